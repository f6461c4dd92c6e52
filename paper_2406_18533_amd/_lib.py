"""ctypes view of the C ABI in include/gs.h (libgs.so). Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs.so")

GS_OK, GS_ERR_ARG, GS_ERR_CAPACITY, GS_ERR_HIP, GS_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
GS_F32, GS_F64 = 0, 1
GS_SCHED_PER_TILE, GS_SCHED_PERSISTENT, GS_SCHED_XCD_SPLIT, GS_SCHED_LPT, GS_SCHED_XCD_LPT = 0, 1, 2, 3, 4
GS_SCHED_LPT_HEAD = 5
GS_REC = 12
GS_MAX_VIEWS = 64

EXPORTS = [
    "gs_version", "gs_last_error", "gs_init", "gs_projected_bytes", "gs_total_tiles", "gs_total_pixels",
    "gs_bin_workspace_bytes", "gs_sched_workspace_bytes", "gs_loss_workspace_bytes",
    "gs_loss_dssim_workspace_bytes", "gs_project",
    "gs_bin_sort", "gs_bins_keys64", "gs_render_fwd", "gs_render_bwd", "gs_render_bwd_pixels", "gs_project_bwd",
    "gs_loss_l1", "gs_loss_l1_dssim", "gs_render_fwd_l1", "gs_render_fwd_l1_noalloc", "gs_adam_step", "gs_project_bwd_adam", "gs_sched_plan",
    "gs_densify_stats", "gs_densify_workspace_bytes", "gs_densify_plan", "gs_densify_apply", "gs_reset_opacity",
]


class GsCamera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("R", C.c_double * 9), ("t", C.c_double * 3),
                ("znear", C.c_double)]


class GsBins(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("tile_keys", C.c_void_p), ("ids", C.c_void_p), ("ranges", C.c_void_p),
                ("n_instances", C.c_void_p), ("overflow", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t)]


class GsSched(C.Structure):
    _fields_ = [("mode", C.c_int32), ("px_per_thread", C.c_int32), ("chunk", C.c_int32), ("workers", C.c_int32),
                ("queues", C.c_int32), ("reserved", C.c_int32), ("tile_cost", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t)]


class GsAdamHparams(C.Structure):
    _fields_ = [("lr", C.c_double * 6), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("batch_size", C.c_int32), ("zero_grad", C.c_int32)]


class GsDensifyHparams(C.Structure):
    _fields_ = [("grad_threshold", C.c_double), ("split_log_scale", C.c_double), ("prune_logit", C.c_double),
                ("prune_log_scale", C.c_double)]


class GsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gs status {status}: {msg}")
        self.status = status


_lib = None


def load() -> C.CDLL:
    """Loads libgs.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    L = C.CDLL(LIB_PATH)
    p, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    cam_p = C.POINTER(GsCamera)
    sig = {
        "gs_version": ([], C.c_char_p),
        "gs_last_error": ([], C.c_char_p),
        "gs_init": ([i32], i32),
        "gs_projected_bytes": ([i32, i64, i32], sz),
        "gs_total_tiles": ([cam_p, i32], i64),
        "gs_total_pixels": ([cam_p, i32], i64),
        "gs_bin_workspace_bytes": ([i64, i32, i64, i64], sz),
        "gs_sched_workspace_bytes": ([i64, i32], sz),
        "gs_loss_workspace_bytes": ([cam_p, i32], sz),
        "gs_loss_dssim_workspace_bytes": ([i32, cam_p, i32], sz),
        "gs_project": ([i32, p, i64, p, cam_p, i32, p, p], i32),
        "gs_bin_sort": ([i32, p, i64, cam_p, i32, C.POINTER(GsBins), i32, p], i32),
        "gs_bins_keys64": ([i32, p, i64, cam_p, i32, C.POINTER(GsBins), p, p], i32),
        "gs_render_fwd": ([i32, p, i64, C.POINTER(GsBins), cam_p, i32, C.POINTER(C.c_float), C.POINTER(GsSched),
                           p, p, p, p, p, p, p], i32),
        "gs_render_fwd_l1": ([i32, p, i64, C.POINTER(GsBins), cam_p, i32, C.POINTER(C.c_float), C.POINTER(GsSched),
                              p, p, p, p, p, p, C.c_double, p, p, p, sz, p], i32),
        "gs_render_fwd_l1_noalloc": ([i32, p, i64, C.POINTER(GsBins), cam_p, i32, C.POINTER(C.c_float),
                                      C.POINTER(GsSched), p, p, p, p, p, p, C.c_double, p, p, p], i32),
        "gs_render_bwd": ([i32, p, i64, p, C.POINTER(GsBins), p, cam_p, i32, C.POINTER(C.c_float),
                           C.POINTER(GsSched), p, p, p, p, p, p], i32),
        "gs_render_bwd_pixels": ([i32, p, i64, C.POINTER(GsBins), cam_p, i32, C.POINTER(C.c_float),
                                  C.POINTER(GsSched), p, p, p, p, p], i32),
        "gs_project_bwd": ([i32, p, i64, p, cam_p, i32, p, p, i32, p, p], i32),
        "gs_loss_l1": ([i32, p, p, cam_p, i32, C.c_double, p, p, p, sz, p], i32),
        "gs_loss_l1_dssim": ([i32, p, p, cam_p, i32, C.c_double, C.c_double, p, p, p, sz, p], i32),
        "gs_adam_step": ([i32, p, p, p, p, i64, C.POINTER(GsAdamHparams), p, p, p, p], i32),
        "gs_project_bwd_adam": ([i32, p, i64, p, cam_p, i32, p, p, p, p, p, C.POINTER(GsAdamHparams), p, p, p, p],
                                i32),
        "gs_sched_plan": ([C.POINTER(GsSched), cam_p, i32, p, p], i32),
        "gs_densify_stats": ([i32, p, p, i64, i32, C.c_double, p, p, p], i32),
        "gs_densify_workspace_bytes": ([i64], sz),
        "gs_densify_plan": ([i32, p, i64, p, p, C.POINTER(GsDensifyHparams), p, sz, p, p], i32),
        "gs_densify_apply": ([i32, p, p, p, i64, p, p, sz, p, p, p, i64, p], i32),
        "gs_reset_opacity": ([i32, p, p, p, i64, C.c_double, p], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(status: int) -> None:
    if status != GS_OK:
        raise GsError(status, load().gs_last_error().decode())
