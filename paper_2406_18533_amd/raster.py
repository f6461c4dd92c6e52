"""Torch-facing binding of the C ABI: one function per entry point, with the
same names. PyTorch only supplies device memory and the current stream;
every step runs in the HIP kernels of libgs.so.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _lib
from ._lib import GsAdamHparams, GsBins, GsCamera, GsDensifyHparams, GsSched, check

TILE = 16


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dtype_code(dt: torch.dtype) -> int:
    if dt == torch.float32:
        return _lib.GS_F32
    if dt == torch.float64:
        return _lib.GS_F64
    raise ValueError(f"unsupported dtype {dt}")


def init(device: int = 0) -> None:
    check(_lib.load().gs_init(device))


# --------------------------------------------------------------------------- cameras
class Cameras:
    """A batch of cameras: host structs (image sizes, launch geometry) and a
    device copy (poses read by the kernels). ``update`` rewrites the poses in
    place, which a captured graph then sees on its next replay."""

    def __init__(self, cams: list, device="cuda"):
        self.n = len(cams)
        self.host = (GsCamera * self.n)()
        self._fill(cams)
        raw = bytes(C.string_at(C.addressof(self.host), C.sizeof(self.host)))
        self.dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
        self.dicts = list(cams)

    def _fill(self, cams):
        for k, c in enumerate(cams):
            h = self.host[k]
            h.width, h.height = int(c["width"]), int(c["height"])
            h.fx, h.fy, h.cx, h.cy = float(c["fx"]), float(c["fy"]), float(c["cx"]), float(c["cy"])
            R = np.asarray(c["R"], dtype=np.float64).reshape(9)
            t = np.asarray(c["t"], dtype=np.float64).reshape(3)
            for j in range(9):
                h.R[j] = float(R[j])
            for j in range(3):
                h.t[j] = float(t[j])
            h.znear = float(c["znear"])

    def update(self, cams: list) -> None:
        assert len(cams) == self.n
        for k, c in enumerate(cams):
            assert (int(c["width"]), int(c["height"])) == (self.host[k].width, self.host[k].height)
        self._fill(cams)
        raw = bytes(C.string_at(C.addressof(self.host), C.sizeof(self.host)))
        self.dev.copy_(torch.frombuffer(bytearray(raw), dtype=torch.uint8), non_blocking=False)
        self.dicts = list(cams)

    @property
    def host_ptr(self):
        return C.cast(self.host, C.POINTER(GsCamera))

    @property
    def dev_ptr(self):
        return C.c_void_p(self.dev.data_ptr())

    def sizes(self):
        return [(self.host[k].width, self.host[k].height) for k in range(self.n)]

    def total_tiles(self) -> int:
        return int(_lib.load().gs_total_tiles(self.host_ptr, self.n))

    def total_pixels(self) -> int:
        return int(_lib.load().gs_total_pixels(self.host_ptr, self.n))

    def tile_base(self) -> list:
        out, b = [], 0
        for (w, h) in self.sizes():
            out.append(b)
            b += ((w + TILE - 1) // TILE) * ((h + TILE - 1) // TILE)
        out.append(b)
        return out

    def pix_base(self) -> list:
        out, b = [], 0
        for (w, h) in self.sizes():
            out.append(b)
            b += w * h
        out.append(b)
        return out


# --------------------------------------------------------------------------- buffers
class Bins:
    """Sorted-instance buffers at a fixed capacity (the Z-buffer)."""

    def __init__(self, n: int, cams: Cameras, capacity: int, device="cuda"):
        L = _lib.load()
        self.capacity = int(capacity)
        self.total_tiles = cams.total_tiles()
        self.tile_keys = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.ids = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.ranges = torch.empty(max(self.total_tiles, 1), 2, dtype=torch.int32, device=device)
        self.n_instances = torch.zeros(1, dtype=torch.int64, device=device)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=device)
        wsb = int(L.gs_bin_workspace_bytes(n, cams.n, self.capacity, self.total_tiles))
        self.workspace = torch.empty(max(wsb, 256), dtype=torch.uint8, device=device)
        self.struct = GsBins(self.capacity, self.tile_keys.data_ptr(), self.ids.data_ptr(), self.ranges.data_ptr(),
                             self.n_instances.data_ptr(), self.overflow.data_ptr(), self.workspace.data_ptr(),
                             self.workspace.numel())

    @staticmethod
    def workspace_bytes(n: int, views: int, capacity: int, total_tiles: int) -> int:
        return int(_lib.load().gs_bin_workspace_bytes(n, views, capacity, total_tiles))


class Sched:
    """Launch shape of the render kernels (+ the scheduler's workspace for the
    persistent, XCD-split and LPT modes)."""

    def __init__(self, cams: Cameras | None = None, mode: int = _lib.GS_SCHED_PER_TILE, px_per_thread: int = 1,
                 chunk: int = 64, workers: int = 0, queues: int = 64, tile_cost: torch.Tensor | None = None,
                 device="cuda"):
        self.mode, self.px, self.chunk, self.workers, self.queues = mode, px_per_thread, chunk, workers, queues
        self.tile_cost = tile_cost
        self.workspace = None
        wsb = 0
        if mode in (_lib.GS_SCHED_PERSISTENT, _lib.GS_SCHED_XCD_SPLIT, _lib.GS_SCHED_LPT, _lib.GS_SCHED_XCD_LPT,
                    _lib.GS_SCHED_LPT_HEAD):
            assert cams is not None
            q = queues if mode == _lib.GS_SCHED_PERSISTENT else 8
            wsb = int(_lib.load().gs_sched_workspace_bytes(cams.total_tiles(), q))
            self.workspace = torch.empty(wsb, dtype=torch.uint8, device=device)
        self.struct = GsSched(mode, px_per_thread, chunk, workers, queues, 0,
                              tile_cost.data_ptr() if tile_cost is not None else None,
                              self.workspace.data_ptr() if self.workspace is not None else None, wsb)

    def with_cost(self, tile_cost: torch.Tensor | None) -> "Sched":
        self.tile_cost = tile_cost
        self.struct.tile_cost = tile_cost.data_ptr() if tile_cost is not None else None
        return self


def _bg(bg):
    return (C.c_float * 3)(*[float(x) for x in bg])


def alloc_projected(n: int, views: int, dtype=torch.float32, device="cuda") -> torch.Tensor:
    """A projected buffer of gs_projected_bytes(n, views); returns the
    [views][n][12] record view (the planar side arrays follow it in the same
    allocation)."""
    nbytes = int(_lib.load().gs_projected_bytes(_dtype_code(dtype), n, views))
    item = torch.empty(0, dtype=dtype).element_size()
    flat = torch.empty(max((nbytes + item - 1) // item, 1), dtype=dtype, device=device)
    return flat[: views * n * _lib.GS_REC].view(views, n, _lib.GS_REC)


def projected_side_arrays(projected: torch.Tensor):
    """(tiles touched, FP32 depth bits) planar side arrays, each [views][n] int32."""
    V, n, _ = projected.shape
    item = projected.element_size()
    total = V * n * _lib.GS_REC + (V * n * 8 + item - 1) // item
    flat = torch.as_strided(projected, (total,), (1,), projected.storage_offset())
    side = flat[V * n * _lib.GS_REC:].view(torch.int32)[: 2 * V * n]
    return side[: V * n].view(V, n), side[V * n:].view(V, n)


def instance_count(projected: torch.Tensor) -> int:
    """Sorted instances the projected buffer will produce: the sum of the
    tiles touched over every (view, Gaussian) (a host synchronisation)."""
    tiles, _ = projected_side_arrays(projected)
    return int(tiles.sum(dtype=torch.int64).item())


def records_on_screen(projected: torch.Tensor) -> torch.Tensor:
    """[views][n] bool: the pairs whose record gs_project wrote (tiles touched > 0)."""
    tiles, _ = projected_side_arrays(projected)
    return tiles > 0


# --------------------------------------------------------------------------- entry points
def gs_project(params: torch.Tensor, cams: Cameras, projected: torch.Tensor | None = None, stream=None):
    """Records [views][n][12] (see include/gs.h gs_project)."""
    assert params.is_cuda and params.is_contiguous() and params.shape[0] == 59
    n = params.shape[1]
    if projected is None:
        projected = alloc_projected(n, cams.n, params.dtype, params.device)
    check(_lib.load().gs_project(_dtype_code(params.dtype), _ptr(params), n, cams.dev_ptr, cams.host_ptr, cams.n,
                                 _ptr(projected), _stream(stream)))
    return projected


def gs_bin_sort(projected: torch.Tensor, n: int, cams: Cameras, bins: Bins, check_capacity: bool = True,
                stream=None) -> None:
    check(_lib.load().gs_bin_sort(_dtype_code(projected.dtype), _ptr(projected), n, cams.host_ptr, cams.n,
                                  C.byref(bins.struct), int(check_capacity), _stream(stream)))


def gs_bins_keys64(projected: torch.Tensor, n: int, cams: Cameras, bins: Bins, stream=None) -> torch.Tensor:
    out = torch.zeros(max(bins.capacity, 1), dtype=torch.int64, device=projected.device)
    check(_lib.load().gs_bins_keys64(_dtype_code(projected.dtype), _ptr(projected), n, cams.host_ptr, cams.n,
                                     C.byref(bins.struct), _ptr(out), _stream(stream)))
    return out


def gs_render_fwd(projected: torch.Tensor, n: int, bins: Bins, cams: Cameras, bg=(0.0, 0.0, 0.0),
                  sched: Sched | None = None, rgb=None, final_T=None, last=None, tile_work_fwd=None,
                  tile_work_bwd=None, pair_stats=None, stream=None):
    P = cams.total_pixels()
    dev = projected.device
    if rgb is None:
        rgb = torch.empty(3 * P, dtype=projected.dtype, device=dev)
    if final_T is None:
        final_T = torch.empty(P, dtype=projected.dtype, device=dev)
    if last is None:
        last = torch.empty(P, dtype=torch.int32, device=dev)
    check(_lib.load().gs_render_fwd(_dtype_code(projected.dtype), _ptr(projected), n, C.byref(bins.struct),
                                    cams.host_ptr, cams.n, _bg(bg), C.byref(sched.struct) if sched else None,
                                    _ptr(rgb), _ptr(final_T), _ptr(last), _ptr(tile_work_fwd), _ptr(tile_work_bwd),
                                    _ptr(pair_stats), _stream(stream)))
    return rgb, final_T, last


def gs_render_fwd_l1(projected: torch.Tensor, n: int, bins: Bins, cams: Cameras, target: torch.Tensor,
                     buf: "LossBuffers", bg=(0.0, 0.0, 0.0), sched: Sched | None = None, rgb=None, final_T=None,
                     last=None, tile_work_fwd=None, tile_work_bwd=None, scale: float = 1.0, stream=None):
    """Render forward with the L1 loss fused in: also writes buf.dL and buf.loss."""
    P = cams.total_pixels()
    dev = projected.device
    if rgb is None:
        rgb = torch.empty(3 * P, dtype=projected.dtype, device=dev)
    if final_T is None:
        final_T = torch.empty(P, dtype=projected.dtype, device=dev)
    if last is None:
        last = torch.empty(P, dtype=torch.int32, device=dev)
    check(_lib.load().gs_render_fwd_l1(_dtype_code(projected.dtype), _ptr(projected), n, C.byref(bins.struct),
                                       cams.host_ptr, cams.n, _bg(bg), C.byref(sched.struct) if sched else None,
                                       _ptr(rgb), _ptr(final_T), _ptr(last), _ptr(tile_work_fwd),
                                       _ptr(tile_work_bwd), _ptr(target), float(scale), _ptr(buf.dL),
                                       _ptr(buf.loss), _ptr(buf.workspace), buf.workspace.numel(), _stream(stream)))
    return rgb, final_T, last


def gs_render_fwd_l1_noalloc(projected: torch.Tensor, n: int, bins: Bins, cams: Cameras, target: torch.Tensor,
                             rgb: torch.Tensor, final_T: torch.Tensor, last: torch.Tensor, dL_drgb: torch.Tensor,
                             loss: torch.Tensor, bg=(0.0, 0.0, 0.0), sched: Sched | None = None, tile_work_fwd=None,
                             tile_work_bwd=None, scale: float = 1.0, stream=None):
    """gs_render_fwd_l1 on the library's fixed per-device scratch: the caller
    passes every output (nothing is allocated here or in the library)."""
    check(_lib.load().gs_render_fwd_l1_noalloc(_dtype_code(projected.dtype), _ptr(projected), n,
                                               C.byref(bins.struct), cams.host_ptr, cams.n, _bg(bg),
                                               C.byref(sched.struct) if sched else None, _ptr(rgb), _ptr(final_T),
                                               _ptr(last), _ptr(tile_work_fwd), _ptr(tile_work_bwd), _ptr(target),
                                               float(scale), _ptr(dL_drgb), _ptr(loss), _stream(stream)))
    return rgb, final_T, last


def gs_render_bwd(params: torch.Tensor, projected: torch.Tensor, bins: Bins, cams: Cameras, final_T, last, dL_drgb,
                  grad: torch.Tensor, bg=(0.0, 0.0, 0.0), sched: Sched | None = None, dprojected=None, stream=None):
    """Both backward halves; accumulates (+=) into ``grad``. ``dprojected``
    must be all zero on entry and is all zero on return."""
    n = params.shape[1]
    if dprojected is None:
        dprojected = torch.zeros(cams.n, n, _lib.GS_REC, dtype=params.dtype, device=params.device)
    check(_lib.load().gs_render_bwd(_dtype_code(params.dtype), _ptr(params), n, _ptr(projected),
                                    C.byref(bins.struct), cams.dev_ptr, cams.host_ptr, cams.n, _bg(bg),
                                    C.byref(sched.struct) if sched else None, _ptr(final_T), _ptr(last),
                                    _ptr(dL_drgb), _ptr(dprojected), _ptr(grad), _stream(stream)))
    return dprojected


def gs_render_bwd_pixels(projected: torch.Tensor, n: int, bins: Bins, cams: Cameras, final_T, last, dL_drgb,
                         dprojected: torch.Tensor | None = None, bg=(0.0, 0.0, 0.0), sched: Sched | None = None,
                         stream=None):
    """Render backward: adds the per-(view, Gaussian) record gradients into
    ``dprojected`` (zeroed here when not given)."""
    if dprojected is None:
        dprojected = torch.zeros(cams.n, n, _lib.GS_REC, dtype=projected.dtype, device=projected.device)
    check(_lib.load().gs_render_bwd_pixels(_dtype_code(projected.dtype), _ptr(projected), n, C.byref(bins.struct),
                                           cams.host_ptr, cams.n, _bg(bg), C.byref(sched.struct) if sched else None,
                                           _ptr(final_T), _ptr(last), _ptr(dL_drgb), _ptr(dprojected),
                                           _stream(stream)))
    return dprojected


def gs_project_bwd(params: torch.Tensor, cams: Cameras, projected: torch.Tensor, dprojected: torch.Tensor,
                   grad: torch.Tensor, clear: bool = False, stream=None):
    n = params.shape[1]
    check(_lib.load().gs_project_bwd(_dtype_code(params.dtype), _ptr(params), n, cams.dev_ptr, cams.host_ptr,
                                     cams.n, _ptr(projected), _ptr(dprojected), int(clear), _ptr(grad),
                                     _stream(stream)))
    return grad


class LossBuffers:
    def __init__(self, cams: Cameras, dtype=torch.float32, device="cuda"):
        P = cams.total_pixels()
        self.dL = torch.empty(3 * P, dtype=dtype, device=device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        wsb = int(_lib.load().gs_loss_workspace_bytes(cams.host_ptr, cams.n))
        self.workspace = torch.empty(wsb, dtype=torch.uint8, device=device)


def gs_loss_l1(rgb: torch.Tensor, target: torch.Tensor, cams: Cameras, buf: LossBuffers, scale: float = 1.0,
               stream=None):
    check(_lib.load().gs_loss_l1(_dtype_code(rgb.dtype), _ptr(rgb), _ptr(target), cams.host_ptr, cams.n,
                                 float(scale), _ptr(buf.dL), _ptr(buf.loss), _ptr(buf.workspace),
                                 buf.workspace.numel(), _stream(stream)))
    return buf.loss, buf.dL


class DssimBuffers:
    """Outputs and workspace of gs_loss_l1_dssim for one camera set."""

    def __init__(self, cams: Cameras, dtype=torch.float32, device="cuda"):
        P = cams.total_pixels()
        self.dL = torch.empty(3 * P, dtype=dtype, device=device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        wsb = int(_lib.load().gs_loss_dssim_workspace_bytes(_dtype_code(dtype), cams.host_ptr, cams.n))
        if wsb == 0:
            check(_lib.GS_ERR_ARG)
        self.workspace = torch.empty(wsb, dtype=torch.uint8, device=device)


def gs_loss_l1_dssim(rgb: torch.Tensor, target: torch.Tensor, cams: Cameras, buf: DssimBuffers, lam: float = 0.2,
                     scale: float = 1.0, stream=None):
    check(_lib.load().gs_loss_l1_dssim(_dtype_code(rgb.dtype), _ptr(rgb), _ptr(target), cams.host_ptr, cams.n,
                                       float(lam), float(scale), _ptr(buf.dL), _ptr(buf.loss),
                                       _ptr(buf.workspace), buf.workspace.numel(), _stream(stream)))
    return buf.loss, buf.dL


def adam_hparams(lr6, beta1=0.9, beta2=0.999, eps=1e-15, batch_size=1, zero_grad=True) -> GsAdamHparams:
    return GsAdamHparams((C.c_double * 6)(*[float(x) for x in lr6]), beta1, beta2, eps, int(batch_size),
                         int(zero_grad))


def gs_adam_step(params, grad, m, v, h: GsAdamHparams, step: torch.Tensor, scratch: torch.Tensor,
                 skip_flag: torch.Tensor | None = None, stream=None):
    n = params.shape[1]
    check(_lib.load().gs_adam_step(_dtype_code(params.dtype), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), n,
                                   C.byref(h), _ptr(step), _ptr(scratch), _ptr(skip_flag), _stream(stream)))


def gs_project_bwd_adam(params, cams: Cameras, projected: torch.Tensor, dprojected: torch.Tensor, grad, m, v,
                        h: GsAdamHparams, step: torch.Tensor, scratch: torch.Tensor,
                        skip_flag: torch.Tensor | None = None, stream=None):
    """Transformation backward + Adam in one pass (grad: all-zero scratch)."""
    n = params.shape[1]
    check(_lib.load().gs_project_bwd_adam(_dtype_code(params.dtype), _ptr(params), n, cams.dev_ptr, cams.host_ptr,
                                          cams.n, _ptr(projected), _ptr(dprojected), _ptr(grad), _ptr(m), _ptr(v),
                                          C.byref(h), _ptr(step), _ptr(scratch), _ptr(skip_flag),
                                          _stream(stream)))


# --------------------------------------------------------------------------- densification
def densify_hparams(grad_threshold: float, split_log_scale: float, prune_logit: float,
                    prune_log_scale: float = math.inf) -> GsDensifyHparams:
    return GsDensifyHparams(float(grad_threshold), float(split_log_scale), float(prune_logit),
                            float(prune_log_scale))


def gs_densify_stats(projected: torch.Tensor, dprojected: torch.Tensor, n: int, views: int, accum: torch.Tensor,
                     count: torch.Tensor, scale: float = 1.0, stream=None):
    assert accum.dtype == torch.float32 and count.dtype == torch.int32 and accum.numel() >= n and count.numel() >= n
    check(_lib.load().gs_densify_stats(_dtype_code(dprojected.dtype), _ptr(projected), _ptr(dprojected), int(n),
                                       int(views), float(scale), _ptr(accum), _ptr(count), _stream(stream)))
    return accum, count


class DensifyPlan:
    """Workspace and device counts of one densification."""

    def __init__(self, n: int, device="cuda"):
        self.n = int(n)
        wsb = int(_lib.load().gs_densify_workspace_bytes(self.n))
        self.workspace = torch.empty(max(wsb, 256), dtype=torch.uint8, device=device)
        self.counts = torch.zeros(3, dtype=torch.int64, device=device)


def gs_densify_plan(params: torch.Tensor, accum: torch.Tensor, count: torch.Tensor, h: GsDensifyHparams,
                    plan: DensifyPlan, stream=None) -> DensifyPlan:
    n = params.shape[1]
    assert n == plan.n and params.is_contiguous()
    check(_lib.load().gs_densify_plan(_dtype_code(params.dtype), _ptr(params), n, _ptr(accum), _ptr(count),
                                      C.byref(h), _ptr(plan.workspace), plan.workspace.numel(), _ptr(plan.counts),
                                      _stream(stream)))
    return plan


def gs_densify_apply(params, m, v, noise: torch.Tensor, plan: DensifyPlan, n_out: int, stream=None):
    """New (params, m, v) [59][n_out]; n_out = K + C + 2 S from the plan's counts."""
    n = params.shape[1]
    assert noise.dtype == params.dtype and noise.numel() == 6 * n
    po = torch.empty(59, n_out, dtype=params.dtype, device=params.device)
    mo, vo = torch.empty_like(po), torch.empty_like(po)
    check(_lib.load().gs_densify_apply(_dtype_code(params.dtype), _ptr(params), _ptr(m), _ptr(v), n, _ptr(noise),
                                       _ptr(plan.workspace), plan.workspace.numel(), _ptr(po), _ptr(mo), _ptr(vo),
                                       int(n_out), _stream(stream)))
    return po, mo, vo


def gs_reset_opacity(params, m, v, max_logit: float, stream=None):
    check(_lib.load().gs_reset_opacity(_dtype_code(params.dtype), _ptr(params), _ptr(m), _ptr(v), params.shape[1],
                                       float(max_logit), _stream(stream)))


def gs_sched_plan(sched: Sched, cams: Cameras, dp_out: torch.Tensor | None = None, stream=None):
    check(_lib.load().gs_sched_plan(C.byref(sched.struct), cams.host_ptr, cams.n, _ptr(dp_out), _stream(stream)))
