"""Helpers that run the HIP path through the C ABI and bring results to numpy
for comparison with the oracle. No oracle code is imported here."""
from __future__ import annotations

import numpy as np
import torch

from paper_2406_18533_amd import raster as R
from paper_2406_18533_amd import _lib


def to_dev(x: torch.Tensor, dtype=torch.float32) -> torch.Tensor:
    return x.to(dtype).contiguous().cuda()


def estimate_capacity(projected: torch.Tensor) -> int:
    return R.instance_count(projected) + 16


def forward(params: torch.Tensor, cams_list: list, bg=(0.0, 0.0, 0.0), sched_kw=None, capacity=None):
    """Project + bin + render on the GPU. Returns a dict of device tensors."""
    cams = R.Cameras(cams_list)
    proj = R.gs_project(params, cams)
    n = params.shape[1]
    cap = capacity if capacity is not None else estimate_capacity(proj)
    bins = R.Bins(n, cams, cap)
    R.gs_bin_sort(proj, n, cams, bins, check_capacity=True)
    T_all = cams.total_tiles()
    wf = torch.zeros(max(T_all, 1), dtype=torch.int32, device="cuda")
    wb = torch.zeros(max(T_all, 1), dtype=torch.int32, device="cuda")
    sched = None
    if sched_kw:
        sched = R.Sched(cams, **sched_kw)
    rgb, T, last = R.gs_render_fwd(proj, n, bins, cams, bg, sched, tile_work_fwd=wf, tile_work_bwd=wb)
    torch.cuda.synchronize()
    return {"cams": cams, "proj": proj, "bins": bins, "rgb": rgb, "T": T, "last": last, "work_fwd": wf,
            "work_bwd": wb, "n": n, "sched": sched}


def backward(params: torch.Tensor, f: dict, dL_drgb: torch.Tensor, bg=(0.0, 0.0, 0.0), sched=None):
    """Render backward, then transformation backward; returns (grad, record grads)."""
    grad = torch.zeros_like(params)
    dproj = R.gs_render_bwd_pixels(f["proj"], f["n"], f["bins"], f["cams"], f["T"], f["last"], dL_drgb, bg=bg,
                                   sched=sched)
    R.gs_project_bwd(params, f["cams"], f["proj"], dproj, grad, clear=False)
    torch.cuda.synchronize()
    return grad, dproj


def split_views(flat: torch.Tensor, cams_list: list, channels: int):
    out, o = [], 0
    for c in cams_list:
        k = channels * c["width"] * c["height"]
        a = flat[o:o + k].detach().cpu().numpy()
        out.append(a.reshape(channels, c["height"], c["width"]) if channels > 1 else a.reshape(c["height"], c["width"]))
        o += k
    return out


def bins_numpy(f: dict):
    b = f["bins"]
    K = int(b.n_instances.item())
    keys = R.gs_bins_keys64(f["proj"], f["n"], f["cams"], b)
    torch.cuda.synchronize()
    return (keys[:K].cpu().numpy().view(np.uint64), b.ids[:K].cpu().numpy().view(np.uint32),
            b.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)[:f["cams"].total_tiles()])


def proj_fields(proj: torch.Tensor):
    """[V][n][12] -> dict of [V][n] numpy arrays. Records exist only for the
    pairs that touch a tile (the side array's tiles touched > 0); the others
    read as all zero here (radius 0, tiles 0)."""
    p = proj.detach().cpu().numpy().copy()
    tiles = R.projected_side_arrays(proj)[0].cpu().numpy()
    p[tiles == 0] = 0
    names = ["u", "v", "a", "b", "c", "opac", "r", "g", "bl", "radius", "depth", "tiles"]
    return {k: p[..., j] for j, k in enumerate(names)}
