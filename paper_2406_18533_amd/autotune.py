"""Autotuner for the render kernels' launch shape.

For a trainer's workload it times every (scheduler mode, pixels per thread,
LDS chunk) of the forward and of the backward render with HIP events on the
real buffers, picks the fastest of each, and caches the choice in a JSON file
keyed by (architecture, resolution class, Gaussian-count bucket).
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import _lib
from . import raster as R

PX = (1, 2, 4)
CHUNKS = (32, 64, 128, 256)
MODES = (_lib.GS_SCHED_PER_TILE, _lib.GS_SCHED_PERSISTENT, _lib.GS_SCHED_XCD_SPLIT)


def cache_path() -> str:
    return os.environ.get("GSMI_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "gsmi_autotune.json"))


def workload_key(cams: R.Cameras, n: int) -> str:
    pix = cams.total_pixels() / cams.n
    res = "4k+" if pix >= 6e6 else "1080p" if pix >= 1.5e6 else "720p" if pix >= 6e5 else "small"
    nb = 2 ** int(math.log2(max(n, 1)))
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "gfx950").split(":")[0]
    return f"{arch}|{res}|v{cams.n}|n{nb}|modes{len(MODES)}"


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d):
    os.makedirs(os.path.dirname(cache_path()), exist_ok=True)
    tmp = cache_path() + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, cache_path())


def _time(fn, reps: int) -> float:
    fn()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps


def tune(tr, reps: int = 3, use_cache: bool = True, verbose: bool = False) -> dict:
    """Picks (mode, px, chunk) for forward and backward of a BatchedTrainer."""
    key = workload_key(tr.cams, tr.n)
    cache = _load() if use_cache else {}
    if key in cache:
        best = cache[key]
    else:
        tr.warmup()          # every kernel once with the Adam update skipped: the training state is unchanged
        torch.cuda.synchronize()
        R.gs_loss_l1(tr.rgb, tr.targets, tr.cams, tr.loss_buf)
        results = {"fwd": [], "bwd": []}
        for mode in MODES:
            for px in PX:
                for ch in CHUNKS:
                    sf = R.Sched(tr.cams, mode, px, ch, tr.cfg.workers, tr.cfg.queues, tile_cost=tr.work_fwd)
                    sb = R.Sched(tr.cams, mode, px, ch, tr.cfg.workers, tr.cfg.queues, tile_cost=tr.work_bwd)
                    tf = _time(lambda: R.gs_render_fwd(tr.proj, tr.n, tr.bins, tr.cams, tr.cfg.bg, sf, tr.rgb, tr.T,
                                                       tr.last, tr.work_fwd, tr.work_bwd), reps)
                    tb = _time(lambda: R.gs_render_bwd_pixels(tr.proj, tr.n, tr.bins, tr.cams, tr.T, tr.last,
                                                              tr.loss_buf.dL, tr.dproj, tr.cfg.bg, sb), reps)
                    results["fwd"].append((tf, mode, px, ch))
                    results["bwd"].append((tb, mode, px, ch))
                    if verbose:
                        print(f"autotune mode={mode} px={px} chunk={ch}: fwd {tf:.3f} ms bwd {tb:.3f} ms", flush=True)
        tr.dproj.zero_()
        bf, bb = _pick(results["fwd"]), _pick(results["bwd"])
        best = {"fwd": {"mode": bf[1], "px": bf[2], "chunk": bf[3], "ms": bf[0]},
                "bwd": {"mode": bb[1], "px": bb[2], "chunk": bb[3], "ms": bb[0]},
                "table": results}
        if use_cache:
            cache[key] = best
            _save(cache)
    apply(tr, best)
    return best


MARGIN = 0.03   # a cost-driven mode must beat the best per-tile shape by this fraction


def _pick(rows):
    """Fastest (ms, mode, px, chunk); a scheduler mode other than per-tile
    only when it beats the best per-tile shape by MARGIN (timings of a few
    back-to-back launches move by about that much, and the per-tile launch
    needs no plan)."""
    best = min(rows)
    tile = min(r for r in rows if r[1] == _lib.GS_SCHED_PER_TILE)
    return best if best[0] < (1.0 - MARGIN) * tile[0] else tile


def apply(tr, best: dict) -> None:
    f, b = best["fwd"], best["bwd"]
    c = tr.cfg
    c.fwd_shape = (f["px"], f["chunk"])
    c.bwd_shape = (b["px"], b["chunk"])
    c.extra["fwd_mode"], c.extra["bwd_mode"] = f["mode"], b["mode"]
    tr.sched_fwd = R.Sched(tr.cams, f["mode"], f["px"], f["chunk"], c.workers, c.queues, tile_cost=tr.work_fwd)
    tr.sched_bwd = R.Sched(tr.cams, b["mode"], b["px"], b["chunk"], c.workers, c.queues, tile_cost=tr.work_bwd)
    tr.graph = None
