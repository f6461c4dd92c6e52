"""Autotuner for the render kernels' launch shape.

For a trainer's workload it times every launch shape (pixels per thread, LDS
chunk) of the forward and of the backward render on the per-tile launch with
HIP events on the real buffers, then five scheduler modes at the best
shape in interleaved rounds, each pass timed after the kernels that precede
it in the step (a cost-driven mode is taken only when it beats
per-tile by 1%), and caches the choice in a JSON file keyed by (architecture,
resolution class, view count, Gaussian-count bucket).
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
# (LPT-head is left out: its timing here has favoured it while the graph-replayed step ran slower)
MODES = (_lib.GS_SCHED_PER_TILE, _lib.GS_SCHED_PERSISTENT, _lib.GS_SCHED_XCD_SPLIT, _lib.GS_SCHED_LPT,
         _lib.GS_SCHED_XCD_LPT)


def cache_path() -> str:
    return os.environ.get("GSMI_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "gsmi_autotune.json"))


def workload_key(cams: R.Cameras, n: int) -> str:
    pix = cams.total_pixels() / cams.n
    res = "4k+" if pix >= 6e6 else "1080p" if pix >= 1.5e6 else "720p" if pix >= 6e5 else "small"
    nb = 2 ** int(math.log2(max(n, 1)))
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "gfx950").split(":")[0]
    return f"{arch}|{res}|v{cams.n}|n{nb}|modes{len(MODES)}-in-step"


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


def tune(tr, reps: int = 3, use_cache: bool = True, verbose: bool = False, mode_rounds: int = 6) -> dict:
    """Picks (mode, px, chunk) for forward and backward of a BatchedTrainer:
    the launch shape (pixels per thread, LDS chunk) on the per-tile launch,
    then the scheduler mode at that shape, the modes timed in interleaved
    rounds so that drift between launches does not favour one, each pass
    after the kernels that precede it in the step."""
    key = workload_key(tr.cams, tr.n)
    cache = _load() if use_cache else {}
    if key in cache:
        best = cache[key]
    else:
        tr.warmup()          # every kernel once with the Adam update skipped: the training state is unchanged
        torch.cuda.synchronize()
        R.gs_loss_l1(tr.rgb, tr.targets, tr.cams, tr.loss_buf)

        def fwd(sf):
            return lambda: R.gs_render_fwd(tr.proj, tr.n, tr.bins, tr.cams, tr.cfg.bg, sf, tr.rgb, tr.T, tr.last,
                                           tr.work_fwd, tr.work_bwd)

        def bwd(sb):
            return lambda: R.gs_render_bwd_pixels(tr.proj, tr.n, tr.bins, tr.cams, tr.T, tr.last, tr.loss_buf.dL,
                                                  tr.dproj, tr.cfg.bg, sb)

        def sched(mode, px, ch, cost):
            return R.Sched(tr.cams, mode, px, ch, tr.cfg.workers, tr.cfg.queues, tile_cost=cost)
        results = {"fwd": [], "bwd": []}
        for px in PX:
            for ch in CHUNKS:
                tf = _time(fwd(sched(_lib.GS_SCHED_PER_TILE, px, ch, tr.work_fwd)), reps)
                tb = _time(bwd(sched(_lib.GS_SCHED_PER_TILE, px, ch, tr.work_bwd)), reps)
                results["fwd"].append((tf, _lib.GS_SCHED_PER_TILE, px, ch))
                results["bwd"].append((tb, _lib.GS_SCHED_PER_TILE, px, ch))
                if verbose:
                    print(f"autotune px={px} chunk={ch}: fwd {tf:.3f} ms bwd {tb:.3f} ms", flush=True)
        # the modes at the best shapes, each timed where the step runs it:
        # after the transformation and binning (which displace the render
        # kernels' data from the caches) for the forward, after the forward
        # for the backward; modes interleaved over the rounds
        best = {}
        _, _, fpx, fch = min(results["fwd"])
        _, _, bpx, bch = min(results["bwd"])
        fns = {m: (fwd(sched(m, fpx, fch, tr.work_fwd)), bwd(sched(m, bpx, bch, tr.work_bwd))) for m in MODES}
        acc = {m: [0.0, 0.0] for m in MODES}
        for r in range(mode_rounds + 1):
            for m in MODES:
                R.gs_project(tr.P, tr.cams, tr.proj)
                R.gs_bin_sort(tr.proj, tr.n, tr.cams, tr.bins, check_capacity=False)
                tf = _time(fns[m][0], 1)
                tb = _time(fns[m][1], 1)
                tr.dproj.zero_()
                if r > 0:                      # round 0 warms every mode's plan and kernels
                    acc[m][0] += tf / mode_rounds
                    acc[m][1] += tb / mode_rounds
        for j, (p, px, ch) in enumerate((("fwd", fpx, fch), ("bwd", bpx, bch))):
            rows = [(acc[m][j], m, px, ch) for m in MODES]
            results[p + "_modes"] = rows
            b = _pick(rows)
            best[p] = {"mode": b[1], "px": b[2], "chunk": b[3], "ms": b[0]}
        tr.dproj.zero_()
        best["table"] = results
        if use_cache:
            cache[key] = best
            _save(cache)
    apply(tr, best)
    return best


MARGIN = 0.01   # a cost-driven mode must beat the per-tile launch of the same shape by this fraction


def _pick(rows):
    """Fastest (ms, mode, px, chunk); a scheduler mode other than per-tile
    only when it beats the per-tile launch by MARGIN (the per-tile launch
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
