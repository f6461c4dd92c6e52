"""Benchmark of the batched 3DGS training step on one MI355X.

Default workload: 1,000,000 clustered Gaussians, a batch of 16 views at
1920x1080 (synthetic, seeded), L1 loss against a jittered-scene target, Adam
with lr * sqrt(16) and beta^16. One step = transformation of every view,
binning + sort, render forward, loss, render backward, transformation
backward, Adam - the whole hot path, replayed as one captured HIP graph.

Prints one JSON line: train views/s (value), the plain per-view path's
views/s beside it, per-entry-point timings, the roofline of the dominant
kernel and the FP64 CPU oracle timed on a sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name: str):
    from synthetic import scenes
    if name == "batched_1080p":
        return scenes.batched_1080p()
    if name == "aerial_4k":
        return scenes.aerial_4k()
    if name == "small":
        return scenes.Workload("small_4x256", scenes.clustered_gaussians(100_000, 1),
                               scenes.sphere_cameras(4, 12, 256, 256), None)
    raise SystemExit(f"unknown workload {name}")


def render_targets(P_target, cams_list):
    """Target images: the jittered scene rendered by the same rasterizer (setup, untimed)."""
    import torch
    from paper_2406_18533_amd import raster as R
    cams = R.Cameras(cams_list)
    proj = R.gs_project(P_target, cams)
    K = R.instance_count(proj)
    bins = R.Bins(P_target.shape[1], cams, K + 1024)
    R.gs_bin_sort(proj, P_target.shape[1], cams, bins)
    rgb, _, _ = R.gs_render_fwd(proj, P_target.shape[1], bins, cams)
    torch.cuda.synchronize()
    del bins, proj
    return rgb


def entry_timings(tr, reps: int):
    """Average duration of every entry point of the step, from HIP events on
    the stream the kernels run on (eager steps, same kernels as the graph)."""
    import torch
    from paper_2406_18533_amd import raster as R
    fused = tr.cfg.fused_adam
    fused_loss = tr.cfg.fused_loss
    names = ["gs_project", "gs_bin_sort"]
    names += ["gs_render_fwd_l1"] if fused_loss else ["gs_render_fwd", "gs_loss_l1"]
    names += ["gs_render_bwd_pixels"]
    names += ["gs_project_bwd_adam"] if fused else ["gs_project_bwd", "gs_adam_step"]
    acc = {k: 0.0 for k in names}
    c = tr.cfg
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        ev[0].record()
        R.gs_project(tr.P, tr.cams, tr.proj)
        ev[1].record()
        R.gs_bin_sort(tr.proj, tr.n, tr.cams, tr.bins, check_capacity=False)
        ev[2].record()
        e = 3
        if fused_loss:
            R.gs_render_fwd_l1(tr.proj, tr.n, tr.bins, tr.cams, tr.targets, tr.loss_buf, c.bg, tr.sched_fwd, tr.rgb,
                               tr.T, tr.last, tr.work_fwd, tr.work_bwd)
        else:
            R.gs_render_fwd(tr.proj, tr.n, tr.bins, tr.cams, c.bg, tr.sched_fwd, tr.rgb, tr.T, tr.last,
                            tr.work_fwd, tr.work_bwd)
            ev[e].record()
            e += 1
            R.gs_loss_l1(tr.rgb, tr.targets, tr.cams, tr.loss_buf)
        ev[e].record()
        e += 1
        R.gs_render_bwd_pixels(tr.proj, tr.n, tr.bins, tr.cams, tr.T, tr.last, tr.loss_buf.dL, tr.dproj, c.bg,
                               tr.sched_bwd)
        ev[e].record()
        if fused:
            R.gs_project_bwd_adam(tr.P, tr.cams, tr.proj, tr.dproj, tr.grad, tr.m, tr.v, tr.hp, tr.step_dev,
                                  tr.scratch, skip_flag=tr.bins.overflow)
        else:
            R.gs_project_bwd(tr.P, tr.cams, tr.proj, tr.dproj, tr.grad, clear=True)
            ev[e + 1].record()
            R.gs_adam_step(tr.P, tr.grad, tr.m, tr.v, tr.hp, tr.step_dev, tr.scratch, skip_flag=tr.bins.overflow)
        ev[len(names)].record()
        torch.cuda.synchronize()
        for j, k in enumerate(names):
            acc[k] += ev[j].elapsed_time(ev[j + 1])
    return {k: v / reps for k, v in acc.items()}


def dssim_side(tr, P, cams_list, targets, steps: int, warmup: int, lam: float = 0.2):
    """The L1 + D-SSIM loss: its entry's average time on the step's rendered
    images (HIP events) against the HBM roofline of its algorithmic bytes
    (44 per image value: the forward reads both images and writes three
    coefficient maps, the backward reads the maps and both images and writes
    the gradient), and the whole step with that loss in place of L1."""
    import dataclasses
    import torch
    from paper_2406_18533_amd import raster as R
    from paper_2406_18533_amd import train
    buf = R.DssimBuffers(tr.cams)
    R.gs_loss_l1_dssim(tr.rgb, tr.targets, tr.cams, buf, lam=lam)
    c0 = tr.cams.dicts[0]
    per = 3 * c0["width"] * c0["height"]
    shape = (3, c0["height"], c0["width"])
    sample = (tr.rgb[:per].double().cpu().numpy().reshape(shape),
              tr.targets[:per].double().cpu().numpy().reshape(shape), tr.V)
    reps = 10
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        R.gs_loss_l1_dssim(tr.rgb, tr.targets, tr.cams, buf, lam=lam)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    nbytes = 44 * 3 * tr.cams.total_pixels()
    gbs = nbytes / (ms / 1e3) / 1e9
    del buf
    t2 = train.BatchedTrainer(P.clone(), cams_list, targets, dataclasses.replace(tr.cfg, ssim_lambda=lam, extra=dict(tr.cfg.extra)))
    for _ in range(max(warmup, 1)):
        t2.step()
        t2.check_overflow()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t2.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out = {"lambda": lam, "views_per_s": round(t2.V * steps / (t1 - t0), 2),
           "ms_per_step": round((t1 - t0) * 1e3 / steps, 4), "loss_ms": round(ms, 4),
           "loss_bytes": nbytes, "loss_GBps": round(gbs, 1), "loss_hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
           "loss_traffic": measured_traffic("gs_loss_l1_dssim")}
    del t2
    return out, sample


def densify_side(tr, reps: int = 5):
    """One densification of the step's Gaussians after a step that
    accumulates the statistic (selection at its 90th percentile, split above
    the median largest log-scale, prune below opacity 0.005): average times
    of the plan and apply entries (HIP events; the host reads the counts in
    between) and the HBM rate of their algorithmic bytes: plan 25 B per
    Gaussian (four parameter rows, the statistic, the class byte); apply the
    class byte and 236 B of parameters per Gaussian, 472 B of moments per kept
    original, 24 B of noise per split pair and 708 B written per output
    Gaussian."""
    import math
    import torch
    from paper_2406_18533_amd import raster as R
    tr.enable_densify_stats()
    tr.step_eager()
    torch.cuda.synchronize()
    acc, cnt = tr.stats
    seen = cnt > 0
    thr = float(torch.quantile((acc[seen] / cnt[seen]).float(), 0.9))
    split_ls = float(torch.quantile(tr.P[3:6].max(dim=0).values.float(), 0.5))
    h = R.densify_hparams(thr, split_ls, math.log(0.005 / 0.995))
    gen = torch.Generator(device="cuda").manual_seed(0)
    noise = torch.randn(2, 3, tr.n, generator=gen, device="cuda")
    plan = R.DensifyPlan(tr.n)
    t_plan = t_apply = 0.0
    for _ in range(reps + 1):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        R.gs_densify_plan(tr.P, acc, cnt, h, plan)
        ev[1].record()
        K, C, S = (int(x) for x in plan.counts.cpu())
        ev[2].record()
        out = R.gs_densify_apply(tr.P, tr.m, tr.v, noise, plan, K + C + 2 * S)
        ev[3].record()
        torch.cuda.synchronize()
        del out
        if _:
            t_plan += ev[0].elapsed_time(ev[1]) / reps
            t_apply += ev[2].elapsed_time(ev[3]) / reps
    sample = {"P": tr.P.double().cpu().numpy(), "m": tr.m.double().cpu().numpy(), "v": tr.v.double().cpu().numpy(),
              "accum": acc.double().cpu().numpy(), "count": cnt.cpu().numpy(),
              "noise": noise.double().cpu().numpy(),
              "hp": (h.grad_threshold, h.split_log_scale, h.prune_logit, h.prune_log_scale)}
    n, n_out = tr.n, K + C + 2 * S
    b_plan = 25 * n
    b_apply = n + 236 * n + 472 * K + 24 * S + 708 * n_out
    tr.enable_densify_stats(False)
    return ({"gaussians": n, "kept": K, "clones": C, "split_pairs": S, "output": n_out,
            "plan_ms": round(t_plan, 4), "apply_ms": round(t_apply, 4),
            "plan_GBps": round(b_plan / (t_plan / 1e3) / 1e9, 1),
            "apply_GBps": round(b_apply / (t_apply / 1e3) / 1e9, 1),
            "apply_hbm_frac": round(b_apply / (t_apply / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}, sample)


def workload_counts(tr):
    """Exact counts of the step's work units, for the algorithmic bytes/flops."""
    import torch
    from paper_2406_18533_amd import raster as R
    stats = torch.zeros(2, dtype=torch.int64, device="cuda")
    R.gs_project(tr.P, tr.cams, tr.proj)
    R.gs_bin_sort(tr.proj, tr.n, tr.cams, tr.bins, check_capacity=True)
    R.gs_render_fwd(tr.proj, tr.n, tr.bins, tr.cams, tr.cfg.bg, tr.sched_fwd, tr.rgb, tr.T, tr.last,
                    tr.work_fwd, tr.work_bwd, pair_stats=stats)
    torch.cuda.synchronize()
    tiles, _ = R.projected_side_arrays(tr.proj)
    return {
        "N": tr.n, "V": tr.V, "pixels": tr.cams.total_pixels(), "tiles": tr.cams.total_tiles(),
        "K": int(tr.bins.n_instances.item()),
        "records_on_screen": int((tiles > 0).sum().item()),
        "gaussians_on_screen": int((tiles > 0).any(dim=0).sum().item()),
        "pairs_evaluated_fwd": int(stats[0].item()),
        "pairs_blended": int(stats[1].item()),
        "pairs_evaluated_bwd": int(tr.last.double().sum().item()),
    }


def algorithmic(c: dict) -> dict:
    """Algorithmic work of each entry point (bytes the method must move, or
    FP32 flops it must execute), per launch, from the exact counts."""
    VN, M, K, T, Pn = c["V"] * c["N"], c["records_on_screen"], c["K"], c["tiles"], c["pixels"]
    N, Ns = c["N"], c["gaussians_on_screen"]
    radix_passes_depth = 4
    return {
        # read means of all, the other 224 B of Gaussians on screen; write a 48-B record per on-screen
        # (view, Gaussian) and a 4-B "no tiles" marker for the rest
        "gs_project": ("hbm", 12 * N + 224 * Ns + 48 * M + 4 * (VN - M)),
        # compaction (4 B flag + 4 B depth in, 8 B out per pair), 4 depth passes over pairs (20 B each),
        # offsets (16 B per pair), emission (20 B per pair + a 2-B tile key and 4-B id per instance),
        # 2 tile passes over instances (2-B key counted, then 2+4 B read and written: 14 B; the last
        # pass writes the 4-B global tile ids: 16 B), ranges (4 B per instance + 8 B per tile)
        "gs_bin_sort": ("hbm", 4 * VN + 12 * M + radix_passes_depth * 20 * M + 16 * M + 20 * M + 6 * K
                        + 14 * K + 16 * K + 4 * K + 8 * T),
        # 17 flops to evaluate a pair (offset, circle, quadratic form, exp, opacity), 9 more to blend it
        "gs_render_fwd": ("alu", 17 * c["pairs_evaluated_fwd"] + 9 * c["pairs_blended"]),
        # the same, with the L1 loss and its gradient (a few flops per pixel channel) in the output stage
        "gs_render_fwd_l1": ("alu", 17 * c["pairs_evaluated_fwd"] + 9 * c["pairs_blended"] + 12 * c["pixels"]),
        "gs_loss_l1": ("hbm", 36 * Pn),
        # re-evaluate every pair up to `last` (17 flops), 53 more for each blended pair's gradients
        "gs_render_bwd_pixels": ("alu", 17 * c["pairs_evaluated_bwd"] + 53 * c["pairs_blended"]),
        # params of on-screen Gaussians (236 B), their gradient read + write (472 B), tiles field of every
        # record (4 B), the 36-B record gradient read and cleared per on-screen record
        "gs_project_bwd": ("hbm", 708 * Ns + 4 * VN + 72 * M),
        # read p, g, m, v and write p, m, v (+ g cleared): 32 B per parameter float, 59 per Gaussian
        "gs_adam_step": ("hbm", 32 * 59 * N),
        # both in one pass: read p, m, v and write p, m, v for every parameter float (24 B), tiles field
        # of every record, the record gradient read and cleared per on-screen record
        "gs_project_bwd_adam": ("hbm", 24 * 59 * N + 4 * VN + 72 * M),
    }


# Kernel sources whose HBM traffic per launch was measured with hardware counters.
TRAFFIC_SOURCES = {"gs_render_bwd_pixels": ["render.hip", "common.hpp"],
                   "gs_render_fwd": ["render.hip", "common.hpp"],
                   "gs_render_fwd_l1": ["render.hip", "common.hpp"],
                   "gs_loss_l1_dssim": ["ssim.hip", "common.hpp"]}


def source_digest(entry: str):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES.get(entry, []):
        with open(os.path.join(ROOT, "paper_2406_18533_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(entry: str):
    """HBM bytes per launch of the entry's kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading), or
    None when there is none or the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", "train_step_16x1080p_1M_hbm_traffic.md")
    if entry not in TRAFFIC_SOURCES or not os.path.exists(path):
        return None
    rows = {}
    with open(path) as f:
        for line in f:
            if line.startswith("| `gs_"):
                cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
                rows[cells[0]] = cells
    r = rows.get(entry)
    if r is None or r[1] != source_digest(entry):
        return None
    return int(float(r[-1]))


def roofline(timings: dict, counts: dict):
    work = algorithmic(counts)
    dom = max(timings, key=lambda k: timings[k])
    bound, amount = work[dom]
    sec = timings[dom] / 1e3
    if bound == "hbm":
        achieved = amount / sec / 1e9
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        achieved = amount / sec / 1e12
        out = {"bound": "alu", "achieved": round(achieved, 2), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s"}
    out["frac"] = round(achieved / out["peak"], 4)
    out["traffic"] = measured_traffic(dom)
    out["kernel"] = dom
    out["ms"] = round(timings[dom], 4)
    # the render pair against the HBM roofline, literally: its algorithmic bytes
    # (40 B per sorted instance for the gathered id and record and 20 B per pixel
    # written by the forward, plus 24 B per pixel for the fused L1's target and
    # gradient; the backward the same 40 B per instance, 36 B of gradient
    # atomics per instance and 20 B per pixel read) over the two kernels' time
    fwd = "gs_render_fwd_l1" if "gs_render_fwd_l1" in timings else "gs_render_fwd"
    if fwd in timings and "gs_render_bwd_pixels" in timings:
        K, Pn = counts["K"], counts["pixels"]
        b_fwd = 40 * K + 20 * Pn + (24 * Pn if fwd == "gs_render_fwd_l1" else 0)
        b_bwd = 76 * K + 20 * Pn
        ms2 = timings[fwd] + timings["gs_render_bwd_pixels"]
        gbs = (b_fwd + b_bwd) / (ms2 / 1e3) / 1e9
        out["render_hbm"] = {"kernels": [fwd, "gs_render_bwd_pixels"], "bytes": b_fwd + b_bwd, "ms": round(ms2, 4),
                             "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(gbs / HBM_PEAK_GBS, 4)}
    per = {}
    for k, (b, a) in work.items():
        if k not in timings:
            continue
        t = timings[k] / 1e3
        per[k] = {"bound": b, "ms": round(timings[k], 4),
                  "achieved": round(a / t / (1e9 if b == "hbm" else 1e12), 2 if b == "alu" else 1),
                  "unit": "GB/s" if b == "hbm" else "TFLOP/s"}
    return out, per


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_step(P, cams, seed: int = 0) -> float:
    """Seconds of one FP64 oracle training step on the host: transformation,
    binning, render, L1 loss against seeded random targets, render and
    transformation backward over every view, then one Adam step with the
    batch's scaling rules."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    f = oracle.forward(P, cams)
    targets = [rng.uniform(size=v["rgb"].shape) for v in f["views"]]
    _, g = oracle.l1_loss([v["rgb"] for v in f["views"]], targets)
    grad, _ = oracle.backward(P, cams, f, g)
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    oracle.adam(P.copy(), grad, m, v, [1e-4] * 6, 0.9, 0.999, 1e-15, len(cams), 1)
    return time.perf_counter() - t0


ORACLE_C1_CHILD = (
    "import json, sys; sys.path.insert(0, {root!r}); import bench; from synthetic import scenes; "
    "w = scenes.plain_single_view(); P = w.params.double().numpy(); bench.oracle_step(P, w.cameras); "
    "print(json.dumps(min(bench.oracle_step(P, w.cameras) for _ in range(3))))")


def cpu_baseline(workload, side: dict | None = None):
    """The FP64 oracle (never tuned) on the host cores: one whole training
    step of the batch (every view), the plain single-view configuration on
    all cores and on one core (a child process with OMP_NUM_THREADS=1), and,
    with `side` (inputs the side lines captured), the oracle of the L1 +
    D-SSIM loss on one view of the batch and of one densification of the
    step's Gaussians."""
    import subprocess
    import oracle
    from synthetic import scenes
    P = workload.params.double().numpy()
    cams = workload.cameras
    step = oracle_step(P, cams)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": round(len(cams) / step, 5), "unit": "views/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"one whole training step of the batch ({len(cams)} views {cams[0]['width']}x{cams[0]['height']}, "
                     f"N={P.shape[1]}, FP64) in {step:.1f} s"}
    c1 = scenes.plain_single_view()
    P1 = c1.params.double().numpy()
    oracle_step(P1, c1.cameras)
    t_all = min(oracle_step(P1, c1.cameras) for _ in range(3))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", ORACLE_C1_CHILD.format(root=ROOT)], env=env, capture_output=True,
                       text=True, timeout=600)
    t_one = float(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
    out["single_view_256_10k"] = {"all_cores_ms": round(t_all * 1e3, 2), "cores": threads,
                                  "one_core_ms": round(t_one * 1e3, 2) if t_one else None,
                                  "kind": "oracle", "sample": "one whole training step, best of 3"}
    side = side or {}
    if "dssim" in side:
        x, y, V = side["dssim"]
        t0 = time.perf_counter()
        oracle.l1_dssim_loss([x], [y], 0.2)
        dt = time.perf_counter() - t0
        out["l1_dssim"] = {"value": round(1.0 / (dt * V), 5), "unit": "batches/s", "kind": "oracle",
                           "sample": f"1 of {V} views ({x.shape[2]}x{x.shape[1]}): loss and gradient in {dt:.1f} s, "
                                     f"extrapolated to the batch"}
    if "densify" in side:
        a = side["densify"]
        t0 = time.perf_counter()
        oracle.densify(a["P"], a["m"], a["v"], a["accum"], a["count"], a["noise"], *a["hp"])
        dt = time.perf_counter() - t0
        out["densify"] = {"value": round(a["P"].shape[1] / dt, 1), "unit": "Gaussians/s", "kind": "oracle",
                          "sample": f"one densification of all {a['P'].shape[1]} Gaussians in {dt:.2f} s"}
    return out


def serve_bench(n_gaussians: int, requests: int, warmup: int, slots: int = 4, max_views: int = 8):
    """Render-only serving of a device-resident model (5M clustered
    Gaussians): one-at-a-time capacity, then Poisson arrivals at 0.7x that
    rate through the continuous-batching server (p50/p99 latency = completion
    minus arrival), then saturation throughput."""
    import threading
    import torch
    from paper_2406_18533_amd.serve import GPUBackend, RenderServer, percentile
    from synthetic import scenes
    P = scenes.serving_scene(n_gaussians).cuda()
    be = GPUBackend(P, slots=slots, max_views=max_views, budget_bytes=16 << 30)
    probe = [c for _, c in scenes.serving_requests(warmup + 100, qps=1.0, seed=16)]
    # one at a time: service time of single-request batches
    for c in probe[:warmup]:
        be.render_now(0, [c])
    t0 = time.perf_counter()
    for c in probe[warmup:]:
        be.render_now(0, [c])
    single = (time.perf_counter() - t0) / (len(probe) - warmup)
    qps = 0.7 / single
    reqs = scenes.serving_requests(requests + warmup, qps=qps, seed=15)
    srv = RenderServer(be, max_batch_views=max_views).start()
    for _, c in reqs[:warmup]:
        srv.submit(c).result()
    srv.completed.clear()
    srv.batches.clear()
    reqs = reqs[warmup:]
    t_first = reqs[0][0]
    reqs = [(arr - t_first, c) for arr, c in reqs]
    done = threading.Semaphore(0)

    def consume(f):       # a client takes each image as it completes and lets it go
        f.result()
        done.release()

    def client():
        t_start = time.perf_counter()
        for arr, c in reqs:
            d = t_start + arr - time.perf_counter()
            if d > 0:
                time.sleep(d)
            srv.submit(c).add_done_callback(consume)
    th = threading.Thread(target=client)
    t0 = time.perf_counter()
    th.start()
    th.join()
    for _ in reqs:
        done.acquire()
    t_fixed = time.perf_counter() - t0
    lat = srv.latencies_ms()
    p50, p99 = percentile(lat, 50), percentile(lat, 99)
    waits = [(st - arr) * 1e3 for arr, st, _ in srv.completed]        # queue: arrival to launch
    service = [(dn - st) * 1e3 for _, st, dn in srv.completed]        # launch to result on the host
    mean_batch = sum(srv.batches) / max(len(srv.batches), 1)
    # saturation: everything queued at once
    srv.completed.clear()
    burst = reqs[: min(len(reqs), 200)]
    t0 = time.perf_counter()
    for _, c in burst:
        srv.submit(c).add_done_callback(consume)
    for _ in burst:
        done.acquire()
    sat = len(burst) / (time.perf_counter() - t0)
    srv.stop()
    torch.cuda.synchronize()
    return {"workload": f"serving_{n_gaussians // 1_000_000}M_mixed_res", "qps": round(qps, 2),
            "requests": requests, "p50_ms": round(p50, 3), "p99_ms": round(p99, 3),
            "queue_wait_p50_p99_ms": [round(percentile(waits, 50), 3), round(percentile(waits, 99), 3)],
            "service_p50_p99_ms": [round(percentile(service, 50), 3), round(percentile(service, 99), 3)],
            "views_per_s_at_qps": round(requests / t_fixed, 2), "saturation_views_per_s": round(sat, 2),
            "one_at_a_time_views_per_s": round(1.0 / single, 2), "mean_batch": round(mean_batch, 2),
            "slots": slots, "sort_buffer_bytes_per_slot": be.capacity * 16, "peak_sort_bytes": srv.peak_mem,
            "pinned_image_buffers": be.pool.allocated,
            "resolutions": ["512x512", "1280x720", "1920x1080", "3840x2160"]}


def small_configs(reps: int = 50):
    """The two configurations beside the batch: the plain single view (10,000
    Gaussians in [-1, 1]^3, one 256x256 view) and the differentiation check's
    large view (1,000,000 clustered Gaussians, one 1920x1080 view). For each,
    fwd + bwd of one view through the autograd Function (transformation,
    binning, render, then the L1 gradient back through render and
    transformation backward), and one whole training step of the batched
    trainer with that single view (graph replay, Adam included)."""
    import torch
    from paper_2406_18533_amd import raster as R
    from paper_2406_18533_amd import train
    from paper_2406_18533_amd.autograd import rasterize
    from synthetic import scenes
    out = {}
    for name, w in [("single_view_256_10k", scenes.plain_single_view()), ("diff_check_1080p_1M", scenes.diff_check_large())]:
        P = w.params.cuda()
        targets = render_targets(w.target_params.cuda(), w.cameras)
        cams = R.Cameras(w.cameras)
        buf = R.LossBuffers(cams)
        k = reps if P.shape[1] < 100_000 else max(5, reps // 5)

        def fwd_bwd():
            Pg = P.detach().requires_grad_(True)
            rgb = rasterize(Pg, cams)
            _, dL = R.gs_loss_l1(rgb.detach(), targets, cams, buf)
            rgb.backward(dL)
            return Pg.grad
        fwd_bwd()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fwd_bwd()
        torch.cuda.synchronize()
        ab = (time.perf_counter() - t0) * 1e3 / k
        tr = train.BatchedTrainer(P.clone(), w.cameras, targets, train.TrainConfig())
        for _ in range(3):
            tr.step()
            tr.check_overflow()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            tr.step()
        torch.cuda.synchronize()
        st = (time.perf_counter() - t0) * 1e3 / k
        c = w.cameras[0]
        out[name] = {"gaussians": P.shape[1], "resolution": f"{c['width']}x{c['height']}",
                     "autograd_fwd_bwd_ms": round(ab, 4), "train_step_ms": round(st, 4),
                     "views_per_s": round(1e3 / st, 1)}
        del tr, P, targets, buf
        torch.cuda.empty_cache()
    return out


def aerial_bench(steps: int, warmup: int, plain: bool):
    """The large aerial scene (20M Gaussians, 2 views 4608x3456 + 2 views
    3840x2160): batched graph-captured step vs the plain per-view path."""
    import torch
    from paper_2406_18533_amd import autotune, train
    w = make_workload("aerial_4k")
    P = w.params.cuda()
    targets = render_targets(w.target_params.cuda(), w.cameras)
    tr = train.BatchedTrainer(P.clone(), w.cameras, targets, train.TrainConfig())
    autotune.tune(tr)
    for _ in range(warmup):
        tr.step()
        tr.check_overflow()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tr.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tr.check_overflow()
    out = {"workload": w.name, "gaussians": P.shape[1], "views": len(w.cameras),
           "views_per_s": round(tr.V * steps / dt, 2), "ms_per_step": round(dt * 1e3 / steps, 3),
           "instances": int(tr.bins.n_instances.item()),
           "scheduler": {"fwd": list(tr.cfg.fwd_shape), "bwd": list(tr.cfg.bwd_shape), "modes": dict(tr.cfg.extra)}}
    del tr
    torch.cuda.empty_cache()
    if plain:
        pt = train.PlainTrainer(P.clone(), w.cameras, targets, train.TrainConfig())
        pt.step()
        torch.cuda.synchronize()
        k = max(2, min(steps, 3))
        t0 = time.perf_counter()
        for _ in range(k):
            pt.step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["plain_views_per_s"] = round(pt.V * k / dt, 2)
        out["speedup_vs_plain"] = round(out["views_per_s"] / out["plain_views_per_s"], 3)
        del pt
    del P, targets
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched_1080p")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--mode", type=int, default=None,
                    help="force scheduler mode of both render passes (0 per-tile, 1 persistent, 2 XCD split, 3 LPT, "
                         "4 XCD-LPT, 5 LPT-head)")
    ap.add_argument("--fwd-mode", type=int, default=None, help="force the forward render's scheduler mode")
    ap.add_argument("--bwd-mode", type=int, default=None, help="force the backward render's scheduler mode")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-aerial", action="store_true")
    ap.add_argument("--no-dssim", action="store_true")
    ap.add_argument("--no-densify", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="end with a fill and a copy of this many MiB (calibration for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU only; --gpus must be 1 (a multi-GPU run would "
                                   "shard Gaussians and tiles across GPUs, which is not built)"}))
        sys.exit(2)
    import torch
    from paper_2406_18533_amd import _lib, autotune, train
    from paper_2406_18533_amd import raster as R

    _lib.load()
    R.init(0)
    log(f"workload {args.workload}: generating")
    w = make_workload(args.workload)
    P = w.params.cuda()
    log(f"N={P.shape[1]} views={len(w.cameras)}; rendering targets")
    targets = render_targets(w.target_params.cuda() if w.target_params is not None else P.clone(), w.cameras)
    cfg = train.TrainConfig(graph=not args.no_graph)
    if args.mode is not None:
        cfg.mode = args.mode
    tr = train.BatchedTrainer(P.clone(), w.cameras, targets, cfg)
    tuned = None
    if not args.no_autotune:
        log("autotuning render launch shapes")
        tuned = autotune.tune(tr, verbose=False)
        log(f"autotune: fwd {tuned['fwd']} bwd {tuned['bwd']}")
    if args.mode is not None:
        tr.set_shapes(mode=args.mode)
    if args.fwd_mode is not None or args.bwd_mode is not None:
        if args.fwd_mode is not None:
            tr.cfg.extra["fwd_mode"] = args.fwd_mode
        if args.bwd_mode is not None:
            tr.cfg.extra["bwd_mode"] = args.bwd_mode
        tr.set_shapes()
    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        tr.step()
        tr.check_overflow()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tr.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    redo = tr.check_overflow()
    ms = (t1 - t0) * 1e3 / args.steps
    views_s = tr.V * args.steps / (t1 - t0)
    log(f"{ms:.3f} ms/step, {views_s:.1f} views/s, loss {tr.loss():.5f}, overflow redo {redo}")
    log("per-entry timings (eager, HIP events)")
    timings = entry_timings(tr, reps=min(5, max(args.steps, 1)))
    counts = workload_counts(tr)
    roof, per = roofline(timings, counts)
    log(f"timings {json.dumps(timings)}")
    dssim, side = None, {}
    if not args.no_dssim:
        log("step with the L1 + D-SSIM loss")
        dssim, side["dssim"] = dssim_side(tr, P, w.cameras, targets, args.steps, args.warmup)
        log(f"l1+dssim {json.dumps(dssim)}")
    dens = None
    if not args.no_densify:
        log("densification of the step's Gaussians")
        dens, side["densify"] = densify_side(tr)
        log(f"densify {json.dumps(dens)}")
    plain = None
    if not args.no_plain:
        log("plain per-view path")
        pt = train.PlainTrainer(P.clone(), w.cameras, targets, cfg)
        pt.step()
        torch.cuda.synchronize()
        k = max(2, min(args.steps, 5))
        t0 = time.perf_counter()
        for _ in range(k):
            pt.step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain = {"views_per_s": round(pt.V * k / (t1 - t0), 2), "ms_per_step": round((t1 - t0) * 1e3 / k, 3)}
        del pt
    serving = None
    sched_cfg = {"fwd": list(tr.cfg.fwd_shape), "bwd": list(tr.cfg.bwd_shape), "modes": dict(tr.cfg.extra)}
    n_gauss = P.shape[1]
    del tr, P, targets
    torch.cuda.empty_cache()
    if not args.no_serve:
        log("serving (render-only, continuous batching)")
        serving = serve_bench(5_000_000, args.serve_requests, warmup=args.serve_warmup)
        log(f"serving {json.dumps(serving)}")
    aerial = None
    if not args.no_aerial and args.workload == "batched_1080p":
        log("aerial 4K-class scene (20M Gaussians)")
        aerial = aerial_bench(max(3, min(args.steps, 10)), 2, not args.no_plain)
        log(f"aerial {json.dumps(aerial)}")
    small = None
    if not args.no_small and args.workload == "batched_1080p":
        log("single-view configurations (256x256 10k, 1080p 1M)")
        small = small_configs()
        log(f"small {json.dumps(small)}")
    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline (whole step of the batch)")
        cpu = cpu_baseline(w, side=side)
    if args.copy_mib:
        log(f"calibration: fill then copy of {args.copy_mib} MiB")
        a = torch.empty(args.copy_mib * 2 ** 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    cams = w.cameras
    out = {
        "metric": "train views/s fwd+bwd (1080p, 4K) vs plain path; render p50/p99 ms at fixed QPS",
        "value": round(views_s, 2), "unit": "views/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "gaussians": n_gauss, "views": len(cams),
                   "resolution": sorted({f"{c['width']}x{c['height']}" for c in cams}),
                   "global_batch": len(cams), "parallelism": "single-gpu",
                   "graph": not args.no_graph, "scheduler": sched_cfg},
        "plain_path": plain,
        "speedup_vs_plain": round(views_s / plain["views_per_s"], 3) if plain else None,
        "aerial_4k": aerial,
        "single_view": small,
        "l1_dssim": dssim,
        "densify": dens,
        "serving": serving,
        "roofline": roof,
        "render_hbm_frac": roof.get("render_hbm", {}).get("frac"),
        "per_kernel": per,
        "counts": counts,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
