"""Training steps over a batch of views.

BatchedTrainer: the batched step of the paper's training loop (section 2.1:
transformation, rendering, loss, back-propagation; section 4: Adam with
lr * sqrt(b) and beta^b) over all b views at once - one projection launch
for every view, one (view, tile) work list for the whole batch, render
kernels launched in an order driven by the previous iteration's per-tile work
(heaviest tiles first, or split over the XCDs: whichever the autotuner
measured faster for that pass), and the whole step captured once as a HIP
graph and replayed.

PlainTrainer: the same batched step computed view by view with eager
launches and one workgroup per tile (the baseline the batched path is
measured against).

Every arithmetic step runs in libgs.so; torch only owns the buffers and the
stream.
"""
from __future__ import annotations

import json
import math
import time
from dataclasses import dataclass, field

import torch

from . import _lib
from . import raster as R


@dataclass
class TrainConfig:
    lr: tuple = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 1.25e-4)   # mean, log-scale, quat, opacity, SH0, SH rest
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    bg: tuple = (0.0, 0.0, 0.0)
    headroom: float = 1.25          # instance capacity = headroom * first K
    mode: int = _lib.GS_SCHED_PER_TILE    # the autotuner may pick another per pass
    fwd_shape: tuple = (1, 64)      # (px_per_thread, chunk) of render forward
    bwd_shape: tuple = (1, 64)      # (px_per_thread, chunk) of render backward
    queues: int = 64
    workers: int = 0
    graph: bool = True
    fused_adam: bool = True         # transformation backward and Adam in one pass (gs_project_bwd_adam)
    fused_loss: bool = True         # L1 loss in the render forward's output stage (gs_render_fwd_l1)
    ssim_lambda: float = 0.0        # > 0: loss (1 - lambda) L1 + lambda (1 - SSIM) (gs_loss_l1_dssim)
    extra: dict = field(default_factory=dict)


class StepLog:
    """Per-step training metrics as JSON lines appended to `path`: the
    optimizer step count, the batch loss, milliseconds per step and views
    per second since the previous record, overflow re-runs so far and the
    number of Gaussians."""

    def __init__(self, path: str, every: int = 1):
        assert every >= 1
        self.path, self.every = path, every

    def write(self, tr, steps: int, seconds: float) -> dict:
        rec = {"step": int(tr.step_dev.item()), "loss": tr.loss(), "ms_per_step": seconds * 1e3 / max(steps, 1),
               "views_per_s": tr.V * steps / seconds if seconds > 0 else None, "overflow_redos": int(tr.overflows),
               "gaussians": int(tr.n)}
        with open(self.path, "a") as f:
            f.write(json.dumps(rec) + "\n")
        return rec


class BatchedTrainer:
    def __init__(self, params: torch.Tensor, cams_list: list, targets: torch.Tensor, cfg: TrainConfig | None = None):
        self.cfg = cfg or TrainConfig()
        assert params.is_cuda and params.dtype in (torch.float32, torch.float64) and params.shape[0] == 59
        self.P = params.contiguous()
        self.n = self.P.shape[1]
        self.V = len(cams_list)
        self.cams = R.Cameras(cams_list)
        self.targets = targets.contiguous()
        dev = self.P.device
        self.grad = torch.zeros_like(self.P)
        self.m = torch.zeros_like(self.P)
        self.v = torch.zeros_like(self.P)
        self.step_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        self.scratch = torch.zeros(2, dtype=torch.float64, device=dev)
        dt = self.P.dtype              # float32 for training; float64 for checks against the FP64 oracle
        self.proj = R.alloc_projected(self.n, self.V, dt, dev)
        self.dproj = torch.zeros(self.V, self.n, _lib.GS_REC, dtype=dt, device=dev)
        P_all = self.cams.total_pixels()
        self.rgb = torch.empty(3 * P_all, dtype=dt, device=dev)
        self.T = torch.empty(P_all, dtype=dt, device=dev)
        self.last = torch.empty(P_all, dtype=torch.int32, device=dev)
        if self.cfg.ssim_lambda > 0.0:
            self.loss_buf = R.DssimBuffers(self.cams, dtype=dt, device=dev)
        else:
            self.loss_buf = R.LossBuffers(self.cams, dtype=dt, device=dev)
        T_all = self.cams.total_tiles()
        self.work_fwd = torch.zeros(T_all, dtype=torch.int32, device=dev)
        self.work_bwd = torch.zeros(T_all, dtype=torch.int32, device=dev)
        self.hp = R.adam_hparams(self.cfg.lr, self.cfg.beta1, self.cfg.beta2, self.cfg.eps, batch_size=self.V,
                                 zero_grad=True)
        self._make_sched()
        self._size_bins()
        self.stats = None                 # densification statistic (accum, count) while enabled
        self.graph = None
        self.overflows = 0
        self._flag_host = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        self._skip_flag = torch.ones(1, dtype=torch.int32, device=dev)

    def _size_bins(self):
        R.gs_project(self.P, self.cams, self.proj)
        K = R.instance_count(self.proj)
        self.bins = R.Bins(self.n, self.cams, max(int(K * self.cfg.headroom), 1024))

    def _make_sched(self):
        """Schedulers of the two render passes: the per-pass modes the
        autotuner recorded in cfg.extra, else cfg.mode for both."""
        c = self.cfg
        fm, bm = c.extra.get("fwd_mode", c.mode), c.extra.get("bwd_mode", c.mode)
        self.sched_fwd = R.Sched(self.cams, fm, c.fwd_shape[0], c.fwd_shape[1], c.workers, c.queues,
                                 tile_cost=self.work_fwd)
        self.sched_bwd = R.Sched(self.cams, bm, c.bwd_shape[0], c.bwd_shape[1], c.workers, c.queues,
                                 tile_cost=self.work_bwd)

    def set_shapes(self, fwd_shape=None, bwd_shape=None, mode=None):
        if fwd_shape:
            self.cfg.fwd_shape = tuple(fwd_shape)
        if bwd_shape:
            self.cfg.bwd_shape = tuple(bwd_shape)
        if mode is not None:
            self.cfg.mode = mode
            self.cfg.extra.pop("fwd_mode", None)
            self.cfg.extra.pop("bwd_mode", None)
        self._make_sched()
        self.graph = None

    # -- the step -------------------------------------------------------------------------
    def forward(self, check: bool = False):
        R.gs_project(self.P, self.cams, self.proj)
        R.gs_bin_sort(self.proj, self.n, self.cams, self.bins, check_capacity=check)
        self._render()

    def _render(self):
        """Render forward, and the loss with its gradient (fused or after)."""
        if self.cfg.ssim_lambda > 0.0:
            R.gs_render_fwd(self.proj, self.n, self.bins, self.cams, self.cfg.bg, self.sched_fwd, self.rgb, self.T,
                            self.last, self.work_fwd, self.work_bwd)
            R.gs_loss_l1_dssim(self.rgb, self.targets, self.cams, self.loss_buf, lam=self.cfg.ssim_lambda)
        elif self.cfg.fused_loss:
            R.gs_render_fwd_l1(self.proj, self.n, self.bins, self.cams, self.targets, self.loss_buf, self.cfg.bg,
                               self.sched_fwd, self.rgb, self.T, self.last, self.work_fwd, self.work_bwd)
        else:
            R.gs_render_fwd(self.proj, self.n, self.bins, self.cams, self.cfg.bg, self.sched_fwd, self.rgb, self.T,
                            self.last, self.work_fwd, self.work_bwd)
            R.gs_loss_l1(self.rgb, self.targets, self.cams, self.loss_buf)

    def backward_and_update(self):
        R.gs_render_bwd_pixels(self.proj, self.n, self.bins, self.cams, self.T, self.last, self.loss_buf.dL,
                               self.dproj, self.cfg.bg, self.sched_bwd)
        self._accumulate_stats()
        self._update(self.bins.overflow)

    def _accumulate_stats(self):
        if self.stats is not None:
            R.gs_densify_stats(self.proj, self.dproj, self.n, self.V, self.stats[0], self.stats[1],
                               scale=float(self.V))

    # -- densification (appendix A.1) -------------------------------------------------------
    def enable_densify_stats(self, on: bool = True):
        """Accumulate the position-gradient statistic in every step from now on."""
        dev = self.P.device
        self.stats = (torch.zeros(self.n, dtype=torch.float32, device=dev),
                      torch.zeros(self.n, dtype=torch.int32, device=dev)) if on else None
        self.graph = None

    def densify(self, h, seed: int = 0):
        """Clone / split / prune with the accumulated statistic; resizes every
        per-Gaussian buffer, restarts the statistic and re-captures the step.
        Returns the class counts (kept, clones, split pairs)."""
        assert self.stats is not None, "enable_densify_stats first"
        torch.cuda.synchronize()
        plan = R.DensifyPlan(self.n)
        R.gs_densify_plan(self.P, self.stats[0], self.stats[1], h, plan)
        gen = torch.Generator(device=self.P.device).manual_seed(seed)
        noise = torch.randn(2, 3, self.n, generator=gen, device=self.P.device, dtype=self.P.dtype)
        K, C, S = (int(x) for x in plan.counts.cpu())
        self.P, self.m, self.v = R.gs_densify_apply(self.P, self.m, self.v, noise, plan, K + C + 2 * S)
        self._resize()
        return K, C, S

    def reset_opacity(self, max_opacity: float = 0.01):
        R.gs_reset_opacity(self.P, self.m, self.v, math.log(max_opacity / (1.0 - max_opacity)))

    def _resize(self):
        dev = self.P.device
        self.n = self.P.shape[1]
        self.grad = torch.zeros_like(self.P)
        self.proj = R.alloc_projected(self.n, self.V, self.P.dtype, dev)
        self.dproj = torch.zeros(self.V, self.n, _lib.GS_REC, dtype=self.P.dtype, device=dev)
        self._size_bins()
        if self.stats is not None:
            self.enable_densify_stats()
        self.graph = None

    def _update(self, skip_flag):
        if self.cfg.fused_adam:
            R.gs_project_bwd_adam(self.P, self.cams, self.proj, self.dproj, self.grad, self.m, self.v, self.hp,
                                  self.step_dev, self.scratch, skip_flag=skip_flag)
        else:
            R.gs_project_bwd(self.P, self.cams, self.proj, self.dproj, self.grad, clear=True)
            R.gs_adam_step(self.P, self.grad, self.m, self.v, self.hp, self.step_dev, self.scratch,
                           skip_flag=skip_flag)

    def _body(self, check: bool):
        self.forward(check)
        self.backward_and_update()

    def _grow(self):
        K = int(self.bins.n_instances.item())
        self.bins = R.Bins(self.n, self.cams, int(K * self.cfg.headroom) + 1024)
        self.graph = None

    def step_eager(self):
        """One eager step; grows the instance buffers first if they are too small."""
        while True:
            try:
                R.gs_project(self.P, self.cams, self.proj)
                R.gs_bin_sort(self.proj, self.n, self.cams, self.bins, check_capacity=True)
                break
            except _lib.GsError as e:
                if e.status != _lib.GS_ERR_CAPACITY:
                    raise
                self.overflows += 1
                self._grow()
        self._render()
        self.backward_and_update()

    def warmup(self):
        """Runs every kernel of the step once (sizing the instance buffers on
        the way) without changing the training state: the Adam launch gets a
        skip flag, so parameters, moments and the step counter stay as they
        were and the gradient is cleared."""
        while True:
            try:
                R.gs_project(self.P, self.cams, self.proj)
                R.gs_bin_sort(self.proj, self.n, self.cams, self.bins, check_capacity=True)
                break
            except _lib.GsError as e:
                if e.status != _lib.GS_ERR_CAPACITY:
                    raise
                self.overflows += 1
                self._grow()
        self._render()
        R.gs_render_bwd_pixels(self.proj, self.n, self.bins, self.cams, self.T, self.last, self.loss_buf.dL,
                               self.dproj, self.cfg.bg, self.sched_bwd)
        self._update(self._skip_flag)

    def capture(self):
        """Captures one whole step as a HIP graph (after a state-preserving
        warm-up of every kernel)."""
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.warmup()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._body(check=False)
        torch.cuda.synchronize()
        self.graph = g

    def step(self):
        if self.cfg.graph:
            if self.graph is None:
                self.capture()
            self.graph.replay()
        else:
            self.step_eager()

    def check_overflow(self) -> bool:
        """After a step: if its bins overflowed, the update was skipped on the
        device; grow the buffers, re-capture and redo the step eagerly."""
        self._flag_host.copy_(self.bins.overflow)
        if int(self._flag_host.item()) == 0:
            return False
        self.overflows += 1
        self._grow()
        self.step_eager()
        return True

    def loss(self) -> float:
        return float(self.loss_buf.loss.item())

    def train(self, steps: int, log: "StepLog | None" = None) -> None:
        """Runs `steps` steps, each followed by the overflow check (one small
        device-to-host read); with a StepLog, appends a record every
        log.every steps (timed from the previous record, after a device
        synchronisation)."""
        t0, done = time.perf_counter(), 0
        for k in range(1, steps + 1):
            self.step()
            self.check_overflow()
            if log is not None and k % log.every == 0:
                torch.cuda.synchronize()
                t = time.perf_counter()
                log.write(self, k - done, t - t0)
                t0, done = t, k

    # -- checkpoint / resume --------------------------------------------------------------------
    def state_dict(self) -> dict:
        """Parameters, both Adam moments, the device step counter and the
        per-tile cost history the scheduler uses (all that a resumed run needs
        to continue the same trajectory)."""
        return {"params": self.P.detach().clone(), "m": self.m.clone(), "v": self.v.clone(),
                "step": self.step_dev.clone(), "work_fwd": self.work_fwd.clone(), "work_bwd": self.work_bwd.clone(),
                "lr": tuple(self.cfg.lr), "batch": self.V}

    def load_state_dict(self, sd: dict) -> None:
        assert sd["params"].shape == self.P.shape and sd["batch"] == self.V
        with torch.no_grad():
            self.P.copy_(sd["params"])
            self.m.copy_(sd["m"])
            self.v.copy_(sd["v"])
            self.step_dev.copy_(sd["step"])
            self.work_fwd.copy_(sd["work_fwd"])
            self.work_bwd.copy_(sd["work_bwd"])
            self.grad.zero_()
        torch.cuda.synchronize()


class PlainTrainer:
    """The batched step computed one view at a time, eagerly, with one
    workgroup per tile: same loss (per-view losses scaled by 1/b), same
    gradient, one Adam step with the same scaled hyper-parameters."""

    def __init__(self, params: torch.Tensor, cams_list: list, targets: torch.Tensor, cfg: TrainConfig | None = None):
        self.cfg = cfg or TrainConfig()
        self.P = params.contiguous()
        self.n = self.P.shape[1]
        self.V = len(cams_list)
        dev = self.P.device
        self.cams = [R.Cameras([c]) for c in cams_list]
        self.targets = []
        o = 0
        for c in cams_list:
            k = 3 * c["width"] * c["height"]
            self.targets.append(targets[o:o + k])
            o += k
        self.grad = torch.zeros_like(self.P)
        self.m = torch.zeros_like(self.P)
        self.v = torch.zeros_like(self.P)
        self.step_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        self.scratch = torch.zeros(2, dtype=torch.float64, device=dev)
        self.proj = R.alloc_projected(self.n, 1, self.P.dtype, dev)
        self.dproj = torch.zeros(1, self.n, _lib.GS_REC, dtype=self.P.dtype, device=dev)
        self.hp = R.adam_hparams(self.cfg.lr, self.cfg.beta1, self.cfg.beta2, self.cfg.eps, batch_size=self.V,
                                 zero_grad=True)
        Kmax = 0
        for cm in self.cams:
            R.gs_project(self.P, cm, self.proj)
            Kmax = max(Kmax, R.instance_count(self.proj))
        self.bins = R.Bins(self.n, max(self.cams, key=lambda c: c.total_tiles()), max(int(Kmax * self.cfg.headroom), 1024))
        self.bins_tiles = self.bins.total_tiles
        self.bufs = [R.LossBuffers(cm, dtype=self.P.dtype, device=dev) for cm in self.cams]
        self.loss_total = torch.zeros(1, dtype=torch.float64, device=dev)

    def step(self):
        bg = self.cfg.bg
        for cm, tg, lb in zip(self.cams, self.targets, self.bufs):
            R.gs_project(self.P, cm, self.proj)
            while True:
                try:
                    if cm.total_tiles() > self.bins_tiles:
                        raise _lib.GsError(_lib.GS_ERR_CAPACITY, "tiles")
                    R.gs_bin_sort(self.proj, self.n, cm, self.bins, check_capacity=True)
                    break
                except _lib.GsError as e:
                    if e.status != _lib.GS_ERR_CAPACITY:
                        raise
                    K = int(self.bins.n_instances.item())
                    self.bins = R.Bins(self.n, cm, int(max(K, self.bins.capacity) * self.cfg.headroom))
                    self.bins_tiles = self.bins.total_tiles
            rgb, T, last = R.gs_render_fwd(self.proj, self.n, self.bins, cm, bg)
            R.gs_loss_l1(rgb, tg, cm, lb, scale=1.0 / self.V)
            R.gs_render_bwd(self.P, self.proj, self.bins, cm, T, last, lb.dL, self.grad, bg, dprojected=self.dproj)
        R.gs_adam_step(self.P, self.grad, self.m, self.v, self.hp, self.step_dev, self.scratch)

    def loss(self) -> float:
        return float(sum(b.loss.item() for b in self.bufs))
