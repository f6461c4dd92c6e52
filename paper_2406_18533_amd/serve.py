"""Continuous-batching render server for a device-resident trained model.

Requests (one camera each, any resolution) arrive at any time. A loop
thread forms batches from the queue in arrival order and admits them while
both a render slot (a stream with its own buffers) and sort-buffer memory
(the instance capacity the batch needs, at 16 bytes per instance) are free;
requests that arrive while earlier batches are still on the GPU join the
next batch as soon as a slot and memory free up, so batches overlap on the
device. Each batch is one gs_project + gs_bin_sort + gs_render_fwd over all
its views: the (view, tile) work queue of the batch is flattened exactly as
in training. A request's image does not depend on what else is in its batch
(tiles are per view and every pixel's list is ordered by (depth, index)), so
a result is the same alone and in the mix.

The backend is separate from the loop: GPUBackend calls libgs.so; tests also
drive the loop with a CPU fake to check admission and ordering without a GPU.
"""
from __future__ import annotations

import collections
import threading
import time
import weakref
from concurrent.futures import Future
from dataclasses import dataclass, field

BYTES_PER_INSTANCE = 16     # tile key + id, and their sort alternates


@dataclass
class Request:
    cam: dict
    arrival: float
    future: Future = field(default_factory=Future)
    est_instances: int = 0
    start: float = 0.0
    done: float = 0.0


class InstanceEstimator:
    """Running estimate of sorted instances per pixel, by resolution."""

    def __init__(self, per_pixel: float = 8.0, margin: float = 1.3):
        self.rate = {}
        self.default = per_pixel
        self.margin = margin

    def estimate(self, cam: dict) -> int:
        px = cam["width"] * cam["height"]
        r = self.rate.get((cam["width"], cam["height"]), self.default)
        return int(px * r * self.margin) + 4096

    def observe(self, cam: dict, k: int):
        key = (cam["width"], cam["height"])
        px = cam["width"] * cam["height"]
        old = self.rate.get(key)
        new = k / max(px, 1)
        self.rate[key] = new if old is None else max(new, 0.8 * old + 0.2 * new)


class PinnedPool:
    """Page-locked host buffers for finished images, reused by size. A result
    image is a NumPy view of one buffer (no host copy); the buffer goes back
    to the pool when the caller drops the image."""

    def __init__(self, torch):
        self.torch = torch
        self.free = collections.defaultdict(list)
        self.lock = threading.Lock()
        self.allocated = 0

    def take(self, numel: int):
        with self.lock:
            lst = self.free.get(numel)
            if lst:
                return lst.pop()
            self.allocated += 1
        return self.torch.empty(numel, dtype=self.torch.float32, pin_memory=True)

    def give(self, buf):
        with self.lock:
            self.free[buf.numel()].append(buf)

    def lend(self, buf, shape):
        """NumPy view of buf with the given shape; buf returns to the pool
        once the view (and everything derived from it) is gone."""
        arr = buf.view(*shape).numpy()
        weakref.finalize(arr, self.give, buf)
        return arr


class GPUBackend:
    """Render slots on separate streams over one device-resident model. Each
    slot owns a projected buffer sized for max_views views; a smaller batch
    uses its front (records, then the side arrays right after them). Images
    come back to the host in pooled page-locked buffers (see PinnedPool)."""

    def __init__(self, params, slots: int = 2, max_views: int = 8, bg=(0.0, 0.0, 0.0)):
        import torch
        from . import raster as R
        self.torch, self.R = torch, R
        self.P = params.contiguous()
        self.n = self.P.shape[1]
        self.bg = bg
        self.max_views = max_views
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.flat = [R.alloc_projected(self.n, max_views, torch.float32, self.P.device) for _ in range(slots)]
        self.counts = [torch.empty(2, dtype=torch.int64, pin_memory=True) for _ in range(slots)]
        self.pool = PinnedPool(torch)
        self.inflight = {}

    @property
    def slots(self) -> int:
        return len(self.streams)

    def _proj_view(self, slot: int, V: int):
        base = self.flat[slot]
        flat = self.torch.as_strided(base, (base.numel(),), (1,), base.storage_offset())
        return flat[: V * self.n * 12].view(V, self.n, 12)

    def launch(self, slot: int, cams_list: list, capacity: int):
        """Renders a batch on the slot's stream (returns at once)."""
        torch, R = self.torch, self.R
        s = self.streams[slot]
        assert len(cams_list) <= self.max_views
        with torch.cuda.stream(s):
            cams = R.Cameras(cams_list)
            view = self._proj_view(slot, len(cams_list))
            R.gs_project(self.P, cams, view)
            bins = R.Bins(self.n, cams, capacity)
            R.gs_bin_sort(view, self.n, cams, bins, check_capacity=False)
            rgb, _, _ = R.gs_render_fwd(view, self.n, bins, cams, self.bg)
            host, o = [], 0
            for c in cams_list:
                k = 3 * c["width"] * c["height"]
                buf = self.pool.take(k)
                buf.copy_(rgb[o:o + k], non_blocking=True)
                host.append(buf)
                o += k
            k_host = self.counts[slot]
            k_host[0:1].copy_(bins.n_instances, non_blocking=True)
            k_host[1:2].copy_(bins.overflow.to(torch.int64), non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        self.inflight[slot] = (ev, host, k_host, cams_list, bins, rgb, cams)

    def poll(self, slot: int):
        """None while running; else (images, instance count, overflowed)."""
        ev, host, k_host, cams_list, *_ = self.inflight[slot]
        if not ev.query():
            return None
        del self.inflight[slot]
        out = [self.pool.lend(buf, (3, c["height"], c["width"])) for buf, c in zip(host, cams_list)]
        return out, int(k_host[0]), bool(k_host[1])

    def render_now(self, slot: int, cams_list: list, capacity: int):
        self.launch(slot, cams_list, capacity)
        while True:
            r = self.poll(slot)
            if r is not None:
                return r


class RenderServer:
    def __init__(self, backend, mem_budget_bytes: int, max_batch_views: int = 8, estimator=None):
        self.backend = backend
        self.budget = int(mem_budget_bytes)
        self.max_views = max_batch_views
        self.est = estimator or InstanceEstimator()
        self.queue = collections.deque()
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.free_slots = list(range(backend.slots))
        self.running = {}            # slot -> (requests, bytes)
        self.mem_used = 0
        self.peak_mem = 0
        self.completed = []
        self.batches = []
        self._stop = False
        self._thread = None

    # -- client side ------------------------------------------------------------------------
    def submit(self, cam: dict) -> Future:
        r = Request(cam, time.perf_counter())
        r.est_instances = self.est.estimate(cam)
        with self.cv:
            self.queue.append(r)
            self.cv.notify()
        return r.future

    def start(self):
        self._thread = threading.Thread(target=self._loop, daemon=True)
        self._thread.start()
        return self

    def stop(self):
        with self.cv:
            self._stop = True
            self.cv.notify()
        if self._thread:
            self._thread.join()

    # -- the loop ----------------------------------------------------------------------------
    def _admit(self):
        """Forms the next batch in arrival order within the free memory."""
        batch, need = [], 0
        free = self.budget - self.mem_used
        while self.queue and len(batch) < self.max_views:
            r = self.queue[0]
            b = r.est_instances * BYTES_PER_INSTANCE
            if b > self.budget:
                b = self.budget          # a request larger than the pool runs alone
            if need + b > free:
                break
            batch.append(self.queue.popleft())
            need += b
        return batch, need

    def _loop(self):
        while True:
            with self.cv:
                if self._stop and not self.queue and not self.running:
                    return
                launch = None
                if self.free_slots and self.queue:
                    batch, need = self._admit()
                    if batch:
                        slot = self.free_slots.pop()
                        self.mem_used += need
                        self.peak_mem = max(self.peak_mem, self.mem_used)
                        self.running[slot] = (batch, need)
                        launch = (slot, batch, need)
                if launch is None and not self.running:
                    self.cv.wait(timeout=0.001)
                    continue
            if launch is not None:
                slot, batch, need = launch
                now = time.perf_counter()
                for r in batch:
                    r.start = now
                self.backend.launch(slot, [r.cam for r in batch], need // BYTES_PER_INSTANCE)
                self.batches.append(len(batch))
            self._reap()
            if launch is None:
                time.sleep(0.0001)

    def _reap(self):
        for slot in list(self.running.keys()):
            res = self.backend.poll(slot)
            if res is None:
                continue
            images, k, overflow = res
            batch, need = self.running[slot]
            if overflow:
                # the estimate was too small: render the batch again on the same
                # slot with the exact count (nothing was written past capacity)
                images, k, overflow = self.backend.render_now(slot, [r.cam for r in batch], int(k * 1.05) + 1024)
            with self.cv:
                self.running.pop(slot)
                self.mem_used -= need
                self.free_slots.append(slot)
            now = time.perf_counter()
            per = k / max(sum(r.cam["width"] * r.cam["height"] for r in batch), 1)
            for r, img in zip(batch, images):
                self.est.observe(r.cam, int(per * r.cam["width"] * r.cam["height"]))
                r.done = now
                self.completed.append((r.arrival, r.start, r.done))   # timestamps only, not the image
                r.future.set_result(img)
            del images, batch

    # -- statistics -------------------------------------------------------------------------
    def latencies_ms(self):
        return sorted((done - arrival) * 1e3 for arrival, _, done in self.completed)


def percentile(xs, q):
    if not xs:
        return None
    xs = sorted(xs)
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]
