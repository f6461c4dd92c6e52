"""Continuous-batching render server for a device-resident trained model.

Requests (one camera each, any resolution) arrive at any time. A loop
thread keeps up to `slots` batches on the GPU at once, each on a render slot
of its own (a stream with its own projected buffer and a fixed share of the
sort-buffer memory: budget / slots bytes, 16 per sorted instance). A batch
goes through two stages:

1. probe: the requests at the head of the queue (arrival order, up to
   max_views) are projected together (gs_project) and the exact number of
   sorted instances K of each view is read back (the sum of its tiles
   touched);
2. render: the longest prefix of those views whose instances fit the slot's
   sort buffers is admitted (the rest go back to the head of the queue, and
   the prefix is projected again on its own when it is shorter), then
   gs_bin_sort + gs_render_fwd run over its flattened (view, tile) work queue
   exactly as in training and the images are copied to page-locked host
   memory.

Admission is thus by measured sort-buffer memory (no estimate, no overflow,
no re-render). Requests that arrive while batches are on the GPU join the
next batch as soon as a slot frees up, so batches overlap on the device. A
request's image does not depend on what else is in its batch (tiles are per
view and every pixel's list is ordered by (depth, index)), so a result is
the same alone and in the mix. A single view whose K exceeds a slot's share
fails with ValueError.

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
    start: float = 0.0
    done: float = 0.0


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
    slot owns a projected buffer for max_views views (a smaller batch uses
    its front) and sort buffers for `capacity` instances (the memory budget
    split evenly over the slots) and up to max_tiles tiles. Images come back
    to the host in pooled page-locked buffers (see PinnedPool)."""

    def __init__(self, params, slots: int = 4, max_views: int = 8, budget_bytes: int = 16 << 30,
                 max_tiles: int = 8 * 240 * 135, bg=(0.0, 0.0, 0.0)):
        import torch
        from . import _lib
        from . import raster as R
        self.torch, self.R, self._lib = torch, R, _lib
        self.P = params.contiguous()
        self.n = self.P.shape[1]
        self.bg = bg
        self.max_views = max_views
        self.max_tiles = max_tiles
        self.capacity = max(int(budget_bytes) // max(slots, 1) // BYTES_PER_INSTANCE, 1)
        dev = self.P.device
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.flat = [R.alloc_projected(self.n, max_views, torch.float32, dev) for _ in range(slots)]
        wsb = int(_lib.load().gs_bin_workspace_bytes(self.n, max_views, self.capacity, max_tiles))
        self.bufs = []
        for _ in range(slots):
            self.bufs.append({
                "keys": torch.empty(self.capacity, dtype=torch.int32, device=dev),
                "ids": torch.empty(self.capacity, dtype=torch.int32, device=dev),
                "ranges": torch.empty(max_tiles, 2, dtype=torch.int32, device=dev),
                "k": torch.zeros(1, dtype=torch.int64, device=dev),
                "over": torch.zeros(1, dtype=torch.int32, device=dev),
                "ws": torch.empty(max(wsb, 256), dtype=torch.uint8, device=dev)})
        self.kview = [torch.zeros(max_views, dtype=torch.int64, pin_memory=True) for _ in range(slots)]
        self.counts = [torch.zeros(2, dtype=torch.int64, pin_memory=True) for _ in range(slots)]
        self.pool = PinnedPool(torch)
        self.probing = {}
        self.probed = {}
        self.inflight = {}

    @property
    def slots(self) -> int:
        return len(self.streams)

    def _proj_view(self, slot: int, V: int):
        base = self.flat[slot]
        flat = self.torch.as_strided(base, (base.numel(),), (1,), base.storage_offset())
        return flat[: V * self.n * 12].view(V, self.n, 12)

    def _bins(self, slot: int, cams):
        """A Bins-like view of the slot's sort buffers for this camera set."""
        b = self.bufs[slot]
        T = cams.total_tiles()
        if T > self.max_tiles:
            raise ValueError(f"{T} tiles exceed the slot's {self.max_tiles}")

        class _B:
            pass
        x = _B()
        x.capacity, x.total_tiles = self.capacity, T
        x.ids, x.ranges, x.n_instances, x.overflow = b["ids"], b["ranges"], b["k"], b["over"]
        x.struct = self._lib.GsBins(self.capacity, b["keys"].data_ptr(), b["ids"].data_ptr(), b["ranges"].data_ptr(),
                                    b["k"].data_ptr(), b["over"].data_ptr(), b["ws"].data_ptr(), b["ws"].numel())
        return x

    def probe(self, slot: int, cams_list: list):
        """Projects the views on the slot's stream and reads back each view's
        instance count (returns at once; see probe_result)."""
        torch, R = self.torch, self.R
        V = len(cams_list)
        assert V <= self.max_views
        with torch.cuda.stream(self.streams[slot]):
            cams = R.Cameras(cams_list)
            view = self._proj_view(slot, V)
            R.gs_project(self.P, cams, view)
            tiles, _ = R.projected_side_arrays(view)
            self.kview[slot][:V].copy_(tiles.sum(dim=1, dtype=torch.int64), non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.streams[slot])
        self.probing[slot] = (ev, cams, V)

    def probe_result(self, slot: int):
        """None while the probe runs; else the exact K of each view."""
        ev, cams, V = self.probing[slot]
        if not ev.query():
            return None
        del self.probing[slot]
        self.probed[slot] = cams          # reused by a launch of the same views
        return [int(k) for k in self.kview[slot][:V]]

    def launch(self, slot: int, cams_list: list, reproject: bool):
        """Bins and renders the views on the slot's stream (returns at once).
        The projected records must be the slot's for exactly these views:
        from the probe, or projected again here when reproject is set."""
        torch, R = self.torch, self.R
        s = self.streams[slot]
        probed = self.probed.pop(slot, None)
        with torch.cuda.stream(s):
            if reproject or probed is None or probed.n != len(cams_list):
                cams = R.Cameras(cams_list)
            else:
                cams = probed
            view = self._proj_view(slot, len(cams_list))
            if reproject:
                R.gs_project(self.P, cams, view)
            bins = self._bins(slot, cams)
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
        self.inflight[slot] = (ev, host, k_host, cams_list, rgb, cams)

    def poll(self, slot: int):
        """None while running; else (images, instance count, overflowed)."""
        ev, host, k_host, cams_list, *_ = self.inflight[slot]
        if not ev.query():
            return None
        del self.inflight[slot]
        out = [self.pool.lend(buf, (3, c["height"], c["width"])) for buf, c in zip(host, cams_list)]
        return out, int(k_host[0]), bool(k_host[1])

    def render_now(self, slot: int, cams_list: list):
        """Probe and render one batch, waiting for each (one at a time)."""
        self.probe(slot, cams_list)
        while True:
            ks = self.probe_result(slot)
            if ks is not None:
                break
        if sum(ks) > self.capacity:
            raise ValueError(f"{sum(ks)} instances exceed a slot's {self.capacity}")
        self.launch(slot, cams_list, reproject=False)
        while True:
            r = self.poll(slot)
            if r is not None:
                return r


class RenderServer:
    def __init__(self, backend, mem_budget_bytes: int | None = None, max_batch_views: int = 8):
        self.backend = backend
        self.max_views = max_batch_views
        self.budget = mem_budget_bytes if mem_budget_bytes is not None else \
            backend.slots * backend.capacity * BYTES_PER_INSTANCE
        self.queue = collections.deque()
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.state = {s: None for s in range(backend.slots)}     # None, ("probe", batch), ("render", batch, bytes)
        self.mem_used = 0
        self.peak_mem = 0
        self.completed = []
        self.batches = []
        self.probes = 0
        self._stop = False
        self._thread = None

    # -- client side ------------------------------------------------------------------------
    def submit(self, cam: dict) -> Future:
        r = Request(cam, time.perf_counter())
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
    def _busy(self) -> bool:
        return any(st is not None for st in self.state.values())

    def _loop(self):
        while True:
            with self.cv:
                if self._stop and not self.queue and not self._busy():
                    return
                probe = None
                free = [s for s, st in self.state.items() if st is None]
                if free and self.queue:
                    batch = [self.queue.popleft() for _ in range(min(self.max_views, len(self.queue)))]
                    self.state[free[0]] = ("probe", batch)
                    probe = (free[0], batch)
                if probe is None and not self._busy():
                    self.cv.wait(timeout=0.001)
                    continue
            if probe is not None:
                slot, batch = probe
                self.backend.probe(slot, [r.cam for r in batch])
                self.probes += 1
            self._advance()
            if probe is None:
                time.sleep(0.00002)

    def _advance(self):
        cap = self.backend.capacity
        for slot, st in list(self.state.items()):
            if st is None:
                continue
            if st[0] == "probe":
                ks = self.backend.probe_result(slot)
                if ks is None:
                    continue
                batch = st[1]
                m, total = 0, 0
                while m < len(batch) and total + ks[m] <= cap:
                    total += ks[m]
                    m += 1
                if m == 0:                      # one view alone needs more than a slot's sort buffers
                    r = batch[0]
                    r.future.set_exception(ValueError(
                        f"a {r.cam['width']}x{r.cam['height']} view needs {ks[0]} sorted instances, more than a "
                        f"render slot's {cap}"))
                    with self.cv:
                        self.queue.extendleft(reversed(batch[1:]))
                        self.state[slot] = None
                    continue
                with self.cv:
                    if m < len(batch):          # the rest waits at the head of the queue
                        self.queue.extendleft(reversed(batch[m:]))
                    need = total * BYTES_PER_INSTANCE
                    self.mem_used += need
                    self.peak_mem = max(self.peak_mem, self.mem_used)
                    self.state[slot] = ("render", batch[:m], need)
                now = time.perf_counter()
                for r in batch[:m]:
                    r.start = now
                self.backend.launch(slot, [r.cam for r in batch[:m]], reproject=m < len(batch))
                self.batches.append(m)
            else:
                res = self.backend.poll(slot)
                if res is None:
                    continue
                images, k, overflow = res
                _, batch, need = st
                assert not overflow, "a batch admitted by its measured instance count overflowed"
                with self.cv:
                    self.state[slot] = None
                    self.mem_used -= need
                now = time.perf_counter()
                for r, img in zip(batch, images):
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
