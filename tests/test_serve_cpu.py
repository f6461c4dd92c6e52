"""The render server's request loop driven by a CPU fake backend: every
request completes, batches are formed in arrival order and admitted by their
measured instance counts within a slot's sort buffers (never beyond the
budget), a batch that does not fit is split with the rest kept at the head
of the queue, and a view larger than a slot fails alone."""
import threading
import time

import numpy as np
import pytest

from paper_2406_18533_amd.serve import BYTES_PER_INSTANCE, RenderServer, percentile


class FakeBackend:
    """Renders a cam to a deterministic image after a short delay; a view
    has K = 2 instances per pixel, known after a probe."""

    def __init__(self, slots=2, capacity=10 ** 9, delay=0.002):
        self.slots = slots
        self.capacity = capacity
        self.delay = delay
        self.probing, self.inflight = {}, {}
        self.launches = []
        self.probes = []

    @staticmethod
    def image(cam):
        return np.full((3, cam["height"], cam["width"]), cam["id"], dtype=np.float32)

    @staticmethod
    def k(cam):
        return 2 * cam["width"] * cam["height"]

    def probe(self, slot, cams):
        assert slot not in self.probing and slot not in self.inflight
        self.probes.append((slot, [c["id"] for c in cams]))
        self.probing[slot] = (time.perf_counter() + self.delay / 4, cams)

    def probe_result(self, slot):
        t, cams = self.probing[slot]
        if time.perf_counter() < t:
            return None
        del self.probing[slot]
        return [self.k(c) for c in cams]

    def launch(self, slot, cams, reproject):
        assert slot not in self.inflight
        k = sum(self.k(c) for c in cams)
        assert k <= self.capacity
        self.launches.append((slot, [c["id"] for c in cams], reproject))
        self.inflight[slot] = (time.perf_counter() + self.delay, cams, k)

    def poll(self, slot):
        t, cams, k = self.inflight[slot]
        if time.perf_counter() < t:
            return None
        del self.inflight[slot]
        return [self.image(c) for c in cams], k, False


def _cam(i, w=32, h=24):
    return {"id": i, "width": w, "height": h}


def test_all_requests_complete_in_order_within_budget():
    cap = 5 * 2 * 64 * 24                  # a few requests' worth of instances per slot
    be = FakeBackend(slots=2, capacity=cap)
    srv = RenderServer(be, max_batch_views=4).start()
    futs = []
    for i in range(40):
        futs.append(srv.submit(_cam(i, 32 + (i % 3) * 16, 24)))
        if i % 7 == 0:
            time.sleep(0.001)
    for i, f in enumerate(futs):
        img = f.result(timeout=10)
        assert img.shape[0] == 3 and (img == i).all()
    srv.stop()
    assert srv.budget == 2 * cap * BYTES_PER_INSTANCE and srv.peak_mem <= srv.budget
    order = [i for _, ids, _ in be.launches for i in ids]
    assert order == sorted(order) and len(order) == 40
    assert max(srv.batches) > 1                    # requests were batched
    lat = srv.latencies_ms()
    assert percentile(lat, 50) <= percentile(lat, 99)


def test_batch_larger_than_a_slot_is_split_and_the_rest_waits_first():
    """Four queued 32x24 views (1536 instances each) against a slot of 3500:
    the probe of all four admits the first two, re-projected on their own,
    and the other two form the next batch ahead of later arrivals."""
    be = FakeBackend(slots=1, capacity=3500, delay=0.01)
    srv = RenderServer(be, max_batch_views=4)
    futs = [srv.submit(_cam(i)) for i in range(4)]       # queued before the loop starts
    srv.start()
    time.sleep(0.002)
    futs.append(srv.submit(_cam(4)))
    for i, f in enumerate(futs):
        assert (f.result(timeout=10) == i).all()
    srv.stop()
    assert be.probes[0] == (0, [0, 1, 2, 3])
    assert be.launches[0] == (0, [0, 1], True)           # a prefix: projected again
    assert be.launches[1][1] == [2, 3]                   # the rest, before request 4
    assert [i for _, ids, _ in be.launches for i in ids] == [0, 1, 2, 3, 4]


def test_view_larger_than_a_slot_fails_alone():
    be = FakeBackend(slots=1, capacity=2 * 32 * 24)
    srv = RenderServer(be, max_batch_views=4).start()
    big = srv.submit(_cam(0, 64, 64))
    small = srv.submit(_cam(1))
    with pytest.raises(ValueError):
        big.result(timeout=10)
    assert (small.result(timeout=10) == 1).all()
    srv.stop()


def test_concurrent_submitters():
    be = FakeBackend(slots=3, capacity=4 * 2 * 32 * 24)
    srv = RenderServer(be, max_batch_views=8).start()
    results = {}

    def client(base):
        fs = [(base + k, srv.submit(_cam(base + k))) for k in range(20)]
        for i, f in fs:
            results[i] = f.result(timeout=10)
    th = [threading.Thread(target=client, args=(100 * t,)) for t in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    srv.stop()
    assert len(results) == 80 and all((img == i).all() for i, img in results.items())
    assert srv.peak_mem <= srv.budget
