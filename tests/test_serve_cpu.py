"""The render server's request loop driven by a CPU fake backend: every
request completes, batches are formed in arrival order, sort-buffer memory
never exceeds the budget, and an undersized estimate is re-rendered."""
import threading
import time

import numpy as np

from paper_2406_18533_amd.serve import BYTES_PER_INSTANCE, InstanceEstimator, RenderServer, percentile


class FakeBackend:
    """Renders a cam to a deterministic image after a short delay; reports K =
    2 instances per pixel."""

    def __init__(self, slots=2, delay=0.002):
        self.slots = slots
        self.delay = delay
        self.inflight = {}
        self.launches = []
        self.lock = threading.Lock()

    @staticmethod
    def image(cam):
        return np.full((3, cam["height"], cam["width"]), cam["id"], dtype=np.float32)

    def launch(self, slot, cams, capacity):
        assert slot not in self.inflight
        k = sum(2 * c["width"] * c["height"] for c in cams)
        self.launches.append((slot, [c["id"] for c in cams], capacity))
        self.inflight[slot] = (time.perf_counter() + self.delay, cams, k, k > capacity)

    def poll(self, slot):
        t, cams, k, over = self.inflight[slot]
        if time.perf_counter() < t:
            return None
        del self.inflight[slot]
        return [self.image(c) for c in cams], k, over

    def render_now(self, slot, cams, capacity):
        self.launch(slot, cams, capacity)
        while True:
            r = self.poll(slot)
            if r is not None:
                return r


def _cam(i, w=32, h=24):
    return {"id": i, "width": w, "height": h}


def test_all_requests_complete_in_order_within_budget():
    be = FakeBackend(slots=2)
    budget = 40 * 32 * 24 * BYTES_PER_INSTANCE      # a few requests' worth of instances
    srv = RenderServer(be, budget, max_batch_views=4, estimator=InstanceEstimator(per_pixel=2.0, margin=1.0)).start()
    futs = []
    for i in range(40):
        futs.append(srv.submit(_cam(i, 32 + (i % 3) * 16, 24)))
        if i % 7 == 0:
            time.sleep(0.001)
    for i, f in enumerate(futs):
        img = f.result(timeout=10)
        assert img.shape[0] == 3 and (img == i).all()
    srv.stop()
    assert srv.peak_mem <= budget
    order = [i for _, ids, _ in be.launches for i in ids]
    assert order == sorted(order) and len(order) == 40
    assert max(srv.batches) > 1                    # requests were batched
    lat = srv.latencies_ms()
    assert percentile(lat, 50) <= percentile(lat, 99)


def test_tiny_budget_still_serves_one_at_a_time():
    be = FakeBackend(slots=2)
    srv = RenderServer(be, 1, max_batch_views=8).start()
    futs = [srv.submit(_cam(i)) for i in range(6)]
    for i, f in enumerate(futs):
        assert (f.result(timeout=10) == i).all()
    srv.stop()
    assert max(srv.batches) == 1


def test_underestimated_batch_is_rendered_again():
    be = FakeBackend(slots=1)
    est = InstanceEstimator(per_pixel=0.1, margin=1.0)   # far below the true 2 per pixel
    srv = RenderServer(be, 10 ** 9, max_batch_views=2, estimator=est).start()
    f = srv.submit(_cam(3, 64, 64))
    assert (f.result(timeout=10) == 3).all()
    srv.stop()
    assert len(be.launches) == 2 and be.launches[1][2] >= 2 * 64 * 64
    assert est.rate[(64, 64)] >= 1.9
