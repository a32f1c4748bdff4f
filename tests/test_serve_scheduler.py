"""CPU tests of the serving scheduler (admission by HBM footprint, slots,
continuous batching, rejection, latency accounting) with a fake executor
that computes results with the oracle and completes after a simulated time."""
import time

import numpy as np
import pytest

import oracle
from paper_1609_03986_amd import serve, synth


class FakeExecutor:
    """Oracle results after a simulated duration.  Memory figures: `retained`
    bytes kept across requests, and `extra(n_kps)` workspace beyond it."""

    def __init__(self, db, triplets, duration=0.01, retained=0, extra=lambda n: 0):
        self.db, self.trip, self.duration = db, triplets, duration
        self.retained, self.extra = retained, extra
        self.slots = {}
        self.started = []

    def workspace_bytes(self, n_kps):
        return self.extra(n_kps)

    def retained_bytes(self):
        return self.retained

    def start(self, slot, req):
        assert slot not in self.slots, "slot reused while busy"
        d, _ = oracle.extract(req.image, req.kps, self.trip)
        out = oracle.knn(d, self.db, k=2, ratio=0.8)
        self.slots[slot] = (time.perf_counter() + self.duration, out)
        self.started.append(req.rid)

    def poll(self, slot):
        return time.perf_counter() >= self.slots[slot][0]

    def finish(self, slot):
        return self.slots.pop(slot)[1]


def small_requests(n, gap, seed=0, size=(60, 80), kp=20):
    g = np.random.default_rng(seed)
    img = synth.smoothed_noise(g, *size)
    return [serve.Request(i, img, synth.random_keypoints(g, kp, *size), i * gap) for i in range(n)]


@pytest.fixture(scope="module")
def db():
    return synth.random_descriptors(np.random.default_rng(1), 300)


def test_results_match_oracle_and_arrive_in_order(db, triplets):
    ex = FakeExecutor(db, triplets, 0.005)
    reqs = small_requests(6, 0.002)
    sched = serve.Scheduler(ex, n_slots=2, hbm_budget=1 << 30, db_rows=len(db))
    results, rejected, stats = sched.run(reqs)
    assert not rejected and stats["served"] == 6
    assert ex.started == list(range(6))                        # FIFO admission
    for r in results:
        d, _ = oracle.extract(reqs[r.rid].image, reqs[r.rid].kps, triplets)
        wi, wd, wa = oracle.knn(d, db)
        assert np.array_equal(r.idx, wi) and np.array_equal(r.dist, wd)
        assert r.arrival <= r.admitted <= r.done


def test_overlapping_arrivals_run_concurrently(db, triplets):
    ex = FakeExecutor(db, triplets, 0.03)
    sched = serve.Scheduler(ex, n_slots=3, hbm_budget=1 << 30, db_rows=len(db))
    _, _, stats = sched.run(small_requests(6, 0.001))
    assert stats["max_inflight"] == 3


def test_hbm_budget_limits_inflight_work(db, triplets):
    reqs = small_requests(5, 0.0)
    fp = serve.footprint_bytes(60, 80, 20)
    ex = FakeExecutor(db, triplets, 0.01)
    sched = serve.Scheduler(ex, n_slots=4, hbm_budget=2 * fp, db_rows=len(db))
    results, rejected, stats = sched.run(reqs)
    assert stats["served"] == 5 and not rejected
    assert stats["max_inflight"] == 2                          # memory, not slots, binds
    # queued requests wait: admissions are at least one duration apart per pair
    adm = sorted(r.admitted for r in results)
    assert adm[2] - adm[0] >= 0.009


def test_request_larger_than_budget_is_rejected(db, triplets):
    g = np.random.default_rng(2)
    big = serve.Request(0, synth.smoothed_noise(g, 200, 300), synth.random_keypoints(g, 50, 200, 300), 0.0)
    small = small_requests(2, 0.0, seed=3)
    for i, r in enumerate(small):
        r.rid = i + 1
    budget = serve.footprint_bytes(60, 80, 20) + 10
    sched = serve.Scheduler(FakeExecutor(db, triplets, 0.001), 2, budget, len(db))
    results, rejected, stats = sched.run([big] + small)
    assert rejected == [0]
    assert sorted(r.rid for r in results) == [1, 2]


def test_poisson_arrivals_and_request_mix_are_seeded():
    pool = {hw: [np.zeros((4, 4), np.uint8)] for hw in serve.SIZES}
    a = serve.make_requests(50, 100.0, pool, seed=4)
    b = serve.make_requests(50, 100.0, pool, seed=4)
    assert [r.arrival for r in a] == [r.arrival for r in b]
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert 0.3 / 100 < gaps.mean() < 3.0 / 100
    n = np.array([len(r.kps) for r in a])
    assert n.min() >= 500 and n.max() <= 50000


def test_footprint_counts_image_keypoints_results_and_workspace():
    assert serve.footprint_bytes(10, 20, 0) == 200
    assert serve.footprint_bytes(10, 20, 3) == 200 + 3 * (16 + 64 + 17)
    assert serve.footprint_bytes(10, 20, 3, workspace_bytes=1000) == 200 + 3 * 97 + 1000


def test_retained_memory_and_extra_workspace_count_against_the_budget(db, triplets):
    fp = serve.footprint_bytes(60, 80, 20)
    # Retained memory leaves room for exactly one request at a time.
    ex = FakeExecutor(db, triplets, 0.01, retained=10_000_000)
    sched = serve.Scheduler(ex, n_slots=4, hbm_budget=10_000_000 + fp + fp // 2, db_rows=len(db))
    results, rejected, stats = sched.run(small_requests(3, 0.0))
    assert stats["served"] == 3 and not rejected and stats["max_inflight"] == 1
    # Retained memory above the budget: every request is rejected.
    ex = FakeExecutor(db, triplets, 0.001, retained=1 << 40)
    results, rejected, stats = serve.Scheduler(ex, 2, 1 << 30, len(db)).run(small_requests(2, 0.0))
    assert rejected == [0, 1] and not results
    # A request whose extra workspace does not fit is rejected; the others run.
    ex = FakeExecutor(db, triplets, 0.001, extra=lambda n: 1 << 40 if n == 21 else 0)
    reqs = small_requests(3, 0.0)
    g = np.random.default_rng(9)
    reqs[1].kps = synth.random_keypoints(g, 21, 60, 80)
    results, rejected, stats = serve.Scheduler(ex, 2, 1 << 30, len(db)).run(reqs)
    assert rejected == [1] and sorted(r.rid for r in results) == [0, 2]
    assert serve.Scheduler(ex, 2, 1 << 30, len(db)).footprint(reqs[1]) == \
        serve.footprint_bytes(60, 80, 21, 1 << 40)


def test_waiting_requests_time_out(db, triplets):
    # One slot, each request takes 30 ms: with a 10 ms timeout the requests
    # queued behind the first are dropped before admission.
    ex = FakeExecutor(db, triplets, 0.03)
    sched = serve.Scheduler(ex, n_slots=1, hbm_budget=1 << 30, db_rows=len(db), timeout_s=0.01)
    results, rejected, stats = sched.run(small_requests(4, 0.0))
    assert [r.rid for r in results] == [0]
    assert sorted(stats["timed_out"]) == [1, 2, 3] and ex.started == [0]


def test_cancelled_requests_are_dropped(db, triplets):
    ex = FakeExecutor(db, triplets, 0.02)
    sched = serve.Scheduler(ex, n_slots=1, hbm_budget=1 << 30, db_rows=len(db))
    sched.cancel(2)
    results, rejected, stats = sched.run(small_requests(4, 0.001))
    assert sorted(r.rid for r in results) == [0, 1, 3]
    assert stats["cancelled"] == [2] and 2 not in ex.started


def test_cancelled_in_flight_result_is_discarded(db, triplets):
    class CancelOnStart(FakeExecutor):
        def start(self, slot, req):
            super().start(slot, req)
            if req.rid == 1:
                sched.cancel(1)
    ex = CancelOnStart(db, triplets, 0.005)
    sched = serve.Scheduler(ex, n_slots=2, hbm_budget=1 << 30, db_rows=len(db))
    results, rejected, stats = sched.run(small_requests(3, 0.0))
    assert sorted(r.rid for r in results) == [0, 2] and stats["cancelled"] == [1]
    assert 1 in ex.started
