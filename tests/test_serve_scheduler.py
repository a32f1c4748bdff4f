"""CPU tests of the serving scheduler (admission by HBM footprint, slots,
continuous batching, rejection, latency accounting) with a fake executor
that computes results with the oracle and completes after a simulated time."""
import time

import numpy as np
import pytest

import oracle
from paper_1609_03986_amd import serve, synth


class FakeExecutor:
    def __init__(self, db, triplets, duration=0.01):
        self.db, self.trip, self.duration = db, triplets, duration
        self.slots = {}
        self.started = []

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
    fp = serve.footprint_bytes(60, 80, 20, len(db))
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
    budget = serve.footprint_bytes(60, 80, 20, len(db)) + 10
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
