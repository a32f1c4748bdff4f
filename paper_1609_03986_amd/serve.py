"""Serving: continuous batching of extract + match requests against a
device-resident descriptor database.

A request is one u8 image with its keypoints.  Serving it means:
  * extracting its LATCH descriptors (latch_extract);
  * matching them 2-NN with the ratio test against the resident database
    (hamming_knn);
  * returning (idx, dist, accept) per keypoint.
The paper runs detection, description and matching of several images
concurrently on self-contained streams (Sec. 4, "CUDA Integration").  Here
that becomes a request loop.

  * Scheduler.  FIFO over arrived requests.  A request is admitted when a slot
    is free and its HBM footprint fits what the budget leaves after the
    memory the executor keeps (the slots' reserved workspaces).  A request
    larger than that is rejected; one that waits longer than the timeout, or
    that is cancelled, is dropped (a cancelled request already on the GPU
    finishes there, and its result is discarded).
  * Slots.  Each slot owns a HIP stream and a library handle whose workspace
    is reserved once, at creation, for the largest request of the mix (the
    library's own figure, hamming_knn_workspace_size), so admitted requests
    run concurrently on the device and no request makes the library allocate
    or wait.  A request that arrives while others are in flight starts as
    soon as a slot and memory free up (continuous batching).
  * Executors.  GpuExecutor drives the C ABI through the binding.  The
    scheduler only needs start / poll / finish and the memory figures, so
    tests can drive it with a fake executor on the CPU.

Latency is measured from a request's arrival to the completion of its results
on the host.
"""
import collections
import dataclasses
import json
import sys
import time

import numpy as np

DESC_BYTES = 64
KEYPOINT_BYTES = 16
RESULT_BYTES_PER_QUERY = 2 * 4 + 2 * 4 + 1      # idx, dist (k = 2), accept


@dataclasses.dataclass
class Request:
    rid: int
    image: np.ndarray          # uint8 [H, W]
    kps: np.ndarray            # float32 [n, 4]
    arrival: float = 0.0       # seconds from the start of the run


@dataclasses.dataclass
class Result:
    rid: int
    idx: np.ndarray
    dist: np.ndarray
    accept: np.ndarray
    arrival: float
    admitted: float
    done: float

    @property
    def latency(self):
        return self.done - self.arrival


def footprint_bytes(height, width, n_kps, workspace_bytes=0):
    """Device bytes a request holds while in flight: its image, keypoints,
    descriptors and results, plus any matcher workspace it needs beyond what
    its slot has reserved (`workspace_bytes`, from the executor, which asks
    the library)."""
    return (height * width + n_kps * (KEYPOINT_BYTES + DESC_BYTES + RESULT_BYTES_PER_QUERY)
            + workspace_bytes)


class Scheduler:
    """FIFO admission by slot and HBM footprint, with a waiting timeout and
    cancellation; polls in-flight work."""

    def __init__(self, executor, n_slots, hbm_budget, db_rows, clock=time.perf_counter,
                 idle_sleep=50e-6, timeout_s=None):
        self.ex = executor
        self.n_slots = n_slots
        self.budget = hbm_budget
        self.db_rows = db_rows
        self.clock = clock
        self.idle_sleep = idle_sleep
        self.timeout_s = timeout_s
        self.cancelled = set()

    def footprint(self, req):
        h, w = req.image.shape
        return footprint_bytes(h, w, len(req.kps), self.ex.workspace_bytes(len(req.kps)))

    def cancel(self, rid):
        """Drop request `rid`: before admission it never runs; in flight, its
        result is discarded when it completes."""
        self.cancelled.add(rid)

    def run(self, requests):
        """Serve `requests` (sorted by arrival).  Returns (results, rejected ids,
        stats); stats lists the ids that timed out or were cancelled."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
        free = list(range(self.n_slots))
        inflight = {}                           # slot -> (request, footprint, admit time)
        used = 0
        results, rejected, timed_out, dropped = [], [], [], []
        max_inflight = 0
        t0 = self.clock()
        while pending or waiting or inflight:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # completions
            for slot in list(inflight):
                if self.ex.poll(slot):
                    req, fp, t_adm = inflight.pop(slot)
                    idx, dist, acc = self.ex.finish(slot)
                    if req.rid in self.cancelled:
                        dropped.append(req.rid)
                    else:
                        results.append(Result(req.rid, idx, dist, acc, req.arrival, t_adm,
                                              self.clock() - t0))
                    used -= fp
                    free.append(slot)
            # cancellations and time-outs of waiting requests
            if waiting and (self.cancelled or self.timeout_s is not None):
                now = self.clock() - t0
                keep = collections.deque()
                for r in waiting:
                    if r.rid in self.cancelled:
                        dropped.append(r.rid)
                    elif self.timeout_s is not None and now - r.arrival > self.timeout_s:
                        timed_out.append(r.rid)
                    else:
                        keep.append(r)
                waiting = keep
            # admissions, in arrival order
            while waiting and free:
                req = waiting[0]
                fp = self.footprint(req)
                room = self.budget - self.ex.retained_bytes()
                if fp > room:
                    rejected.append(waiting.popleft().rid)
                    continue
                if used + fp > room:
                    break
                waiting.popleft()
                slot = free.pop()
                self.ex.start(slot, req)
                inflight[slot] = (req, fp, self.clock() - t0)
                used += fp
            max_inflight = max(max_inflight, len(inflight))
            if not inflight and not waiting and pending:
                # idle until the next arrival
                delay = pending[0].arrival - (self.clock() - t0)
                if delay > 0:
                    time.sleep(min(delay, 0.01))
            elif inflight:
                time.sleep(self.idle_sleep)
        wall = self.clock() - t0
        lat = np.array([r.latency for r in results]) if results else np.zeros(1)
        stats = {"served": len(results), "rejected": len(rejected), "wall_s": wall,
                 "throughput_rps": len(results) / wall if wall > 0 else 0.0,
                 "p50_ms": float(np.percentile(lat, 50) * 1e3),
                 "p99_ms": float(np.percentile(lat, 99) * 1e3),
                 "max_inflight": max_inflight, "timed_out": timed_out, "cancelled": dropped}
        return results, rejected, stats


class GpuExecutor:
    """Runs requests on the GPU, one library handle and one HIP stream per slot,
    matching against a device-resident database (torch int32 [N, 16]).  Each
    slot's workspace is reserved at creation for every request of up to
    `max_kps` keypoints."""

    def __init__(self, db, triplets, n_slots, ratio=0.8, path="auto", max_kps=50000):
        import torch
        from . import autotune
        from .binding import Latch
        self.torch = torch
        self.db = db
        self.ratio = ratio
        self.path = path
        self.slots = []
        for _ in range(n_slots):
            lat = Latch(triplets)
            self.tuning = autotune.load(lat, autotune.IN_TREE)
            self.slots.append({"stream": torch.cuda.Stream(), "lat": lat, "event": None,
                               "out": None})
        self.reserved = self.largest_workspace(max_kps)
        for s in self.slots:
            s["lat"].reserve(self.reserved)

    def workspace_need(self, n_kps):
        """The library's workspace figure for matching n_kps queries against the database."""
        return self.slots[0]["lat"].knn_workspace_size(n_kps, self.db.shape[0], self.path)

    def largest_workspace(self, max_kps):
        """The largest need of any request of 1 .. max_kps keypoints.  The need
        grows with the query count while the number of query groups (256 or
        384 queries, multiples of 128) stays fixed, so the largest of each
        group count is at a multiple of 128 or at max_kps."""
        counts = sorted({min(max_kps, 128 * g) for g in range(1, -(-max_kps // 128) + 1)})
        return max(self.workspace_need(n) for n in counts)

    def workspace_bytes(self, n_kps):
        """Workspace a request needs beyond its slot's reservation."""
        return max(0, self.workspace_need(n_kps) - self.reserved)

    def retained_bytes(self):
        """Device memory the slots keep across requests (their workspaces)."""
        return sum(s["lat"].reserve(0) for s in self.slots)

    def start(self, slot, req):
        torch = self.torch
        s = self.slots[slot]
        with torch.cuda.stream(s["stream"]):
            img = torch.from_numpy(req.image).pin_memory().to("cuda", non_blocking=True)
            kps = torch.from_numpy(req.kps).pin_memory().to("cuda", non_blocking=True)
            desc = s["lat"].extract(img, kps, stream=s["stream"])
            idx, dist, acc = s["lat"].knn(desc, self.db, k=2, ratio=self.ratio, path=self.path,
                                          stream=s["stream"])
            host = (torch.empty(idx.shape, dtype=idx.dtype, pin_memory=True),
                    torch.empty(dist.shape, dtype=dist.dtype, pin_memory=True),
                    torch.empty(acc.shape, dtype=acc.dtype, pin_memory=True))
            host[0].copy_(idx, non_blocking=True)
            host[1].copy_(dist, non_blocking=True)
            host[2].copy_(acc, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s["stream"])
        s["event"] = ev
        s["out"] = host
        s["keep"] = (img, kps, desc, idx, dist, acc)

    def poll(self, slot):
        return self.slots[slot]["event"].query()

    def finish(self, slot):
        s = self.slots[slot]
        s["event"].synchronize()
        out = tuple(t.numpy().copy() for t in s["out"])
        s["out"] = s["keep"] = s["event"] = None
        return out

    def close(self):
        for s in self.slots:
            s["lat"].close()


# --------------------------------------------------------------------------
# The serving workload: database of 1,000,000 descriptors, requests drawn from
# the uneven image mix, Poisson arrivals.
# --------------------------------------------------------------------------
SIZES = [(240, 320), (480, 640), (720, 1280), (1080, 1920), (3000, 4000)]


def request_pool(seed=5, per_size=3):
    """A few seeded images per size of the mix (requests reuse them)."""
    from . import synth
    g = np.random.default_rng(seed)
    return {hw: [synth.smoothed_noise(g, *hw) for _ in range(per_size)] for hw in SIZES}


def make_requests(n, qps, pool, seed=11):
    """n requests with Poisson arrivals at `qps`, image size uniform over the
    mix, keypoint count round(LogNormal(ln 5000, 1)) clipped to [500, 50000]."""
    from . import synth
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0 / qps, n))
    reqs = []
    for i in range(n):
        hw = SIZES[int(g.integers(0, len(SIZES)))]
        img = pool[hw][int(g.integers(0, len(pool[hw])))]
        m = int(np.clip(np.rint(g.lognormal(np.log(5000), 1.0)), 500, 50000))
        kps = synth.random_keypoints(g, m, hw[0], hw[1])
        reqs.append(Request(i, img, kps, float(t[i])))
    return reqs


def max_requests(n, pool, seed=98):
    """n simultaneous requests of the mix's largest size (4000x3000, 50,000
    keypoints): a warm-up that touches every slot at its largest footprint."""
    from . import synth
    g = np.random.default_rng(seed)
    hw = SIZES[-1]
    return [Request(i, pool[hw][0], synth.random_keypoints(g, 50000, *hw), 0.0) for i in range(n)]


def build_database(lat, rows=1_000_000, images=50, seed=3):
    """`rows` descriptors extracted on the GPU from `images` seeded 1920x1080
    images (20,000 keypoints each for the default sizes)."""
    import torch
    from . import synth
    g = np.random.default_rng(seed)
    per = -(-rows // images)
    out = torch.empty((images * per, 16), dtype=torch.int32, device="cuda")
    for i in range(images):
        img = torch.from_numpy(synth.smoothed_noise(g, 1080, 1920)).cuda()
        kps = torch.from_numpy(synth.random_keypoints(g, per, 1080, 1920)).cuda()
        lat.extract(img, kps, desc=out[i * per:(i + 1) * per])
    torch.cuda.synchronize()
    return out[:rows]


def main(argv=None):
    import argparse
    import torch
    from . import synth
    from .binding import Latch
    ap = argparse.ArgumentParser(description="Serve extract + match requests against a "
                                             "device-resident database; print one JSON line per rate.")
    ap.add_argument("--qps", type=float, nargs="+", default=[50, 200, 800])
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--db-rows", type=int, default=1_000_000)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--hbm-budget-gb", type=float, default=8.0)
    ap.add_argument("--path", default="auto", choices=["auto", "mfma", "fp4", "popcount"])
    ap.add_argument("--timeout-s", type=float, default=None,
                    help="drop requests that wait longer than this before admission")
    args = ap.parse_args(argv)
    trip = synth.triplet_table()
    builder = Latch(trip)
    db = build_database(builder, args.db_rows)
    import hashlib
    db_sha256 = hashlib.sha256(db.cpu().numpy().tobytes()).hexdigest()   # record of the inputs
    pool = request_pool()
    ex = GpuExecutor(db, trip, args.slots, path=args.path)
    sched = Scheduler(ex, args.slots, int(args.hbm_budget_gb * 2 ** 30), args.db_rows,
                      timeout_s=args.timeout_s)
    warm = max_requests(args.slots, pool)
    sched.run(warm)
    for qps in args.qps:
        reqs = make_requests(args.requests, qps, pool, seed=int(qps))
        results, rejected, stats = sched.run(reqs)
        pairs = sum(len(r.idx) for r in results) * args.db_rows
        stats.update({"offered_qps": qps, "db_rows": args.db_rows, "slots": args.slots,
                      "pairs_per_s": pairs / stats["wall_s"], "path": args.path,
                      "slot_workspace_bytes": ex.reserved, "db_sha256": db_sha256,
                      "tuning": "in-tree table" if ex.tuning is not None else "library default",
                      "timed_out": len(stats["timed_out"]), "cancelled": len(stats["cancelled"])})
        print(json.dumps(stats), flush=True)
    ex.close()
    builder.close()


if __name__ == "__main__":
    sys.exit(main())
