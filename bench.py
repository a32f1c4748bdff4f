"""Benchmark: LATCH extraction + 2-NN Hamming matching on one MI355X.

One step is one replay of the SfM batch plan (a HIP graph captured once by
latch_plan_create): extraction of 20,000 oriented, scaled keypoints in each of
64 images of 3000x2000 u8 (1.28 M descriptors, one batched launch), then 2-NN
matching with ratio 0.8 over the 63 consecutive image pairs, 20,000 x 20,000
each (2.52e10 pairs, one persistent batched launch).  The images are crops of
one textured mosaic (a synthetic stand-in for a photogrammetry scene, the
setting of the paper's Sec. 5).  Inputs are resident in HBM before the timed
region starts.

Prints one JSON line.  `value` is descriptors extracted and matched per
second for the whole step; `pairs_per_s` the matched pairs per second.  The
roofline object covers the step's dominant kernel: its average duration
comes from HIP events the library records on its launch stream around each
kernel, in a run of the same launches (the graph holds the same two kernels
with the same arguments).  Components: the same batch as one call per image
and per pair (the plain form), the PCIe-inclusive step, a 1920x1080 image
pair (extraction, and matching on every matcher path), the uneven 256-image
batch as a plan, a short serving run against a 1,000,000-row resident
database, FAST detection, the weighted 64 x 64 / 8 x 8 geometry and dense
per-pixel descriptors with windowed matching.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LATCH desc/s + Hamming pairs/s (MFMA vs popcount) at 1 GPU; p50/p99 ms"
WORKLOAD = ("SfM batch: 64 images of 3000x2000 u8 (crops of one textured mosaic), 20,000 "
            "keypoints each (angle U[0,360), scale 1.2^U{0..7}), 512-bit LATCH over 48x48 "
            "windows with 7x7 patches (1.28 M descriptors), then brute-force 2-NN Hamming "
            "matching with ratio 0.8 over the 63 consecutive image pairs (20,000 x 20,000 each), "
            "replayed as one captured plan")

# MI355X published peaks and chip constants.
PEAK_HBM_GBS = 8000.0
PEAK_INT8_MFMA_TOPS = 5000.0           # dense int8 MFMA, 10^12 ops/s
PEAK_FP4_MFMA_TOPS = 10100.0           # dense FP4 MFMA, 10^12 ops/s
PEAK_VECTOR_TOPS = 157.3               # published vector peak (fp32), 10^12 ops/s
CUS, CLOCK_GHZ, LANES = 256, 2.4, 64
# One 32-bit integer VALU operation per lane per cycle.
PEAK_INT_TOPS = CUS * LANES * CLOCK_GHZ / 1000.0         # 39.3
# Integer VALU with v_dot4_u32_u8: 4 byte MACs = 8 ops per lane per cycle.
PEAK_DOT4_TOPS = PEAK_INT_TOPS * 8                       # 314.6
# v_dot2_i32_i16: 2 MACs = 4 ops per lane per cycle.
PEAK_DOT2_TOPS = PEAK_INT_TOPS * 4                       # 157.3
# Algorithmic work per unit.  Extraction: per descriptor 512 triplets x 2
# patch distances x 49 squared differences, 2 operations each (subtract,
# multiply-accumulate).  Matching: per pair the 512 multiply-accumulates of
# a.b (1,024 operations).
EXTRACT_OPS_PER_DESC = 512 * 2 * 49 * 2                  # 100,352
MATCH_OPS_PER_PAIR = 512 * 2
POPCOUNT_OPS_PER_PAIR = 32                               # 16 XOR + 16 popcount-accumulate
DETECT_THRESHOLD = 20                                    # FAST threshold of the detection component
# Weighted CLATCH geometry: per descriptor 512 x 2 x 64 weighted squared
# differences x 4 ops (sub, square, weight, add), against the v_dot2_i32_i16 rate.
WEIGHTED_OPS_PER_DESC = 512 * 2 * 64 * 4
# Dense CLATCH: per pixel and triplet, G = (C1 - C2)(C1 + C2 - 2A) (4 ops), a
# running sum down the rows (2), one across the columns (2) and the compare
# (1); dense matching: 32 ops per candidate.  Both against the 32-bit integer
# VALU rate.
DENSE_OPS_PER_PIXEL = 512 * 9
DENSE_RADIUS = 4
TUNING_TABLE = os.path.join(ROOT, "paper_1609_03986_amd", "tuning.json")
PAPER = {"clatch_extraction_us_per_desc": 0.5, "desc_per_s": 2.0e6,
         "hardware": "NVIDIA GTX 970M", "source": "Table 1",
         "matching": "no standalone matching rate reported (Sec. 4 describes the kernel only)"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--path", default="auto", choices=["auto", "mfma", "fp4", "popcount"],
                    help="matcher path of the plan (auto: the handle's tuning table)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="approximate CPU time budget of the oracle baseline (0 = skip)")
    ap.add_argument("--components", default="all",
                    help="comma-separated components to run besides the headline step "
                         "(all, none, or any of: plain, pcie, hd, uneven, serve, match_1m, "
                         "detect, weighted, dense)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (3 times) and exit; "
                         "its FETCH_SIZE / WRITE_SIZE readings calibrate the HBM traffic counters")
    return ap.parse_args()


def copy_calibration(mib):
    import torch
    x = torch.full((mib << 20,), 7, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_mib": mib, "bytes": mib << 20}), flush=True)


def recorded_traffic(kernel, workload):
    """HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE) recorded in
    profiles/traffic.json for this kernel on this workload, or None when
    missing or when the kernel's source has changed since the counters were
    taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["kernels"]
        rec = rec["%s@%s" % (kernel, workload)]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


def log(msg):
    """Progress of the run, on stderr (the JSON line alone goes to stdout)."""
    print("[bench %.1fs] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr, flush=True)


T_START = time.perf_counter()


def percentile(xs, p):
    return float(np.percentile(np.asarray(xs), p))


def load_tuning(lat):
    """Install the in-tree autotuned table when it was measured on this
    device and library version; returns a description of the table in use."""
    from paper_1609_03986_amd import autotune
    t = autotune.load(lat, TUNING_TABLE)
    if t is None:
        return {"source": "library default", "table": lat.get_tuning().to_dict()}
    return {"source": os.path.relpath(TUNING_TABLE, ROOT), "key": autotune.cache_key(), "table": t}


class Timer:
    """Wall time of repeated calls, bracketed by device synchronisation."""

    def __init__(self, torch):
        self.torch = torch

    def loop(self, fn, steps, warmup=0, per_step=False):
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        if per_step:
            starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
            stops = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        t0 = time.perf_counter()
        for i in range(steps):
            if per_step:
                starts[i].record(stream)
            fn()
            if per_step:
                stops[i].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat_ms = [s.elapsed_time(e) for s, e in zip(starts, stops)] if per_step else None
        return wall, lat_ms


def kernel_times(lat, torch, fn, reps, names):
    """Average durations of the library's kernels over `reps` calls of fn,
    from the HIP events the library records on its launch stream."""
    lat.timing(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    out = {}
    for name in names:
        n, total = lat.timing_read(name)
        if n:
            out[name] = {"launches_per_step": n / reps, "avg_ms": total / n,
                         "ms_per_step": total / reps}
    lat.timing(False)
    return out


class Batch:
    """A batch of images on the device: image table, keypoints, image ids,
    consecutive-pair table and output buffers, with its captured plan and the
    same work as eager batched calls and as one call per image and pair."""

    def __init__(self, torch, lat, imgs, kps, path):
        from paper_1609_03986_amd.binding import image_table, pair_table
        self.torch, self.lat, self.path = torch, lat, path
        self.counts = [len(k) for k in kps]
        self.first = np.concatenate([[0], np.cumsum(self.counts)[:-1]]).astype(np.int64)
        self.total = int(sum(self.counts))
        self.n_img = len(imgs)
        self.dimgs = [torch.from_numpy(im).cuda() for im in imgs]
        self.kp_all = torch.from_numpy(np.concatenate(kps).astype(np.float32)).cuda()
        self.ids = torch.from_numpy(np.repeat(np.arange(self.n_img, dtype=np.int32),
                                              self.counts)).cuda()
        self.table = image_table(self.dimgs)
        self.pairs_np = np.array([(self.first[i], self.counts[i], self.first[i + 1],
                                   self.counts[i + 1], self.first[i])
                                  for i in range(self.n_img - 1)], np.int64)
        self.pairs = pair_table(self.pairs_np)
        self.n_pairs = int(sum(self.counts[i] * self.counts[i + 1] for i in range(self.n_img - 1)))
        self.desc = torch.empty((self.total, 16), dtype=torch.int32, device="cuda")
        self.idx = torch.full((self.total, 2), -2, dtype=torch.int32, device="cuda")
        self.dist = torch.full((self.total, 2), -2, dtype=torch.int32, device="cuda")
        self.acc = torch.zeros(self.total, dtype=torch.uint8, device="cuda")
        self.plan = lat.plan(self.table, self.n_img, self.ids, self.kp_all, self.desc, self.pairs,
                             self.idx, self.dist, self.acc, path=path)
        lat.reserve(max(lat.knn_batch_workspace_size(self.n_img - 1, self.total),
                        lat.extract_batch_workspace_size(self.n_img, self.total)))

    def run_plan(self):
        self.plan.run()

    def run_eager(self):
        """The plan's two launches as eager calls (same kernels and arguments)."""
        self.lat.extract_batch(self.table, self.n_img, self.ids, self.kp_all, self.desc)
        self.lat.knn_batch(self.desc, self.desc, self.pairs, self.total, path=self.path,
                           idx=self.idx, dist=self.dist, accept=self.acc)

    def per_image_form(self):
        """One latch_extract per image and one hamming_knn per pair, into
        separate outputs; returns (run, outputs)."""
        torch, lat = self.torch, self.lat
        desc = torch.empty_like(self.desc)
        idx = torch.full_like(self.idx, -2)
        dist = torch.full_like(self.dist, -2)
        acc = torch.zeros_like(self.acc)
        ks = [self.kp_all[self.first[i]:self.first[i] + self.counts[i]] for i in range(self.n_img)]
        ds = [desc[self.first[i]:self.first[i] + self.counts[i]] for i in range(self.n_img)]
        need = max(lat.knn_workspace_size(self.counts[i], self.counts[i + 1], self.path)
                   for i in range(self.n_img - 1))
        lat.reserve(need)

        def run():
            for i in range(self.n_img):
                lat.extract(self.dimgs[i], ks[i], ds[i])
            for i in range(self.n_img - 1):
                o = slice(int(self.first[i]), int(self.first[i] + self.counts[i]))
                lat.knn(ds[i], ds[i + 1], path=self.path, idx=idx[o], dist=dist[o], accept=acc[o])
        return run, (desc, idx, dist, acc)

    def same_as(self, outs):
        d, i, di, a = outs
        t = self.torch
        return (t.equal(d, self.desc) and t.equal(i, self.idx) and t.equal(di, self.dist) and
                t.equal(a, self.acc))

    def close(self):
        self.plan.close()


def roofline_of(kernels, desc_per_launch, pairs_per_launch, workload, kernel=None):
    """Roofline object of `kernel`, by default the kernel with the largest time per step."""
    dom = kernel or max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    kd = kernels[dom]
    sec = kd["avg_ms"] * 1e-3
    if dom in ("knn_batch_fp4", "knn_fp4"):
        achieved = pairs_per_launch * MATCH_OPS_PER_PAIR / sec / 1e12
        roof = {"bound": "mfma", "peak": PEAK_FP4_MFMA_TOPS, "unit": "TFLOP/s",
                "work": "%d pairs x 1,024 ops (FP4 MFMA)" % pairs_per_launch}
    elif dom in ("knn_batch_mfma", "knn_mfma"):
        achieved = pairs_per_launch * MATCH_OPS_PER_PAIR / sec / 1e12
        roof = {"bound": "mfma", "peak": PEAK_INT8_MFMA_TOPS, "unit": "TFLOP/s",
                "work": "%d pairs x 1,024 ops (int8 MFMA)" % pairs_per_launch}
    elif dom in ("knn_batch_popcount", "knn_popcount"):
        achieved = pairs_per_launch * POPCOUNT_OPS_PER_PAIR / sec / 1e12
        roof = {"bound": "alu", "peak": PEAK_INT_TOPS, "unit": "TFLOP/s",
                "work": "%d pairs x 32 VALU ops" % pairs_per_launch}
    else:
        achieved = desc_per_launch * EXTRACT_OPS_PER_DESC / sec / 1e12
        roof = {"bound": "alu", "peak": PEAK_VECTOR_TOPS, "unit": "TFLOP/s",
                "work": "%d descriptors x 100,352 ops" % desc_per_launch,
                "frac_of_dot4_peak": achieved / PEAK_DOT4_TOPS}
    roof.update({"kernel": dom, "achieved": achieved, "frac": achieved / roof["peak"],
                 "avg_ms": kd["avg_ms"], "traffic": recorded_traffic(dom, workload),
                 "traffic_unit": "bytes/launch"})
    return roof


def cpu_baseline_sfm(imgs, kps, triplets, total_desc, total_pairs, budget_s):
    """The oracle on a bounded sample of the SfM batch, extrapolated to one
    whole step: extraction of a keypoint sample of several images, and 2-NN
    of query samples of several pairs against their whole train image."""
    import oracle
    ex_t = ex_n = m_t = m_n = 0.0
    rounds = 0
    t_start = time.perf_counter()
    n_img = len(imgs)
    while time.perf_counter() - t_start < budget_s and rounds < n_img - 1:
        i = rounds
        t0 = time.perf_counter()
        q, _ = oracle.extract(imgs[i], kps[i][:5000], triplets)
        t, _ = oracle.extract(imgs[i + 1], kps[i + 1], triplets)
        ex_t += time.perf_counter() - t0
        ex_n += len(q) + len(t)
        t0 = time.perf_counter()
        oracle.knn(q, t, k=2, ratio=0.8)
        m_t += time.perf_counter() - t0
        m_n += len(q) * len(t)
        rounds += 1
    cores = oracle.num_threads()
    ex_rate, m_rate = ex_n / ex_t, m_n / m_t
    step_s = total_desc / ex_rate + total_pairs / m_rate
    # The same sample kinds on one thread (a smaller sample).
    oracle.set_threads(1)
    t0 = time.perf_counter()
    q1, _ = oracle.extract(imgs[0], kps[0][:200], triplets)
    t1, _ = oracle.extract(imgs[1], kps[1][:2000], triplets)
    ex1 = 2200 / (time.perf_counter() - t0)
    t0 = time.perf_counter()
    oracle.knn(q1, t1, k=2, ratio=0.8)
    m1 = 200 * 2000 / (time.perf_counter() - t0)
    oracle.set_threads(cores)
    return {"value": total_desc / step_s, "unit": "desc/s", "cores": cores, "kind": "oracle",
            "sample": "%d image pairs: 5,000 query keypoints of image i and all 20,000 of image "
                      "i + 1 extracted (%d descriptors, %.1f s), then 2-NN of the 5,000 queries "
                      "against the 20,000 (%.3g pairs, %.1f s); one whole step extrapolated "
                      "linearly as 1.28 M / extraction rate + 2.52e10 / matching rate"
                      % (rounds, ex_n, ex_t, m_n, m_t),
            "extrapolated": True, "extract_desc_per_s": ex_rate, "match_pairs_per_s": m_rate,
            "pairs_per_s": total_pairs / step_s, "ms_per_step": step_s * 1e3,
            "value_1_core": total_desc / (total_desc / ex1 + total_pairs / m1),
            "extract_desc_per_s_1_core": ex1, "match_pairs_per_s_1_core": m1}


def hd_component(torch, lat, timer, trip, steps, cpu_seconds):
    """A 1920x1080 image pair: both images' 10,000 keypoints in one batched
    extraction, then 10,000 x 10,000 2-NN on every matcher path."""
    from paper_1609_03986_amd import synth
    from paper_1609_03986_amd.binding import image_table
    w = synth.workload_hd()
    nq, nt = len(w["query_kps"]), len(w["train_kps"])
    img_q = torch.from_numpy(w["query_image"]).cuda()
    img_t = torch.from_numpy(w["train_image"]).cuda()
    kps = torch.from_numpy(np.concatenate([w["query_kps"], w["train_kps"]])).cuda()
    image_id = torch.from_numpy(np.repeat(np.arange(2, dtype=np.int32), [nq, nt])).cuda()
    table = image_table([img_q, img_t])
    desc = torch.empty((nq + nt, 16), dtype=torch.int32, device="cuda")
    desc_q, desc_t = desc[:nq], desc[nq:]
    idx = torch.empty((nq, 2), dtype=torch.int32, device="cuda")
    dist = torch.empty((nq, 2), dtype=torch.int32, device="cuda")
    acc = torch.empty((nq,), dtype=torch.uint8, device="cuda")
    for p in ("mfma", "fp4", "popcount", "auto"):
        lat.reserve(lat.knn_workspace_size(nq, nt, p))

    def extract_both():
        lat.extract_batch(table, 2, image_id, kps, desc)

    def match(path):
        lat.knn(desc_q, desc_t, k=2, ratio=0.8, path=path, idx=idx, dist=dist, accept=acc)

    def step():
        extract_both()
        match("auto")

    wall, _ = timer.loop(step, steps, 300)
    _, step_ms = timer.loop(step, steps, 0, per_step=True)
    kern = kernel_times(lat, torch, step, steps, ("extract", "knn_mfma", "knn_fp4", "knn_popcount",
                                                  "knn_merge"))
    ex_wall, _ = timer.loop(extract_both, steps, 2)
    pairs = nq * nt
    rates, kms = {}, {}
    for path in ("mfma", "fp4", "popcount"):
        m_wall, _ = timer.loop(lambda: match(path), steps, 2)
        rates[path] = pairs / (m_wall / steps)
        name = {"mfma": "knn_mfma", "fp4": "knn_fp4", "popcount": "knn_popcount"}[path]
        kt = kernel_times(lat, torch, lambda: match(path), steps, (name,))
        kms[path] = kt[name]["avg_ms"]
    roof = roofline_of(kern, (nq + nt) / kern["extract"]["launches_per_step"], pairs, "hd")
    out = {"workload": "1920x1080 u8 image pair, 10,000 keypoints each, 10,000 x 10,000 2-NN",
           "desc_per_s": (nq + nt) / (wall / steps), "ms_per_step": wall / steps * 1e3,
           "latency_ms": {"p50": percentile(step_ms, 50), "p99": percentile(step_ms, 99)},
           "extract_desc_per_s": (nq + nt) / (ex_wall / steps),
           "match_pairs_per_s": rates, "match_kernel_avg_ms": kms, "kernels": kern,
           "roofline": roof}
    if cpu_seconds > 0:
        import oracle
        t0 = time.perf_counter()
        oq, _ = oracle.extract(w["query_image"], w["query_kps"], synth.triplet_table())
        ot, _ = oracle.extract(w["train_image"], w["train_kps"], synth.triplet_table())
        oracle.knn(oq, ot, k=2, ratio=0.8)
        out["cpu_oracle_desc_per_s"] = (nq + nt) / (time.perf_counter() - t0)
    return out, (w, img_q, img_t, kps, image_id, table, desc, torch)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)." % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    comps = set()
    if args.components != "none":
        comps = ({"plain", "pcie", "hd", "uneven", "serve", "match_1m", "detect", "weighted",
                  "dense"}
                 if args.components == "all" else set(args.components.split(",")))

    import torch
    from paper_1609_03986_amd import synth
    from paper_1609_03986_amd.binding import Latch

    torch.cuda.set_device(0)
    timer = Timer(torch)
    trip = synth.triplet_table()
    lat = Latch(trip)
    tuning = load_tuning(lat)

    # --- The SfM batch and its captured plan. ---
    log("generating the SfM batch")
    imgs, kps = synth.sfm_workload()
    inputs = {"triplets_sha256": digest([trip]),
              "sfm": {"images_sha256": digest(imgs), "keypoints_sha256": digest(kps)}}
    sfm = Batch(torch, lat, imgs, kps, args.path)
    total, n_pairs = sfm.total, sfm.n_pairs
    # One run of the plain form and of the plan on the same inputs: the two
    # must agree (and the GPU leaves its idle clocks before the warm-up).
    plain_run, plain_out = sfm.per_image_form()
    plain_run()
    sfm.run_plan()
    torch.cuda.synchronize()
    identical = sfm.same_as(plain_out)
    flags = lat.check_errors(clear=True)

    log("plan and plain form agree: %s" % identical)
    # --- The timed region: W untimed steps, then exactly K steps. ---
    wall, _ = timer.loop(sfm.run_plan, args.steps, args.warmup)
    ms_per_step = wall / args.steps * 1e3
    value = total / (wall / args.steps)
    # Step latency (p50 / p99) from a second run of K steps with an event pair
    # around each replay.
    _, step_ms = timer.loop(sfm.run_plan, args.steps, 0, per_step=True)
    # Kernel durations: the plan's launches as eager calls, with the library's events.
    kernels = kernel_times(lat, torch, sfm.run_eager, args.steps,
                           ("extract_order", "extract", "knn_batch_fp4", "knn_batch_mfma",
                            "knn_batch_popcount"))
    eager_wall, _ = timer.loop(sfm.run_eager, args.steps, 1)
    roof = roofline_of(kernels, total, n_pairs, "sfm")
    # Every kernel of the step against its own roof; the extraction also
    # against HBM, with the algorithmic bytes of a descriptor: its share of
    # the images read once, its 16-byte keypoint and its 64-byte descriptor.
    step_roofs = {k: roofline_of(kernels, total, n_pairs, "sfm", kernel=k)
                  for k in kernels if k != "extract_order"}
    if "extract" in kernels:
        ex_bytes = sum(im.nbytes for im in imgs) + total * (16 + 64)
        ex_sec = kernels["extract"]["avg_ms"] * 1e-3
        step_roofs["extract"]["hbm"] = {
            "algorithmic_bytes": ex_bytes, "achieved_gbs": ex_bytes / ex_sec / 1e9,
            "frac": ex_bytes / ex_sec / 1e9 / PEAK_HBM_GBS}
    log("timed %d steps: %.3f ms per step" % (args.steps, ms_per_step))

    components = {"sfm_identical_to_plain_form": bool(identical), "sfm_error_flags": flags,
                  "sfm_kernel_rooflines": step_roofs,
                  "sfm_eager_batched_ms_per_step": eager_wall / args.steps * 1e3}
    if "plain" in comps:
        p_wall, _ = timer.loop(plain_run, max(3, args.steps // 4), 1)
        p_ms = p_wall / max(3, args.steps // 4) * 1e3
        components["sfm_plain_form"] = {"ms_per_step": p_ms, "desc_per_s": total / p_ms * 1e3,
                                        "plan_speedup": p_ms / ms_per_step}
    del plain_out, plain_run

    if "pcie" in comps:
        # The same step with images and keypoints starting in pinned host
        # memory and descriptors and matches copied back (not the headline).
        h_imgs = [torch.from_numpy(im).pin_memory() for im in imgs]
        h_kps = sfm.kp_all.cpu().pin_memory()
        h_out = [torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
                 for t in (sfm.desc, sfm.idx, sfm.dist, sfm.acc)]

        def step_pcie():
            for d, h in zip(sfm.dimgs, h_imgs):
                d.copy_(h, non_blocking=True)
            sfm.kp_all.copy_(h_kps, non_blocking=True)
            sfm.run_plan()
            for h, d in zip(h_out, (sfm.desc, sfm.idx, sfm.dist, sfm.acc)):
                h.copy_(d, non_blocking=True)

        pc_wall, _ = timer.loop(step_pcie, max(3, args.steps // 4), 1)
        components["sfm_pcie_inclusive_desc_per_s"] = total / (pc_wall / max(3, args.steps // 4))
        del h_imgs, h_out

    cpu = None
    if args.cpu_seconds > 0:
        log("oracle baseline")
        cpu = cpu_baseline_sfm(imgs, kps, trip, total, n_pairs, args.cpu_seconds)
    sfm.close()
    del sfm, imgs, kps
    torch.cuda.empty_cache()

    if "uneven" in comps:
        log("uneven batch")
        u_imgs, u_kps = synth.uneven_workload()
        inputs["uneven"] = {"images_sha256": digest(u_imgs), "keypoints_sha256": digest(u_kps)}
        ub = Batch(torch, lat, u_imgs, u_kps, args.path)
        u_run, u_out = ub.per_image_form()
        u_run()
        ub.run_plan()
        torch.cuda.synchronize()
        u_same = ub.same_as(u_out)
        reps = max(3, args.steps // 2)
        u_plan, _ = timer.loop(ub.run_plan, reps, 2)
        u_plain, _ = timer.loop(u_run, reps, 1)
        ub.close()
        # The same plan captured under the library's default tuning table.
        tuned = lat.get_tuning()
        fresh = Latch(trip)
        lat.set_tuning(fresh.get_tuning())
        fresh.close()
        ub_default = Batch(torch, lat, u_imgs, u_kps, args.path)
        u_plan_default, _ = timer.loop(ub_default.run_plan, reps, 2)
        ub_default.close()
        lat.set_tuning(tuned)
        del ub_default
        components["uneven_batch"] = {
            "workload": "256 images, sizes uniform over {320x240, 640x480, 1280x720, 1920x1080, "
                        "4000x3000}, keypoints round(LogNormal(ln 5000, 1)) clipped to "
                        "[500, 50000], 2-NN over the 255 consecutive pairs",
            "descriptors": ub.total, "pairs": ub.n_pairs,
            "plan_ms": u_plan / reps * 1e3, "plain_form_ms": u_plain / reps * 1e3,
            "plan_speedup": u_plain / u_plan, "plan_desc_per_s": ub.total / (u_plan / reps),
            "plan_pairs_per_s": ub.n_pairs / (u_plan / reps), "identical": bool(u_same),
            "tuning": tuning["source"],
            "plan_ms_library_default_tuning": u_plan_default / reps * 1e3}
        del ub, u_out, u_run, u_imgs, u_kps
        torch.cuda.empty_cache()

    hd = None
    if comps & {"hd", "match_1m", "detect", "weighted", "dense"}:
        log("1920x1080 pair")
        hd_out, hd = hd_component(torch, lat, timer, trip, max(args.steps, 200),
                                  args.cpu_seconds if "hd" in comps else 0)
        if "hd" in comps:
            components["image_pair_hd"] = hd_out

    db = None
    if "serve" in comps:
        log("serving")
        components["serving"], db = serving_component(torch, trip)
    if hd is not None and "match_1m" in comps:
        log("1,000,000-row database matching")
        if db is None:
            from paper_1609_03986_amd import serve
            db = serve.build_database(lat)
        components["match_1m"] = match_db_component(torch, lat, hd_desc_q(hd), db)
    del db
    torch.cuda.empty_cache()

    log("detection, weighted geometry, dense")
    if hd is not None and "detect" in comps:
        components["detection"] = detection_component(torch, lat, timer, hd)
    if hd is not None and "weighted" in comps:
        components["weighted_extraction"] = weighted_component(torch, timer, hd)
    if hd is not None and "dense" in comps:
        components["dense"] = dense_component(torch, lat, timer, hd)

    out = {
        "metric": METRIC, "value": value, "unit": "desc/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": WORKLOAD, "images": 64, "descriptors_per_step": total,
                   "pairs_per_step": n_pairs, "image_pairs": 63, "match_path": args.path,
                   "parallelism": "single GPU"},
        "arithmetic": "u8 images, exact int32 patch sums; matching on exact MXFP4 MFMA "
                      "(0 / +-1 operands, f32 sums of integers < 2^24) unless the tuning "
                      "table picks int8 MFMA or popcount",
        "pairs_per_s": n_pairs / (wall / args.steps),
        "latency_ms": {"p50": percentile(step_ms, 50), "p99": percentile(step_ms, 99)},
        "tuning": tuning,
        "kernels": kernels,
        "roofline": roof,
        "cpu_baseline": cpu,
        "paper": PAPER,
        "components": components,
        "inputs": inputs,
        "versions": versions(torch),
    }
    print(json.dumps(out), flush=True)
    lat.close()


def digest(arrays):
    """SHA-256 over the bytes of the given arrays, in order (the record of the
    seeded synthetic inputs a run used)."""
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def serving_component(torch, trip, rates=((50, 200), (200, 400), (800, 400)), slots=4):
    """A short serving run: Poisson requests of the uneven mix matched against
    a 1,000,000-row resident database (serve.py runs the full 2,000-request
    rates)."""
    from paper_1609_03986_amd import serve
    from paper_1609_03986_amd.binding import Latch
    builder = Latch(trip)
    db = serve.build_database(builder)
    pool = serve.request_pool()
    ex = serve.GpuExecutor(db, trip, slots)
    sched = serve.Scheduler(ex, slots, 8 << 30, db.shape[0])
    sched.run(serve.max_requests(slots, pool))
    out = {"db_rows": int(db.shape[0]), "slots": slots, "slot_workspace_bytes": ex.reserved,
           "db_sha256": digest([db.cpu().numpy()]), "rates": []}
    for qps, n in rates:
        results, rejected, stats = sched.run(serve.make_requests(n, qps, pool, seed=int(qps)))
        pairs = sum(len(r.idx) for r in results) * db.shape[0]
        out["rates"].append({"offered_qps": qps, "requests": n, "served_qps": stats["throughput_rps"],
                             "p50_ms": stats["p50_ms"], "p99_ms": stats["p99_ms"],
                             "pairs_per_s": pairs / stats["wall_s"], "rejected": len(rejected),
                             "max_inflight": stats["max_inflight"]})
    ex.close()
    builder.close()
    return out, db


def hd_desc_q(hd):
    """The 10,000 query descriptors of the 1920x1080 pair."""
    return hd[6][:10000].clone()


def match_db_component(torch, lat, query, db, reps=5):
    """10,000 queries against the 1,000,000-row database on every matcher path:
    the split matchers at the serving shape (kernel times from the library's
    events, including the merge of the train splits)."""
    nq, nt = query.shape[0], db.shape[0]
    out = {"nq": nq, "nt": nt, "pairs": nq * nt}
    for path, names in (("fp4", ("knn_fp4", "knn_merge")), ("mfma", ("knn_mfma", "knn_merge")),
                        ("popcount", ("knn_popcount", "knn_merge"))):
        lat.reserve(lat.knn_workspace_size(nq, nt, path))
        lat.knn(query, db, path=path)
        kt = kernel_times(lat, torch, lambda: lat.knn(query, db, path=path), reps, names)
        main_ms = kt[names[0]]["avg_ms"]
        merge_ms = kt.get("knn_merge", {"ms_per_step": 0.0})["ms_per_step"]
        peak = {"fp4": PEAK_FP4_MFMA_TOPS, "mfma": PEAK_INT8_MFMA_TOPS, "popcount": PEAK_INT_TOPS}[path]
        ops = MATCH_OPS_PER_PAIR if path != "popcount" else POPCOUNT_OPS_PER_PAIR
        achieved = nq * nt * ops / (main_ms * 1e-3) / 1e12
        out[path] = {"kernel_avg_ms": main_ms, "merge_ms": merge_ms,
                     "pairs_per_s": nq * nt / ((main_ms + merge_ms) * 1e-3),
                     "frac_of_peak": achieved / peak, "achieved_tops": achieved}
    return out


def detection_component(torch, lat, timer, hd):
    """FAST-9 detection, suppression and orientation of both 1920x1080 images,
    appended into one keypoint array with image ids."""
    w, img_q, img_t = hd[0], hd[1], hd[2]
    det_cap = 1 << 17
    det_kps = torch.empty((det_cap, 4), dtype=torch.float32, device="cuda")
    det_ids = torch.empty((det_cap,), dtype=torch.int32, device="cuda")
    det_n = torch.zeros((1,), dtype=torch.int64, device="cuda")
    lat.reserve(lat.detect_workspace_size(*img_q.shape))

    def detect_both():
        det_n.zero_()
        lat.detect(img_q, DETECT_THRESHOLD, det_cap, kps=det_kps, n_kps=det_n, image_id=det_ids,
                   image_index=0)
        lat.detect(img_t, DETECT_THRESHOLD, det_cap, kps=det_kps, n_kps=det_n, image_id=det_ids,
                   image_index=1)

    steps = 200
    d_wall, _ = timer.loop(detect_both, steps, 20)
    n_found = int(det_n.item())
    kt = kernel_times(lat, torch, detect_both, steps, ("detect",))
    det_ms = kt["detect"]["avg_ms"]
    image_bytes = img_q.numel() + img_t.numel()
    # Algorithmic HBM bytes per image: the image read once, 20 bytes per
    # keypoint written (keypoint and image id).
    det_bytes = (image_bytes + 20 * n_found) / 2
    return {"threshold": DETECT_THRESHOLD, "keypoints_per_step": n_found,
            "images_per_s": 2 / (d_wall / steps), "avg_ms_per_image": det_ms,
            "roofline": {"bound": "hbm", "achieved": det_bytes / (det_ms * 1e-3) / 1e9,
                         "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": det_bytes / (det_ms * 1e-3) / 1e9 / PEAK_HBM_GBS}}


def weighted_component(torch, timer, hd):
    """The paper's CLATCH geometry: the 20,000 keypoints of the 1920x1080 pair
    from 64 x 64 windows with 8 x 8 patches and Gaussian integer weights."""
    from paper_1609_03986_amd import synth
    from paper_1609_03986_amd.binding import Latch
    kps, image_id, table = hd[3], hd[4], hd[5]
    n = kps.shape[0]
    geo = Latch(synth.triplet_table_geom(64, 8), window=64, patch=8,
                weights=synth.gaussian_weights(8, 2.0, 128))
    out_desc = torch.empty((n, 16), dtype=torch.int32, device="cuda")

    def extract_geometry():
        geo.extract_batch(table, 2, image_id, kps, out_desc)

    steps = 200
    g_wall, _ = timer.loop(extract_geometry, steps, 20)
    kt = kernel_times(geo, torch, extract_geometry, steps, ("extract",))
    geo.close()
    g_ms = kt["extract"]["avg_ms"]
    g_ops = n * WEIGHTED_OPS_PER_DESC / (g_ms * 1e-3) / 1e12
    return {"geometry": "64x64 window, 8x8 patches, Gaussian weights (sigma 2, peak 128)",
            "desc_per_s": n / (g_wall / steps), "avg_ms": g_ms,
            "roofline": {"bound": "alu", "achieved": g_ops, "peak": PEAK_DOT2_TOPS,
                         "unit": "TFLOP/s", "frac": g_ops / PEAK_DOT2_TOPS}}


def dense_component(torch, lat, timer, hd):
    """Dense CLATCH (Sec. 6): descriptors at every pixel of both 1920x1080
    images by box filters, then windowed 2-NN matching (radius DENSE_RADIUS)."""
    img_q, img_t = hd[1], hd[2]
    H, W = img_q.shape
    npx = H * W
    dq = torch.empty((npx, 16), dtype=torch.int32, device="cuda")
    dt = torch.empty((npx, 16), dtype=torch.int32, device="cuda")

    def dense_both():
        lat.extract_dense(img_q, 0, 0, W, H, dq)
        lat.extract_dense(img_t, 0, 0, W, H, dt)

    def dense_match():
        lat.knn_window(dq, dt, W, H, DENSE_RADIUS)

    steps = 20
    de_wall, _ = timer.loop(dense_both, steps, 2)
    dm_wall, _ = timer.loop(dense_match, steps, 2)
    ke = kernel_times(lat, torch, dense_both, steps, ("dense_extract",))
    km = kernel_times(lat, torch, dense_match, steps, ("knn_window",))
    de_ms, dm_ms = ke["dense_extract"]["avg_ms"], km["knn_window"]["avg_ms"]
    de_ops = npx * DENSE_OPS_PER_PIXEL / (de_ms * 1e-3) / 1e12
    cand = (2 * DENSE_RADIUS + 1) ** 2
    dm_ops = npx * cand * POPCOUNT_OPS_PER_PAIR / (dm_ms * 1e-3) / 1e12
    return {"image": "%dx%d, every pixel" % (W, H), "radius": DENSE_RADIUS,
            "desc_per_s": 2 * npx / (de_wall / steps), "extract_avg_ms": de_ms,
            "match_pairs_per_s": npx * cand / (dm_wall / steps), "match_avg_ms": dm_ms,
            "extract_roofline": {"bound": "alu", "achieved": de_ops, "peak": PEAK_INT_TOPS,
                                 "unit": "TFLOP/s", "frac": de_ops / PEAK_INT_TOPS,
                                 "traffic": recorded_traffic("dense_extract", "hd")},
            "match_roofline": {"bound": "alu", "achieved": dm_ops, "peak": PEAK_INT_TOPS,
                               "unit": "TFLOP/s", "frac": dm_ops / PEAK_INT_TOPS}}


def versions(torch):
    """ROCm, HIP runtime, driver and device names for the record."""
    props = torch.cuda.get_device_properties(0)
    out = {"torch": torch.__version__, "hip": getattr(torch.version, "hip", None),
           "device": torch.cuda.get_device_name(0),
           "arch": getattr(props, "gcnArchName", None), "compute_units": props.multi_processor_count}
    try:
        out["rocm"] = open("/opt/rocm/.info/version").read().strip()
    except OSError:
        out["rocm"] = None
    try:
        out["amdgpu_driver"] = open("/sys/module/amdgpu/version").read().strip()
    except OSError:
        out["amdgpu_driver"] = None
    try:
        # The HIP runtime's own report of the driver stack it runs on.
        import ctypes
        v = ctypes.c_int(0)
        rc = ctypes.CDLL("libamdhip64.so").hipDriverGetVersion(ctypes.byref(v))
        out["hip_driver_version"] = v.value if rc == 0 else None
    except (OSError, AttributeError):
        out["hip_driver_version"] = None
    try:
        from paper_1609_03986_amd.binding import latch_version
        out["library"] = latch_version()
    except Exception:
        out["library"] = None
    return out


if __name__ == "__main__":
    main()
