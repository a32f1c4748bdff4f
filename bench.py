"""Benchmark: LATCH extraction + 2-NN Hamming matching on one MI355X.

One step is one pass of the whole path over one synthetic image pair:
  extract 10,000 descriptors from each of two 1920x1080 u8 images (angle
  U[0, 360), scale 1.2^U{0..7}) in one batched launch, then match the 10,000
  query descriptors 2-NN against the 10,000 train descriptors with ratio 0.8
  (matcher path from the handle's tuning table unless --path is given).
Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  `value` is descriptors extracted and matched per
second for the whole step (20,000 descriptors per step).  Extra fields give
the component rates (extraction desc/s, matching pairs/s per path,
FAST detection of both images, the weighted 64 x 64 / 8 x 8 geometry, dense
per-pixel descriptors and windowed matching), step
latency percentiles, per-kernel durations from HIP events recorded by the
library on its launch stream, the roofline of the dominant kernel and the
CPU oracle baseline.

    python bench.py [--gpus 1] [--steps 500] [--warmup 300] [--path mfma|fp4|popcount]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LATCH desc/s + Hamming pairs/s (MFMA vs popcount) at 1 GPU; p50/p99 ms"
WORKLOAD = ("1920x1080 u8 image pair, 10,000 keypoints each (angle U[0,360), scale 1.2^U{0..7}), "
            "512-bit LATCH over 48x48 windows with 7x7 patches, then 10,000 x 10,000 "
            "brute-force 2-NN Hamming matching with ratio 0.8")

# MI355X published peaks and chip constants.
PEAK_HBM_GBS = 8000.0
PEAK_INT8_MFMA_TOPS = 5000.0           # dense int8 MFMA, 10^12 ops/s
PEAK_FP4_MFMA_TOPS = 10100.0           # dense FP4 MFMA, 10^12 ops/s
CUS, CLOCK_GHZ, LANES = 256, 2.4, 64
# Integer VALU with v_dot4_u32_u8: 4 byte MACs = 8 ops per lane per cycle.
PEAK_DOT4_TOPS = CUS * LANES * CLOCK_GHZ * 8 / 1000.0   # 314.6
# Algorithmic work per unit: per descriptor, 512 triplets x 2 distances x 49 squared
# differences x 3 integer ops; per matched pair, the 512 MACs of a.b.
EXTRACT_OPS_PER_DESC = 512 * 2 * 49 * 3                  # sub, mul, add per squared difference
MATCH_OPS_PER_PAIR = 512 * 2                             # 512 MACs of a.b
DETECT_THRESHOLD = 20                                    # FAST threshold of the detection component
# Weighted CLATCH geometry: per descriptor 512 x 2 x 64 weighted squared
# differences x 4 ops (sub, square, weight, add), against the chip's
# v_dot2_i32_i16 rate (2 MACs = 4 ops per lane per cycle).
WEIGHTED_OPS_PER_DESC = 512 * 2 * 64 * 4
PEAK_DOT2_TOPS = CUS * LANES * CLOCK_GHZ * 4 / 1000.0   # 157.3
# Dense CLATCH: per pixel and triplet, G = (C1 - C2)(C1 + C2 - 2A) (4 ops), a
# running sum down the rows (2), one across the columns (2) and the compare
# (1); dense matching: 32 ops per candidate (16 XOR + 16 popcount-add).  Both
# against the 32-bit integer VALU rate (one op per lane per cycle).
DENSE_OPS_PER_PIXEL = 512 * 9
DENSE_RADIUS = 4
PEAK_INT_TOPS = CUS * LANES * CLOCK_GHZ / 1000.0         # 39.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # Defaults: 300 untimed steps (about 40 ms) bring the GPU to its steady
    # clocks before the 500 timed ones (about 60 ms).
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--path", default="auto", choices=["auto", "mfma", "fp4", "popcount"],
                    help="matcher path of the step (auto: the handle's tuning table)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="approximate CPU time budget of the oracle baseline (0 = skip)")
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


def recorded_traffic(kernel):
    """HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE) recorded in
    profiles/traffic.json for this kernel, or None when missing or when the
    kernel's source has changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["kernels"][kernel]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


def percentile(xs, p):
    return float(np.percentile(np.asarray(xs), p))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d)." % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    import torch
    from paper_1609_03986_amd import synth
    from paper_1609_03986_amd.binding import Latch, image_table

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    w = synth.workload_hd()
    trip = synth.triplet_table()
    nq, nt = len(w["query_kps"]), len(w["train_kps"])

    img_q = torch.from_numpy(w["query_image"]).to(dev)
    img_t = torch.from_numpy(w["train_image"]).to(dev)
    # Both images' keypoints in one array, extracted by one batched launch
    # (latch_extract_batch with a two-image table and per-keypoint image ids).
    kps = torch.from_numpy(np.concatenate([w["query_kps"], w["train_kps"]])).to(dev)
    kps_q, kps_t = kps[:nq], kps[nq:]
    image_id = torch.from_numpy(np.repeat(np.arange(2, dtype=np.int32), [nq, nt])).to(dev)
    table = image_table([img_q, img_t])
    desc = torch.empty((nq + nt, 16), dtype=torch.int32, device=dev)
    desc_q, desc_t = desc[:nq], desc[nq:]
    idx = torch.empty((nq, 2), dtype=torch.int32, device=dev)
    dist = torch.empty((nq, 2), dtype=torch.int32, device=dev)
    acc = torch.empty((nq,), dtype=torch.uint8, device=dev)
    lat = Latch(trip)
    stream = torch.cuda.current_stream()

    def extract_both():
        lat.extract_batch(table, 2, image_id, kps, desc)

    def match(path):
        lat.knn(desc_q, desc_t, k=2, ratio=0.8, path=path, idx=idx, dist=dist, accept=acc)

    def step():
        extract_both()
        match(args.path)

    def timed_loop(fn, steps, warmup, per_step=False):
        """Wall time of `steps` calls, bracketed by device synchronisation.
        With per_step, also each call's GPU time from an event pair around it
        (the event packets themselves cost several microseconds per step, so
        throughput is measured without them)."""
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
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

    # --- The timed region: exactly K whole steps. ---
    wall, _ = timed_loop(step, args.steps, args.warmup)
    # Step latency (p50 / p99) from a second, event-instrumented run of K steps.
    _, step_ms = timed_loop(step, args.steps, 0, per_step=True)
    ms_per_step = wall / args.steps * 1e3
    value = (nq + nt) / (wall / args.steps)

    # --- Per-kernel durations from the library's HIP events (same workload). ---
    lat.timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    kernels = {}
    for name in ("extract", "knn_mfma", "knn_fp4", "knn_popcount", "knn_merge"):
        n, total = lat.timing_read(name)
        if n:
            kernels[name] = {"launches_per_step": n / args.steps, "avg_ms": total / n,
                             "ms_per_step": total / args.steps}
    lat.timing(False)

    # --- Component rates. ---
    ex_wall, _ = timed_loop(extract_both, args.steps, 2)
    extract_desc_s = (nq + nt) / (ex_wall / args.steps)
    pairs = nq * nt
    match_rates, match_kernel_ms = {}, {}
    for path in ("mfma", "fp4", "popcount"):
        m_wall, _ = timed_loop(lambda: match(path), args.steps, 2)
        match_rates[path] = pairs / (m_wall / args.steps)
        lat.timing(True)
        for _ in range(args.steps):
            match(path)
        torch.cuda.synchronize()
        name = {"mfma": "knn_mfma", "fp4": "knn_fp4", "popcount": "knn_popcount"}[path]
        n, total = lat.timing_read(name)
        match_kernel_ms[path] = total / max(n, 1)
        lat.timing(False)

    # --- Keypoint detection (FAST-9, suppression, orientation) of both images,
    # appended into one array with image ids. ---
    det_cap = 1 << 17
    det_kps = torch.empty((det_cap, 4), dtype=torch.float32, device=dev)
    det_ids = torch.empty((det_cap,), dtype=torch.int32, device=dev)
    det_n = torch.zeros((1,), dtype=torch.int64, device=dev)

    def detect_both():
        det_n.zero_()
        lat.detect(img_q, DETECT_THRESHOLD, det_cap, kps=det_kps, n_kps=det_n, image_id=det_ids,
                   image_index=0)
        lat.detect(img_t, DETECT_THRESHOLD, det_cap, kps=det_kps, n_kps=det_n, image_id=det_ids,
                   image_index=1)

    d_wall, _ = timed_loop(detect_both, args.steps, 2)
    n_found = int(det_n.item())
    lat.timing(True)
    for _ in range(args.steps):
        detect_both()
    torch.cuda.synchronize()
    n_det, det_total = lat.timing_read("detect")
    lat.timing(False)
    det_ms = det_total / max(n_det, 1)
    image_bytes = img_q.numel() + img_t.numel()
    # Algorithmic HBM bytes per image: the image read once, 20 bytes per
    # keypoint written (keypoint and image id).
    det_bytes = (image_bytes + 20 * n_found) / 2
    detection = {"threshold": DETECT_THRESHOLD, "keypoints_per_step": n_found,
                 "images_per_s": 2 / (d_wall / args.steps),
                 "avg_ms_per_image": det_ms,
                 "roofline": {"bound": "hbm", "achieved": det_bytes / (det_ms * 1e-3) / 1e9,
                              "peak": PEAK_HBM_GBS, "unit": "GB/s",
                              "frac": det_bytes / (det_ms * 1e-3) / 1e9 / PEAK_HBM_GBS}}

    # --- The paper's CLATCH geometry: the same 20,000 keypoints extracted
    # from 64 x 64 windows with 8 x 8 patches and Gaussian integer weights
    # (one batched launch of the weighted kernel). ---
    geo_trip = synth.triplet_table_geom(64, 8)
    geo = Latch(geo_trip, window=64, patch=8, weights=synth.gaussian_weights(8, 2.0, 128))
    geo_desc = torch.empty_like(desc)

    def extract_geometry():
        geo.extract_batch(table, 2, image_id, kps, geo_desc)

    g_wall, _ = timed_loop(extract_geometry, args.steps, 2)
    geo.timing(True)
    for _ in range(args.steps):
        extract_geometry()
    torch.cuda.synchronize()
    n_g, g_total = geo.timing_read("extract")
    geo.timing(False)
    geo.close()
    g_ms = g_total / max(n_g, 1)
    g_ops = (nq + nt) * WEIGHTED_OPS_PER_DESC / (g_ms * 1e-3) / 1e12
    weighted = {"geometry": "64x64 window, 8x8 patches, Gaussian weights (sigma 2, peak 128)",
                "desc_per_s": (nq + nt) / (g_wall / args.steps), "avg_ms": g_ms,
                "roofline": {"bound": "alu", "achieved": g_ops, "peak": PEAK_DOT2_TOPS,
                             "unit": "TFLOP/s", "frac": g_ops / PEAK_DOT2_TOPS}}

    # --- Dense CLATCH (Sec. 6): descriptors at every pixel of both images by
    # box filters, then windowed 2-NN matching (radius DENSE_RADIUS). ---
    H_img, W_img = img_q.shape
    npx = H_img * W_img
    dq = torch.empty((npx, 16), dtype=torch.int32, device=dev)
    dt = torch.empty((npx, 16), dtype=torch.int32, device=dev)

    def dense_both():
        lat.extract_dense(img_q, 0, 0, W_img, H_img, dq)
        lat.extract_dense(img_t, 0, 0, W_img, H_img, dt)

    dense_steps = max(3, min(args.steps // 5, 20))
    de_wall, _ = timed_loop(dense_both, dense_steps, 1)
    dm_wall, _ = timed_loop(lambda: lat.knn_window(dq, dt, W_img, H_img, DENSE_RADIUS), dense_steps, 1)
    lat.timing(True)
    for _ in range(dense_steps):
        dense_both()
        lat.knn_window(dq, dt, W_img, H_img, DENSE_RADIUS)
    torch.cuda.synchronize()
    n_de, t_de = lat.timing_read("dense_extract")
    n_dm, t_dm = lat.timing_read("knn_window")
    lat.timing(False)
    de_ms, dm_ms = t_de / max(n_de, 1), t_dm / max(n_dm, 1)
    de_ops = npx * DENSE_OPS_PER_PIXEL / (de_ms * 1e-3) / 1e12
    cand = (2 * DENSE_RADIUS + 1) ** 2
    dm_ops = npx * cand * 32 / (dm_ms * 1e-3) / 1e12
    dense = {"image": "%dx%d, every pixel" % (W_img, H_img), "radius": DENSE_RADIUS,
             "desc_per_s": 2 * npx / (de_wall / dense_steps), "extract_avg_ms": de_ms,
             "match_pairs_per_s": npx * cand / (dm_wall / dense_steps), "match_avg_ms": dm_ms,
             "extract_roofline": {"bound": "alu", "achieved": de_ops, "peak": PEAK_INT_TOPS,
                                  "unit": "TFLOP/s", "frac": de_ops / PEAK_INT_TOPS},
             "match_roofline": {"bound": "alu", "achieved": dm_ops, "peak": PEAK_INT_TOPS,
                                "unit": "TFLOP/s", "frac": dm_ops / PEAK_INT_TOPS}}
    del dq, dt

    # --- The same step with the inputs starting in pinned host memory and the
    # results copied back (PCIe-inclusive; not the headline value). ---
    h_img_q = torch.from_numpy(w["query_image"]).pin_memory()
    h_img_t = torch.from_numpy(w["train_image"]).pin_memory()
    h_kps_q = torch.from_numpy(w["query_kps"]).pin_memory()
    h_kps_t = torch.from_numpy(w["train_kps"]).pin_memory()
    h_idx = torch.empty(idx.shape, dtype=idx.dtype, pin_memory=True)
    h_dist = torch.empty(dist.shape, dtype=dist.dtype, pin_memory=True)
    h_acc = torch.empty(acc.shape, dtype=acc.dtype, pin_memory=True)
    h_desc_q = torch.empty(desc_q.shape, dtype=desc_q.dtype, pin_memory=True)
    h_desc_t = torch.empty(desc_t.shape, dtype=desc_t.dtype, pin_memory=True)

    def step_pcie():
        img_q.copy_(h_img_q, non_blocking=True)
        img_t.copy_(h_img_t, non_blocking=True)
        kps_q.copy_(h_kps_q, non_blocking=True)
        kps_t.copy_(h_kps_t, non_blocking=True)
        step()
        h_desc_q.copy_(desc_q, non_blocking=True)
        h_desc_t.copy_(desc_t, non_blocking=True)
        h_idx.copy_(idx, non_blocking=True)
        h_dist.copy_(dist, non_blocking=True)
        h_acc.copy_(acc, non_blocking=True)

    pcie_wall, _ = timed_loop(step_pcie, args.steps, 2)
    pcie_desc_s = (nq + nt) / (pcie_wall / args.steps)

    # --- Roofline of the dominant kernel of the step. ---
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    kd = kernels[dom]
    if dom in ("knn_mfma", "knn_fp4"):
        peak = PEAK_INT8_MFMA_TOPS if dom == "knn_mfma" else PEAK_FP4_MFMA_TOPS
        achieved = pairs * MATCH_OPS_PER_PAIR / (kd["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None}
    elif dom == "extract":
        per_launch = (nq + nt) / kd["launches_per_step"]     # keypoints per extraction launch
        achieved = per_launch * EXTRACT_OPS_PER_DESC / (kd["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": PEAK_DOT4_TOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_DOT4_TOPS, "traffic": None}
    else:  # popcount: 16 xor + 16 popcount-accumulate per pair on the VALU
        peak = CUS * LANES * CLOCK_GHZ / 1000.0
        achieved = pairs * 32 / (kd["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None}

    roof["traffic"] = recorded_traffic(dom)
    roof["traffic_unit"] = "bytes/launch"

    # --- CPU oracle baseline: whole steps on the host cores. ---
    cpu = None
    if args.cpu_seconds > 0:
        import oracle
        reps, t_cpu = 0, 0.0
        while t_cpu < args.cpu_seconds and reps < 100:
            t0 = time.perf_counter()
            oq, _ = oracle.extract(w["query_image"], w["query_kps"], trip)
            ot, _ = oracle.extract(w["train_image"], w["train_kps"], trip)
            oracle.knn(oq, ot, k=2, ratio=0.8)
            t_cpu += time.perf_counter() - t0
            reps += 1
        cores = oracle.num_threads()
        # One whole step on a single thread as well.
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oq, _ = oracle.extract(w["query_image"], w["query_kps"], trip)
        ot, _ = oracle.extract(w["train_image"], w["train_kps"], trip)
        oracle.knn(oq, ot, k=2, ratio=0.8)
        t_one = time.perf_counter() - t0
        oracle.set_threads(cores)
        # The oracle on bounded samples of the components, all host cores.
        def rate(fn, units):
            t0 = time.perf_counter()
            fn()
            return units / (time.perf_counter() - t0)
        geo_sample = np.concatenate([w["query_kps"], w["train_kps"]])[:2000]
        comp = {
            "detection_images_per_s": rate(lambda: oracle.detect(w["query_image"], DETECT_THRESHOLD), 1),
            "weighted_extraction_desc_per_s": rate(
                lambda: oracle.extract_geom(w["query_image"], geo_sample, geo_trip, 64, 8,
                                            synth.gaussian_weights(8, 2.0, 128)), len(geo_sample)),
            "dense_extraction_desc_per_s": rate(
                lambda: oracle.extract_dense(w["query_image"], 900, 500, 64, 32, trip), 64 * 32),
        }
        dq_s = oracle.extract_dense(w["query_image"], 900, 500, 64, 32, trip)
        dt_s = oracle.extract_dense(w["train_image"], 900, 500, 64, 32, trip)
        comp["dense_match_pairs_per_s"] = rate(
            lambda: oracle.knn_window(dq_s, dt_s, 64, 32, DENSE_RADIUS),
            sum(min(32, y + DENSE_RADIUS + 1) - max(0, y - DENSE_RADIUS) for y in range(32)) *
            sum(min(64, x + DENSE_RADIUS + 1) - max(0, x - DENSE_RADIUS) for x in range(64)))
        cpu = {"value": (nq + nt) * reps / t_cpu, "unit": "desc/s", "cores": cores,
               "kind": "oracle",
               "sample": "%d whole steps (2 x 10,000 extractions + 10,000 x 10,000 2-NN) in %.1f s; "
                         "components: detection of one 1920x1080 image, weighted extraction of "
                         "2,000 keypoints, dense extraction and radius-%d matching of a 64x32 "
                         "region" % (reps, t_cpu, DENSE_RADIUS),
               "value_1_core": (nq + nt) / t_one,
               "components": comp}

    out = {
        "metric": METRIC, "value": value, "unit": "desc/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": WORKLOAD, "descriptors_per_step": nq + nt, "pairs_per_step": pairs,
                   "match_path": args.path, "parallelism": "single GPU"},
        "pairs_per_s": pairs / (wall / args.steps),
        "latency_ms": {"p50": percentile(step_ms, 50), "p99": percentile(step_ms, 99)},
        "components": {"extract_desc_per_s": extract_desc_s,
                       "pcie_inclusive_desc_per_s": pcie_desc_s,
                       "match_pairs_per_s": match_rates,
                       "match_kernel_avg_ms": match_kernel_ms,
                       "detection": detection,
                       "weighted_extraction": weighted,
                       "dense": dense},
        "kernels": kernels,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    lat.close()


if __name__ == "__main__":
    main()
