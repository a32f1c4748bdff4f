"""Batched workloads: the per-image form (one latch_extract per image, one
hamming_knn per image pair) against one captured plan (batched extraction +
batched matching replayed from a HIP graph), on the same inputs.  Prints one
JSON line per workload; both forms must give identical descriptors and
matches.

Workloads (stand-ins for the paper's Strecha scenes, Sec. 5):
  sfm:    64 crops of 3000x2000 from one textured mosaic (offsets 16 px / 8 px,
          +-4 noise), 20,000 keypoints each (angle U[0,360), scale 1.2^U{0..7}),
          2-NN over the 63 consecutive image pairs (20k x 20k each).
  uneven: 256 images, sizes uniform over {320x240, 640x480, 1280x720,
          1920x1080, 4000x3000}, keypoints per image round(LogNormal(ln 5000, 1))
          clipped to [500, 50000], 2-NN over the 255 consecutive pairs.

    python -m paper_1609_03986_amd.batchbench [--workload sfm uneven] [--reps 5]
"""
import argparse
import json
import sys
import time

import numpy as np

def run(name, imgs, kps, reps, triplets):
    import torch
    from .binding import Latch, image_table, pair_table
    from . import autotune
    lat = Latch(triplets)
    tuned = autotune.load(lat, autotune.IN_TREE)
    dimgs = [torch.from_numpy(im).cuda() for im in imgs]
    counts = [len(k) for k in kps]
    first = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    total = int(sum(counts))
    kp_all = torch.from_numpy(np.concatenate(kps).astype(np.float32)).cuda()
    ids = torch.from_numpy(np.repeat(np.arange(len(imgs), dtype=np.int32), counts)).cuda()
    pairs_np = np.array([(first[i], counts[i], first[i + 1], counts[i + 1], first[i])
                         for i in range(len(imgs) - 1)], np.int64)
    pairs = pair_table(pairs_np)
    out_rows = total
    n_pairs_total = int(sum(counts[i] * counts[i + 1] for i in range(len(imgs) - 1)))

    # Per-image form.
    desc_a = torch.empty((total, 16), dtype=torch.int32, device="cuda")
    idx_a = torch.full((out_rows, 2), -2, dtype=torch.int32, device="cuda")
    dist_a = torch.full((out_rows, 2), -2, dtype=torch.int32, device="cuda")
    acc_a = torch.zeros(out_rows, dtype=torch.uint8, device="cuda")
    kslices = [kp_all[first[i]:first[i] + counts[i]] for i in range(len(imgs))]
    dslices = [desc_a[first[i]:first[i] + counts[i]] for i in range(len(imgs))]

    def per_image():
        for i in range(len(imgs)):
            lat.extract(dimgs[i], kslices[i], dslices[i])
        for i in range(len(imgs) - 1):
            o = slice(first[i], first[i] + counts[i])
            lat.knn(dslices[i], dslices[i + 1], idx=idx_a[o], dist=dist_a[o], accept=acc_a[o])

    # Batched form: one plan.
    table = image_table(dimgs)
    desc_b = torch.empty((total, 16), dtype=torch.int32, device="cuda")
    idx_b = torch.full((out_rows, 2), -2, dtype=torch.int32, device="cuda")
    dist_b = torch.full((out_rows, 2), -2, dtype=torch.int32, device="cuda")
    acc_b = torch.zeros(out_rows, dtype=torch.uint8, device="cuda")
    plan = lat.plan(table, len(imgs), ids, kp_all, desc_b, pairs, idx_b, dist_b, acc_b)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_a = timed(per_image)
    t_b = timed(plan.run)
    same = (torch.equal(desc_a, desc_b) and torch.equal(idx_a, idx_b) and
            torch.equal(dist_a, dist_b) and torch.equal(acc_a, acc_b))
    flags = lat.check_errors()
    plan.close()
    lat.close()
    return {"workload": name, "images": len(imgs), "descriptors": total,
            "pairs_matched": n_pairs_total, "image_pairs": len(imgs) - 1,
            "per_image_ms": t_a * 1e3, "batched_graph_ms": t_b * 1e3,
            "speedup": t_a / t_b, "batched_desc_per_s": total / t_b,
            "batched_pairs_per_s": n_pairs_total / t_b, "identical": bool(same),
            "error_flags": flags,
            "tuning": "in-tree table" if tuned is not None else "library default"}


def main(argv=None):
    from . import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", nargs="+", default=["sfm", "uneven"], choices=["sfm", "uneven"])
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    trip = synth.triplet_table()
    for name in args.workload:
        t0 = time.perf_counter()
        imgs, kps = synth.sfm_workload() if name == "sfm" else synth.uneven_workload()
        gen = time.perf_counter() - t0
        out = run(name, imgs, kps, args.reps, trip)
        out["input_generation_s"] = gen
        print(json.dumps(out), flush=True)
        if not out["identical"]:
            return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
