"""Autotuner for the matcher: picks, per (query count, train count) size
bucket, the fastest of the int8-MFMA, MXFP4-MFMA and popcount paths, the
path for batched matching, the MXFP4 tile shape (2 or 3 blocks of 32
queries per wavefront), the split planner's workgroups-per-CU target and the
persistent workgroups per CU of batched matching.  It measures the library's
own kernels (HIP events recorded by the library on its launch stream) on
random descriptors and caches the result per device kind (architecture and
compute-unit count) and library version.

Tuning never changes results (every path is exact), only speed.

    python -m paper_1609_03986_amd.autotune [--cache PATH] [--quick]

The table the benchmark and the batch and serving drivers load sits in the
package (tuning.json); `--cache paper_1609_03986_amd/tuning.json` rewrites it.
"""
import json
import os
import sys

import numpy as np

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "latch_gfx950", "autotune.json")
IN_TREE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
MFMA, POPCOUNT, FP4 = 1, 2, 3


def bucket_shape(b):
    """A representative size of bucket b (bucket(n) = floor(log2 n / 2))."""
    return 2 ** (2 * b + 1)


def choose(timings):
    """timings: {candidate: seconds}.  The fastest candidate; ties go to the
    first candidate in insertion order."""
    best = None
    for c, t in timings.items():
        if best is None or t < timings[best]:
            best = c
    return best


def fill_table(measured):
    """measured: {(qb, tb): path}.  An 8 x 8 table whose unmeasured cells take
    the choice of the nearest measured cell (ties to the larger bucket)."""
    table = [[FP4] * 8 for _ in range(8)]
    if not measured:
        return table
    keys = list(measured)
    for i in range(8):
        for j in range(8):
            k = min(keys, key=lambda ab: (abs(ab[0] - i) + abs(ab[1] - j), -ab[0], -ab[1]))
            table[i][j] = measured[k]
    return table


def _time_knn(lat, q, t, path, reps):
    import torch
    lat.knn(q, t, path=path)                         # warm-up, workspace growth
    torch.cuda.synchronize()
    lat.timing(True)
    for _ in range(reps):
        lat.knn(q, t, path=path)
    torch.cuda.synchronize()
    total = 0.0
    for name in ("knn_mfma", "knn_fp4", "knn_popcount", "knn_merge"):
        n, ms = lat.timing_read(name)
        total += ms
    lat.timing(False)
    return total / reps * 1e-3


def _time_batch(lat, desc, pairs, path, reps):
    import torch
    out_rows = desc.shape[0]
    lat.knn_batch(desc, desc, pairs, out_rows, path=path)        # warm-up
    torch.cuda.synchronize()
    lat.timing(True)
    for _ in range(reps):
        lat.knn_batch(desc, desc, pairs, out_rows, path=path)
    torch.cuda.synchronize()
    n, ms = lat.timing_read("knn_batch_" + ("fp4" if path == "fp4" else path))
    lat.timing(False)
    return ms / max(n, 1) * 1e-3


def tune(lat, buckets=None, reps=5, seed=0, log=None):
    """Measure and install a tuning on the handle `lat` (binding.Latch);
    returns it as a dict."""
    import torch
    from . import synth
    from .binding import Tuning, pair_table
    g = np.random.default_rng(seed)
    if buckets is None:
        buckets = [(qb, tb) for qb in (2, 4, 6, 7) for tb in (4, 6, 7)]
    cap = 1 << 17
    rows = max(min(bucket_shape(b), cap) for ab in buckets for b in ab)
    pool = torch.from_numpy(synth.random_descriptors(g, rows).view(np.int32)).cuda()
    base = lat.get_tuning().to_dict()
    measured = {}
    for qb, tb in buckets:
        nq, nt = min(bucket_shape(qb), cap), min(bucket_shape(tb), cap)
        q, t = pool[:nq], pool[rows - nt:]
        ts = {MFMA: _time_knn(lat, q, t, "mfma", reps),
              FP4: _time_knn(lat, q, t, "fp4", reps),
              POPCOUNT: _time_knn(lat, q, t, "popcount", reps)}
        measured[(qb, tb)] = choose(ts)
        if log:
            log("bucket (%d, %d) nq=%d nt=%d: mfma %.1f us, fp4 %.1f us, popcount %.1f us" %
                (qb, tb, nq, nt, ts[MFMA] * 1e6, ts[FP4] * 1e6, ts[POPCOUNT] * 1e6))
    tuning = dict(base)
    tuning["path"] = fill_table(measured)
    tuning["batch_path"] = tuning["path"][6][6]

    def trial(**kw):
        t = dict(tuning, **kw)
        lat.set_tuning(Tuning.from_dict(t))
        return t

    # MXFP4 tile shape: the split matcher at 10,000 x 10,000 plus the batched
    # matcher on a batch shaped like structure from motion (64 images of
    # 20,000 descriptors, the 63 consecutive pairs; random bits).
    q, t = pool[:10000], pool[rows - 10000:] if rows >= 20000 else pool[:10000]
    bsize, bsets = 20000, 64
    bdesc = torch.from_numpy(g.integers(0, 2 ** 32, size=(bsize * bsets, 16), dtype=np.uint32)
                             .view(np.int32)).cuda()
    bpairs = pair_table([(i * bsize, bsize, (i + 1) * bsize, bsize, i * bsize)
                         for i in range(bsets - 1)])
    lat.reserve(lat.knn_batch_workspace_size(bsets - 1, bsize * bsets))
    shapes = {}
    for qb in (2, 3):
        trial(fp4_query_blocks=qb)
        shapes[qb] = (_time_knn(lat, q, t, "fp4", reps) +
                      _time_batch(lat, bdesc, bpairs, "fp4", reps))
    tuning["fp4_query_blocks"] = choose(shapes)
    if log:
        log("fp4 query blocks: %s -> %d" % ({k: round(v * 1e6, 1) for k, v in shapes.items()},
                                             tuning["fp4_query_blocks"]))
    # Split planner target on the 10,000 x 10,000 shape, for the faster MFMA path there.
    mfma_path = "fp4" if tuning["path"][6][6] == FP4 else "mfma"
    targets = {}
    for w in (1, 2, 3, 4):
        trial(mfma_groups_per_cu=w)
        targets[w] = _time_knn(lat, q, t, mfma_path, reps)
    tuning["mfma_groups_per_cu"] = choose(targets)
    if log:
        log("mfma workgroups per CU: %s -> %d" %
            ({w: round(v * 1e6, 1) for w, v in targets.items()}, tuning["mfma_groups_per_cu"]))
    # Persistent workgroups per CU of batched matching.
    bpath = {FP4: "fp4", MFMA: "mfma", POPCOUNT: "popcount"}[tuning["batch_path"]]
    groups = {}
    for w in (1, 2, 3, 4):
        trial(batch_groups_per_cu=w)
        groups[w] = _time_batch(lat, bdesc, bpairs, bpath, reps)
    tuning["batch_groups_per_cu"] = choose(groups)
    if log:
        log("batch workgroups per CU: %s -> %d" %
            ({w: round(v * 1e6, 1) for w, v in groups.items()}, tuning["batch_groups_per_cu"]))
    lat.set_tuning(Tuning.from_dict(tuning))
    return tuning


def cache_key():
    """Device architecture, compute-unit count and library version.  (Not the
    marketing name: it comes from a libdrm table that an installation may
    lack, and under rocprofv3 it reads as an empty string.)"""
    import torch
    from .binding import latch_version
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "").split(":")[0]
    return "%s|%d CUs|%s" % (arch, p.multi_processor_count, latch_version())


def load(lat, path=DEFAULT_CACHE):
    """Install a cached tuning for this device and library version, if any."""
    from .binding import Tuning
    try:
        entries = json.load(open(path))
    except (OSError, ValueError):
        return None
    t = entries.get(cache_key())
    if t is not None:
        lat.set_tuning(Tuning.from_dict(t))
    return t


def save(tuning, path=DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    try:
        entries = json.load(open(path))
    except (OSError, ValueError):
        entries = {}
    entries[cache_key()] = tuning
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1)
    os.replace(tmp, path)


def main(argv=None):
    import argparse
    from . import synth
    from .binding import Latch
    ap = argparse.ArgumentParser()
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--quick", action="store_true", help="three buckets only")
    args = ap.parse_args(argv)
    lat = Latch(synth.triplet_table())
    buckets = [(2, 6), (6, 6), (7, 7)] if args.quick else None
    t = tune(lat, buckets, log=lambda m: print(m, flush=True))
    save(t, args.cache)
    print(json.dumps({"cache": args.cache, "tuning": t}), flush=True)
    lat.close()


if __name__ == "__main__":
    sys.exit(main())
