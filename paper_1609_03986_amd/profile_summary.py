"""Summaries of rocprofv3 CSV output for the profiles/ folder.

    python -m paper_1609_03986_amd.profile_summary stats KERNEL_STATS_CSV
        Markdown table of per-kernel dispatch durations (from --stats).
    python -m paper_1609_03986_amd.profile_summary counters COUNTER_CSV [COUNTER_CSV ...]
        Markdown table of each counter's average per dispatch, by kernel
        (from --pmc runs; several runs of the same command merge).
    python -m paper_1609_03986_amd.profile_summary traffic --fetch F.csv --write W.csv \\
            --fetch-copy FC.csv --write-copy WC.csv --workload NAME [--json profiles/traffic.json]
        HBM bytes per launch of each library launch (FETCH_SIZE and WRITE_SIZE
        in KiB per dispatch, each scaled by what the same counter reads for a
        plain 64 MiB device copy), as markdown; with --json, also recorded as
        "<launch>@<workload>" entries with the sha256 of the kernel's source,
        which bench.py reads for the roofline's `traffic`.

A library launch is named as the library's timing events name it: the
order's five kernels are one "extract_order" launch, and so on.
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 64 << 20

# HIP kernel -> (library launch name, source file).
LAUNCHES = [
    (r"^extract_kernel<", "extract", "extract.hip"),
    (r"^extract_weighted_kernel<", "extract_weighted", "extract_weighted.hip"),
    (r"^order_\w+_kernel", "extract_order", "order.hip"),
    (r"^knn_batch_fp4_kernel<", "knn_batch_fp4", "knn.hip"),
    (r"^knn_batch_mfma_kernel", "knn_batch_mfma", "knn.hip"),
    (r"^knn_batch_popcount_kernel", "knn_batch_popcount", "knn.hip"),
    (r"^knn_batch_(setup|fill)_kernel", "knn_batch_setup", "knn.hip"),
    (r"^knn_fp4_kernel<", "knn_fp4", "knn.hip"),
    (r"^knn_mfma_kernel", "knn_mfma", "knn.hip"),
    (r"^knn_popcount_kernel", "knn_popcount", "knn.hip"),
    (r"^knn_merge_kernel", "knn_merge", "knn.hip"),
    (r"^detect_tile_kernel", "detect_tile", "detect.hip"),
    (r"^detect_scan_kernel", "detect_scan", "detect.hip"),
    (r"^detect_emit_kernel", "detect_emit", "detect.hip"),
    (r"^dense_extract_kernel", "dense_extract", "dense.hip"),
    (r"^dense_match_kernel", "knn_window", "dense.hip"),
]


def short(name):
    """`void latch::(anonymous namespace)::knn_fp4_kernel<3>(...)` -> `knn_fp4_kernel<3>`."""
    name = re.sub(r"^void ", "", name)
    name = name.replace("latch::(anonymous namespace)::", "").replace("latch::", "")
    depth, out = 0, []
    for ch in name:                      # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out)


def launch_of(kernel):
    for pattern, launch, source in LAUNCHES:
        if re.search(pattern, kernel):
            return launch, source
    return None, None


def stats_table(path):
    rows = list(csv.DictReader(open(path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows) or 1.0
    out = ["| Kernel | Calls | Average (us) | Min (us) | Max (us) | Share of GPU time |",
           "|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        out.append("| %s | %s | %.2f | %.2f | %.2f | %.1f%% |" % (
            short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, 100.0 * float(r["TotalDurationNs"]) / total))
    return "\n".join(out)


def per_dispatch(paths, counter=None):
    """{kernel: {counter: [values per dispatch]}} and {kernel: [durations ns]}."""
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    dur = collections.defaultdict(dict)
    for path in paths:
        for r in csv.DictReader(open(path)):
            if counter and r["Counter_Name"] != counter:
                continue
            k = short(r["Kernel_Name"])
            vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
            dur[k][(path, r["Dispatch_Id"])] = (float(r["End_Timestamp"]) -
                                                float(r["Start_Timestamp"]))
    return vals, {k: list(v.values()) for k, v in dur.items()}


def counters_table(paths):
    vals, dur = per_dispatch(paths)
    names = sorted({c for k in vals for c in vals[k]})
    out = ["| Kernel | Dispatches | Average (us) | " + " | ".join(names) + " |",
           "|---|---|---|" + "---|" * len(names)]
    for k in sorted(vals, key=lambda k: -sum(dur[k])):
        if k.startswith("__amd") or not launch_of(k)[0]:
            continue
        cells = []
        for c in names:
            v = vals[k].get(c)
            cells.append("%.4g" % (sum(v) / len(v)) if v else "")
        n = max(len(v) for v in vals[k].values())
        out.append("| %s | %d | %.2f | %s |" % (k, n, sum(dur[k]) / len(dur[k]) / 1e3,
                                               " | ".join(cells)))
    return "\n".join(out)


def copy_kib(path, counter):
    """The counter's reading for the largest device copy in the run (the 64 MiB one)."""
    vals, _ = per_dispatch([path], counter)
    copies = [v for k, cs in vals.items() if "copyBuffer" in k for v in cs.get(counter, [])]
    if not copies:
        raise SystemExit("%s: no copy kernel in %s" % (counter, path))
    return max(copies)


def traffic(args):
    ff = COPY_BYTES / 1024.0 / copy_kib(args.fetch_copy, "FETCH_SIZE")
    wf = COPY_BYTES / 1024.0 / copy_kib(args.write_copy, "WRITE_SIZE")
    fv, _ = per_dispatch([args.fetch], "FETCH_SIZE")
    wv, _ = per_dispatch([args.write], "WRITE_SIZE")
    # Per library launch: the sum over its kernels of their average per
    # dispatch.  The kernels of one launch run equally often; where kernels of
    # one launch name run a different number of times (the batched and the
    # single-image extraction kernel, say), the most frequent ones are that
    # launch on this workload and the others are listed on their own.
    groups = collections.defaultdict(lambda: collections.defaultdict(list))
    for k in fv:
        launch, source = launch_of(k)
        if launch and k in wv:
            groups[launch][len(fv[k]["FETCH_SIZE"])].append(k)
    per = {}
    for launch, by_count in groups.items():
        for count, ks in sorted(by_count.items(), reverse=True):
            name = launch if count == max(by_count) else "%s [%s]" % (launch, ", ".join(ks))
            r = sum(sum(fv[k]["FETCH_SIZE"]) / count for k in ks) * 1024.0 * ff
            w = sum(sum(wv[k]["WRITE_SIZE"]) / len(wv[k]["WRITE_SIZE"]) for k in ks) * 1024.0 * wf
            per[name] = [r, w, set(ks), launch_of(ks[0])[1]]
    lines = ["Calibration: a %d MiB device copy reads FETCH_SIZE %.1f KiB and WRITE_SIZE %.1f KiB, "
             "so bytes = FETCH_SIZE x %.4f KiB and WRITE_SIZE x %.4f KiB." % (
                 COPY_BYTES >> 20, COPY_BYTES / 1024.0 / ff, COPY_BYTES / 1024.0 / wf, ff, wf), "",
             "| Launch (%s) | Kernels | Read MB per launch | Written MB per launch |" % args.workload,
             "|---|---|---|---|"]
    for launch in sorted(per):
        r, w, ks, _ = per[launch]
        lines.append("| %s | %s | %.2f | %.2f |" % (launch, ", ".join(sorted(ks)), r / 1e6, w / 1e6))
    if args.json:
        try:
            doc = json.load(open(args.json))
        except (OSError, ValueError):
            doc = {}
        doc["calibration"] = {"fetch_factor": ff, "write_factor": wf, "copy_bytes": COPY_BYTES}
        kern = doc.setdefault("kernels", {})
        for launch, (r, w, ks, source) in per.items():
            if "[" in launch:
                continue
            src = os.path.join("paper_1609_03986_amd", "csrc", source)
            kern["%s@%s" % (launch, args.workload)] = {
                "read_bytes_per_launch": r, "write_bytes_per_launch": w, "source": src,
                "source_sha256": hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()}
        with open(args.json, "w") as f:
            json.dump(doc, f, indent=1, sort_keys=True)
            f.write("\n")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+")
    t = sub.add_parser("traffic")
    for name in ("fetch", "write", "fetch-copy", "write-copy", "workload"):
        t.add_argument("--" + name, required=True)
    t.add_argument("--json")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(stats_table(args.csv))
    elif args.cmd == "counters":
        print(counters_table(args.csv))
    else:
        print(traffic(args))


if __name__ == "__main__":
    sys.exit(main())
