"""Build the gfx950 HIP library liblatch.so in-tree with hipcc.

    python -m paper_1609_03986_amd.build [-v]

Compiler diagnostics are always shown, except the host pass's notice that it
does not know the device-only target feature -packed-fp32-ops (harmless: the
flag is meant for the gfx950 pass).
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblatch.so")
SOURCES = ["runtime.hip", "extract.hip", "extract_weighted.hip", "order.hip", "knn.hip", "detect.hip",
           "dense.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep hand-written float code away from packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
_HARMLESS = "'-packed-fp32-ops' is not a recognized feature for this target"


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    diag = "\n".join(l for l in p.stdout.splitlines() if _HARMLESS not in l)
    if diag:
        print(diag, file=sys.stderr, flush=True)
    if p.returncode != 0:
        raise subprocess.CalledProcessError(p.returncode, cmd)


def build(verbose=False):
    """Compile every source to an object (in parallel), then link liblatch.so
    (always rebuilds)."""
    jobs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-c",
                                         os.path.join(CSRC, src), "-o", obj]
        jobs.append((cmd, obj))
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        for f in [pool.submit(_run, cmd, verbose) for cmd, _ in jobs]:
            f.result()
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
