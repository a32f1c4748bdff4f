"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU, no GPU): every library source is compiled with its host pass sanitized,
linked with a driver (tests/sanitize/runtime_host_driver.hip) that runs the
rotation table, the gather order tables, the triplet slot search, the split
planner, the workspace sizes and the C ABI's argument checks.  It must exit 0
with no sanitizer report."""
import concurrent.futures
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1609_03986_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
KERNEL_SOURCES = ["extract.hip", "extract_weighted.hip", "order.hip", "knn.hip", "detect.hip",
                  "dense.hip"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
         "-I", os.path.join(ROOT, "include")]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="ROCm compilers not available")
def test_runtime_host_code_clean_under_asan_and_ubsan(tmp_path):
    jobs = [(os.path.join(CSRC, s), str(tmp_path / s.replace(".hip", ".o"))) for s in KERNEL_SOURCES]
    jobs.append((os.path.join(HERE, "sanitize", "runtime_host_driver.hip"), str(tmp_path / "driver.o")))

    def compile_one(job):
        src, obj = job
        return subprocess.run([HIPCC] + FLAGS + ["-c", src, "-o", obj], capture_output=True,
                              text=True)

    with concurrent.futures.ThreadPoolExecutor(min(8, len(jobs))) as pool:
        for r in pool.map(compile_one, jobs):
            assert r.returncode == 0, r.stdout + r.stderr
    exe = str(tmp_path / "driver")
    link = subprocess.run([CLANG, "-fsanitize=address,undefined"] + [o for _, o in jobs] +
                          ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                          capture_output=True, text=True)
    assert link.returncode == 0, link.stdout + link.stderr
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                         env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    report = run.stderr
    assert run.returncode == 0, report
    assert "AddressSanitizer" not in report and "runtime error" not in report, report
    assert len(run.stdout.strip()) == 16
