"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc): a driver (tests/sanitize/oracle_driver.c) calls every oracle
entry point on seeded edge-case inputs.  The plain and the sanitized builds
must both exit 0, print the same digest of all outputs, and report nothing."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "sanitize", "oracle_driver.c"),
           os.path.join(ROOT, "oracle", "latch_oracle.c")]
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
            "-g"]


def build_and_run(tmp_path, name, extra):
    exe = str(tmp_path / name)
    subprocess.run(["gcc", "-O1", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-Wall", "-Wextra", *extra,
                    *SOURCES, "-lm", "-o", exe], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    plain = build_and_run(tmp_path, "plain", [])
    assert plain.returncode == 0, plain.stderr
    san = build_and_run(tmp_path, "sanitized", SANITIZE)
    report = san.stderr
    assert san.returncode == 0, report
    assert "AddressSanitizer" not in report and "runtime error" not in report, report
    assert "LeakSanitizer" not in report, report
    assert san.stdout.strip() == plain.stdout.strip() != ""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_sanitized_driver_catches_a_planted_overread(tmp_path):
    """The check has teeth: a copy of the oracle whose window clamp lets the
    row index reach `height` (one row past the image) fails under ASan."""
    with open(SOURCES[1]) as f:
        src = f.read()
    clamp = "clamp64(cy + round_q22(dy), 0, height - 1)"
    assert src.count(clamp) == 1
    planted = tmp_path / "planted_oracle.c"
    planted.write_text(src.replace(clamp, "clamp64(cy + round_q22(dy), 0, height)"))
    exe = str(tmp_path / "planted")
    subprocess.run(["gcc", "-O1", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", *SANITIZE, SOURCES[0],
                    str(planted), "-lm", "-o", exe], check=True, capture_output=True, text=True)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                         env=dict(os.environ, OMP_NUM_THREADS="2"))
    assert run.returncode != 0
    assert "heap-buffer-overflow" in run.stderr
