"""The CPU oracle and the library's host code under AddressSanitizer (with
LeakSanitizer) and UndefinedBehaviorSanitizer.

Each driver under tests/sanitize/ is built with gcc/g++,
-fsanitize=address,undefined and -Wall -Werror (no GPU code is involved) and
run; the run must pass its own functional checks and print no sanitizer
report.  The oracle's
driver runs rank with the f/g, minimax and Chebyshev comparators, a
tie-corrected order statistic, sort, multi-ciphertext rank and the error
paths (too few levels, bad N, missing rotation keys) on a ring of 2^10; the
host driver runs the prime chain, the ChaCha20 streams, the slot encoder and
the Chebyshev coefficients."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-Wall", "-Werror", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=undefined"]
REPORTS = ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, **kw)


def _build_and_run(tmp_path, compiler, sources, extra, timeout):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not found")
    exe = str(tmp_path / "driver")
    b = _run([compiler] + SAN + extra + sources + ["-o", exe, "-lquadmath", "-lm"], cwd=ROOT, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = _run([exe], env=env, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert not any(s in out for s in REPORTS), out[-4000:]
    return r.stdout


@pytest.mark.slow
def test_oracle_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "gcc", ["tests/sanitize/ora_driver.c"], ["-fopenmp"], 600)
    assert "all checks passed" in out


def test_host_code_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "g++", ["tests/sanitize/host_driver.cpp",
                                           "paper_2412_15126_amd/csrc/host_math.cpp"],
                         ["-std=gnu++17", "-ffp-contract=off"], 120)
    assert "all checks passed" in out
