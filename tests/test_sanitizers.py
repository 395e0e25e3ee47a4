"""AddressSanitizer + UBSan runs of the host-side C/C++ (CPU only).

The CPU oracle and the host planner (argument checks, M/N/K groups, offset
tables, features) are compiled with -fsanitize=address,undefined together
with the random-signature drivers under tests/sanitize/, which give every
buffer exactly its viewed footprint; any out-of-bounds access or undefined
operation aborts the driver.  The planner driver also checks that
canonicalisation keeps the set of (A, B, C) offset triples of every term.
A planted one-element-short buffer is caught (the run is shown to detect).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    return r.returncode, r.stdout + r.stderr


@pytest.fixture(scope="module")
def tmp(tmp_path_factory):
    if not shutil.which("gcc") or not shutil.which("g++"):
        pytest.skip("no host compiler")
    return tmp_path_factory.mktemp("san")


def test_oracle_under_asan_ubsan(tmp):
    exe = str(tmp / "oracle_fuzz")
    _build(["gcc", "-std=c11", *SAN, "-fopenmp", "-ffp-contract=off",
            os.path.join(ROOT, "tests", "sanitize", "oracle_fuzz.c"),
            os.path.join(ROOT, "oracle", "gett_oracle.c"), "-lm", "-o", exe])
    rc, out = _run(exe)
    assert rc == 0, out[-3000:]
    assert "valid contractions run" in out


def test_planner_under_asan_ubsan(tmp):
    exe = str(tmp / "plan_fuzz")
    _build(["g++", "-std=c++17", *SAN, f"-I{os.path.join(ROOT, 'include')}",
            f"-I{os.path.join(ROOT, 'paper_2410_06770_amd', 'csrc')}",
            os.path.join(ROOT, "tests", "sanitize", "plan_fuzz.cpp"),
            os.path.join(ROOT, "paper_2410_06770_amd", "csrc", "gett_plan.cpp"), "-o", exe])
    rc, out = _run(exe)
    assert rc == 0, out[-3000:]
    assert "plan fuzz:" in out


def test_sanitized_run_detects_a_short_buffer(tmp):
    """The same oracle driver with A allocated one element short must fail."""
    src = open(os.path.join(ROOT, "tests", "sanitize", "oracle_fuzz.c")).read()
    bad = src.replace("double *A = malloc(na * sizeof(double))",
                      "double *A = malloc((na > 1 ? na - 1 : na) * sizeof(double))")
    bad = bad.replace("Af[i] = (float)(A[i] = (double)rint_in(-4, 4));",
                      "{ Af[i] = (float)rint_in(-4, 4); if (i < na - 1 || na == 1) A[i] = Af[i]; }")
    assert bad != src
    path = tmp / "oracle_fuzz_short.c"
    path.write_text(bad)
    exe = str(tmp / "oracle_fuzz_short")
    _build(["gcc", "-std=c11", *SAN, "-fopenmp", "-ffp-contract=off", str(path),
            os.path.join(ROOT, "oracle", "gett_oracle.c"), "-lm", "-o", exe])
    rc, out = _run(exe)
    assert rc != 0 and "AddressSanitizer" in out
