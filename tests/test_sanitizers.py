"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two programs are built with gcc/g++ and run: one drives the CPU oracle's C
code (assembly for the three target kinds, sampled rows, element matrices,
Jacobi-PCG), the other the library's host-side bisection refiner (several
Doerfler refinements, the queries and the argument checks).  Any sanitizer
report aborts the program (-fno-sanitize-recover=all) and fails the test.
The refiner's source is copied to a .cpp file first: it is plain host C++.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, cwd):
    return subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=300)


def _build_and_run(tmp_path, compiler, sources, out, extra=()):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    exe = str(tmp_path / out)
    b = _run([compiler, *SAN, *extra, "-I", os.path.join(HERE, "sanitize"), "-I", os.path.join(ROOT, "include"),
              *sources, "-o", exe, "-lm"], str(tmp_path))
    if b.returncode != 0 and "asan" in b.stderr.lower() and "cannot find" in b.stderr.lower():
        pytest.skip("sanitizer runtime not installed")
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, \
        (r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_oracle_c_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc", [os.path.join(ROOT, "oracle", "oracle.c"),
                                           os.path.join(HERE, "sanitize", "oracle_driver.c")], "oracle_driver",
                         extra=["-std=gnu11"])
    assert "oracle driver: ok" in out


def test_refiner_under_sanitizers(tmp_path):
    src = tmp_path / "refine_host.cpp"
    shutil.copyfile(os.path.join(ROOT, "paper_2102_03515_amd", "csrc", "refine.hip"), src)
    out = _build_and_run(tmp_path, "g++", [str(src), os.path.join(HERE, "sanitize", "refiner_driver.cpp")],
                         "refiner_driver", extra=["-std=c++17"])
    assert "refiner driver: ok" in out
