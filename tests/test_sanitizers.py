"""Host sanitizer builds (no GPU): the CPU pre-pass under AddressSanitizer + UndefinedBehavior-
Sanitizer and under ThreadSanitizer (its loops run on up to 16 threads), and the CPU oracle
under AddressSanitizer + UndefinedBehaviorSanitizer. Each build is a small driver in
``tests/sanitize/`` compiled with g++/gcc; a finding makes the driver exit non-zero
(-fno-sanitize-recover) and the report is shown in the assertion."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2007_12266_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs g++ and gcc")


def _build_and_run(tmp_path, compiler, sources, flags, name, env=None):
    exe = str(tmp_path / name)
    cmd = [compiler, "-O1", "-g", "-fno-omit-frame-pointer", *flags, *sources, "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                       env={**os.environ, **(env or {})})
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer"):
        assert marker not in out, out[-6000:]
    return out


def test_prepass_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "g++",
                         [os.path.join(SAN, "prepass_driver.cpp"),
                          os.path.join(CSRC, "lbm_prepass.cpp")],
                         ["-std=c++17", "-pthread", "-fsanitize=address,undefined",
                          "-fno-sanitize-recover=all"], "prepass_asan")
    assert out.count("ok ") == 5


def test_prepass_threads_under_thread_sanitizer(tmp_path):
    out = _build_and_run(tmp_path, "g++",
                         [os.path.join(SAN, "prepass_driver.cpp"),
                          os.path.join(CSRC, "lbm_prepass.cpp")],
                         ["-std=c++17", "-pthread", "-fsanitize=thread"], "prepass_tsan",
                         env={"TSAN_OPTIONS": "halt_on_error=1"})
    assert out.count("ok ") == 5


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    # OpenMP's runtime is not instrumented for ThreadSanitizer, so the oracle is checked for
    # memory and undefined-behaviour errors only, with two OpenMP threads.
    out = _build_and_run(tmp_path, "gcc",
                         [os.path.join(SAN, "oracle_driver.c"),
                          os.path.join(ROOT, "oracle", "colorlbm_oracle.c")],
                         ["-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp", "-ffp-contract=off",
                          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-lm"],
                         "oracle_asan", env={"OMP_NUM_THREADS": "2"})
    assert out.count("ok ") == 4
