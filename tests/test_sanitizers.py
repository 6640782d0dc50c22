"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle's C source (oracle/asf_oracle.c) with a C driver that calls every
  entry point on small inputs, valid and invalid (tests/sanitize/oracle_main.c).
* The library's host-side plan arithmetic (paper_1203_3583_amd/csrc/plan_host.cpp:
  parameter checks, workspace layouts, Gauss-Legendre rules, the kernel's Fourier
  transform, FFT twiddle tables), which has no HIP dependency, with a C++ driver
  over every supported grid size and invalid parameters (tests/sanitize/plan_main.cpp).

Both are built with gcc/g++ (no GPU code is involved) and must exit cleanly; the
sanitizers abort on the first error, and leak detection is on.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _build_and_run(tmp_path, compiler, sources, extra):
    exe = str(tmp_path / "driver")
    r = subprocess.run([compiler] + SAN + extra + sources + ["-o", exe, "-lm"], capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("compiler without sanitizer runtime: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    run = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "ok" in run.stdout
    assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr


def test_oracle_under_sanitizers(tmp_path):
    _build_and_run(tmp_path, "gcc", [os.path.join(ROOT, "oracle", "asf_oracle.c"),
                                     os.path.join(ROOT, "tests", "sanitize", "oracle_main.c")],
                   ["-std=c11", "-fopenmp"])


def test_plan_arithmetic_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1203_3583_amd", "csrc")
    _build_and_run(tmp_path, "g++", [os.path.join(csrc, "plan_host.cpp"),
                                     os.path.join(ROOT, "tests", "sanitize", "plan_main.cpp")],
                   ["-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", csrc])
