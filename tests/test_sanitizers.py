"""The FP64 oracle and the host twin of the kernels' per-tetrahedron code,
built with AddressSanitizer and UndefinedBehaviorSanitizer (host code only)
and run on small cases of every view kind and form (CPU only)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = "/opt/rocm/bin/hipcc"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r.stdout


def test_oracle_under_asan_and_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    exe = str(tmp_path / "orc_asan")
    run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", os.path.join(HERE, "sanitize", "orc_main.c"), "-o", exe, "-lm"], str(tmp_path))
    out = run([exe], str(tmp_path))
    assert "0 failures" in out


def test_host_twin_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("no hipcc")
    exe = str(tmp_path / "hc_asan")
    # sanitizers on the host side only (the device side is not run)
    run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xarch_host", "-fno-sanitize-recover=all",
         "-I", os.path.join(ROOT, "paper_1208_3206_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
         os.path.join(HERE, "sanitize", "hostcheck_main.cpp"), "-o", exe], str(tmp_path))
    out = run([exe], str(tmp_path))
    assert "0 failures" in out
