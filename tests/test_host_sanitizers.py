"""The library's host code (coefficients, the M rule, pole plans, slot and
workspace sizing, argument checks, the circulant premises) built with the
address and undefined-behaviour sanitizers on the host side only (device
code is built as usual) and exercised by tests/sanitize/host_check.cpp.  No
GPU is needed: nothing in the driver reaches the device."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2008_11607_amd", "csrc")
SOURCES = ["coeffs.cpp", "kernels.hip", "kernels_vh.hip", "kernels_fft.hip", "kernels_lz.hip", "circulant.hip", "precond.hip",
           "solver.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# host-side sanitizers only: each -fsanitize= goes to the host compilation
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_check")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC"] + SAN + [
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
        "-I", os.path.join(ROOT, "include")] + [os.path.join(CSRC, s) for s in SOURCES] + [
        os.path.join(ROOT, "tests", "sanitize", "host_check.cpp"),
        "-L/opt/rocm/lib", "-lrocfft", "-Wl,-rpath,/opt/rocm/lib", "-pthread", "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert res.returncode == 0, res.stderr[-4000:]
    env = dict(os.environ)
    # leaks of process-lifetime caches (FFT plans, pinned tables) are by design
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "host checks passed" in run.stdout
