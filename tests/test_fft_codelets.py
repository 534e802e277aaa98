"""Host check of the HIP FFT building blocks (csrc/fft_device.h): every radix
codelet, forward and inverse, against the DFT by its definition in double, and
the pass plan of every transform length the canvas edges use (at most two LDS
passes up to the 180 edge, three above).  Compiles tests/native/fft_codelets.cpp
for the host with hipcc and runs it; no GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _hipcc():
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if p and os.path.exists(p):
            return p
    return None


def test_codelets_and_plans(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "fft_codelets")
    r = subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                        "-I" + os.path.join(ROOT, "paper_2605_21398_amd", "csrc"), "-I" + os.path.join(ROOT, "include"),
                        os.path.join(HERE, "native", "fft_codelets.cpp"), "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert r.stdout.count(" ok") == 11 + 28
