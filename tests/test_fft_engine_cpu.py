"""Host emulation of the workgroup FFT engine (tests/native/fft_engine_check.hip):
every stage of the device transforms run thread by thread on the CPU and
compared with a float64 O(N^2) DFT, plus the float32 convolution-energy bias
of the codelet constants and the gain bias of every float32 codelet (Parseval
over 10^6 random butterflies).  Compiled with hipcc as host code (no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_fft_engine_host_emulation(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "fft_engine_check")
    src = os.path.join(HERE, "native", "fft_engine_check.hip")
    subprocess.run([hipcc, "-std=c++17", "-O1", src, "-o", exe], check=True,
                   capture_output=True, timeout=600)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-2000:]
    assert "ALL OK" in r.stdout
