"""The FFT building blocks of the kernels (csrc/fft.h: the small DFTs, both
four-step pass schemes, the lane-pair split and the spectrum index map),
compiled for the host and checked against a direct double-precision DFT by
tests/native/fft_host_check.cpp."""
import os
import subprocess

import pytest

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native", "fft_host_check")


def test_fft_blocks_on_host():
    if not os.path.exists(EXE):
        pytest.skip("tests/native/fft_host_check is not built (run __graft_entry__.build())")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("OK")
