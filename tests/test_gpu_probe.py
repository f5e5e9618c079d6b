"""The benchmark's matrix-core probe on the device: its three kinds run and
give rates that respect what they measure -- products alone below the bf16
peak, and products followed by SiLU rows no faster than either part alone
(the mixed kind does the work of both).  The rates themselves are
measurements, not asserted values."""
import ctypes
import os

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PEAK_BF16 = 2.5e15


def test_mfma_mix_probe_rates_are_consistent():
    import torch
    assert torch.cuda.is_available()
    path = os.path.join(ROOT, "paper_2304_06835_amd", "libvaluprobe.so")
    assert os.path.exists(path), "build libvaluprobe.so first"
    L = ctypes.CDLL(path)
    f = L.mfma_mix_rate
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    rates = []
    for kind in range(3):
        r = ctypes.c_double(0.0)
        assert f(0, kind, 1024, ctypes.byref(r)) == 0
        rates.append(r.value)
    mfma, silu, both = rates
    print("wave-iterations/s: products %.3e, SiLU rows %.3e, both %.3e" % (mfma, silu, both))
    flops = 24 * 16 * 16 * 32 * 2  # per wave-iteration of the product kinds
    assert 0.2 * PEAK_BF16 < mfma * flops < 1.05 * PEAK_BF16
    # the mixed kind does both parts' work: at best it overlaps them fully
    assert both < mfma and both < silu
