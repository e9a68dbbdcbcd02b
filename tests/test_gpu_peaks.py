"""GPU check of the device peak measurement (the rates roofline fractions are
quoted against): plausible magnitudes, and the copy really copies."""

import ctypes

import pytest
import torch

import paper_2206_04827_amd as cyl
from tests.gpu_common import banner, need_gpu

pytestmark = pytest.mark.gpu


def test_device_peaks_are_plausible():
    need_gpu()
    banner("device peaks")
    pk = cyl.device_peaks(n=1 << 25, reps=3)
    print("  measured", pk)
    assert 5.0 < pk["fp64_tflops"] < 200.0
    assert 500.0 < pk["copy_gbs"] < 20000.0


def test_device_peak_copy_copies_odd_lengths():
    need_gpu()
    n = 1001
    src = torch.arange(n + 2, dtype=torch.float64, device="cuda")
    dst = torch.full((n + 2,), -1.0, dtype=torch.float64, device="cuda")
    gb = ctypes.c_double()
    lib = cyl.load()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.cyl_device_peaks(s, cyl._ptr(src), cyl._ptr(dst), n, 1, None, ctypes.byref(gb)) == 0
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src[:n]) and bool((dst[n:] == -1.0).all())
    assert gb.value > 0.0
