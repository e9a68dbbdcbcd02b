"""GPU parity of the value <-> coefficient transforms (Section 2) against the oracle."""

import numpy as np
import pytest

import paper_2206_04827_amd as cyl
from oracle import transforms as tr
from tests.gpu_common import banner, dev, host, need_gpu

pytestmark = pytest.mark.gpu

# power-of-two, mixed-radix, prime-pass and Bluestein lengths, odd/even/1/2
# theta counts, ragged tails.  DFT lengths (r: m - 1, z: n - 1, theta: p) and
# their passes: 255 = 17 x 15, 17, 34 = 17 x 2; 11, 22 = 11 x 2; 13, 26 =
# 13 x 2; 7, 35 = 7 x 5, 45 = 15 x 3; 65 = 13 x 5; 39 = 13 x 3; 30 = 2 x 15;
# direct prime passes 47, 19, 31, 37, 191, 129 = 43 x 3, 511 = 73 x 7,
# 146 = 73 x 2; Bluestein where no plan exists: 119 = 7 x 17 (two factors of
# 7 .. 17).
SIZES = [(4, 4, 1), (8, 6, 4), (9, 7, 5), (17, 33, 16), (33, 20, 12), (32, 32, 32),
         (48, 40, 30), (65, 17, 2), (20, 129, 7), (130, 66, 64), (256, 18, 34),
         (12, 23, 22), (14, 27, 26), (8, 36, 45), (120, 10, 6), (10, 9, 37),
         (192, 40, 6), (24, 192, 2), (512, 20, 4), (30, 512, 3), (8, 8, 146)]


@pytest.mark.parametrize("m,n,p", SIZES)
def test_forward_and_inverse_match_oracle(m, n, p):
    need_gpu()
    banner("transforms m=%d n=%d p=%d" % (m, n, p))
    f = np.random.default_rng(m * 1000 + n * 10 + p).standard_normal((p, n, m))
    plan = cyl.Plan(m, n, p)
    c = host(plan.transform_fwd(dev(f)))
    ref = tr.to_half(tr.forward(f))
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(c - ref)) / scale
    print("  fwd rel max %.3e" % err)
    assert err < 1e-13
    v = host(plan.transform_inv(dev(ref)))
    err2 = np.max(np.abs(v - f)) / np.max(np.abs(f))
    print("  inv rel max %.3e" % err2)
    assert err2 < 1e-13
    # the inverse does not modify its input
    r = dev(ref)
    plan.transform_inv(r)
    assert np.array_equal(host(r), ref)


def test_inverse_ignores_imaginary_parts_of_real_slots():
    need_gpu()
    m, n, p = 10, 8, 6
    h = np.random.default_rng(0).standard_normal((p // 2 + 1, n, m)) * (1 + 1j)
    plan = cyl.Plan(m, n, p)
    v = host(plan.transform_inv(dev(h)))
    hr = h.copy()
    hr[0] = hr[0].real
    hr[p // 2] = hr[p // 2].real
    assert np.max(np.abs(v - tr.inverse(tr.from_half(hr, p)))) < 1e-13 * np.max(np.abs(v))


def test_mixed_radix_equals_bluestein_at_256():
    """n = 256 (DFT length 255 = 17 x 15): the mixed-radix transforms agree
    with the Bluestein ones to rounding."""
    import os
    need_gpu()
    m, n, p = 256, 256, 6
    f = np.random.default_rng(7).standard_normal((p, n, m))
    a = host(cyl.Plan(m, n, p).transform_fwd(dev(f)))
    os.environ["CYLSPEC_DFT_MIXED"] = "0"
    try:
        b = host(cyl.Plan(m, n, p).transform_fwd(dev(f)))
    finally:
        os.environ.pop("CYLSPEC_DFT_MIXED")
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(b))


@pytest.mark.parametrize("m,n,p", [(512, 40, 4), (192, 96, 6)])
def test_prime_pass_equals_bluestein(m, n, p):
    """DFT lengths 511 = 73 x 7 and 191 (prime): the direct prime-radix pass
    agrees with the Bluestein transforms to rounding, forward and inverse."""
    import os
    need_gpu()
    banner("prime pass vs Bluestein m=%d n=%d p=%d" % (m, n, p))
    f = np.random.default_rng(m + n).standard_normal((p, n, m))
    pa = cyl.Plan(m, n, p)
    a = host(pa.transform_fwd(dev(f)))
    ia = host(pa.transform_inv(dev(a)))
    os.environ["CYLSPEC_DFT_MIXED"] = "0"
    try:
        pb = cyl.Plan(m, n, p)
        b = host(pb.transform_fwd(dev(f)))
        ib = host(pb.transform_inv(dev(a)))
    finally:
        os.environ.pop("CYLSPEC_DFT_MIXED")
    print("  fwd %.3e inv %.3e" % (np.max(np.abs(a - b)) / np.max(np.abs(b)), np.max(np.abs(ia - ib)) / np.max(np.abs(ib))))
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(b))
    assert np.max(np.abs(ia - ib)) < 1e-13 * np.max(np.abs(ib))


@pytest.mark.parametrize("m,n,p", [(256, 36, 8), (36, 256, 96), (66, 10, 30), (17, 20, 256)])
def test_sixteen_points_per_thread_match_oracle(m, n, p):
    """The transform kernels exist for 8 and 16 points per thread; plans take
    8 for direct lengths up to 256 without a prime pass (255 = 17 x 15,
    35 = 7 x 5, 65 = 13 x 5, 96, 256, 30) and 16 otherwise.  The 16-point
    instances of those lengths (CYLSPEC_DFT_POINTS=16) match the oracle too,
    forward and inverse."""
    import os
    need_gpu()
    banner("16 points per thread m=%d n=%d p=%d" % (m, n, p))
    f = np.random.default_rng(m + 3 * n + 7 * p).standard_normal((p, n, m))
    ref = tr.to_half(tr.forward(f))
    os.environ["CYLSPEC_DFT_POINTS"] = "16"
    try:
        plan = cyl.Plan(m, n, p)
        c = host(plan.transform_fwd(dev(f)))
        v = host(plan.transform_inv(dev(ref)))
    finally:
        os.environ.pop("CYLSPEC_DFT_POINTS")
    e1 = np.max(np.abs(c - ref)) / np.max(np.abs(ref))
    e2 = np.max(np.abs(v - f)) / np.max(np.abs(f))
    print("  fwd %.3e inv %.3e" % (e1, e2))
    assert e1 < 1e-13 and e2 < 1e-13
