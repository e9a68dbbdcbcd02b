"""Pins for the oracle's ADI and Zolotarev shifts (Section 3, Algorithm 1)."""

import math

import numpy as np
import pytest
import scipy.special as ss

from oracle import adi
from oracle import operators as ops
from oracle import sylvester as sy


@pytest.mark.parametrize("kp", [0.9, 0.5, 0.3, 0.05])
def test_agm_matches_scipy(kp):
    k2 = 1.0 - kp * kp                       # scipy takes the parameter m = k^2
    K = adi.ellipk_from_kp(kp)
    assert K == pytest.approx(ss.ellipk(k2), rel=1e-14)
    for frac in (0.1, 0.37, 0.5, 0.93):
        u = frac * K
        assert adi.ellip_dn(u, kp) == pytest.approx(ss.ellipj(u, k2)[2], rel=1e-13)
        assert adi.ellip_dn_frac(frac, kp) == pytest.approx(ss.ellipj(u, k2)[2], rel=1e-13)


@pytest.mark.parametrize("kp", [1e-4, 1e-8, 1e-12])
def test_complete_integral_for_tiny_complementary_modulus(kp):
    """K(k) = ln(4/k') + O(k'^2 ln k') as k' -> 0 (the large-gamma regime)."""
    assert adi.ellipk_from_kp(kp) == pytest.approx(math.log(4.0 / kp), rel=1e-7)
    # dn(K, k) = k' at the quarter period, dn(K/2, k) = sqrt(k')
    assert adi.ellip_dn_frac(1.0, kp) == pytest.approx(kp, rel=1e-14)
    assert adi.ellip_dn_frac(0.5, kp) == pytest.approx(math.sqrt(kp), rel=1e-12)
    # the two branches agree where they meet, and dn(x) dn(K - x) = k'
    for t in (0.2, 0.45):
        assert adi.ellip_dn_frac(t, kp) * adi.ellip_dn_frac(1 - t, kp) == pytest.approx(kp, rel=1e-13)


def test_moebius_sends_four_points():
    a, b, c, d = -3.4e3, -40.7, 2.4674, 2.84e3
    gamma, alpha_z, _ = adi.zolotarev_params(a, b, c, d)
    T = adi.T_map(a, b, c, d, alpha_z)
    assert T(-alpha_z) == pytest.approx(a, rel=1e-12)
    assert T(-1.0) == pytest.approx(b, rel=1e-12)
    assert T(1.0 + 1e-9) == pytest.approx(c, rel=1e-6)
    assert T(alpha_z) == pytest.approx(d, rel=1e-10)


def test_symmetric_intervals_reduce_to_classical_shifts():
    """For [a, b] = [-d, -c] the Moebius map is z -> c z and the shifts are the
    classical ones, +-d dn((2j+1) K / (2J), k) with k' = c/d."""
    c, d, J = 1.0, 400.0, 9
    u, v = adi.shifts(-d, -c, c, d, J)
    k2 = 1.0 - (c / d) ** 2
    K = ss.ellipk(k2)
    ref = np.array([d * ss.ellipj((2 * j + 1) * K / (2 * J), k2)[2] for j in range(J)])
    assert np.allclose(u, ref, rtol=1e-12)
    assert np.allclose(v, -ref, rtol=1e-12)


@pytest.mark.parametrize("m,n,w", [(16, 16, 0), (34, 30, 2), (66, 66, 9)])
def test_spectra_real_and_disjoint(m, n, w):
    At, Ct, Bt, Dt = ops.tau_system(m, n, w)
    a, b, c, d, im = adi.spectral_bounds(At, Bt, Ct, Dt)
    assert im < 1e-8 * max(abs(a), d)
    assert a <= b < 0.0 < c <= d
    assert c == pytest.approx(np.pi ** 2 / 4, rel=1e-3)
    u, v = adi.shifts(a, b, c, d, 12)
    assert np.all((u >= c * (1 - 1e-12)) & (u <= d * (1 + 1e-12)))
    assert np.all((v >= a * (1 + 1e-12)) & (v <= b * (1 - 1e-12)))


@pytest.mark.parametrize("eps", [1e-4, 1e-8, 1e-11])
def test_adi_error_within_zolotarev_bound(eps):
    m = n = 34
    At, Ct, Bt, Dt = ops.tau_system(m, n, 2)
    E = np.random.default_rng(1).standard_normal((m - 2, n - 2))
    Xs = sy.solve(At, Bt, Ct, Dt, E)
    X, J = adi.adi_solve(At, Bt, Ct, Dt, E, eps)
    err = np.linalg.norm(X - Xs) / np.linalg.norm(Xs)
    assert err < eps
    # one fewer iteration is measurably worse: J is not wildly over-estimated
    a, b, c, d, _ = adi.spectral_bounds(At, Bt, Ct, Dt)
    u, v = adi.shifts(a, b, c, d, max(1, J // 2))
    err_half = np.linalg.norm(adi.adi(At, Bt, Ct, Dt, E, u, v) - Xs) / np.linalg.norm(Xs)
    assert err_half > 10 * err


def test_heat_pencil_bounds_are_shifted_poisson_bounds():
    m = n = 20
    ka = 1e-3
    At, Ct, Bt, Dt = ops.tau_system(m, n, 3)
    Ah, Ch, _, _ = ops.heat_system(m, n, 3, ka)
    a, b, c, d, _ = adi.spectral_bounds(At, Bt, Ct, Dt)
    ah, bh, ch, dh, _ = adi.spectral_bounds(Ah, Bt, Ch, Dt)
    assert ah == pytest.approx(a - 1 / ka, rel=1e-10)
    assert bh == pytest.approx(b - 1 / ka, rel=1e-10)
    assert (ch, dh) == (pytest.approx(c), pytest.approx(d))


def test_printed_algorithm_signs_and_roles_fail():
    """Documents the two readings: the printed signs converge to -X; the printed
    shift roles do not converge."""
    m = n = 24
    At, Ct, Bt, Dt = ops.tau_system(m, n, 1)
    E = np.random.default_rng(2).standard_normal((m - 2, n - 2))
    Xs = sy.solve(At, Bt, Ct, Dt, E)
    a, b, c, d, _ = adi.spectral_bounds(At, Bt, Ct, Dt)
    gamma, _, _ = adi.zolotarev_params(a, b, c, d)
    J = adi.num_iterations(gamma, 1e-10)
    u, v = adi.shifts(a, b, c, d, J)
    # printed signs: +E in step 1, -E in step 2  == corrected algorithm on -E
    X_printed = adi.adi(At, Bt, Ct, Dt, -E, u, v)
    assert np.linalg.norm(X_printed + Xs) < 1e-8 * np.linalg.norm(Xs)
    # printed roles: u in [a, b], v in [c, d]
    X_swapped = adi.adi(At, Bt, Ct, Dt, E, v, u)
    assert np.linalg.norm(X_swapped - Xs) > 1e2 * np.linalg.norm(Xs)
