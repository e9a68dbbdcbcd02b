"""Pins for the oracle's transforms (Section 2): interpolation and convergence.

The interpolant is evaluated with numpy's Chebyshev Vandermonde matrices and
explicit exponentials, which share nothing with the DCT/FFT route.
"""

import numpy as np
import pytest

from oracle import transforms as tr


@pytest.mark.parametrize("m,n,p", [(5, 4, 1), (9, 7, 6), (8, 11, 5), (6, 6, 8)])
def test_interpolation_property(m, n, p):
    """f* equals f on CCF_(m,n,p) (Section 2, the unique interpolant)."""
    f = np.random.default_rng(m * 100 + n * 10 + p).standard_normal((p, n, m))
    c = tr.forward(f)
    r, z, th = tr.grid(m, n, p)
    TH, Z, Rr = np.meshgrid(th, z, r, indexing="ij")
    vals = tr.evaluate(c, Rr.ravel(), Z.ravel(), TH.ravel())
    assert np.max(np.abs(vals - f.ravel())) < 1e-13
    assert np.max(np.abs(tr.inverse(c) - f)) < 1e-13


def test_grid_definition():
    r, z, th = tr.grid(5, 3, 4)
    assert np.allclose(r, [-1, -np.sqrt(0.5), 0, np.sqrt(0.5), 1], atol=1e-15)
    assert np.allclose(z, [-1, 0, 1], atol=1e-15)
    assert np.allclose(th, [-np.pi, -np.pi / 2, 0, np.pi / 2])


def test_known_polynomial_coefficients():
    """f = T_3(r) T_2(z) cos(2 theta) has coefficient 1/2 at (3, 2, w = +-2)."""
    m, n, p = 7, 6, 8
    r, z, th = tr.grid(m, n, p)
    TH, Z, Rr = np.meshgrid(th, z, r, indexing="ij")
    f = (4 * Rr ** 3 - 3 * Rr) * (2 * Z ** 2 - 1) * np.cos(2 * TH)
    c = tr.forward(f)
    w = tr.wavenumbers(p)
    ref = np.zeros_like(c)
    ref[list(w).index(2), 2, 3] = 0.5
    ref[list(w).index(-2), 2, 3] = 0.5
    assert np.max(np.abs(c - ref)) < 1e-14


def test_theta_phase_convention():
    """e^{i w theta} with theta_0 = -pi: a single Fourier mode lands on its own w."""
    m, n, p = 4, 4, 7
    r, z, th = tr.grid(m, n, p)
    TH = th[:, None, None] * np.ones((1, n, m))
    for w in range(-3, 4):
        c = tr.forward(np.cos(w * TH)) if w >= 0 else tr.forward(np.sin(-w * TH))
        wn = tr.wavenumbers(p)
        nz = {int(wn[l]) for l in range(p) if np.max(np.abs(c[l])) > 1e-12}
        assert nz == ({w, -w} if w != 0 else {0})


def test_spectral_convergence_off_grid():
    """Off-grid interpolation error decays spectrally for an analytic field."""
    def f(r, z, th):
        return np.exp(r * np.cos(th) - 0.5 * r * np.sin(th)) * np.cos(1.3 * z)

    rng = np.random.default_rng(3)
    P = 40
    rp, zp, tp = rng.uniform(-1, 1, P), rng.uniform(-1, 1, P), rng.uniform(-np.pi, np.pi, P)
    errs = []
    for N in (8, 12, 16, 20, 24):
        r, z, th = tr.grid(N, N, N)
        TH, Z, Rr = np.meshgrid(th, z, r, indexing="ij")
        c = tr.forward(f(Rr, Z, TH))
        errs.append(np.max(np.abs(tr.evaluate(c, rp, zp, tp) - f(rp, zp, tp))))
    assert errs[-1] < 1e-11
    assert all(errs[i + 1] < errs[i] * 0.05 for i in range(len(errs) - 1))


@pytest.mark.parametrize("p", [1, 2, 5, 8])
def test_hermitian_half_roundtrip(p):
    f = np.random.default_rng(p).standard_normal((p, 5, 6))
    c = tr.forward(f)
    h = tr.to_half(c)
    assert h.shape[0] == p // 2 + 1
    assert np.max(np.abs(h[0].imag)) < 1e-15
    if p % 2 == 0:
        assert np.max(np.abs(h[p // 2].imag)) < 1e-15
    assert np.max(np.abs(tr.inverse(tr.from_half(h, p)) - f)) < 1e-13


def test_physical_parity_of_smooth_fields():
    """Fields smooth through the axis have zero coefficients for j + w odd."""
    m, n, p = 12, 6, 10
    r, z, th = tr.grid(m, n, p)
    TH, Z, Rr = np.meshgrid(th, z, r, indexing="ij")
    x, y = Rr * np.cos(TH), Rr * np.sin(TH)
    c = tr.forward(np.exp(0.3 * x - 0.7 * y + x * y) * (1 + Z))
    w = tr.wavenumbers(p)
    j = np.arange(m)
    odd = (j[None, None, :] + w[:, None, None]) % 2 == 1
    assert np.max(np.abs(c * odd)) < 1e-14
