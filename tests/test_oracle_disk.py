"""Pins for the oracle's horizontal (disk) Poisson solve (Section 4,
eq. (ptpoisson): Delta_h = nabla^2 - d_zz, solved by diagonalising in theta
and z).

Pinned by closed forms, not by the oracle: polynomial solutions in the trial
space (exact), a Bessel eigenfunction of Delta_h (spectral accuracy), a
Cartesian polynomial whose horizontal Laplacian is worked out by hand, and
the independence of the z levels.
"""

import numpy as np
import pytest
import scipy.special as ss

from oracle import problems as pb
from oracle import transforms as tr


def _mesh(m, n, p):
    r, z, th = tr.grid(m, n, p)
    return np.meshgrid(th, z, r, indexing="ij")


@pytest.mark.parametrize("w", [0, 1, 2, 5])
def test_polynomial_solutions_are_exact(w):
    """u = (1 - r^2) r^w h(z) cos(w theta): Delta_h u = -(4w + 4) r^w h(z) cos(w theta)."""
    m, n, p = 14, 9, 12
    TH, Z, R = _mesh(m, n, p)
    h = 1.0 + Z - 2.0 * Z ** 3 + 0.5 * Z ** 6
    u = (1 - R ** 2) * R ** w * h * np.cos(w * TH)
    f = -(4 * w + 4) * R ** w * h * np.cos(w * TH)
    assert np.max(np.abs(pb.disk_poisson(f) - u)) < 1e-12


def test_bessel_eigenfunction():
    """J_w(j r) with J_w(j) = 0 is an eigenfunction of Delta_h with eigenvalue -j^2."""
    m, n, p = 48, 6, 8
    TH, Z, R = _mesh(m, n, p)
    for w in (0, 3):
        j1 = ss.jn_zeros(w, 1)[0]
        u = ss.jv(w, j1 * R) * (1 + Z ** 2) * np.cos(w * TH + 0.3)
        assert np.max(np.abs(pb.disk_poisson(-j1 ** 2 * u) - u)) < 1e-12


def test_cartesian_polynomial():
    """u = (1 - x^2 - y^2)(x + y z^2 + 1): Delta_h u = -4 (x + y z^2 + 1) - 4x - 4 y z^2."""
    m, n, p = 12, 8, 10
    TH, Z, R = _mesh(m, n, p)
    X, Y = R * np.cos(TH), R * np.sin(TH)
    q = X + Y * Z ** 2 + 1
    u = (1 - X ** 2 - Y ** 2) * q
    f = -4 * q - 4 * X - 4 * Y * Z ** 2
    assert np.max(np.abs(pb.disk_poisson(f) - u)) < 1e-12


def test_z_coefficients_are_independent():
    """Changing the forcing's z-coefficient k changes only the solution's
    z-coefficient k (no coupling in z)."""
    m, n, p = 16, 10, 6
    c = tr.forward(np.random.default_rng(5).standard_normal((p, n, m)))
    u0 = pb.disk_poisson_coeffs(c)
    c2 = c.copy()
    c2[:, 4, :] *= 3.0
    u1 = pb.disk_poisson_coeffs(c2)
    d = np.max(np.abs(u1 - u0), axis=(0, 2))
    assert np.all(d[np.arange(n) != 4] == 0.0) and d[4] > 0
