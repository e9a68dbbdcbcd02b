"""Pins for the oracle's poloidal-toroidal decomposition (Section 4, eqs. (pt)
and (ptpoisson)).

Pinned by closed forms, not by the oracle: fields built from potentials that
vanish on the side wall (Cartesian polynomials, derivatives by numpy's
polynomial routines) are decomposed back into those potentials; a purely
toroidal or poloidal field has no component of the other kind; the r^2-weighted
curl right side summed in scipy's Gegenbauer C^(2) polynomials equals the
curl formula evaluated with numpy's Chebyshev derivative; the Nyquist mode's
theta derivative vanishes on the grid; the potentials of a real field have
Hermitian coefficients (real at the Nyquist slot).
"""

import numpy as np
import numpy.polynomial.chebyshev as C
import numpy.polynomial.polynomial as P
import pytest
import scipy.special as ss

from oracle import pt
from oracle import transforms as tr


def _mesh(m, n, p):
    r, z, th = tr.grid(m, n, p)
    return np.meshgrid(th, z, r, indexing="ij")


def _poly(rng, dxy=3, dz=3):
    """Random x^i y^j z^k coefficients with i + j <= dxy, k <= dz."""
    c = rng.standard_normal((dxy + 1, dxy + 1, dz + 1))
    i, j = np.meshgrid(np.arange(dxy + 1), np.arange(dxy + 1), indexing="ij")
    c[i + j > dxy] = 0.0
    return c


def _ev(c, X, Y, Z, dx=0, dy=0, dz=0):
    if dx:
        c = P.polyder(c, dx, axis=0)
    if dy:
        c = P.polyder(c, dy, axis=1)
    if dz:
        c = P.polyder(c, dz, axis=2)
    return P.polyval3d(X, Y, Z, c)


def pt_field(cl, cg, TH, Z, R):
    """(lambda, gamma, V_r, V_theta, V_z) for lambda = s P_l, gamma = s P_g,
    s = 1 - x^2 - y^2, V = curl(lambda z) + curl curl(gamma z)
    = (lambda_y + gamma_xz, -lambda_x + gamma_yz, -gamma_xx - gamma_yy)."""
    X, Y = R * np.cos(TH), R * np.sin(TH)
    s, sx, sy = 1 - X ** 2 - Y ** 2, -2 * X, -2 * Y
    ev = lambda c, **d: _ev(c, X, Y, Z, **d)
    lam = s * ev(cl)
    gam = s * ev(cg)
    lx = sx * ev(cl) + s * ev(cl, dx=1)
    ly = sy * ev(cl) + s * ev(cl, dy=1)
    gxz = sx * ev(cg, dz=1) + s * ev(cg, dx=1, dz=1)
    gyz = sy * ev(cg, dz=1) + s * ev(cg, dy=1, dz=1)
    gxx = -2 * ev(cg) + 2 * sx * ev(cg, dx=1) + s * ev(cg, dx=2)
    gyy = -2 * ev(cg) + 2 * sy * ev(cg, dy=1) + s * ev(cg, dy=2)
    vx, vy, vz = ly + gxz, -lx + gyz, -(gxx + gyy)
    vr = vx * np.cos(TH) + vy * np.sin(TH)
    vt = -vx * np.sin(TH) + vy * np.cos(TH)
    return lam, gam, vr, vt, vz


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_manufactured_potentials_are_recovered(seed):
    m, n, p = 14, 9, 12
    rng = np.random.default_rng(100 + seed)
    lam, gam, vr, vt, vz = pt_field(_poly(rng), _poly(rng), *_mesh(m, n, p))
    l2, g2 = pt.pt_decompose(vr, vt, vz)
    assert np.max(np.abs(g2 - gam)) < 1e-11 * max(1.0, np.max(np.abs(gam)))
    assert np.max(np.abs(l2 - lam)) < 1e-11 * max(1.0, np.max(np.abs(lam)))


def test_toroidal_and_poloidal_parts_separate():
    m, n, p = 14, 9, 12
    rng = np.random.default_rng(7)
    mesh = _mesh(m, n, p)
    zero = np.zeros_like(_poly(rng))
    lam, _, vr, vt, vz = pt_field(_poly(rng), zero, *mesh)     # toroidal only
    l2, g2 = pt.pt_decompose(vr, vt, vz)
    assert np.max(np.abs(g2)) < 1e-13 and np.max(np.abs(l2 - lam)) < 1e-11
    _, gam, vr, vt, vz = pt_field(zero, _poly(rng), *mesh)     # poloidal only
    l2, g2 = pt.pt_decompose(vr, vt, vz)
    assert np.max(np.abs(l2)) < 1e-11 and np.max(np.abs(g2 - gam)) < 1e-11


@pytest.mark.parametrize("w", [0, 1, 3, -4])
def test_curl_right_side_in_gegenbauer_polynomials(w):
    """sum_k E_k C^(2)_k(r) = -(r V_theta + r^2 V_theta' - i w r V_r) for V of
    degree <= m - 5 (all of the right side then lies in the kept rows)."""
    m = 16
    rng = np.random.default_rng(40 + w)
    fr = np.zeros(m, complex)
    ft = np.zeros(m, complex)
    fr[: m - 4] = rng.standard_normal(m - 4) + 1j * rng.standard_normal(m - 4)
    ft[: m - 4] = rng.standard_normal(m - 4) + 1j * rng.standard_normal(m - 4)
    E = pt.curl_z_rhs(m, w, fr[:, None], ft[:, None])[:, 0]
    r = np.linspace(-0.97, 0.99, 23)
    lhs = sum(E[k] * ss.eval_gegenbauer(k, 2.0, r) for k in range(m - 2))
    vt, dvt, vr = C.chebval(r, ft), C.chebval(r, C.chebder(ft)), C.chebval(r, fr)
    rhs = -(r * vt + r ** 2 * dvt - 1j * w * r * vr)
    assert np.max(np.abs(lhs - rhs)) < 1e-11 * np.max(np.abs(rhs))


def test_nyquist_theta_derivative_vanishes_on_the_grid():
    """V_r = cos(p theta / 2) h(r, z) has d_theta V_r = 0 at every grid angle:
    lambda = 0 (and gamma = 0 with V_z = 0)."""
    m, n, p = 12, 7, 8
    TH, Z, R = _mesh(m, n, p)
    vr = np.cos(p * TH / 2) * (1 + R ** 2) * (1 - Z)
    l2, g2 = pt.pt_decompose(vr, np.zeros_like(vr), np.zeros_like(vr))
    assert np.max(np.abs(l2)) < 1e-13 and np.max(np.abs(g2)) == 0.0


def test_coefficients_of_a_real_field_are_hermitian():
    """A real field's potentials are real: their coefficients satisfy
    c(-w) = conj(c(w)), and the Nyquist coefficient (even p) is real."""
    m, n, p = 12, 7, 8
    rng = np.random.default_rng(11)
    v = [rng.standard_normal((p, n, m)) for _ in range(3)]
    lam, gam = pt.pt_decompose_coeffs(*[tr.forward(x) for x in v])
    wn = tr.wavenumbers(p)
    for c in (lam, gam):
        for l in range(p):
            if wn[l] == -(p // 2):
                assert np.max(np.abs(c[l].imag)) < 1e-13 * np.max(np.abs(c))
            else:
                l2 = int(np.nonzero(wn == -wn[l])[0][0])
                assert np.max(np.abs(c[l] - np.conj(c[l2]))) < 1e-13 * np.max(np.abs(c))
