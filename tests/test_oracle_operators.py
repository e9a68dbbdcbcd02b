"""Pins for the oracle's operators (Section 3) against printed values and identities.

The identities are checked by evaluating polynomials with scipy's independent
Chebyshev / Gegenbauer evaluators at random points.
"""

import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.special as ss

from oracle import operators as ops


def _load(golden_dir):
    with open(os.path.join(golden_dir, "printed_operators.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("name,builder", [
    ("C12", ops.C12), ("R", ops.R), ("D1", ops.D1), ("D2", ops.D2),
    ("C01_printed", ops.printed_C01)])
def test_printed_entries(golden_dir, name, builder):
    g = _load(golden_dir)
    n = g["n"]
    M = builder(n)[:n, :n]
    for i, j, num, den in g[name]["lead"] + g[name]["end"]:
        assert M[i, j] == pytest.approx(float(Fraction(num, den)), abs=1e-15), (name, i, j)


def _T(k, x):
    return ss.eval_chebyt(k, x)


def _U(k, x):
    return ss.eval_chebyu(k, x)


def _C2(k, x):
    return ss.eval_gegenbauer(k, 2.0, x)


def _series(basis, coef, x):
    return sum(c * basis(i, x) for i, c in enumerate(coef))


@pytest.fixture
def pts():
    return np.random.default_rng(7).uniform(-1, 1, 25)


N = 12


def test_C01_is_T_to_U(pts):
    a = np.random.default_rng(1).standard_normal(N)
    b = ops.C01(N)[:N + 2, :N] @ a
    assert np.allclose(_series(_U, b, pts), _series(_T, a, pts), atol=1e-13, rtol=0)


def test_printed_C01_is_not_the_conversion(pts):
    a = np.random.default_rng(1).standard_normal(N)
    b = ops.printed_C01(N) @ a
    assert np.max(np.abs(_series(_U, b, pts) - _series(_T, a, pts))) > 1e-2


def test_C12_is_U_to_C2(pts):
    a = np.random.default_rng(2).standard_normal(N)
    b = ops.C12(N)[:N + 2, :N] @ a
    assert np.allclose(_series(_C2, b, pts), _series(_U, a, pts), atol=1e-13, rtol=0)


def test_R_multiplies_by_x(pts):
    a = np.random.default_rng(3).standard_normal(N)
    b = ops.R(N)[:N + 2, :N] @ a
    assert np.allclose(_series(_C2, b, pts), pts * _series(_C2, a, pts), atol=1e-12, rtol=0)


def test_D1_D2_differentiate(pts):
    a = np.random.default_rng(4).standard_normal(N)
    d1 = np.polynomial.chebyshev.chebval(pts, np.polynomial.chebyshev.chebder(a, 1))
    d2 = np.polynomial.chebyshev.chebval(pts, np.polynomial.chebyshev.chebder(a, 2))
    assert np.allclose(_series(_U, ops.D1(N)[:N, :N] @ a, pts), d1, atol=1e-11, rtol=0)
    assert np.allclose(_series(_C2, ops.D2(N)[:N, :N] @ a, pts), d2, atol=1e-9, rtol=1e-13)


def test_C02_R2_compose(pts):
    a = np.random.default_rng(5).standard_normal(N)
    t = _series(_T, a, pts)
    assert np.allclose(_series(_C2, ops.C02(N)[:N + 4, :N] @ a, pts), t, atol=1e-13, rtol=0)
    assert np.allclose(_series(_C2, ops.R2(N)[:N + 6, :N] @ a, pts), pts ** 2 * t, atol=1e-12, rtol=0)


@pytest.mark.parametrize("w", [0, 1, 3])
def test_radial_operator(pts, w):
    """r^2 u'' + r u' - w^2 u in C^(2) coefficients (eq. HelmholtzMatEqn)."""
    a = np.random.default_rng(6 + w).standard_normal(N)
    cd = np.polynomial.chebyshev
    u = cd.chebval(pts, a)
    du = cd.chebval(pts, cd.chebder(a, 1))
    ddu = cd.chebval(pts, cd.chebder(a, 2))
    ref = pts ** 2 * ddu + pts * du - w * w * u
    got = _series(_C2, ops.radial_operator(N, w)[:N + 6, :N] @ a, pts)
    assert np.allclose(got, ref, atol=1e-9, rtol=1e-13)


def test_dirichlet_basis_vanishes_on_boundary():
    Q = ops.dirichlet_basis(N)[:N]
    for x in (-1.0, 1.0):
        vals = np.array([_series(_T, Q[:, j], np.array([x]))[0] for j in range(N - 2)])
        assert np.max(np.abs(vals)) < 1e-14


@pytest.mark.parametrize("m,n,w", [(12, 10, 0), (13, 11, 2), (20, 16, 5)])
def test_parity_decoupling_and_bandwidths(m, n, w):
    """Parity blocks decouple; the block bandwidths the library relies on."""
    At, Ct, Bt, Dt = ops.tau_system(m, n, w)

    def bw(M):
        idx = np.argwhere(np.abs(M) > 0)
        d = idx[:, 1] - idx[:, 0]
        return int(-d.min()), int(d.max())

    for pr in (0, 1):
        for M in (At, Ct):
            assert np.max(np.abs(M[pr::2, 1 - pr::2])) == 0.0
        for M in (Bt, Dt):
            assert np.max(np.abs(M[pr::2, 1 - pr::2])) == 0.0
        assert bw(At[pr::2, pr::2]) == (1, 2)
        assert bw(Ct[pr::2, pr::2]) == (2, 3)
        assert bw(Bt[pr::2, pr::2]) == (2, 1)
        lo, hi = bw(Dt[pr::2, pr::2])
        assert lo == 1 and hi <= 0
