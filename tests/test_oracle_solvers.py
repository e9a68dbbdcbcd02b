"""Pins for the oracle's Poisson and heat solves (Sections 2-3).

Each pin is fixed by something other than the oracle itself: closed-form
solutions, a Galerkin characterisation evaluated by quadrature, a 3-D system
built with a different theta discretisation, or exact scalar recurrences.
"""

import numpy as np
import pytest
import scipy.special as ss

from oracle import operators as ops
from oracle import problems as pb
from oracle import sylvester as sy
from oracle import transforms as tr


def _mesh(m, n, p):
    r, z, th = tr.grid(m, n, p)
    return np.meshgrid(th, z, r, indexing="ij")   # TH, Z, R with shape (p, n, m)


# ----------------------------------------------------------------------------
# manufactured polynomial solutions (exactly in the trial space)
# ----------------------------------------------------------------------------

def _manufactured(m, n, p, w, a):
    """u = (1 - r^2) r^w (1 - z^2) z^a cos(w theta) and its Laplacian (closed form)."""
    TH, Z, R = _mesh(m, n, p)
    g = (1 - R ** 2) * R ** w                       # radial factor
    # g'' + g'/r - w^2 g / r^2 for g = r^w - r^(w+2):
    #   = [w(w-1) + w - w^2] r^(w-2) - [(w+2)(w+1) + (w+2) - w^2] r^w = -(4w + 4) r^w
    lap_r = -(4 * w + 4) * R ** w
    hz = (1 - Z ** 2) * Z ** a
    hzz = a * (a - 1) * Z ** (a - 2) - (a + 2) * (a + 1) * Z ** a if a >= 2 else \
        -(a + 2) * (a + 1) * Z ** a
    u = g * hz * np.cos(w * TH)
    f = (lap_r * hz + g * hzz) * np.cos(w * TH)
    return u, f


@pytest.mark.parametrize("m,n,p,w,a", [(10, 9, 4, 0, 2), (12, 10, 6, 1, 3), (14, 12, 8, 3, 1),
                                       (16, 16, 9, 4, 4)])
@pytest.mark.parametrize("method", ["bs", "kron"])
def test_manufactured_polynomial_is_recovered(m, n, p, w, a, method):
    u, f = _manufactured(m, n, p, w, a)
    got = pb.poisson(f, method=method)
    assert np.max(np.abs(got - u)) < 1e-13 * max(1.0, np.max(np.abs(u)))


def test_kron_and_bs_agree():
    for (m, n, w) in [(18, 14, 0), (20, 22, 3), (34, 34, 7)]:
        At, Ct, Bt, Dt = ops.tau_system(m, n, w)
        E = np.random.default_rng(m + w).standard_normal((m - 2, n - 2))
        Xk = sy.kron_solve(At, Bt, Ct, Dt, E)
        Xb = sy.bs_solve(At, Bt, Ct, Dt, E)
        assert np.max(np.abs(Xk - Xb)) < 1e-12 * np.max(np.abs(Xk))


def test_refined_bs_backward_stable_larger_size():
    """Componentwise backward error at rounding level, and a further refinement
    step no longer moves the solution."""
    m = n = 130
    At, Ct, Bt, Dt = ops.tau_system(m, n, 2)
    E = np.random.default_rng(0).standard_normal((m - 2, n - 2))
    X = sy.solve(At, Bt, Ct, Dt, E)
    res = np.abs(sy.residual_ld(At, Bt, Ct, Dt, X, E).astype(np.float64))
    aX = np.abs(X)
    scale = np.abs(At) @ aX @ np.abs(Bt) + np.abs(Ct) @ aX @ np.abs(Dt) + np.abs(E)
    assert np.max(res / scale) < 1e-15
    X2 = sy.refine(At, Bt, Ct, Dt, E, X, steps=1)
    assert np.max(np.abs(X2 - X)) < 1e-14 * np.max(np.abs(X))


# ----------------------------------------------------------------------------
# Galerkin characterisation of the tau system, by quadrature
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,w", [(10, 8, 0), (11, 9, 2), (14, 12, 5)])
def test_tau_solution_satisfies_weighted_orthogonality(m, n, w):
    """The discrete solution vanishes on r = +-1, z = +-1 and the r^2-weighted
    residual r^2 (nabla^2 u - f) is orthogonal, in the C^(2) weight
    (1 - x^2)^(3/2), to every C^(2)_a(r) C^(2)_b(z) with a < m-2, b < n-2.
    Evaluated with Gauss-Gegenbauer quadrature and numpy's Chebyshev calculus."""
    rng = np.random.default_rng(m * n + w)
    F = rng.standard_normal((m, n))
    U = pb.poisson_mode(m, n, w, F)
    cd = np.polynomial.chebyshev
    xq, wq = ss.roots_gegenbauer(m + 4, 2.0)
    yq, vq = ss.roots_gegenbauer(n + 4, 2.0)

    def ev(C, dr=0, dz=0):
        Cr = cd.chebder(C, dr, axis=0) if dr else C
        Crz = cd.chebder(Cr, dz, axis=1) if dz else Cr
        return cd.chebgrid2d(xq, yq, Crz)

    r = xq[:, None]
    res = r ** 2 * ev(U, 2, 0) + r * ev(U, 1, 0) - w * w * ev(U) + r ** 2 * ev(U, 0, 2) - r ** 2 * ev(F)
    scale = np.abs(r ** 2 * ev(F))
    Pa = np.array([ss.eval_gegenbauer(a, 2.0, xq) for a in range(m - 2)])
    Pb = np.array([ss.eval_gegenbauer(b, 2.0, yq) for b in range(n - 2)])
    mom = (Pa * wq) @ res @ (Pb * vq).T
    ref = (np.abs(Pa) * wq) @ scale @ (np.abs(Pb) * vq).T
    assert np.max(np.abs(mom) / ref) < 1e-12
    for x in (-1.0, 1.0):
        assert np.max(np.abs(cd.chebgrid2d([x], yq, U))) < 1e-13
        assert np.max(np.abs(cd.chebgrid2d(xq, [x], U))) < 1e-13


# ----------------------------------------------------------------------------
# theta decoupling against a 3-D system with theta in value space
# ----------------------------------------------------------------------------

def _fourier_d2(p):
    """Second-derivative matrix of the trigonometric interpolant on p equispaced
    points (closed form; p even)."""
    h = 2 * np.pi / p
    D = np.empty((p, p))
    for i in range(p):
        for j in range(p):
            if i == j:
                D[i, j] = -np.pi ** 2 / (3 * h ** 2) - 1.0 / 6.0
            else:
                D[i, j] = -0.5 * (-1) ** (i - j) / np.sin((i - j) * h / 2) ** 2
    return D


@pytest.mark.parametrize("m,n,p", [(8, 7, 6), (7, 8, 8)])
def test_theta_decoupling_matches_3d_system(m, n, p):
    """Per-wavenumber solves (eq. HelmholtzMatEqn decoupled in theta) equal the
    solution of one 3-D system in which theta is kept in value space and
    d^2/dtheta^2 is the Fourier differentiation matrix."""
    rng = np.random.default_rng(11)
    f = rng.standard_normal((p, n, m))
    u_modes = pb.poisson(f)

    cd = np.polynomial.chebyshev
    r, z, th = tr.grid(m, n, p)
    Vr = cd.chebvander(r, m - 1)
    Vz = cd.chebvander(z, n - 1)
    Fc = [np.linalg.solve(Vr, np.linalg.solve(Vz, f[l]).T) for l in range(p)]  # m x n each

    Qm = ops.dirichlet_basis(m)
    Qn = ops.dirichlet_basis(n)
    A0 = ((ops.R(m) @ ops.C12(m) @ ops.D1(m) + ops.R(m) @ ops.R(m) @ ops.D2(m)) @ Qm)[: m - 2]
    Cc = (ops.C02(m) @ Qm)[: m - 2]
    Ct = (ops.R2(m) @ Qm)[: m - 2]
    Bt = ((ops.C02(n) @ Qn)[: n - 2]).T
    Dt = ((ops.D2(n) @ Qn)[: n - 2]).T
    Dth = _fourier_d2(p)
    K = np.kron(np.eye(p), np.kron(A0, Bt.T) + np.kron(Ct, Dt.T)) + np.kron(Dth, np.kron(Cc, Bt.T))
    E = np.concatenate([ops.tau_rhs(m, n, Fc[l]).ravel() for l in range(p)])
    Xs = np.linalg.solve(K, E).reshape(p, m - 2, n - 2)
    u3 = np.stack([Vz @ (Vr @ ops.recombine(Xs[l])).T for l in range(p)])
    assert np.max(np.abs(u3 - u_modes)) < 1e-12 * np.max(np.abs(u_modes))


# ----------------------------------------------------------------------------
# spectral accuracy against Bessel x sine eigenfunctions
# ----------------------------------------------------------------------------

def _eigfun(m, n, p, w, s, q):
    TH, Z, R = _mesh(m, n, p)
    j = ss.jn_zeros(w, s)[-1]
    lam = j * j + (q * np.pi / 2) ** 2
    phi = ss.jv(w, j * R) * np.sin(q * np.pi * (Z + 1) / 2) * np.cos(w * TH)
    return phi, lam


def test_poisson_spectral_convergence_bessel_sine():
    errs = []
    for N in (12, 16, 20, 24, 28):
        phi, lam = _eigfun(N, N, 8, 3, 2, 1)
        u = pb.poisson(-lam * phi)
        errs.append(np.max(np.abs(u - phi)))
    assert errs[-1] < 1e-11
    assert all(errs[i + 1] < 0.1 * errs[i] for i in range(len(errs) - 1))


def test_real_data_gives_hermitian_output():
    f = np.random.default_rng(5).standard_normal((7, 9, 10))
    c = pb.poisson_coeffs(tr.forward(f))
    wn = tr.wavenumbers(7)
    for l, w in enumerate(wn):
        if w > 0:
            lm = list(wn).index(-w)
            assert np.max(np.abs(c[l] - np.conj(c[lm]))) < 1e-13 * np.max(np.abs(c))
    v = tr.inverse(c, real=False)
    assert np.max(np.abs(v.imag)) < 1e-13 * np.max(np.abs(v.real))


# ----------------------------------------------------------------------------
# non-homogeneous Dirichlet data through a lift
# ----------------------------------------------------------------------------

def test_lift_recovers_polynomial_with_boundary_data():
    """u polynomial with nonzero boundary values; the lift is a different field
    with the same boundary values; the solve must return u exactly."""
    m, n, p = 12, 10, 6
    TH, Z, R = _mesh(m, n, p)
    X, Y = R * np.cos(TH), R * np.sin(TH)
    u = 1.0 + X + 2 * Y * Z + X * X - Y * Y + 3 * Z ** 3          # Laplacian: 18 z
    f = 18.0 * Z
    bump = (1 - R ** 2) * (1 - Z ** 2) * (0.3 + X * Z - Y ** 2)
    got = pb.poisson(f, lift=u + bump)
    assert np.max(np.abs(got - u)) < 1e-12


# ----------------------------------------------------------------------------
# heat stepping
# ----------------------------------------------------------------------------

def test_bdf1_eigenmode_decay_is_exact():
    """g = 0, T0 = Bessel x sine eigenfunction: BDF1 gives (1 + h a lam)^-N T0."""
    m, n, p = 24, 16, 6
    phi, lam = _eigfun(m, n, p, 1, 1, 1)
    alpha, h, N = 1.0, 1e-3, 60
    T = pb.heat([phi], np.zeros_like(phi), alpha, h, N, order=1)
    ref = (1 + h * alpha * lam) ** (-N) * phi
    assert np.max(np.abs(T - ref)) < 1e-12
    assert np.max(np.abs(T - np.exp(-alpha * lam * h * N) * phi)) < 1e-2 * np.max(np.abs(phi))


def test_bdf4_eigenmode_follows_scalar_recurrence(golden_dir):
    import json
    import os
    with open(os.path.join(golden_dir, "bdf.json")) as fh:
        g = json.load(fh)["bdf4"]
    kfac = g["kappa_over_h"][0] / g["kappa_over_h"][1]
    beta = [a / b for a, b in g["delta"]]
    m, n, p = 24, 16, 6
    phi, lam = _eigfun(m, n, p, 0, 1, 1)
    alpha, h, N = 0.5, 2e-3, 30
    x = [np.exp(alpha * lam * h * k) for k in range(4)]            # newest first
    hist = [xk * phi for xk in x]
    T = pb.heat(hist, np.zeros_like(phi), alpha, h, N, order=4)
    for _ in range(N):
        xn = sum(b * xk for b, xk in zip(beta, x)) / (1 + kfac * h * alpha * lam)
        x = [xn] + x[:-1]
    assert np.max(np.abs(T - x[0] * phi)) < 1e-12
    # fourth order in time: much closer to the true decay than BDF1 would be
    assert abs(x[0] - np.exp(-alpha * lam * h * N)) < 1e-6


@pytest.mark.parametrize("order", [1, 4])
def test_heat_steady_state_with_forcing_and_lift(order):
    """T0 = psi and g = -alpha nabla^2 psi: psi is a fixed point of every step
    (pins the sign and the kappa factor on g, and the lift term)."""
    m, n, p = 10, 9, 6
    TH, Z, R = _mesh(m, n, p)
    X, Y = R * np.cos(TH), R * np.sin(TH)
    psi = 2.0 + X * Z + Y * Y * Z + Z ** 2             # Laplacian: 2 z + 2
    alpha = 0.7
    g = -alpha * (2 * Z + 2.0)
    lift = psi + (1 - R ** 2) * (1 - Z ** 2) * X
    T = pb.heat([psi] * order, g, alpha, 1e-2, 5, order=order, lift=lift)
    assert np.max(np.abs(T - psi)) < 1e-12
