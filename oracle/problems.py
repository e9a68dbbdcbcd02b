"""Poisson and heat solves on the closed cylinder (Sections 2 and 3).

Oracle module (test infrastructure only; see the package docstring).

Every wavenumber is solved independently (the theta decoupling of
eq. (HelmholtzMatEqn)); for real data nothing exploits Hermitian symmetry, so
the symmetry of the output is itself a check.

Boundary data (READING: the paper states no boundary closure for these two
problems): homogeneous Dirichlet through the Dirichlet basis; non-homogeneous
Dirichlet data is given as a lift field L (values on the grid) whose boundary
values are the data; the solver then solves for u - L with the right side
reduced by r^2 nabla^2 L.  The discrete solution depends only on L's boundary
values.

Heat (Section 3, BDF paragraphs and eq. (Helmholtz)):
kappa^(1) = h, delta^(1) X = X(t);
kappa^(4) = 12 h / 25, delta^(4) X = (48 X(t) - 36 X(t-h) + 16 X(t-2h) - 3 X(t-3h)) / 25.
The forcing is time independent (the paper's g(t+h) ~ g(t) is then exact).
READING (BDF4 start-up is not stated): the caller supplies all four history
levels.
"""

import numpy as np

from . import operators as ops
from . import sylvester
from . import transforms as tr


def _mode_matrix(c, l):
    """X_l[j, k] = c[l, k, j] (Section 3: rows are r-degrees, columns z-degrees)."""
    return np.asarray(c[l]).T


def poisson_mode(m, n, w, F, L=None, method="bs", refine_steps=2):
    """Solve r^2 nabla^2 u = r^2 f for one wavenumber; F, L are m x n T-coeffs.

    Returns the full T coefficients U (m x n) of the discrete solution.
    """
    At, Ct, Bt, Dt = ops.tau_system(m, n, w)
    E = ops.tau_rhs(m, n, F)
    if L is not None:
        E = E - ops.lift_rhs(m, n, w, L)
    Xt = sylvester.solve(At, Bt, Ct, Dt, E, method=method, refine_steps=refine_steps)
    U = ops.recombine(Xt)
    if L is not None:
        U = U + L
    return U


def poisson_coeffs(c_f, c_lift=None, modes=None, method="bs", refine_steps=2):
    """Full-coefficient Poisson solve.  ``modes``: optional subset of storage indices."""
    p, n, m = c_f.shape
    out = np.zeros((p, n, m), dtype=np.complex128)
    wn = tr.wavenumbers(p)
    for l in (range(p) if modes is None else modes):
        L = None if c_lift is None else _mode_matrix(c_lift, l)
        U = poisson_mode(m, n, wn[l], _mode_matrix(c_f, l), L, method, refine_steps)
        out[l] = U.T
    return out


def poisson(f, lift=None, method="bs", refine_steps=2):
    """Value-space Poisson solve nabla^2 u = f (lift: boundary data field or None)."""
    c_f = tr.forward(f)
    c_l = None if lift is None else tr.forward(lift)
    return tr.inverse(poisson_coeffs(c_f, c_l, None, method, refine_steps))


BDF = {
    1: (1.0, (1.0,)),
    4: (12.0 / 25.0, (48.0 / 25.0, -36.0 / 25.0, 16.0 / 25.0, -3.0 / 25.0)),
}


def heat_coeffs(history, c_g, alpha, h, steps, order=1, c_lift=None, modes=None,
                method="bs", refine_steps=2):
    """BDF heat stepping in full coefficients.

    history: list of ``order`` full-coefficient fields, newest first.
    Returns the list of history levels after ``steps`` steps (newest first).
    """
    kfac, beta = BDF[order]
    kappa = kfac * h
    ka = kappa * alpha
    p, n, m = c_g.shape
    wn = tr.wavenumbers(p)
    hist = [np.array(x, dtype=np.complex128) for x in history]
    if c_lift is not None:
        hist = [x - c_lift for x in hist]
    assert len(hist) == order
    ls = range(p) if modes is None else list(modes)
    systems = {l: ops.heat_system(m, n, wn[l], ka) for l in ls}
    lifts = {}
    if c_lift is not None:
        for l in ls:
            lifts[l] = ka * ops.lift_rhs(m, n, wn[l], _mode_matrix(c_lift, l))
    for _ in range(steps):
        new = np.zeros((p, n, m), dtype=np.complex128)
        for l in ls:
            delta = sum(bk * _mode_matrix(hk, l) for bk, hk in zip(beta, hist))
            E = ops.tau_rhs(m, n, delta + kappa * _mode_matrix(c_g, l))
            if c_lift is not None:
                E = E + lifts[l]
            Ah, Ch, Bt, Dt = systems[l]
            Xt = sylvester.solve(Ah, Bt, Ch, Dt, E, method=method, refine_steps=refine_steps)
            new[l] = ops.recombine(Xt).T
        hist = [new] + hist[:-1]
    if c_lift is not None:
        hist = [x + c_lift for x in hist]
    return hist


def heat(history_values, g, alpha, h, steps, order=1, lift=None, method="bs", refine_steps=2):
    """Value-space heat run; returns the final temperature values."""
    hist_c = [tr.forward(v) for v in history_values]
    c_g = tr.forward(g)
    c_l = None if lift is None else tr.forward(lift)
    out = heat_coeffs(hist_c, c_g, alpha, h, steps, order, c_l, None, method, refine_steps)
    return tr.inverse(out[0])


# ----------------------------------------------------------------------------
# Horizontal (disk) Poisson (Section 4, eq. (ptpoisson))
# ----------------------------------------------------------------------------

def disk_poisson_mode(m, n, w, F):
    """Solve Delta_h u = f for one wavenumber, u = 0 at r = +-1.

    Delta_h = nabla^2 - d_zz has no z derivative, so after the theta DFT every
    Chebyshev z coefficient k is its own problem in r (the diagonalisation in
    theta and z of Section 4): r^2 (d_rr + r^-1 d_r - w^2 r^-2) u_k = r^2 f_k,
    in the Dirichlet basis of Section 3 with the first m-2 C^(2) rows kept:
    At x_k = [R2 f_k]_tau, u_k = Q_m x_k.  F: m x n full T coefficients
    (rows r-degrees).  READING: the paper states no boundary condition for
    this solve in isolation; homogeneous Dirichlet at the side wall is used
    (no condition in z, where the operator has no derivative).
    """
    At, _, _, _ = ops.tau_system(m, max(n, 3), w)
    R2m = ops._cut(ops.R2(m), m, m)
    E = (R2m @ F)[: m - 2]
    Xt = np.linalg.solve(At, E)
    Qm = ops.dirichlet_basis(m)[:m]
    return Qm @ Xt


def disk_poisson_coeffs(c_f):
    """Full-coefficient disk solve c[l, k, j] -> c_u[l, k, j] (every wavenumber)."""
    p, n, m = c_f.shape
    wn = tr.wavenumbers(p)
    out = np.zeros_like(c_f)
    for l in range(p):
        out[l] = disk_poisson_mode(m, n, wn[l], _mode_matrix(c_f, l)).T
    return out


def disk_poisson(f):
    """Value-space horizontal Poisson solve Delta_h u = f, u = 0 at r = +-1."""
    return np.real(tr.inverse(disk_poisson_coeffs(tr.forward(f))))
