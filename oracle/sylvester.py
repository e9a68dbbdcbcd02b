"""Exact (to rounding) solution of the per-mode Sylvester equation A X B + C X D = E.

Oracle module (test infrastructure only; see the package docstring).

Eq. (HelmholtzMatEqn) decouples in theta into one generalised Sylvester
equation per wavenumber (Section 3, the remark after the equation).  The
discrete operator is nonsingular, so the equation has exactly one solution;
ADI (Algorithm 1) approximates it.  The oracle computes it by two routes that
share nothing with ADI or with each other:

* ``kron_solve``: the definition written out -- dense LU of the Kronecker
  matrix A (x) B^T + C (x) D^T acting on the row-major vectorisation of X.
  Only for small sizes.
* ``bs_solve``: Bartels-Stewart in diagonalised form.  The z-pencil is
  diagonalised once, D V = B V Lambda; then Y = X B V satisfies
  A Y + C Y Lambda = E V, i.e. one banded solve (A + lambda_i C) y_i = (E V)_i
  per eigenvalue, and X = Y (B V)^{-1}.
* ``refine``: iterative refinement with the residual E - (A X B + C X D)
  formed in 80-bit extended precision from the nonzero diagonals only.
"""

import numpy as np
import scipy.linalg as sl


def kron_solve(A, B, C, D, E):
    """Dense Kronecker solve of A X B + C X D = E (row-major vec(X))."""
    K = np.kron(A, B.T) + np.kron(C, D.T)
    x = np.linalg.solve(K, np.asarray(E).reshape(-1))
    return x.reshape(E.shape)


def _bandwidths(M, tol=0.0):
    idx = np.argwhere(np.abs(M) > tol)
    d = idx[:, 1] - idx[:, 0]
    return int(max(0, -d.min())), int(max(0, d.max()))


def _to_banded(M, l, u):
    n = M.shape[0]
    ab = np.zeros((l + u + 1, n), dtype=M.dtype)
    for d in range(-l, u + 1):
        diag = np.diagonal(M, d)
        if d >= 0:
            ab[u - d, d:] = diag
        else:
            ab[u - d, : n + d] = diag
    return ab


_ZCACHE = {}


def z_eig(B, D):
    """Diagonalise the z-pencil: D V = B V Lambda (eigenvalues real, Section 3)."""
    key = (B.shape[0], B.tobytes(), D.tobytes())
    hit = _ZCACHE.get(key)
    if hit is not None:
        return hit
    lam, V = sl.eig(D, B)
    if np.max(np.abs(lam.imag)) > 1e-8 * np.max(np.abs(lam.real)):
        raise RuntimeError("z-pencil has complex eigenvalues")
    lam = lam.real.copy()
    V = V.real.copy()
    BV = B @ V
    lu = sl.lu_factor(BV)
    out = (lam, V, lu)
    if len(_ZCACHE) > 16:
        _ZCACHE.clear()
    _ZCACHE[key] = out
    return out


def bs_solve(A, B, C, D, E):
    """Diagonalised Bartels-Stewart solve of A X B + C X D = E."""
    lam, V, lu = z_eig(B, D)
    E = np.asarray(E)
    EV = E @ V
    lA, uA = _bandwidths(A)
    lC, uC = _bandwidths(C)
    l, u = max(lA, lC), max(uA, uC)
    Y = np.empty_like(EV, dtype=np.result_type(EV, A))
    for i, li in enumerate(lam):
        M = A + li * C
        Y[:, i] = sl.solve_banded((l, u), _to_banded(M, l, u), EV[:, i])
    # X = Y (B V)^{-1}  <=>  (B V)^T X^T = Y^T
    return sl.lu_solve(lu, Y.T, trans=1).T


def _band_left(M, X):
    """M @ X with M applied through its nonzero diagonals, in extended precision."""
    n = M.shape[0]
    out = np.zeros(X.shape, dtype=X.dtype)
    l, u = _bandwidths(M)
    for d in range(-l, u + 1):
        diag = np.diagonal(M, d).astype(np.longdouble)
        if not np.any(diag):
            continue
        if d >= 0:
            out[: n - d] += diag[:, None] * X[d:]
        else:
            out[-d:] += diag[:, None] * X[: n + d]
    return out


def residual_ld(A, B, C, D, X, E):
    """E - (A X B + C X D) evaluated in 80-bit extended precision."""
    cplx = np.iscomplexobj(X) or np.iscomplexobj(E)
    dt = np.clongdouble if cplx else np.longdouble
    Xl = np.asarray(X).astype(dt)
    El = np.asarray(E).astype(dt)
    AXB = _band_left(B.T, _band_left(A, Xl).T).T
    CXD = _band_left(D.T, _band_left(C, Xl).T).T
    return El - AXB - CXD


def refine(A, B, C, D, E, X, steps=2, solver=bs_solve):
    """Iterative refinement with extended-precision residuals."""
    for _ in range(steps):
        Rl = residual_ld(A, B, C, D, X, E)
        Rd = Rl.astype(np.complex128 if np.iscomplexobj(Rl) else np.float64)
        X = X + solver(A, B, C, D, Rd)
    return X


def solve(A, B, C, D, E, method="bs", refine_steps=2):
    """Oracle solution of A X B + C X D = E (``bs`` or ``kron``), refined."""
    solver = bs_solve if method == "bs" else kron_solve
    X = solver(A, B, C, D, E)
    if refine_steps:
        X = refine(A, B, C, D, E, X, steps=refine_steps, solver=solver)
    return X
