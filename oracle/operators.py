"""Sparse ultraspherical operators and the per-wavenumber tau systems.

Oracle module (test infrastructure only; see the package docstring).

All matrices act on coefficient column vectors indexed from 0, i.e. entry i is
the coefficient of the degree-i basis polynomial.  Operators are built at the
requested size ``n`` by first building them ``PAD`` rows/columns larger and then
cutting, so that every truncated product below equals the same rows of the
infinite-matrix product (the inputs never carry degree >= n).

Section 3, list of operators:

* ``C01`` (T -> U conversion).  READING: the matrix printed in the paper for
  C_01 (symmetric tridiagonal with 1/2 off the diagonal) is the operator
  "multiply by x" in the U basis, not the T -> U conversion it is described as.
  We use the textbook conversion T_0 = U_0, T_1 = U_1 / 2,
  T_k = (U_k - U_{k-2}) / 2, which is the map the text describes.
  ``printed_C01`` returns the printed matrix so that tests can show it is not
  the conversion.
* ``C12`` (U -> C^(2) conversion), ``R`` (multiplication by r in C^(2)),
  ``D1``, ``D2`` (differentiation T -> U and T -> C^(2)) are as printed.
* ``C02 = C12 C01``; ``R2 = R^2 C02``.

Tau / Dirichlet closure (READING: the paper states no boundary closure for the
heat or Poisson problem).  Homogeneous Dirichlet data at r = +-1 and z = +-1 is
imposed through the basis phi_j = T_{j+2} - T_j (``dirichlet_basis``), and the
equation is kept in the first m-2 (n-2) C^(2) coefficient rows.
"""

import numpy as np

PAD = 6


def _zeros(n):
    return np.zeros((n + PAD, n + PAD))


def _cut(M, rows, cols):
    return np.ascontiguousarray(M[:rows, :cols])


def C01(n):
    """T -> U conversion (Section 3; corrected reading of the printed C_01).

    Chebyshev identity T_0 = U_0, T_1 = U_1/2, T_k = (U_k - U_{k-2})/2 (k >= 2):
    column k of the matrix holds the U coefficients of T_k.
    """
    M = _zeros(n)
    M[0, 0] = 1.0
    for k in range(1, n + PAD):
        M[k, k] = 0.5
    for k in range(2, n + PAD):
        M[k - 2, k] = -0.5
    return M


def printed_C01(n):
    """The matrix printed for C_01 in Section 3 (zero diagonal, 1/2 off it)."""
    M = np.zeros((n, n))
    for i in range(n - 1):
        M[i, i + 1] = 0.5
        M[i + 1, i] = 0.5
    return M


def C12(n):
    """U -> C^(2) conversion (Section 3, printed matrix C_12).

    U_k = (C^(2)_k - C^(2)_{k-2}) / (k + 1): diagonal 1/(i+1) and second
    super-diagonal -1/(i+3) in row i.
    """
    M = _zeros(n)
    for i in range(n + PAD):
        M[i, i] = 1.0 / (i + 1)
    for i in range(n + PAD - 2):
        M[i, i + 2] = -1.0 / (i + 3)
    return M


def R(n):
    """Multiplication by r acting on C^(2) coefficients (Section 3, matrix R).

    Row i: R[i, i-1] = i / (2(i+1)), R[i, i+1] = (i+4) / (2(i+3)); the printed
    matrix starts its sub-diagonal with 1/4 and its super-diagonal with 2/3.
    """
    M = _zeros(n)
    for i in range(n + PAD - 1):
        M[i, i + 1] = (i + 4) / (2.0 * (i + 3))
    for i in range(1, n + PAD):
        M[i, i - 1] = i / (2.0 * (i + 1))
    return M


def D1(n):
    """First derivative, T coefficients -> U coefficients (Section 3, D_1)."""
    M = _zeros(n)
    for i in range(n + PAD - 1):
        M[i, i + 1] = i + 1.0
    return M


def D2(n):
    """Second derivative, T coefficients -> C^(2) coefficients (Section 3, D_2).

    d^2/dx^2 T_k = 2k C^(2)_{k-2}; the paper's line with "T_K(x^2)" is read as
    T_K(x).
    """
    M = _zeros(n)
    for i in range(n + PAD - 2):
        M[i, i + 2] = 2.0 * (i + 2)
    return M


def C02(n):
    """T -> C^(2) conversion, C_02 = C_12 C_01 (Section 3)."""
    return C12(n) @ C01(n)


def R2(n):
    """R_2 = R^2 C_02 (Section 3): multiply by r^2 after conversion to C^(2)."""
    return R(n) @ R(n) @ C02(n)


def radial_operator(n, w):
    """r^2 (d_rr + r^-1 d_r - w^2 r^-2) in coefficient form (eq. HelmholtzMatEqn).

    R C_12 D_1 + R^2 D_2 - w^2 C_02, with w the wavenumber l - floor(p/2)
    (READING: the equation writes the storage index l where the wavenumber is
    meant).
    """
    return R(n) @ C12(n) @ D1(n) + R(n) @ R(n) @ D2(n) - float(w) ** 2 * C02(n)


def dirichlet_basis(n):
    """Q: n x (n-2), column j holds phi_j = T_{j+2} - T_j in T coefficients."""
    Q = np.zeros((n + PAD, n - 2))
    for j in range(n - 2):
        Q[j, j] = -1.0
        Q[j + 2, j] = 1.0
    return Q


def full_operators(m, n, w):
    """The m x m and n x n operators of eq. (HelmholtzMatEqn), cut to size.

    Returns (A_w, R2_m, C02_n, D2_n) acting on full T coefficients.
    """
    return (_cut(radial_operator(m, w), m, m), _cut(R2(m), m, m),
            _cut(C02(n), n, n), _cut(D2(n), n, n))


def tau_system(m, n, w):
    """Per-wavenumber Poisson tau system in the Dirichlet basis.

    With X = Q_m Xt Q_n^T substituted into r^2 nabla^2 (eq. HelmholtzMatEqn
    without the identity/time terms) and the first m-2 / n-2 rows kept:

        At Xt Bt + Ct Xt Dt = E,
        At = [A_w Q_m]_{rows < m-2},    Ct = [R2 Q_m]_{rows < m-2},
        Bt = ([C02 Q_n]_{rows < n-2})^T, Dt = ([D2 Q_n]_{rows < n-2})^T.
    """
    Qm = dirichlet_basis(m)
    Qn = dirichlet_basis(n)
    At = (radial_operator(m, w) @ Qm)[: m - 2]
    Ct = (R2(m) @ Qm)[: m - 2]
    Bt = ((C02(n) @ Qn)[: n - 2]).T
    Dt = ((D2(n) @ Qn)[: n - 2]).T
    return (np.ascontiguousarray(At), np.ascontiguousarray(Ct),
            np.ascontiguousarray(Bt), np.ascontiguousarray(Dt))


def heat_system(m, n, w, kappa_alpha):
    """Heat (BDF) tau system: the left side of eq. (HelmholtzMatEqn).

    (R2 - k a A_w) X C02^T - k a R2 X D2^T in the Dirichlet basis:
        (Ct - k a At) Xt Bt + (-k a Ct) Xt Dt.
    Returns (A_h, C_h, Bt, Dt).
    """
    At, Ct, Bt, Dt = tau_system(m, n, w)
    ka = float(kappa_alpha)
    return Ct - ka * At, -ka * Ct, Bt, Dt


def tau_rhs(m, n, F):
    """[R2 F C02^T]_{rows < m-2, cols < n-2}: the r^2-weighted tau right side.

    F holds full T coefficients (m x n, possibly complex).
    """
    R2m = _cut(R2(m), m, m)
    C02n = _cut(C02(n), n, n)
    return (R2m @ F @ C02n.T)[: m - 2, : n - 2]


def lift_rhs(m, n, w, L):
    """[r^2 nabla^2 L]_tau = [A_w L C02^T + R2 L D2^T]_tau for full coeffs L."""
    Aw, R2m, C02n, D2n = full_operators(m, n, w)
    return (Aw @ L @ C02n.T + R2m @ L @ D2n.T)[: m - 2, : n - 2]


def recombine(Xt):
    """U = Q_m Xt Q_n^T: Dirichlet-basis coefficients -> full T coefficients."""
    m = Xt.shape[0] + 2
    n = Xt.shape[1] + 2
    Qm = dirichlet_basis(m)[:m]
    Qn = dirichlet_basis(n)[:n]
    return Qm @ Xt @ Qn.T
