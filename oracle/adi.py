"""ADI (Algorithm 1) with Zolotarev-optimal shifts (Section 3).

Oracle module (test infrastructure only; see the package docstring).

Written in the paper's order and notation: spectral intervals [a, b] of C^-1 A
and [c, d] of -D B^-1; gamma, alpha, k, K(k), dn and the Moebius map T; then
the two half-steps of Algorithm 1.  The paper reuses symbols: its alpha in the
shift formula is called ``alpha_z`` here (alpha is the diffusivity), and its
Moebius map T is called ``T_map``.

READINGS (each is listed with its reason in the project's design notes):

* Sign: as printed, both half-steps of Algorithm 1 have the fixed point
  A X B + C X D = -E.  We use
      (u_j C - A) X_{j+1/2} B = C X_j (u_j B + D) - E,
      C X_{j+1} (v_j B + D)   = (v_j C - A) X_{j+1/2} B + E,
  whose fixed point is A X B + C X D = E.  "X_{k+1}" in the second step is
  read as X_{j+1}.
* Shift roles: the first half-step inverts (u_j C - A), so u_j must lie near
  the spectrum of -D B^-1, i.e. in [c, d]; the printed u_j = T(-alpha dn)
  lies in [a, b] and the iteration diverges.  We take
      u_j = T(+alpha dn_j),  v_j = T(-alpha dn_j).
* dn and K use the modulus k of the cited elliptic-function reference; both
  are computed from the complementary modulus k' = 1/alpha by the
  arithmetic-geometric mean, which stays finite when 1 - 1/alpha^2 rounds to 1.
  For arguments above K/2, dn is taken from the reflection dn(K - x) = k'/dn(x).
* Number of iterations for a tolerance eps (the paper only states
  J = O(log mn)): J = ceil(ln(16 gamma) ln(4/eps) / pi^2), the Zolotarev-number
  bound of the shift reference cited in Section 3.
"""

import math

import numpy as np
import scipy.linalg as sl


# --------------------------------------------------------------------------
# spectral intervals
# --------------------------------------------------------------------------

def spectral_bounds(A, B, C, D):
    """[a, b] = extreme eigenvalues of C^-1 A and [c, d] of -D B^-1 (dense eig)."""
    ev1 = sl.eigvals(A, C)
    ev2 = sl.eigvals(-D.T, B.T)          # spectrum of -D B^-1 equals that of -B^-T D^T
    ev1 = ev1[np.isfinite(ev1)]
    ev2 = ev2[np.isfinite(ev2)]
    return (float(ev1.real.min()), float(ev1.real.max()),
            float(ev2.real.min()), float(ev2.real.max()),
            float(max(np.abs(ev1.imag).max(), np.abs(ev2.imag).max())))


# --------------------------------------------------------------------------
# elliptic functions by the arithmetic-geometric mean
# --------------------------------------------------------------------------

def _agm_sequence(kp):
    """AGM with a_0 = 1, b_0 = k', c_0 = k (k = sqrt((1-k')(1+k')))."""
    a = [1.0]
    b = [float(kp)]
    c = [math.sqrt((1.0 - kp) * (1.0 + kp))]
    while abs(c[-1]) > 2.0 ** -60 * a[-1] and len(a) < 64:
        a_n, b_n = a[-1], b[-1]
        a.append(0.5 * (a_n + b_n))
        b.append(math.sqrt(a_n * b_n))
        c.append(0.5 * (a_n - b_n))
    return a, b, c


def ellipk_from_kp(kp):
    """Complete elliptic integral K(k) = pi / (2 AGM(1, k'))."""
    a, _, _ = _agm_sequence(kp)
    return math.pi / (2.0 * a[-1])


def _dn_descending(u, kp):
    """Jacobi dn(u, k) by the descending AGM recursion on the amplitude.

    phi_N = 2^N a_N u, phi_{n-1} = (phi_n + asin(c_n sin(phi_n) / a_n)) / 2;
    then dn = cos(phi_0) / cos(phi_1 - phi_0).  Accurate for moderate k'.
    """
    a, _, c = _agm_sequence(kp)
    N = len(a) - 1
    if N == 0:
        return 1.0
    phi = (2.0 ** N) * a[N] * u
    phis = [phi]
    for nn in range(N, 0, -1):
        phi = 0.5 * (phi + math.asin(c[nn] * math.sin(phi) / a[nn]))
        phis.append(phi)
    phi0, phi1 = phis[-1], phis[-2]
    return math.cos(phi0) / math.cos(phi1 - phi0)


def _dn_theta(u, kp):
    """Jacobi dn(u, k) from theta functions of the complementary nome.

    Jacobi's imaginary transformation turns dn = sqrt(k') theta_3 / theta_4
    (nome q) into dn(u, k) = sqrt(k') theta_3(i y | q') / theta_2(i y | q') with
    q' = exp(-pi K / K'), y = pi u / (2 K').  For small k' the nome q' is tiny
    and both series are sums of positive terms (no cancellation):
        theta_3(i y) = 1 + 2 sum_{n>=1} q'^(n^2) cosh(2 n y),
        theta_2(i y) = 2 sum_{n>=0} q'^((n+1/2)^2) cosh((2n+1) y).
    """
    k = math.sqrt((1.0 - kp) * (1.0 + kp))
    K = ellipk_from_kp(kp)
    Kp = ellipk_from_kp(k)                      # K(k') has complementary modulus k
    lnq = -math.pi * K / Kp
    y = math.pi * u / (2.0 * Kp)

    def ch(e, x):                               # exp(e) cosh(x) without overflow
        return 0.5 * (math.exp(e + x) + math.exp(e - x))

    t3 = 1.0
    n = 1
    while True:
        term = 2.0 * ch(n * n * lnq, 2.0 * n * y)
        t3 += term
        if term < 1e-18 * t3 or n > 50:
            break
        n += 1
    t2 = 0.0
    n = 0
    while True:
        term = 2.0 * ch((n + 0.5) ** 2 * lnq, (2 * n + 1) * y)
        t2 += term
        if (n > 0 and term < 1e-18 * t2) or n > 50:
            break
        n += 1
    return math.sqrt(kp) * t3 / t2


def ellip_dn(u, kp):
    """Jacobi dn(u, k) for 0 <= u <= K(k), given k' (k = sqrt(1 - k'^2))."""
    if kp >= 0.5:
        return _dn_descending(u, kp)
    return _dn_theta(u, kp)


# --------------------------------------------------------------------------
# Zolotarev shifts
# --------------------------------------------------------------------------

def ellip_dn_frac(t, kp):
    """dn(t K(k), k) for 0 <= t <= 1, accurate to relative rounding.

    The descending recursion loses relative accuracy as u -> K, where both
    cosines vanish; for t > 1/2 the quarter-period reflection
    dn(K - x) = k' / dn(x) is used instead.
    """
    K = ellipk_from_kp(kp)
    if t <= 0.5:
        return ellip_dn(t * K, kp)
    return kp / ellip_dn((1.0 - t) * K, kp)


def zolotarev_params(a, b, c, d):
    """gamma, alpha and k' = 1/alpha from the four spectral endpoints."""
    gamma = abs(c - a) * abs(d - b) / (abs(c - b) * abs(d - a))
    alpha_z = -1.0 + 2.0 * gamma + 2.0 * math.sqrt(gamma * gamma - gamma)
    return gamma, alpha_z, 1.0 / alpha_z


def T_map(a, b, c, d, alpha_z):
    """Moebius map sending (-alpha, -1, 1, alpha) to (a, b, c, d).

    Built from the first three points by equating cross-ratios; the fourth
    point is implied by the definition of gamma.
    """
    def T(zv):
        rho = (zv + alpha_z) * (-2.0) / ((zv - 1.0) * (alpha_z - 1.0))
        s = rho * (b - a) / (b - c)
        return (a - s * c) / (1.0 - s)
    return T


def num_iterations(gamma, eps):
    """J(eps) = ceil(ln(16 gamma) ln(4 / eps) / pi^2)."""
    return max(1, int(math.ceil(math.log(16.0 * gamma) * math.log(4.0 / eps) / math.pi ** 2)))


def shifts(a, b, c, d, J):
    """Shift sequences (u_j, v_j), j = 0..J-1 (Section 3, with corrected roles)."""
    gamma, alpha_z, kp = zolotarev_params(a, b, c, d)
    T = T_map(a, b, c, d, alpha_z)
    u = np.empty(J)
    v = np.empty(J)
    for j in range(J):
        dn = ellip_dn_frac((2 * j + 1) / (2.0 * J), kp)
        u[j] = T(alpha_z * dn)
        v[j] = T(-alpha_z * dn)
    return u, v


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------

def adi(A, B, C, D, E, u, v):
    """Algorithm 1 (corrected): approximately solve A X B + C X D = E."""
    E = np.asarray(E)
    X = np.zeros(E.shape, dtype=np.result_type(E, A))
    Binv = np.linalg.inv(B)
    for uj, vj in zip(u, v):
        rhs = C @ X @ (uj * B + D) - E
        X_half = np.linalg.solve(uj * C - A, rhs) @ Binv
        rhs2 = (vj * C - A) @ X_half @ B + E
        X = np.linalg.solve(C, rhs2) @ np.linalg.inv(vj * B + D)
    return X


def adi_solve(A, B, C, D, E, eps):
    """Bounds by dense eig, J(eps), shifts, then Algorithm 1.  Returns (X, J)."""
    a, b, c, d, _ = spectral_bounds(A, B, C, D)
    gamma, _, _ = zolotarev_params(a, b, c, d)
    J = num_iterations(gamma, eps)
    u, v = shifts(a, b, c, d, J)
    return adi(A, B, C, D, E, u, v), J
