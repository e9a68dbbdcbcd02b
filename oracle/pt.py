"""Poloidal-toroidal (PT) decomposition through horizontal Poisson solves
(Section 4, eqs. (pt) and (ptpoisson)).

Oracle module (test infrastructure only; see the package docstring).

A field V = curl(lambda z) + curl curl(gamma z) has z-component -Delta_h gamma
and the z-component of its curl is -Delta_h lambda (eq. (ptpoisson)).  Given
the cylindrical components (V_r, V_theta, V_z) on the doubled grid, gamma and
lambda are recovered by two disk solves:

    Delta_h gamma  = -V_z,
    Delta_h lambda = -(z . curl V) = -(1/r) (d_r (r V_theta) - d_theta V_r).

The curl term is formed in coefficient space after weighting by r^2, so that
no division by r occurs:

    r^2 Delta_h lambda = -(r V_theta + r^2 d_r V_theta - i w r V_r),

which in the C^(2) rows of the tau system (Section 3 operators) reads

    [A_w Q]_tau x = [ -R (C02 + R C12 D1) F_theta + i w R C02 F_r ]_tau,
    lambda = Q x.

READINGS (the paper gives the two relations only):
* boundary data: lambda = gamma = 0 on the side wall r = 1, the condition of
  the horizontal solve (no condition in z, where Delta_h has no derivative);
  a field whose potentials vanish there is recovered exactly;
* the components on the doubled grid are taken with the signed radius: at
  (r, theta) with r < 0, V_r = V . (cos theta, sin theta) and
  V_theta = V . (-sin theta, cos theta) at the point r (cos theta, sin theta);
  the polar formulas then hold unchanged for r < 0;
* for even p the theta derivative of the Nyquist mode (w = -p/2) of a real
  field is taken as zero (its sine vanishes at every grid angle);
* the input need not be solenoidal: gamma and lambda are defined by the two
  solves for any field.
"""

import numpy as np

from . import operators as ops
from . import problems as pb
from . import transforms as tr


def curl_z_rhs(m, w, Fr, Ft):
    """r^2-weighted right side of Delta_h lambda = -(z . curl V), C^(2) rows.

    Fr, Ft: m x n full T coefficients (rows r-degrees) of V_r and V_theta for
    wavenumber w.  Returns the first m-2 rows of
    -R (C02 + R C12 D1) Ft + i w R C02 Fr  (Section 3 operators; r V_theta +
    r^2 d_r V_theta - i w r V_r weighted as r^2 (z . curl V)).
    """
    Rm = ops.R(m)
    C02 = ops.C02(m)
    Ma = ops._cut(Rm @ (C02 + Rm @ ops.C12(m) @ ops.D1(m)), m, m)
    Mb = ops._cut(Rm @ C02, m, m)
    return (-(Ma @ Ft) + 1j * float(w) * (Mb @ Fr))[: m - 2]


def pt_mode(m, n, w, Fr, Ft, Fz, nyquist=False):
    """(Lambda, Gamma) full T coefficients (m x n) for one wavenumber.

    Gamma: the disk solve of -V_z; Lambda: the tau system with the curl right
    side (w taken as 0 in the curl term for the Nyquist mode).
    """
    Gamma = pb.disk_poisson_mode(m, n, w, -Fz)
    At, _, _, _ = ops.tau_system(m, max(n, 3), w)
    E = curl_z_rhs(m, 0.0 if nyquist else w, Fr, Ft)
    Xt = np.linalg.solve(At, E)
    Lam = ops.dirichlet_basis(m)[:m] @ Xt
    return Lam, Gamma


def pt_decompose_coeffs(c_r, c_t, c_z):
    """Full-coefficient PT decomposition c[l, k, j] -> (c_lambda, c_gamma)."""
    p, n, m = c_z.shape
    wn = tr.wavenumbers(p)
    lam = np.zeros(c_z.shape, dtype=np.complex128)
    gam = np.zeros(c_z.shape, dtype=np.complex128)
    for l in range(p):
        nyq = p % 2 == 0 and wn[l] == -(p // 2)
        L, G = pt_mode(m, n, wn[l], pb._mode_matrix(c_r, l), pb._mode_matrix(c_t, l),
                       pb._mode_matrix(c_z, l), nyquist=nyq)
        lam[l] = L.T
        gam[l] = G.T
    return lam, gam


def pt_decompose(v_r, v_theta, v_z):
    """Value-space PT decomposition of (V_r, V_theta, V_z) -> (lambda, gamma)."""
    lam, gam = pt_decompose_coeffs(tr.forward(v_r), tr.forward(v_theta), tr.forward(v_z))
    return np.real(tr.inverse(lam)), np.real(tr.inverse(gam))
