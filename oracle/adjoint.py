"""Reverse-mode differentiation of a BDF1 heat run (Section 3, heat equation).

Oracle module (test infrastructure only; see the package docstring).

The heat run of Section 3 with BDF1 and a time-independent forcing g is a
chain of linear maps (READING: the paper gives no adjoint; what follows is the
chain rule applied to the discrete method it defines):

    c_0 = F T_0,   G = F g                      (Section 2 transform F)
    E_k = [R2 (U_{k-1} + kappa G) C02^T]_tau     (tau right side, eq. (HelmholtzMatEqn))
    S_w(X_k) = E_k   per wavenumber w            (heat pencil, kappa = h)
    U_k = Q_m X_k Q_n^T                          (Dirichlet basis -> T coefficients)
    T_N = Re(G_inv U_N),  L = sum over grid (T_N - T_target)^2

with S_w(X) = Ct X Bt - kappa alpha (At X Bt + Ct X Dt).  The gradient
follows by transposing each link:

    Ubar_N = G_inv^H Tbar_N,  Tbar_N = 2 (T_N - T_target)
    Xbar_k = Q_m^T Ubar_k Q_n,  Ebar_k = S_w^{-T} Xbar_k (transposed solve)
    Ubar_{k-1} = R2_cut^T Ebar_k C02_cut,   Gbar += kappa R2_cut^T Ebar_k C02_cut
    alphabar += kappa Re <Ebar_k, At X_k Bt + Ct X_k Dt>
    T0bar = Re(F^H Ubar_0),  gbar = Re(F^H Gbar)

Every adjoint is taken with respect to the real inner product Re sum conj(a) b
of the arrays involved.  Complex coefficients are used for all p wavenumbers,
so nothing relies on Hermitian symmetry.

The transform adjoints are written from the definition of the interpolant of
Section 2: G_inv evaluates sum c T_j(r) T_k(z) e^{i w theta} at the grid, so
it is the tensor product of three Vandermonde matrices; F is its inverse.
"""

import numpy as np

from . import operators as ops
from . import sylvester
from . import transforms as tr


def vandermonde(m, n, p):
    """Factors of the evaluation map G_inv = E_theta (x) V_z (x) V_r (Section 2).

    E_theta[l_pt, l] = exp(i w_l theta_pt), V_z[k_pt, k] = T_k(z_pt),
    V_r[j_pt, j] = T_j(r_pt), at the points of Definition "grid".
    """
    r, z, th = tr.grid(m, n, p)
    Vr = np.polynomial.chebyshev.chebvander(r, m - 1)
    Vz = np.polynomial.chebyshev.chebvander(z, n - 1)
    Et = np.exp(1j * np.outer(th, tr.wavenumbers(p)))
    return Et, Vz, Vr


def evaluate_grid(c):
    """G_inv c: values of the interpolant at the grid (complex, no real part taken)."""
    p, n, m = c.shape
    Et, Vz, Vr = vandermonde(m, n, p)
    return np.einsum("Ll,Kk,Jj,lkj->LKJ", Et, Vz, Vr, c)


def inverse_adjoint(v):
    """Adjoint of c -> Re(G_inv c) (``transforms.inverse``): G_inv^H v, complex."""
    p, n, m = v.shape
    Et, Vz, Vr = vandermonde(m, n, p)
    return np.einsum("Ll,Kk,Jj,LKJ->lkj", np.conj(Et), Vz, Vr, np.asarray(v, dtype=float))


def forward_adjoint(cbar):
    """Adjoint of real values -> full coefficients (``transforms.forward``).

    F = G_inv^{-1}, so F^H = (G_inv^H)^{-1} = E^{-H} (x) V_z^{-T} (x) V_r^{-T};
    the result is Re(F^H cbar) because the values are real.
    """
    p, n, m = cbar.shape
    Et, Vz, Vr = vandermonde(m, n, p)
    x = np.linalg.solve(np.conj(Et).T, np.asarray(cbar, dtype=complex).reshape(p, -1)).reshape(p, n, m)
    x = np.linalg.solve(Vz.T, x.transpose(1, 0, 2).reshape(n, -1)).reshape(n, p, m).transpose(1, 0, 2)
    x = np.linalg.solve(Vr.T, x.transpose(2, 0, 1).reshape(m, -1)).reshape(m, p, n).transpose(1, 2, 0)
    return x.real.copy()


def from_half_adjoint(cbar):
    """Adjoint of ``transforms.from_half`` (half -> full coefficients of a real field).

    Slot w > 0 feeds c[w] = h_w and c[-w] = conj(h_w); the w = 0 and Nyquist
    slots feed only through their real part.
    """
    p = cbar.shape[0]
    wn = tr.wavenumbers(p)
    idx = {int(w): l for l, w in enumerate(wn)}
    h = np.zeros((p // 2 + 1,) + cbar.shape[1:], dtype=np.complex128)
    for w in range(p // 2 + 1):
        if w == 0:
            h[0] = cbar[idx[0]].real
        elif p % 2 == 0 and w == p // 2:
            h[w] = cbar[idx[-w]].real
        else:
            h[w] = cbar[idx[w]] + np.conj(cbar[idx[-w]])
    return h


def to_half_adjoint(hbar, p):
    """Adjoint of ``transforms.to_half`` (a selection of storage slots)."""
    c = np.zeros((p,) + hbar.shape[1:], dtype=np.complex128)
    for w in range(p // 2 + 1):
        if p % 2 == 0 and w == p // 2:
            c[0] += hbar[w]
        else:
            c[w + p // 2] += hbar[w]
    return c


def tau_rhs_adjoint(m, n, Ebar):
    """Adjoint of ``operators.tau_rhs``: R2_cut^T Ebar C02_cut, an m x n matrix."""
    R2m = ops._cut(ops.R2(m), m, m)[: m - 2]
    C02n = ops._cut(ops.C02(n), n, n)[: n - 2]
    return R2m.T @ Ebar @ C02n


def recombine_adjoint(Ubar):
    """Adjoint of ``operators.recombine``: Q_m^T Ubar Q_n."""
    m, n = Ubar.shape
    Qm = ops.dirichlet_basis(m)[:m]
    Qn = ops.dirichlet_basis(n)[:n]
    return Qm.T @ Ubar @ Qn


def _modes(c):
    """Per storage index l, the m x n matrix X[j, k] = c[l, k, j]."""
    return [np.asarray(c[l]).T for l in range(c.shape[0])]


def heat_bdf1_run(c0, cg, alpha, h, steps, keep_states=False):
    """BDF1 heat steps in full coefficients (Section 3); optionally keep every X_k."""
    p, n, m = c0.shape
    wn = tr.wavenumbers(p)
    kappa = h
    ka = kappa * alpha
    systems = [ops.heat_system(m, n, wn[l], ka) for l in range(p)]
    U = _modes(c0)
    G = _modes(cg)
    states = []
    for _ in range(steps):
        Xs = []
        for l in range(p):
            E = ops.tau_rhs(m, n, U[l] + kappa * G[l])
            Ah, Ch, Bt, Dt = systems[l]
            Xs.append(sylvester.solve(Ah, Bt, Ch, Dt, E))
        U = [ops.recombine(X) for X in Xs]
        if keep_states:
            states.append(Xs)
    cN = np.stack([u.T for u in U])
    return cN, states


def heat_bdf1_backward(cbar_N, states, cg_shape, alpha, h):
    """Reverse sweep: from the gradient of L w.r.t. the final full coefficients
    to the gradients w.r.t. c_0, G (full coefficients) and alpha."""
    p, n, m = cg_shape
    wn = tr.wavenumbers(p)
    kappa = h
    ka = kappa * alpha
    heat = [ops.heat_system(m, n, wn[l], ka) for l in range(p)]
    pois = [ops.tau_system(m, n, wn[l]) for l in range(p)]
    Ubar = _modes(cbar_N)
    Gbar = [np.zeros((m, n), dtype=np.complex128) for _ in range(p)]
    abar = 0.0
    for Xs in reversed(states):
        new = []
        for l in range(p):
            Xbar = recombine_adjoint(Ubar[l])
            Ah, Ch, Bt, Dt = heat[l]
            Ebar = sylvester.solve(Ah.T, Bt.T, Ch.T, Dt.T, Xbar)
            At, Ct, _, _ = pois[l]
            dS = At @ Xs[l] @ Bt + Ct @ Xs[l] @ Dt
            abar += kappa * float(np.real(np.sum(np.conj(Ebar) * dS)))
            back = tau_rhs_adjoint(m, n, Ebar)
            Gbar[l] = Gbar[l] + kappa * back
            new.append(back)
        Ubar = new
    cbar_0 = np.stack([u.T for u in Ubar])
    gbar_c = np.stack([u.T for u in Gbar])
    return cbar_0, gbar_c, abar


def heat_bdf1_grad(T0, g, T_target, alpha, h, steps):
    """L = sum (T_N - T_target)^2 of a BDF1 run from values T0 with forcing g.

    Returns dict with L, T_final and the gradients T0_bar, g_bar (value space,
    real) and alpha_bar.
    """
    c0 = tr.forward(T0)
    cg = tr.forward(g)
    cN, states = heat_bdf1_run(c0, cg, alpha, h, steps, keep_states=True)
    TN = tr.inverse(cN)
    diff = TN - T_target
    L = float(np.sum(diff * diff))
    cbar_N = inverse_adjoint(2.0 * diff)
    cbar_0, gbar_c, abar = heat_bdf1_backward(cbar_N, states, cg.shape, alpha, h)
    return {"L": L, "T_final": TN, "T0_bar": forward_adjoint(cbar_0),
            "g_bar": forward_adjoint(gbar_c), "alpha_bar": abar}


def heat_bdf1_grad_coeff(h0, hg, h_target, alpha, h, steps, p):
    """The same run with Hermitian-half coefficient inputs and outputs (n_theta = p).

    L = sum over the stored real and imaginary parts of (h_N - h_target)^2 with
    h_N = to_half(c_N).  Returns gradients w.r.t. h0 and hg (half layout, as
    complex arrays holding the real-part and imaginary-part derivatives) and alpha.
    """
    c0 = tr.from_half(h0, p)
    cg = tr.from_half(hg, p)
    cN, states = heat_bdf1_run(c0, cg, alpha, h, steps, keep_states=True)
    hN = tr.to_half(cN)
    diff = hN - h_target
    L = float(np.sum(diff.real ** 2 + diff.imag ** 2))
    cbar_N = to_half_adjoint(2.0 * diff, p)
    cbar_0, gbar_c, abar = heat_bdf1_backward(cbar_N, states, cg.shape, alpha, h)
    return {"L": L, "h_final": hN, "T0_bar": from_half_adjoint(cbar_0),
            "g_bar": from_half_adjoint(gbar_c), "alpha_bar": abar}

