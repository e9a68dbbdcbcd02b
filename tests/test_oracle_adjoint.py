"""Pins for the oracle's reverse-mode differentiation of a BDF1 heat run.

The gradient is fixed by things other than the adjoint code itself:
* the evaluation map built from Chebyshev/Fourier Vandermonde matrices equals
  the DCT/FFT inverse transform (two independent constructions);
* the defining identity <M x, y> = <x, M^T y> of every transposed link;
* central finite differences of the forward loss, which are exact up to
  rounding in T0 and g because the loss is quadratic in them;
* closed forms on a Bessel x sine eigenmode, where BDF1 reduces to the scalar
  recurrence x_k = (x_{k-1} + h eps) / (1 + h alpha lambda).
"""

import numpy as np
import pytest
import scipy.special as ss

from oracle import adjoint as ad
from oracle import operators as ops
from oracle import problems as pb
from oracle import transforms as tr


def _rdot(a, b):
    return float(np.sum(np.real(np.conj(a) * b)))


def _smooth(shape, seed, decay=3.0):
    """A random smooth field: random half coefficients with a decaying envelope."""
    p, n, m = shape
    g = np.random.default_rng(seed)
    nw = p // 2 + 1
    w = np.arange(nw)[:, None, None]
    k = np.arange(n)[None, :, None]
    j = np.arange(m)[None, None, :]
    h = (g.standard_normal((nw, n, m)) + 1j * g.standard_normal((nw, n, m))) * np.exp(-(j + k + w) / decay)
    h[0] = h[0].real
    if p % 2 == 0:
        h[p // 2] = h[p // 2].real
    return tr.inverse(tr.from_half(h, p))


@pytest.mark.parametrize("m,n,p", [(7, 6, 4), (9, 8, 5)])
def test_vandermonde_evaluation_equals_inverse_transform(m, n, p):
    g = np.random.default_rng(1)
    c = g.standard_normal((p, n, m)) + 1j * g.standard_normal((p, n, m))
    assert np.max(np.abs(ad.evaluate_grid(c) - tr.inverse(c, real=False))) < 1e-12


@pytest.mark.parametrize("m,n,p", [(7, 6, 4), (9, 8, 5), (6, 7, 1)])
def test_transform_adjoint_identities(m, n, p):
    g = np.random.default_rng(2)
    f = g.standard_normal((p, n, m))
    v = g.standard_normal((p, n, m))
    c = g.standard_normal((p, n, m)) + 1j * g.standard_normal((p, n, m))
    lhs = _rdot(tr.forward(f), c)
    rhs = _rdot(f, ad.forward_adjoint(c))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))
    lhs = _rdot(tr.inverse(c), v)
    rhs = _rdot(c, ad.inverse_adjoint(v))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("p", [4, 5, 1])
def test_half_layout_adjoint_identities(p):
    g = np.random.default_rng(3)
    nw = p // 2 + 1
    hh = g.standard_normal((nw, 3, 4)) + 1j * g.standard_normal((nw, 3, 4))
    cc = g.standard_normal((p, 3, 4)) + 1j * g.standard_normal((p, 3, 4))
    assert abs(_rdot(tr.from_half(hh, p), cc) - _rdot(hh, ad.from_half_adjoint(cc))) < 1e-12
    assert abs(_rdot(tr.to_half(cc), hh) - _rdot(cc, ad.to_half_adjoint(hh, p))) < 1e-12


def test_operator_adjoint_identities():
    m, n = 9, 8
    g = np.random.default_rng(4)
    F = g.standard_normal((m, n))
    Eb = g.standard_normal((m - 2, n - 2))
    assert abs(_rdot(ops.tau_rhs(m, n, F), Eb) - _rdot(F, ad.tau_rhs_adjoint(m, n, Eb))) < 1e-12
    X = g.standard_normal((m - 2, n - 2))
    U = g.standard_normal((m, n))
    assert abs(_rdot(ops.recombine(X), U) - _rdot(X, ad.recombine_adjoint(U))) < 1e-12


def test_forward_run_matches_heat_solver():
    m, n, p = 9, 8, 5
    T0 = _smooth((p, n, m), 5)
    g = _smooth((p, n, m), 6)
    ref = pb.heat([T0], g, 0.7, 1e-2, 3, order=1)
    cN, _ = ad.heat_bdf1_run(tr.forward(T0), tr.forward(g), 0.7, 1e-2, 3)
    assert np.max(np.abs(tr.inverse(cN) - ref)) < 1e-13 * np.max(np.abs(ref))


def _loss(T0, g, Tt, alpha, h, steps):
    T = pb.heat([T0], g, alpha, h, steps, order=1)
    return float(np.sum((T - Tt) ** 2))


@pytest.mark.parametrize("m,n,p", [(10, 9, 6), (9, 8, 5)])
def test_gradient_matches_central_differences(m, n, p):
    alpha, h, steps = 0.7, 2e-2, 4
    T0 = _smooth((p, n, m), 10)
    g = _smooth((p, n, m), 11)
    Tt = _smooth((p, n, m), 12)
    out = ad.heat_bdf1_grad(T0, g, Tt, alpha, h, steps)
    assert abs(out["L"] - _loss(T0, g, Tt, alpha, h, steps)) < 1e-12 * out["L"]
    d0 = _smooth((p, n, m), 13)
    dg = _smooth((p, n, m), 14)
    # quadratic in T0 and g: central differences are exact up to rounding
    e = 1e-3
    fd = (_loss(T0 + e * d0, g, Tt, alpha, h, steps) - _loss(T0 - e * d0, g, Tt, alpha, h, steps)) / (2 * e)
    an = float(np.sum(out["T0_bar"] * d0))
    assert abs(fd - an) < 1e-9 * max(abs(an), 1e-3 * out["L"])
    fd = (_loss(T0, g + e * dg, Tt, alpha, h, steps) - _loss(T0, g - e * dg, Tt, alpha, h, steps)) / (2 * e)
    an = float(np.sum(out["g_bar"] * dg))
    assert abs(fd - an) < 1e-9 * max(abs(an), 1e-3 * out["L"])
    ea = 1e-5
    fd = (_loss(T0, g, Tt, alpha + ea, h, steps) - _loss(T0, g, Tt, alpha - ea, h, steps)) / (2 * ea)
    assert abs(fd - out["alpha_bar"]) < 1e-7 * abs(out["alpha_bar"])


def test_coefficient_space_gradient_matches_central_differences():
    m, n, p = 9, 8, 6
    alpha, h, steps = 1.3, 1e-2, 3
    fwd = tr.to_half(tr.forward(_smooth((p, n, m), 20)))
    hg = tr.to_half(tr.forward(_smooth((p, n, m), 21)))
    ht = tr.to_half(tr.forward(_smooth((p, n, m), 22)))
    out = ad.heat_bdf1_grad_coeff(fwd, hg, ht, alpha, h, steps, p)

    def loss(a, b, al):
        return ad.heat_bdf1_grad_coeff(a, b, ht, al, h, steps, p)["L"]

    g = np.random.default_rng(23)
    d = g.standard_normal(fwd.shape) + 1j * g.standard_normal(fwd.shape)
    e = 1e-3
    fd = (loss(fwd + e * d, hg, alpha) - loss(fwd - e * d, hg, alpha)) / (2 * e)
    an = _rdot(out["T0_bar"], d)
    assert abs(fd - an) < 1e-9 * max(abs(an), 1e-3 * out["L"])
    fd = (loss(fwd, hg + e * d, alpha) - loss(fwd, hg - e * d, alpha)) / (2 * e)
    an = _rdot(out["g_bar"], d)
    assert abs(fd - an) < 1e-9 * max(abs(an), 1e-3 * out["L"])
    # imaginary parts of the w = 0 and Nyquist slots do not enter the field
    assert np.all(out["T0_bar"][0].imag == 0) and np.all(out["T0_bar"][p // 2].imag == 0)


def _eigfun(m, n, p, w, s, q):
    r, z, th = tr.grid(m, n, p)
    TH, Z, R = np.meshgrid(th, z, r, indexing="ij")
    j = ss.jn_zeros(w, s)[-1]
    lam = j * j + (q * np.pi / 2) ** 2
    return ss.jv(w, j * R) * np.sin(q * np.pi * (Z + 1) / 2) * np.cos(w * TH), lam


def test_gradient_closed_form_on_eigenmode():
    """T0 = phi, g = 0, T_target = 0: with c = 1/(1 + h alpha lambda),
    L = c^(2N) |phi|^2, dL/dalpha = -2 N h lambda c^(2N+1) |phi|^2,
    <dL/dT0, phi> = 2 c^(2N) |phi|^2 and <dL/dg, phi> = 2 c^N h c (1 - c^N)/(1 - c) |phi|^2."""
    m, n, p = 24, 16, 6
    phi, lam = _eigfun(m, n, p, 1, 1, 1)
    alpha, h, N = 1.0, 1e-3, 12
    out = ad.heat_bdf1_grad(phi, np.zeros_like(phi), np.zeros_like(phi), alpha, h, N)
    c = 1.0 / (1.0 + h * alpha * lam)
    nrm = float(np.sum(phi * phi))
    assert abs(out["L"] - c ** (2 * N) * nrm) < 1e-11 * nrm
    ref = -2 * N * h * lam * c ** (2 * N + 1) * nrm
    assert abs(out["alpha_bar"] - ref) < 1e-10 * abs(ref)
    ref = 2 * c ** (2 * N) * nrm
    assert abs(float(np.sum(out["T0_bar"] * phi)) - ref) < 1e-10 * ref
    ref = 2 * c ** N * h * c * (1 - c ** N) / (1 - c) * nrm
    assert abs(float(np.sum(out["g_bar"] * phi)) - ref) < 1e-10 * ref
