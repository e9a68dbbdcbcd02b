"""GPU parity of the differentiated heat run and the transposed transforms.

The library's gradients (transposed ADI on the flipped pencil, transposed tau
right side and recombination, transposed transforms) are compared with the
oracle's reverse-mode chain (dense transposed solves, Vandermonde transform
adjoints) element by element; at the 192^3 / 200-step configuration they are
checked by central finite differences of the library's own forward runs and by
the closed form of a Bessel x sine eigenmode.
"""

import numpy as np
import pytest
import scipy.special as ss
import torch

import paper_2206_04827_amd as cyl
import synth
from oracle import adjoint as ad
from oracle import transforms as tr
from tests.gpu_common import S, TOL, assert_close, banner, dev, host, need_gpu, smooth_values

pytestmark = pytest.mark.gpu


def _zero_single_imag(h, p):
    h = h.copy()
    h[0] = h[0].real
    if p % 2 == 0:
        h[p // 2] = h[p // 2].real
    return h


@pytest.mark.parametrize("m,n,p", [(12, 10, 8), (17, 13, 7), (33, 20, 1), (9, 65, 12)])
def test_transform_adjoints_match_oracle(m, n, p):
    need_gpu()
    banner("transform adjoints %dx%dx%d" % (m, n, p))
    g = np.random.default_rng(m * 1000 + n * 10 + p)
    plan = cyl.Plan(m, n, p)
    hb = g.standard_normal((p // 2 + 1, n, m)) + 1j * g.standard_normal((p // 2 + 1, n, m))
    got = host(plan.transform_fwd_adjoint(dev(hb)))
    ref = ad.forward_adjoint(ad.to_half_adjoint(_zero_single_imag(hb, p), p))
    assert_close(got, ref, 1e-12, "F^T")
    vb = g.standard_normal((p, n, m))
    got = host(plan.transform_inv_adjoint(dev(vb)))
    ref = ad.from_half_adjoint(ad.inverse_adjoint(vb))
    assert_close(got.real, ref.real, 1e-12, "F^-T re")
    assert np.max(np.abs(got.imag - ref.imag)) <= 1e-12 * np.max(np.abs(ref))


def _run(plan, T0, g, Tt, alpha, h, steps, every, space=cyl.CYL_SPACE_VALUE):
    H = cyl.Heat(plan, [dev(T0)], dev(g), alpha, h, 1, 1e-12, space=space)
    G = cyl.HeatGrad(H, steps, every)
    G.forward()
    TN = host(H.read(space))
    Tbar = 2.0 * (TN - Tt)
    T0b, gb, ab = G.backward(dev(Tbar), space)
    return H, G, TN, host(T0b), host(gb), float(host(ab))


@pytest.mark.parametrize("m,n,p,steps,every", [(20, 18, 8, 6, 4), (20, 18, 8, 6, 1), (20, 18, 8, 6, 6),
                                               (21, 17, 7, 5, 3), (14, 22, 6, 3, 10)])
def test_gradients_match_oracle(m, n, p, steps, every):
    need_gpu()
    banner("heat grad %dx%dx%d steps=%d every=%d" % (m, n, p, steps, every))
    alpha, h = 0.8, 1e-2
    T0 = smooth_values(m, n, p, S + 70)
    g = smooth_values(m, n, p, S + 71)
    Tt = smooth_values(m, n, p, S + 72)
    plan = cyl.Plan(m, n, p)
    H, G, TN, T0b, gb, ab = _run(plan, T0, g, Tt, alpha, h, steps, every)
    ref = ad.heat_bdf1_grad(T0, g, Tt, alpha, h, steps)
    assert_close(TN, ref["T_final"], TOL, "T_N")
    assert_close(T0b, ref["T0_bar"], TOL, "dL/dT0")
    assert_close(gb, ref["g_bar"], TOL, "dL/dg")
    print("  dL/dalpha %.15e ref %.15e" % (ab, ref["alpha_bar"]), flush=True)
    assert abs(ab - ref["alpha_bar"]) <= TOL * abs(ref["alpha_bar"])
    # a second backward pass (segments recomputed again) gives the same numbers
    T0b2, gb2, ab2 = G.backward(dev(2.0 * (TN - Tt)))
    assert np.array_equal(host(T0b2), T0b) and np.array_equal(host(gb2), gb) and float(host(ab2)) == ab
    G.close()
    H.close()


def test_gradients_with_fused_residual(monkeypatch):
    """Two passes on the split kernels, each first pass writing its own
    residual (forced here; chosen by itself only with several blocks per
    compute unit): the forward and transposed heat solves agree with the
    oracle."""
    need_gpu()
    monkeypatch.setenv("CYLSPEC_PASSES", "2")
    monkeypatch.setenv("CYLSPEC_ADI_FUSED_RES", "2")
    m, n, p, steps, every = 40, 36, 6, 4, 2
    banner("heat grad fused residual %dx%dx%d" % (m, n, p))
    alpha, h = 0.8, 1e-2
    T0 = smooth_values(m, n, p, S + 75)
    g = smooth_values(m, n, p, S + 76)
    Tt = smooth_values(m, n, p, S + 77)
    plan = cyl.Plan(m, n, p)
    H, G, TN, T0b, gb, ab = _run(plan, T0, g, Tt, alpha, h, steps, every)
    ref = ad.heat_bdf1_grad(T0, g, Tt, alpha, h, steps)
    assert_close(TN, ref["T_final"], TOL, "T_N")
    assert_close(T0b, ref["T0_bar"], TOL, "dL/dT0")
    assert_close(gb, ref["g_bar"], TOL, "dL/dg")
    assert abs(ab - ref["alpha_bar"]) <= TOL * abs(ref["alpha_bar"])
    G.close()
    H.close()


def test_gradients_on_global_state_kernel():
    """Blocks wider than the LDS-resident kernel takes (n above 258): the
    forward and the transposed (flipped-pencil) heat solves run the split
    sweeps with the block state in global memory; coefficient-space
    gradients against the oracle's dense adjoint."""
    need_gpu()
    m, n, p, steps, every = 290, 270, 2, 2, 1
    banner("heat grad global-state kernel %dx%dx%d" % (m, n, p))
    alpha, h = 0.9, 1e-3
    h0 = synth.smooth_coeffs(m, n, p, S + 83)
    hg = synth.smooth_coeffs(m, n, p, S + 84)
    ht = synth.smooth_coeffs(m, n, p, S + 85)
    plan = cyl.Plan(m, n, p)
    H, G, hN, T0b, gb, ab = _run(plan, h0, hg, ht, alpha, h, steps, every, cyl.CYL_SPACE_COEFF)
    ref = ad.heat_bdf1_grad_coeff(h0, hg, ht, alpha, h, steps, p)
    assert_close(hN.view(np.float64), ref["h_final"].view(np.float64), TOL, "h_N")
    assert_close(T0b.view(np.float64), _zero_single_imag(ref["T0_bar"], p).view(np.float64), TOL, "dL/dh0")
    assert_close(gb.view(np.float64), _zero_single_imag(ref["g_bar"], p).view(np.float64), TOL, "dL/dhg")
    print("  dL/dalpha %.15e ref %.15e" % (ab, ref["alpha_bar"]), flush=True)
    assert abs(ab - ref["alpha_bar"]) <= TOL * abs(ref["alpha_bar"])
    G.close()
    H.close()


def test_gradients_coefficient_space():
    need_gpu()
    m, n, p, steps, every = 16, 14, 6, 4, 3
    banner("heat grad coefficient space %dx%dx%d" % (m, n, p))
    alpha, h = 1.3, 1e-2
    h0 = synth.smooth_coeffs(m, n, p, S + 80)
    hg = synth.smooth_coeffs(m, n, p, S + 81)
    ht = synth.smooth_coeffs(m, n, p, S + 82)
    plan = cyl.Plan(m, n, p)
    H, G, hN, T0b, gb, ab = _run(plan, h0, hg, ht, alpha, h, steps, every, cyl.CYL_SPACE_COEFF)
    ref = ad.heat_bdf1_grad_coeff(h0, hg, ht, alpha, h, steps, p)
    assert_close(hN.view(np.float64), ref["h_final"].view(np.float64), TOL, "h_N")
    assert_close(T0b.view(np.float64), ref["T0_bar"].view(np.float64), TOL, "dL/dh0")
    assert_close(gb.view(np.float64), ref["g_bar"].view(np.float64), TOL, "dL/dhg")
    assert abs(ab - ref["alpha_bar"]) <= TOL * abs(ref["alpha_bar"])


def test_autograd_function():
    need_gpu()
    from paper_2206_04827_amd.autograd import heat_run
    m, n, p, steps = 18, 16, 6, 5
    banner("autograd heat_run %dx%dx%d" % (m, n, p))
    T0 = smooth_values(m, n, p, S + 90)
    g = smooth_values(m, n, p, S + 91)
    Tt = smooth_values(m, n, p, S + 92)
    plan = cyl.Plan(m, n, p)
    t0 = dev(T0).requires_grad_(True)
    tg = dev(g).requires_grad_(True)
    ta = torch.tensor(0.6, dtype=torch.float64, requires_grad=True)
    T = heat_run(t0, tg, ta, plan, 1e-2, steps, checkpoint_every=2)
    loss = ((T - dev(Tt)) ** 2).sum()
    loss.backward()
    ref = ad.heat_bdf1_grad(T0, g, Tt, 0.6, 1e-2, steps)
    assert abs(float(loss.detach()) - ref["L"]) <= TOL * ref["L"]
    assert_close(host(t0.grad), ref["T0_bar"], TOL, "autograd dL/dT0")
    assert_close(host(tg.grad), ref["g_bar"], TOL, "autograd dL/dg")
    assert abs(float(ta.grad) - ref["alpha_bar"]) <= TOL * abs(ref["alpha_bar"])


def test_grad_handle_rejects_unsupported():
    need_gpu()
    m, n, p = 10, 9, 4
    plan = cyl.Plan(m, n, p)
    T0 = smooth_values(m, n, p, S + 93)
    H4 = cyl.Heat(plan, [dev(T0)] * 4, dev(T0), 1.0, 1e-2, 4, 1e-12)
    with pytest.raises(cyl.CylError) as e:
        cyl.HeatGrad(H4, 3, 1)
    assert e.value.status == 2
    H1 = cyl.Heat(plan, [dev(T0)], dev(T0), 1.0, 1e-2, 1, 1e-12, bc_lift=dev(T0))
    with pytest.raises(cyl.CylError) as e:
        cyl.HeatGrad(H1, 3, 1)
    assert e.value.status == 2
    H0 = cyl.Heat(plan, [dev(T0)], dev(T0), 1.0, 1e-2, 1, 1e-12)
    G = cyl.HeatGrad(H0, 3, 2)
    with pytest.raises(cyl.CylError) as e:     # backward before forward
        G.backward(dev(T0))
    assert e.value.status == 1


# ----------------------------------------------------------------------------
# the 192^3, 200-step differentiation configuration
# ----------------------------------------------------------------------------

def _loss_gpu(plan, T0, g, Tt, alpha, h, steps):
    H = cyl.Heat(plan, [T0], g, alpha, h, 1, 1e-12)
    H.step(steps)
    d = H.read() - Tt
    val = float(torch.sum(d * d))
    H.close()
    return val


def test_d192_gradients_match_central_differences():
    need_gpu()
    m = n = p = 192
    steps, every, alpha, h = 200, 20, 1.0, 1e-3
    banner("D192 gradients vs central differences")
    T0 = synth.eigenmode_values(synth.eigenmode_params(S + 5), m, n, p)
    g = smooth_values(m, n, p, S + 6)
    Tt = smooth_values(m, n, p, S + 7)
    plan = cyl.Plan(m, n, p)
    dT0, dg, dTt = dev(T0), dev(g), dev(Tt)
    H = cyl.Heat(plan, [dT0], dg, alpha, h, 1, 1e-12)
    G = cyl.HeatGrad(H, steps, every)
    G.forward()
    T0b, gb, ab = G.backward(2.0 * (H.read() - dTt))
    ab = float(host(ab))
    G.close()
    H.close()
    d0 = dev(smooth_values(m, n, p, S + 8))
    d1 = dev(smooth_values(m, n, p, S + 9))
    e = 1e-6
    checks = [
        ("T0", float(torch.sum(T0b * d0)),
         lambda s: _loss_gpu(plan, dT0 + s * d0, dg, dTt, alpha, h, steps)),
        ("g", float(torch.sum(gb * d1)),
         lambda s: _loss_gpu(plan, dT0, dg + s * d1, dTt, alpha, h, steps)),
        ("alpha", ab, lambda s: _loss_gpu(plan, dT0, dg, dTt, alpha + s, h, steps)),
    ]
    L0 = _loss_gpu(plan, dT0, dg, dTt, alpha, h, steps)
    for name, an, f in checks:
        fd = (f(e) - f(-e)) / (2 * e)
        print("  d%s: adjoint %.12e  central difference %.12e  (L = %.6e)" % (name, an, fd, L0), flush=True)
        # rounding in L limits the difference quotient to about 1e-16 L / e
        assert abs(an - fd) <= 1e-6 * abs(an) + 1e-9 * L0, name


def test_d192_alpha_gradient_closed_form_on_eigenmode():
    """T0 = J_1(j r) sin(pi (z+1)/2) cos(theta), g = 0, target 0: with
    c = 1/(1 + h alpha lambda), dL/dalpha = -2 N h lambda c^(2N+1) |T0|^2."""
    need_gpu()
    m = n = p = 192
    steps, every, alpha, h = 200, 20, 1.0, 1e-3
    banner("D192 eigenmode closed form")
    r, z, th = tr.grid(m, n, p)
    TH, Z, R = np.meshgrid(th, z, r, indexing="ij")
    j = ss.jn_zeros(1, 2)[-1]
    lam = j * j + (np.pi / 2) ** 2
    phi = ss.jv(1, j * R) * np.sin(np.pi * (Z + 1) / 2) * np.cos(TH)
    plan = cyl.Plan(m, n, p)
    H = cyl.Heat(plan, [dev(phi)], dev(np.zeros_like(phi)), alpha, h, 1, 1e-12)
    G = cyl.HeatGrad(H, steps, every)
    G.forward()
    T0b, gb, ab = G.backward(2.0 * H.read())
    c = 1.0 / (1.0 + h * alpha * lam)
    nrm = float(np.sum(phi * phi))
    ref = -2 * steps * h * lam * c ** (2 * steps + 1) * nrm
    got = float(host(ab))
    print("  dL/dalpha %.15e closed form %.15e" % (got, ref), flush=True)
    assert abs(got - ref) <= 1e-9 * abs(ref)
    ref0 = 2 * c ** (2 * steps) * nrm
    got0 = float(torch.sum(T0b * dev(phi)))
    assert abs(got0 - ref0) <= 1e-9 * ref0


def test_handles_can_be_destroyed_in_any_order():
    """Destroying a parent handle first (as Python's cycle collector may do)
    leaves the child's destroy call safe."""
    need_gpu()
    m, n, p = 10, 9, 4
    banner("destroy order")
    T0 = smooth_values(m, n, p, S + 94)
    plan = cyl.Plan(m, n, p)
    H = cyl.Heat(plan, [dev(T0)], dev(T0), 1.0, 1e-2, 1, 1e-12)
    G = cyl.HeatGrad(H, 2, 1)
    G.forward()
    H.close()
    G.close()
    plan2 = cyl.Plan(m, n, p)
    H2 = cyl.Heat(plan2, [dev(T0)], dev(T0), 1.0, 1e-2, 1, 1e-12)
    plan2.close()
    H2.close()
    plan.close()
