"""GPU parity of BDF heat stepping (Section 3) against the oracle."""

import numpy as np
import pytest
import scipy.special as ss

import paper_2206_04827_amd as cyl
import synth
from oracle import problems as pb
from oracle import transforms as tr
from tests.gpu_common import S, TOL, assert_close, banner, dev, host, need_gpu, smooth_values

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("order", [1, 4])
def test_small_heat_full_field(order):
    need_gpu()
    m, n, p = 22, 18, 8
    banner("heat small order=%d" % order)
    hist = [smooth_values(m, n, p, S + 50 + i) for i in range(order)]
    g = smooth_values(m, n, p, S + 60)
    alpha, h, steps = 0.8, 2e-3, 12
    plan = cyl.Plan(m, n, p)
    H = cyl.Heat(plan, [dev(x) for x in hist], dev(g), alpha, h, order, 1e-12)
    assert np.max(np.abs(host(H.read()) - hist[0])) < 1e-13 * np.max(np.abs(hist[0]))
    H.step(steps)
    got = host(H.read())
    ref = pb.heat(hist, g, alpha, h, steps, order=order)
    assert_close(got, ref, TOL, "heat order %d" % order)
    # coefficient-space read agrees with the value-space read
    gc = host(H.read(cyl.CYL_SPACE_COEFF))
    assert np.max(np.abs(tr.inverse(tr.from_half(gc, p)) - got)) < 1e-12 * np.max(np.abs(got))


def test_heat_steady_state_with_lift():
    need_gpu()
    m, n, p = 10, 9, 6
    r, z, th = tr.grid(m, n, p)
    TH, Z, R = np.meshgrid(th, z, r, indexing="ij")
    X, Y = R * np.cos(TH), R * np.sin(TH)
    psi = 2.0 + X * Z + Y * Y * Z + Z ** 2
    alpha = 0.7
    g = -alpha * (2 * Z + 2.0)
    lift = psi + (1 - R ** 2) * (1 - Z ** 2) * X
    plan = cyl.Plan(m, n, p)
    H = cyl.Heat(plan, [dev(psi)], dev(g), alpha, 1e-2, 1, 1e-12, bc_lift=dev(lift))
    H.step(5)
    assert np.max(np.abs(host(H.read()) - psi)) < 1e-12


def test_bessel_sine_eigenmode_decay():
    """g = 0, T0 an eigenfunction: BDF1 gives (1 + h alpha lambda)^-N T0."""
    need_gpu()
    m, n, p = 32, 24, 8
    r, z, th = tr.grid(m, n, p)
    TH, Z, R = np.meshgrid(th, z, r, indexing="ij")
    jz = ss.jn_zeros(2, 1)[-1]
    lam = jz * jz + (np.pi / 2) ** 2
    phi = ss.jv(2, jz * R) * np.sin(np.pi * (Z + 1) / 2) * np.cos(2 * TH)
    alpha, h, N = 1.0, 1e-3, 40
    plan = cyl.Plan(m, n, p)
    H = cyl.Heat(plan, [dev(phi)], dev(np.zeros_like(phi)), alpha, h, 1, 1e-12)
    H.step(N)
    got = host(H.read())
    assert np.max(np.abs(got - (1 + h * alpha * lam) ** (-N) * phi)) < 1e-11


def test_h128_config_sampled_modes():
    """128^3, alpha = 1, dt = 1e-3, 100 BDF1 steps; T0 = 8 Bessel x sine
    eigenmodes (seed S+1), g = decaying random forcing (seed S+2)."""
    need_gpu()
    banner("heat H128 sampled")
    m = n = p = 128
    prm = synth.eigenmode_params(S + 1)
    T0 = synth.eigenmode_values(prm, m, n, p)
    g = smooth_values(m, n, p, S + 2)
    plan = cyl.Plan(m, n, p)
    H = cyl.Heat(plan, [dev(T0)], dev(g), 1.0, 1e-3, 1, 1e-12)
    H.step(100)
    got = host(H.read(cyl.CYL_SPACE_COEFF))
    wn = list(tr.wavenumbers(p))
    ws = sorted(set([0, 1, 2, int(prm["w"][0]), -64]))      # -64: the Nyquist mode (slot 64)
    ls = [wn.index(w) for w in ws]
    slots = [w if w >= 0 else p // 2 for w in ws]
    cT = tr.forward(T0)
    cg = tr.forward(g)
    ref = pb.heat_coeffs([cT], cg, 1.0, 1e-3, 100, order=1, modes=ls)[0]
    refh = tr.to_half(ref)
    num = sum(np.linalg.norm(got[s] - refh[s]) ** 2 for s in slots) ** 0.5
    den = sum(np.linalg.norm(refh[s]) ** 2 for s in slots) ** 0.5
    mx = max(np.max(np.abs(got[s] - refh[s])) for s in slots) / max(np.max(np.abs(refh[s])) for s in slots)
    print("  H128 sampled w=%s rel l2 %.3e rel max %.3e" % (ws, num / den, mx), flush=True)
    assert num / den <= TOL and mx <= TOL
