"""GPU parity of BDF heat stepping (Section 3) against the oracle."""

import numpy as np
import pytest
import scipy.special as ss

import paper_2206_04827_amd as cyl
import synth
from oracle import problems as pb
from oracle import transforms as tr
from tests.gpu_common import (S, TOL, assert_close, assert_slots_close, banner, dev, half_slots, host,
                               need_gpu, smooth_values)

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


def test_h128_config_all_slots():
    """128^3, alpha = 1, dt = 1e-3, 100 BDF1 steps; T0 = 8 Bessel x sine
    eigenmodes (seed S+1), g = decaying random forcing (seed S+2); every
    Hermitian-half slot against the oracle (one wavenumber per worker)."""
    need_gpu()
    from tests import oracle_pool
    banner("heat H128 all slots")
    m = n = p = 128
    prm = synth.eigenmode_params(S + 1)
    T0 = synth.eigenmode_values(prm, m, n, p)
    g = smooth_values(m, n, p, S + 2)
    plan = cyl.Plan(m, n, p)
    H = cyl.Heat(plan, [dev(T0)], dev(g), 1.0, 1e-3, 1, 1e-12)
    H.step(100)
    got = host(H.read(cyl.CYL_SPACE_COEFF))
    ref = oracle_pool.heat_modes([tr.forward(T0)], tr.forward(g), 1.0, 1e-3, 100,
                                 [l for _, l in half_slots(p)])
    assert_slots_close(got, ref, p, TOL, "H128")


@pytest.mark.parametrize("m,n,p,order,alpha,steps", [(290, 270, 2, 1, 1.0, 3), (262, 262, 4, 4, 0.7, 3)])
def test_heat_on_global_state_kernel_full_field(m, n, p, order, alpha, steps):
    """Blocks wider than the LDS-resident kernel takes (n above 258): the
    split sweeps with the block state in global memory, on the heat pencil
    (two passes at these sizes), full field against the oracle."""
    need_gpu()
    banner("heat global-state kernel %dx%dx%d order %d" % (m, n, p, order))
    hist = [smooth_values(m, n, p, S + 140 + i) for i in range(order)]
    g = smooth_values(m, n, p, S + 149)
    plan = cyl.Plan(m, n, p)
    H = cyl.Heat(plan, [dev(x) for x in hist], dev(g), alpha, 1e-3, order, 1e-12)
    H.step(steps)
    got = host(H.read())
    ref = pb.heat(hist, g, alpha, 1e-3, steps, order=order)
    assert_close(got, ref, TOL, "heat %dx%dx%d BDF%d" % (m, n, p, order))


def test_b64_member_on_global_state_kernel_matches_oracle():
    """A member of the 64-problem configuration with n_r = n_z >= 259 (its
    sizes, diffusivity, initial eigenmodes and forcing), 3 BDF1 steps, every
    slot against the oracle."""
    need_gpu()
    from tests import oracle_pool
    specs = synth.batch_specs(S + 10)
    i = min((q for q in range(len(specs)) if specs[q][0] >= 259), key=lambda q: specs[q][2])
    m, n, p, alpha = specs[i]
    banner("B64 member %d: %dx%dx%d alpha %.3f" % (i, m, n, p, alpha))
    T0 = synth.eigenmode_values(synth.eigenmode_params(S + 10 + i), m, n, p)
    g = smooth_values(m, n, p, S + 100 + i)
    plan = cyl.Plan(m, n, p)
    H = cyl.Heat(plan, [dev(T0)], dev(g), alpha, 1e-3, 1, 1e-12)
    H.step(3)
    got = host(H.read(cyl.CYL_SPACE_COEFF))
    ref = oracle_pool.heat_modes([tr.forward(T0)], tr.forward(g), alpha, 1e-3, 3,
                                 [l for _, l in half_slots(p)])
    assert_slots_close(got, ref, p, TOL, "B64 member %dx%dx%d" % (m, n, p))
