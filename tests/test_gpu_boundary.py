"""GPU parity of the physical-parity fast path and of the boundary-trace lift
against the oracle (doubled-grid parity j = w mod 2; transfinite lift).

The fast path solves only the j = w (mod 2) parity blocks: for physical
forcing it must agree with the oracle's full solve, and for any forcing with
the oracle's solve of the parity-projected forcing.  The lift kernel is
compared elementwise with the oracle's, and solves with boundary traces with
the oracle's lifted solves.
"""

import numpy as np
import pytest
import torch

import paper_2206_04827_amd as cyl
import synth
from oracle import boundary as bd
from oracle import problems as pb
from oracle import transforms as tr
from tests.gpu_common import S, TOL, assert_close, banner, dev, host, need_gpu, smooth_values

pytestmark = pytest.mark.gpu


def _faces(u):
    rf, zf = bd.faces(u)
    return np.ascontiguousarray(rf), np.ascontiguousarray(zf)


@pytest.mark.parametrize("m,n,p", [(12, 10, 6), (33, 17, 7), (64, 40, 1)])
def test_trace_lift_matches_oracle(m, n, p):
    need_gpu()
    banner("trace lift m=%d n=%d p=%d" % (m, n, p))
    rf, zf = _faces(synth.physical_values(m, n, p, S + 60 + m))
    got = host(cyl.Plan(m, n, p).trace_lift(dev(rf), dev(zf)))
    ref = bd.trace_lift(rf, zf, m, n, p)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_solution_recovered_from_its_traces():
    need_gpu()
    m, n, p = 12, 10, 6
    r, z, th = tr.grid(m, n, p)
    TH, Z, R = np.meshgrid(th, z, r, indexing="ij")
    X, Y = R * np.cos(TH), R * np.sin(TH)
    u = 1.0 + X + 2 * Y * Z + X * X - Y * Y + 3 * Z ** 3 + X * Y * Z
    rf, zf = _faces(u)
    got = host(cyl.Plan(m, n, p).poisson_solve(dev(18.0 * Z), bc_traces=(dev(rf), dev(zf))))
    assert np.max(np.abs(got - u)) < 1e-12


@pytest.mark.parametrize("m,n,p", [(24, 20, 8), (40, 33, 6)])
def test_trace_solve_matches_oracle(m, n, p):
    need_gpu()
    banner("trace solve m=%d n=%d p=%d" % (m, n, p))
    f = smooth_values(m, n, p, S + 70 + m)
    rf, zf = _faces(synth.physical_values(m, n, p, S + 71 + m))
    got = host(cyl.Plan(m, n, p).poisson_solve(dev(f), bc_traces=(dev(rf), dev(zf))))
    ref = pb.poisson(f, lift=bd.trace_lift(rf, zf, m, n, p))
    assert_close(got, ref, TOL, "traces")
    assert np.max(np.abs(got[:, :, 0] - rf[0])) < 1e-12 and np.max(np.abs(got[:, -1, :] - zf[1])) < 1e-12


# sizes covering the three ADI kernels: one thread per line, split in LDS,
# split with the block state in global memory
@pytest.mark.parametrize("m,n,p", [(18, 16, 6), (40, 36, 10), (130, 120, 4), (290, 270, 2)])
def test_physical_fast_path_matches_full_oracle_solve(m, n, p):
    need_gpu()
    banner("physical fast path m=%d n=%d p=%d" % (m, n, p))
    f = synth.physical_values(m, n, p, S + 80 + m)
    plan = cyl.Plan(m, n, p)
    plan.set_physical(True)
    u, info = plan.poisson_solve(dev(f), info=True)
    u = host(u)
    print("  info", info)
    assert info["resid_ratio"] < 1e-9
    assert_close(u, pb.poisson(f), TOL, "physical")
    c = tr.forward(u)
    mask = bd.physical_mask(m, p)
    assert np.max(np.abs(np.where(mask, 0.0, c))) < 1e-13 * np.max(np.abs(c))


def test_physical_fast_path_projects_non_physical_forcing():
    """For arbitrary forcing the fast path returns the solution of the
    parity-projected forcing."""
    need_gpu()
    m, n, p = 26, 22, 8
    f = smooth_values(m, n, p, S + 90)
    plan = cyl.Plan(m, n, p)
    plan.set_physical(True)
    got = host(plan.poisson_solve(dev(f)))
    cf = bd.project_physical(tr.forward(f))
    ref = np.real(tr.inverse(pb.poisson_coeffs(cf)))
    assert_close(got, ref, TOL, "projected")
    plan.set_physical(False)
    full = host(plan.poisson_solve(dev(f)))
    assert np.max(np.abs(full - got)) > 1e-3 * np.max(np.abs(full))


def test_physical_fast_path_at_256():
    """The benchmark size: physical and general solves of physical forcing
    agree to the solver's accuracy."""
    need_gpu()
    m = n = p = 256
    banner("physical fast path 256^3")
    f = dev(synth.physical_values(m, n, p, S + 95))
    plan = cyl.Plan(m, n, p)
    a = plan.poisson_solve(f)
    plan.set_physical(True)
    b, info = plan.poisson_solve(f, info=True)
    print("  info", info)
    rel = float((a - b).abs().max() / a.abs().max())
    print("  physical vs general rel max %.3e" % rel)
    assert rel < TOL
    del a, b, f
    torch.cuda.empty_cache()


def test_physical_needs_even_theta_count():
    need_gpu()
    plan = cyl.Plan(10, 8, 5)
    with pytest.raises(cyl.CylError) as e:
        plan.set_physical(True)
    assert e.value.status == 2


# ----------------------------------------------------------------------------
# heat stepping on the physical-parity blocks
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,p,order", [(24, 20, 8, 1), (21, 17, 6, 4), (130, 120, 4, 1)])
def test_physical_heat_matches_oracle(m, n, p, order):
    """Physical initial state and forcing: the fast path's BDF steps agree
    with the oracle's full heat solve (one thread per line and split kernels)."""
    need_gpu()
    banner("physical heat m=%d n=%d p=%d bdf%d" % (m, n, p, order))
    hist = [synth.physical_values(m, n, p, S + 150 + i) for i in range(order)]
    g = synth.physical_values(m, n, p, S + 159)
    plan = cyl.Plan(m, n, p)
    plan.set_physical(True)
    H = cyl.Heat(plan, [dev(x) for x in hist], dev(g), 0.8, 1e-3, order, 1e-12)
    H.step(5)
    got = host(H.read())
    ref = pb.heat(hist, g, 0.8, 1e-3, 5, order=order)
    assert_close(got, ref, TOL, "physical heat")
    c = tr.forward(got)
    mask = bd.physical_mask(m, p)
    assert np.max(np.abs(np.where(mask, 0.0, c))) < 1e-13 * np.max(np.abs(c))


def test_physical_heat_handles_are_rejected_by_batch_and_grad():
    need_gpu()
    m, n, p = 16, 14, 6
    plan = cyl.Plan(m, n, p)
    plan.set_physical(True)
    T0 = dev(synth.physical_values(m, n, p, S + 160))
    H = cyl.Heat(plan, [T0], torch.zeros_like(T0), 1.0, 1e-3, 1, 1e-12)
    with pytest.raises(cyl.CylError) as e:
        cyl.HeatGrad(H, 4, 2)
    assert e.value.status == 2
    with pytest.raises(cyl.CylError) as e:
        cyl.Batch([H])
    assert e.value.status == 2


@pytest.mark.parametrize("m,n,p", [(10, 9, 6), (40, 36, 8)])
def test_physical_heat_with_lift(m, n, p):
    """Physical-parity stepping with Dirichlet data through a (physical)
    lift: the steady state of a polynomial solution is kept exactly, and a
    run from a physical initial state matches the oracle's lifted heat run."""
    need_gpu()
    banner("physical heat with lift m=%d n=%d p=%d" % (m, n, p))
    r, z, th = tr.grid(m, n, p)
    TH, Z, R = np.meshgrid(th, z, r, indexing="ij")
    X, Y = R * np.cos(TH), R * np.sin(TH)
    psi = 2.0 + X * Z + Y * Y * Z + Z ** 2
    alpha = 0.7
    g = -alpha * (2 * Z + 2.0)
    lift = psi + (1 - R ** 2) * (1 - Z ** 2) * X
    plan = cyl.Plan(m, n, p)
    plan.set_physical(True)
    H = cyl.Heat(plan, [dev(psi)], dev(g), alpha, 1e-2, 1, 1e-12, bc_lift=dev(lift))
    H.step(5)
    assert np.max(np.abs(host(H.read()) - psi)) < 1e-12
    T0 = synth.physical_values(m, n, p, S + 170) * (1 - R ** 2) * (1 - Z ** 2) + lift
    g2 = synth.physical_values(m, n, p, S + 171)
    H2 = cyl.Heat(plan, [dev(T0)], dev(g2), 0.9, 2e-3, 1, 1e-12, bc_lift=dev(lift))
    H2.step(4)
    assert_close(host(H2.read()), pb.heat([T0], g2, 0.9, 2e-3, 4, order=1, lift=lift), TOL, "physical lifted heat")
