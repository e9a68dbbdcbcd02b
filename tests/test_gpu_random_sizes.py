"""Seeded random grid sizes against the oracle: Poisson (general and
physical-parity), BDF4 heat and the horizontal (disk) Poisson solve.

The sizes are drawn around the thresholds where the library changes kernels
(one thread per line below about 18 rows per parity block, split sweeps
above; tile edges of the transforms and of the right-side, recombination and
residual kernels), with odd and even counts and a single theta point."""

import itertools

import numpy as np
import pytest

import paper_2206_04827_amd as cyl
import synth
from oracle import problems as pb
from oracle import transforms as tr
from tests.gpu_common import S, TOL, assert_close, banner, dev, host, need_gpu, smooth_values
from tests.test_oracle_random_polynomials import N_COEFFS, _manufactured, _poly_add, _poly_d2, _poly_eval

pytestmark = pytest.mark.gpu


def _sizes(count, seed):
    g = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = int(g.integers(5, 72))
        n = int(g.integers(5, 72))
        p = int(g.choice([1, 2, 3, 5, 8, 12, 16, 20]))
        out.append((m, n, p))
    return out


@pytest.mark.parametrize("m,n,p", _sizes(6, S + 300))
def test_random_size_poisson(m, n, p):
    need_gpu()
    banner("random poisson m=%d n=%d p=%d" % (m, n, p))
    f = smooth_values(m, n, p, S + 301 + m + n)
    u = host(cyl.Plan(m, n, p).poisson_solve(dev(f)))
    assert_close(u, pb.poisson(f), TOL, "poisson")


@pytest.mark.parametrize("m,n,p", [(m, n, 2 * max(1, p // 2)) for m, n, p in _sizes(3, S + 310)])
def test_random_size_physical(m, n, p):
    need_gpu()
    banner("random physical m=%d n=%d p=%d" % (m, n, p))
    f = synth.physical_values(m, n, p, S + 311 + m)
    plan = cyl.Plan(m, n, p)
    plan.set_physical(True)
    u = host(plan.poisson_solve(dev(f)))
    assert_close(u, pb.poisson(f), TOL, "physical")


@pytest.mark.parametrize("m,n,p", _sizes(3, S + 320))
def test_random_size_heat_bdf4(m, n, p):
    need_gpu()
    banner("random heat m=%d n=%d p=%d" % (m, n, p))
    hist = [smooth_values(m, n, p, S + 321 + i) for i in range(4)]
    g = smooth_values(m, n, p, S + 325)
    H = cyl.Heat(cyl.Plan(m, n, p), [dev(x) for x in hist], dev(g), 0.7, 2e-3, 4, 1e-12)
    H.step(4)
    got = host(H.read())
    assert_close(got, pb.heat(hist, g, 0.7, 2e-3, 4, order=4), TOL, "heat bdf4")


@pytest.mark.parametrize("m,n,p", _sizes(3, S + 330))
def test_random_size_disk(m, n, p):
    need_gpu()
    banner("random disk m=%d n=%d p=%d" % (m, n, p))
    f = smooth_values(m, n, p, S + 331 + m)
    got = host(cyl.Plan(m, n, p).disk_poisson_solve(dev(f)))
    assert_close(got, pb.disk_poisson(f), TOL, "disk")


@pytest.mark.parametrize("m,n,p,seed", [(10, 8, 12, 1), (17, 13, 11, 2), (33, 21, 16, 3), (64, 40, 12, 4)])
def test_random_polynomial_solution_exact(m, n, p, seed):
    """Random cubic q(x, y, z), u = (1 - x^2 - y^2)(1 - z^2) q, Laplacian by
    exact monomial differentiation: the GPU solve returns u to rounding,
    independently of the oracle."""
    need_gpu()
    banner("random polynomial m=%d n=%d p=%d" % (m, n, p))
    coeffs = np.random.default_rng(S + 340 + seed).uniform(-1.0, 1.0, N_COEFFS)
    u, f = _manufactured(m, n, p, coeffs)
    got = host(cyl.Plan(m, n, p).poisson_solve(dev(f)))
    err = np.max(np.abs(got - u)) / max(1.0, np.max(np.abs(u)))
    print("  rel max %.3e" % err)
    assert err <= 1e-11


@pytest.mark.parametrize("m,n,p,seed", [(14, 12, 12, 5), (40, 33, 16, 6)])
def test_random_polynomial_physical_and_traces(m, n, p, seed):
    """The same random polynomials are single-valued smooth fields: the
    physical-parity fast path returns them exactly; and q itself (nonzero on
    the boundary) is recovered from its Laplacian and its boundary traces."""
    need_gpu()
    banner("random polynomial physical/traces m=%d n=%d p=%d" % (m, n, p))
    coeffs = np.random.default_rng(S + 350 + seed).uniform(-1.0, 1.0, N_COEFFS)
    u, f = _manufactured(m, n, p, coeffs)
    plan = cyl.Plan(m, n, p)
    plan.set_physical(True)
    got = host(plan.poisson_solve(dev(f)))
    assert np.max(np.abs(got - u)) <= 1e-11 * max(1.0, np.max(np.abs(u)))
    plan.set_physical(False)
    # v = u + b with b a random cubic that does not vanish on the boundary:
    # lap v = f + lap b, and v's values on the faces are the Dirichlet data
    b_coeffs = np.random.default_rng(S + 360 + seed).uniform(-1.0, 1.0, N_COEFFS)
    exps = [e for e in itertools.product(range(4), repeat=3) if sum(e) <= 3]
    bq = {e: c for e, c in zip(exps, b_coeffs)}
    lap_b = _poly_add(_poly_d2(bq, 0), _poly_d2(bq, 1), _poly_d2(bq, 2))
    r, z, th = tr.grid(m, n, p)
    TH, Z, R = np.meshgrid(th, z, r, indexing="ij")
    X, Y = R * np.cos(TH), R * np.sin(TH)
    v = u + _poly_eval(bq, X, Y, Z)
    fv = f + _poly_eval(lap_b, X, Y, Z)
    rface = np.ascontiguousarray(np.stack([v[:, :, 0], v[:, :, -1]]))
    zface = np.ascontiguousarray(np.stack([v[:, 0, :], v[:, -1, :]]))
    got = host(plan.poisson_solve(dev(fv), bc_traces=(dev(rface), dev(zface))))
    assert np.max(np.abs(got - v)) <= 1e-11 * max(1.0, np.max(np.abs(v)))
