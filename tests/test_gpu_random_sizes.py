"""Seeded random grid sizes against the oracle: Poisson (general and
physical-parity), BDF4 heat and the horizontal (disk) Poisson solve.

The sizes are drawn around the thresholds where the library changes kernels
(one thread per line below about 18 rows per parity block, split sweeps
above; tile edges of the transforms and of the right-side, recombination and
residual kernels), with odd and even counts and a single theta point."""

import numpy as np
import pytest

import paper_2206_04827_amd as cyl
import synth
from oracle import problems as pb
from tests.gpu_common import S, TOL, assert_close, banner, dev, host, need_gpu, smooth_values

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
    from tests.test_oracle_random_polynomials import N_COEFFS, _manufactured
    need_gpu()
    banner("random polynomial m=%d n=%d p=%d" % (m, n, p))
    coeffs = np.random.default_rng(S + 340 + seed).uniform(-1.0, 1.0, N_COEFFS)
    u, f = _manufactured(m, n, p, coeffs)
    got = host(cyl.Plan(m, n, p).poisson_solve(dev(f)))
    err = np.max(np.abs(got - u)) / max(1.0, np.max(np.abs(u)))
    print("  rel max %.3e" % err)
    assert err <= 1e-11
