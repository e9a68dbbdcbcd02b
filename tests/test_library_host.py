"""CPU-side checks of libcylspec: exports, synchronous argument errors, and the
host planner's ADI parameters against the oracle (no GPU needed)."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2206_04827_amd as cyl
from oracle import adi
from oracle import operators as ops

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(cyl.LIB_PATH):
        pytest.skip("libcylspec.so not built")
    return cyl.load()


def _declared():
    with open(os.path.join(ROOT, "include", "cylspec.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(cyl_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(cyl.EXPORTS) == names


def test_status_strings(lib):
    for code in range(7):
        assert lib.cyl_status_string(code)
    assert b"unknown" in lib.cyl_status_string(99)


@pytest.mark.parametrize("dims,code", [((3, 8, 8), 1), ((8, 2, 8), 1), ((8, 8, 0), 1),
                                       ((2000, 8, 8), 2), ((8, 8, 5000), 2), ((8, 8, 3001), 2)])
def test_plan_create_rejects_sizes(lib, dims, code):
    h = ctypes.c_void_p()
    assert lib.cyl_plan_create(ctypes.byref(h), *dims, None) == code
    assert not h.value
    assert lib.cyl_last_error()


def test_plan_create_without_a_device_fails_cleanly(lib):
    """On a machine without a HIP device, creating a valid plan fails with a
    HIP or memory status and returns no handle (the partly built plan is
    freed: the sanitizer build of this test checks that path)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    h = ctypes.c_void_p()
    st = lib.cyl_plan_create(ctypes.byref(h), 16, 14, 8, None)
    assert st in (3, 4), st
    assert not h.value
    assert lib.cyl_last_error()


def test_null_arguments_are_rejected(lib):
    assert lib.cyl_plan_create(None, 8, 8, 8, None) == 1
    assert lib.cyl_plan_destroy(None) == 1
    assert lib.cyl_transform_fwd(None, None, None) == 1
    assert lib.cyl_transform_inv(None, None, None) == 1
    assert lib.cyl_poisson_solve(None, 0, None, None, None, 1e-12, None) == 1
    assert lib.cyl_poisson_solve_noalloc(None, 0, None, None, None, 1e-12, None) == 1
    assert lib.cyl_plan_prepare(None, 1e-12) == 1
    h = ctypes.c_void_p()
    assert lib.cyl_heat_create(ctypes.byref(h), None, 1.0, 1e-3, 1, 1e-12, 0, None, None, None) == 1
    assert lib.cyl_heat_step(None, 1) == 1
    assert lib.cyl_heat_read(None, 0, None) == 1
    assert lib.cyl_heat_destroy(None) == 1
    assert lib.cyl_plan_set_profiling(None, 1) == 1
    assert lib.cyl_plan_get_profile(None, None) == 1
    assert lib.cyl_transform_fwd_adjoint(None, None, None) == 1
    assert lib.cyl_transform_inv_adjoint(None, None, None) == 1
    g = ctypes.c_void_p()
    assert lib.cyl_heat_grad_create(ctypes.byref(g), None, 10, 2) == 1
    assert not g.value
    assert lib.cyl_heat_grad_create(None, None, 10, 2) == 1
    assert lib.cyl_heat_grad_forward(None) == 1
    assert lib.cyl_heat_grad_backward(None, 0, None, None, None, None) == 1
    assert lib.cyl_heat_grad_destroy(None) == 1
    b = ctypes.c_void_p()
    assert lib.cyl_batch_create(ctypes.byref(b), 0, None, 0) == 1
    assert not b.value
    assert lib.cyl_batch_create(None, 1, None, 0) == 1
    assert lib.cyl_batch_step(None, 1) == 1
    assert lib.cyl_batch_describe(None, None, None, None) == 1
    assert lib.cyl_batch_destroy(None) == 1
    assert lib.cyl_plan_set_physical(None, 1) == 1
    assert lib.cyl_trace_lift(None, None, None, None) == 1
    assert lib.cyl_disk_poisson_solve(None, 0, None, None) == 1
    assert lib.cyl_pt_decompose(None, 0, None, None, None, None, None) == 1
    d = ctypes.c_double()
    assert lib.cyl_device_peaks(None, None, None, 16, 0, None, None) == 1        # reps < 1
    assert lib.cyl_device_peaks(None, None, None, 16, 1001, None, None) == 1     # reps > 1000
    assert lib.cyl_device_peaks(None, None, None, 16, 3, None, ctypes.byref(d)) == 1   # copy without buffers
    buf = (ctypes.c_double * 64)()
    base = ctypes.addressof(buf) // 16 * 16 + 16
    assert lib.cyl_device_peaks(None, base, base + 8, 4, 3, None, ctypes.byref(d)) == 1  # misaligned dst
    assert lib.cyl_device_peaks(None, base, base + 16, 4, 3, None, ctypes.byref(d)) == 1  # overlap


def test_adi_parameter_validation():
    with pytest.raises(cyl.CylError) as e:
        cyl.adi_parameters(16, 16, 0, 0.0, 1.0)
    assert e.value.status == 1
    with pytest.raises(cyl.CylError):
        cyl.adi_parameters(3, 16, 0, 0.0, 1e-12)
    with pytest.raises(cyl.CylError):
        cyl.adi_parameters(16, 16, 0, 0.0, 1e-12, cap=2)


@pytest.mark.parametrize("m,n,w,ka", [(16, 16, 0, 0.0), (34, 30, 2, 0.0), (66, 66, 9, 0.0),
                                      (66, 40, 33, 0.0), (130, 130, 0, 0.0), (48, 48, 5, 1e-3),
                                      (40, 56, 0, 0.1)])
def test_planner_bounds_enclose_and_shifts_match_oracle(m, n, w, ka):
    r = cyl.adi_parameters(m, n, w, ka, 1e-12)
    At, Ct, Bt, Dt = ops.tau_system(m, n, w)
    if ka > 0:
        At, Ct, _, _ = ops.heat_system(m, n, w, ka)
    a, b, c, d, _ = adi.spectral_bounds(At, Bt, Ct, Dt)
    A, B, C, D = r["bounds"]
    # enclosing (Section 3 needs the spectra inside [a, b] and [c, d]) and tight
    assert A <= a and B >= b and C <= c and D >= d
    assert A > 1.05 * a and C > 0.95 * c and D < 1.05 * d
    assert abs(B - b) < 0.05 * abs(b)
    g, _, _ = adi.zolotarev_params(A, B, C, D)
    assert r["J"] == adi.num_iterations(g, 1e-12)
    u, v = adi.shifts(A, B, C, D, r["J"])
    assert np.allclose(r["u"], u, rtol=1e-12, atol=0)
    assert np.allclose(r["v"], v, rtol=1e-12, atol=0)


def test_planner_shifts_converge_with_oracle_adi():
    """The planner's parameters drive Algorithm 1 to the tolerance."""
    m = n = 40
    At, Ct, Bt, Dt = ops.tau_system(m, n, 3)
    E = np.random.default_rng(4).standard_normal((m - 2, n - 2))
    from oracle import sylvester
    Xs = sylvester.solve(At, Bt, Ct, Dt, E)
    for eps in (1e-6, 1e-10):
        r = cyl.adi_parameters(m, n, 3, 0.0, eps)
        X = adi.adi(At, Bt, Ct, Dt, E, np.array(r["u"]), np.array(r["v"]))
        assert np.linalg.norm(X - Xs) / np.linalg.norm(Xs) < eps
