"""Pins for the oracle's physical parity and boundary-trace lift.

Physical parity is pinned by fields built from Cartesian coordinates (smooth
on the cylinder by construction, so the parity follows from the mathematics,
not from the oracle), by a field that is not single-valued (its coefficients
must break the parity), and by the Poisson solve of physical forcing.  The
lift is pinned by its face values, by exactness on functions that are
bilinear in (r, z), and by recovering a manufactured polynomial solution from
nothing but its boundary values.
"""

import numpy as np
import pytest

from oracle import boundary as bd
from oracle import problems as pb
from oracle import transforms as tr


def _cart(m, n, p):
    r, z, th = tr.grid(m, n, p)
    TH, Z, R = np.meshgrid(th, z, r, indexing="ij")
    return R * np.cos(TH), R * np.sin(TH), Z, R, TH


def _smooth_cartesian(m, n, p):
    X, Y, Z, _, _ = _cart(m, n, p)
    return np.exp(0.3 * X - 0.2 * Y) * np.cos(1.1 * Z + 0.4 * X * Y) + X ** 3 * Z - 2 * Y ** 2


def _wrong_parity_ratio(c):
    p, n, m = c.shape
    mask = bd.physical_mask(m, p)
    return np.max(np.abs(np.where(mask, 0.0, c))) / np.max(np.abs(c))


@pytest.mark.parametrize("m,n,p", [(24, 20, 16), (25, 17, 12), (30, 22, 10)])
def test_cartesian_fields_have_physical_parity(m, n, p):
    c = tr.forward(_smooth_cartesian(m, n, p))
    assert _wrong_parity_ratio(c) < 1e-13


def test_odd_theta_count_aliases_across_parities():
    """For odd p the grid has no theta + pi and w aliases onto w +- p of the
    other parity: the restriction holds on the grid for even p only."""
    c = tr.forward(_smooth_cartesian(24, 20, 9))
    assert _wrong_parity_ratio(c) > 1e-10


def test_non_single_valued_field_breaks_parity():
    """f = r cos(2 theta)... on the doubled grid f(-r, theta) = -f(r, theta +
    pi): not a function on the cylinder, and its coefficients sit at j != w."""
    m, n, p = 20, 12, 8
    _, _, Z, R, TH = _cart(m, n, p)
    c = tr.forward(R * np.cos(2 * TH) * (1 + Z))
    assert _wrong_parity_ratio(c) > 0.5
    assert np.max(np.abs(bd.project_physical(c))) < 1e-13


def test_projection_is_idempotent_and_splits_fields():
    m, n, p = 18, 14, 10
    c = tr.forward(np.random.default_rng(3).standard_normal((p, n, m)))
    a = bd.project_physical(c)
    assert np.array_equal(bd.project_physical(a), a)
    assert np.max(np.abs(bd.project_physical(c - a))) == 0.0


@pytest.mark.parametrize("m,n,p", [(20, 16, 8), (21, 15, 6)])
def test_poisson_of_physical_forcing_is_physical(m, n, p):
    u = pb.poisson(_smooth_cartesian(m, n, p))
    assert _wrong_parity_ratio(tr.forward(u)) < 1e-11


def test_lift_takes_the_face_values():
    m, n, p = 14, 11, 6
    u = _smooth_cartesian(m, n, p)
    rf, zf = bd.faces(u)
    L = bd.trace_lift(rf, zf, m, n, p)
    assert np.max(np.abs(L[:, :, 0] - u[:, :, 0])) < 1e-14
    assert np.max(np.abs(L[:, :, -1] - u[:, :, -1])) < 1e-14
    assert np.max(np.abs(L[:, 0, :] - u[:, 0, :])) < 1e-14
    assert np.max(np.abs(L[:, -1, :] - u[:, -1, :])) < 1e-14


def test_lift_is_exact_on_bilinear_functions():
    m, n, p = 12, 10, 5
    _, _, Z, R, TH = _cart(m, n, p)
    u = (1.0 + np.sin(TH)) + (2.0 - np.cos(TH)) * R - 0.5 * Z + 3.0 * np.cos(2 * TH) * R * Z
    rf, zf = bd.faces(u)
    assert np.max(np.abs(bd.trace_lift(rf, zf, m, n, p) - u)) < 1e-14


@pytest.mark.parametrize("m,n,p", [(12, 10, 6), (15, 13, 8)])
def test_solution_recovered_from_its_traces(m, n, p):
    """u polynomial in x, y, z with nonzero boundary values: forcing nabla^2 u
    and the four faces of u determine u exactly."""
    X, Y, Z, _, _ = _cart(m, n, p)
    u = 1.0 + X + 2 * Y * Z + X * X - Y * Y + 3 * Z ** 3 + X * Y * Z
    f = 18.0 * Z
    rf, zf = bd.faces(u)
    got = pb.poisson(f, lift=bd.trace_lift(rf, zf, m, n, p))
    assert np.max(np.abs(got - u)) < 1e-12
