"""Seeded synthetic inputs for the cylinder solver (shared by tests and benchmark).

This module holds no step of the solver: it draws random numbers and evaluates
closed-form fields at given sample points.  Both the oracle and the HIP library
receive what it produces as plain arrays.

Workloads (the paper measures on no public dataset; everything is synthetic):

* ``smooth_coeffs``: random smooth forcing given by its CCF coefficients,
  c = (N(0,1) + i N(0,1)) exp(-(j + k + |w|)/4) for w >= 0, with the w = 0 and
  Nyquist slots real so that the field is real.  Layout: Hermitian half
  [floor(p/2)+1][n_z][n_r], complex128, r fastest.
* ``eigenmode_params`` / ``eigenmode_values``: a seeded sum of 8 Laplacian
  eigenfunctions J_w(j_{w,s} r) sin(q pi (z+1)/2) cos(w theta + phi), with
  w in {0..6}, s, q in {1,2,3}, a ~ N(0,1), phi ~ U[0, 2 pi).  On the doubled
  grid J_w(-x) = (-1)^w J_w(x), consistent with (r, theta) ~ (-r, theta + pi).
* ``physical_values``: a seeded smooth function of the Cartesian coordinates
  (x, y, z) = (r cos theta, r sin theta, z), sum over 4 terms of
  a exp(b x + c y) cos(d z + e x y + phi) with a ~ N(0,1), b, c ~ U[-0.6, 0.6],
  d ~ U[0.5, 2.5], e ~ U[-1, 1], phi ~ U[0, 2 pi): single-valued and smooth
  on the cylinder, hence of physical parity on the doubled grid.
* ``ccf_grid``: the sample points x_(j,k,l) of the doubled CCF grid
  (r_j = cos((m-j-1) pi/(m-1)), z_k likewise, theta_l = (2l - p) pi / p).
"""

import numpy as np
import scipy.special as ss

SEED_BASE = 220604827


def rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def ccf_grid(m, n, p):
    """Sample points (r, z, theta) of the doubled m x n x p CCF grid."""
    r = np.cos((m - np.arange(m) - 1) * np.pi / (m - 1))
    z = np.cos((n - np.arange(n) - 1) * np.pi / (n - 1))
    th = (2 * np.arange(p) - p) * np.pi / p
    return r, z, th


def physical_values(m, n, p, seed, terms=4):
    """Seeded smooth Cartesian field on the grid, values [p][n][m] float64."""
    g = rng(seed)
    r, z, th = ccf_grid(m, n, p)
    TH, Z, R = np.meshgrid(th, z, r, indexing="ij")
    X, Y = R * np.cos(TH), R * np.sin(TH)
    f = np.zeros((p, n, m))
    for _ in range(terms):
        a = g.standard_normal()
        b, c = g.uniform(-0.6, 0.6, 2)
        d = g.uniform(0.5, 2.5)
        e = g.uniform(-1.0, 1.0)
        phi = g.uniform(0.0, 2 * np.pi)
        f += a * np.exp(b * X + c * Y) * np.cos(d * Z + e * X * Y + phi)
    return f


def smooth_coeffs(m, n, p, seed, decay=4.0):
    """Hermitian-half CCF coefficients with |c| ~ N(0,1) exp(-(j+k+|w|)/decay)."""
    g = rng(seed)
    nw = p // 2 + 1
    re = g.standard_normal((nw, n, m))
    im = g.standard_normal((nw, n, m))
    w = np.arange(nw)[:, None, None]
    k = np.arange(n)[None, :, None]
    j = np.arange(m)[None, None, :]
    env = np.exp(-(j + k + w) / decay)
    c = (re + 1j * im) * env
    c[0] = c[0].real
    if p % 2 == 0:
        c[p // 2] = c[p // 2].real
    return c


def eigenmode_params(seed, count=8, wmax=6):
    g = rng(seed)
    return {
        "w": g.integers(0, wmax + 1, size=count),
        "s": g.integers(1, 4, size=count),
        "q": g.integers(1, 4, size=count),
        "a": g.standard_normal(count),
        "phi": g.uniform(0.0, 2.0 * np.pi, size=count),
    }


def eigenmode_values(params, m, n, p):
    """Values [p][n][m] of sum_i a_i J_w(j_{w,s} r) sin(q pi (z+1)/2) cos(w th + phi)."""
    r, z, th = ccf_grid(m, n, p)
    out = np.zeros((p, n, m))
    for w, s, q, a, ph in zip(params["w"], params["s"], params["q"], params["a"], params["phi"]):
        jz = ss.jn_zeros(int(w), int(s))[-1]
        fr = ss.jv(int(w), jz * r)
        fz = np.sin(q * np.pi * (z + 1.0) / 2.0)
        ft = np.cos(w * th + ph)
        out += a * ft[:, None, None] * fz[None, :, None] * fr[None, None, :]
    return out


def eigenmode_rates(params):
    """Laplacian eigenvalues lambda_i = j_{w,s}^2 + (q pi / 2)^2 of each term."""
    lam = []
    for w, s, q in zip(params["w"], params["s"], params["q"]):
        jz = ss.jn_zeros(int(w), int(s))[-1]
        lam.append(jz * jz + (q * np.pi / 2.0) ** 2)
    return np.array(lam)


def half_to_planes(c):
    """Complex half coefficients -> float64 interleaved array (same memory layout)."""
    return np.ascontiguousarray(np.asarray(c, dtype=np.complex128)).view(np.float64)


def batch_specs(seed, count=64, n_range=(48, 384), p_range=(32, 256), alpha_range=(0.1, 2.0)):
    """Sizes and diffusivities of a batch of independent heat problems:
    n_r = n_z ~ U{n_range}, n_theta ~ U{p_range}, alpha ~ U[alpha_range].
    Returns a list of (n_r, n_z, n_theta, alpha)."""
    g = rng(seed)
    nn = g.integers(n_range[0], n_range[1] + 1, size=count)
    pp = g.integers(p_range[0], p_range[1] + 1, size=count)
    aa = g.uniform(alpha_range[0], alpha_range[1], size=count)
    return [(int(a), int(a), int(b), float(c)) for a, b, c in zip(nn, pp, aa)]
