"""Physical parity and boundary traces on the doubled grid (Sections 1-2).

Oracle module (test infrastructure only; see the package docstring).

Physical parity.  The doubled grid lets r run over [-1, 1]; a function that is
single-valued and smooth on the cylinder satisfies f(-r, theta) =
f(r, theta + pi).  With f = sum c_(j,k,w) T_j(r) T_k(z) e^{i w theta} and
T_j(-r) = (-1)^j T_j(r), e^{i w (theta + pi)} = (-1)^w e^{i w theta}, this
forces c_(j,k,w) = 0 unless j = w (mod 2): the parity restriction the
introduction cites for the doubled discretization.  On the grid it holds
for even p (theta + pi is then a grid angle, and w aliases onto w +- p of the
same parity); for odd p the sampled field's DFT mixes the parities.  The
Poisson operator
(r^2 nabla^2, Section 3) maps this subspace to itself, so for such forcing
only the r-parity blocks with j = w (mod 2) carry the solution.

Boundary traces (READING: the paper gives no construction for non-homogeneous
Dirichlet data of these problems; the solvers take a lift field whose
boundary values are the data).  Here the data are the four faces of the
doubled (r, z) box of every theta line -- r = -1 and r = +1 (the side wall at
theta + pi and theta), z = -1 and z = +1 (the caps) -- and the lift is their
transfinite (Coons) interpolant in (r, z):

    L = (1-a) R_-(z) + a R_+(z) + (1-b) Z_-(r) + b Z_+(r)
        - [(1-a)(1-b) Z_-(-1) + a(1-b) Z_-(1) + (1-a) b Z_+(-1) + a b Z_+(1)],

a = (1 + r)/2, b = (1 + z)/2, corner values taken from the z-faces.  For
compatible data (the faces agree on the box's edges) L takes the given values
on all four faces.  Since the equations are multiplied by r^2 (Section 3), any
lift with the right boundary values gives a polynomial right-hand side; the
discrete solution depends on the lift's boundary values only.
"""

import numpy as np

from . import transforms as tr


def physical_mask(m, p):
    """Boolean mask [p, 1, m] over full coefficients c[l, k, j]: j = w (mod 2)."""
    w = tr.wavenumbers(p)
    j = np.arange(m)
    return ((j[None, :] - w[:, None]) % 2 == 0)[:, None, :]


def project_physical(c):
    """Zero the full coefficients c[l, k, j] with j != w (mod 2)."""
    p, n, m = c.shape
    return np.where(physical_mask(m, p), c, 0.0)


def faces(u):
    """Boundary faces of a value field u[l, k, j]: rface [2, p, n] (r = -1,
    r = +1) and zface [2, p, m] (z = -1, z = +1)."""
    rface = np.stack([u[:, :, 0], u[:, :, -1]])
    zface = np.stack([u[:, 0, :], u[:, -1, :]])
    return rface, zface


def trace_lift(rface, zface, m, n, p):
    """Coons lift [p, n, m] of the faces (see the module docstring)."""
    r, z, _ = tr.grid(m, n, p)
    a = (0.5 * (1.0 + r))[None, None, :]
    b = (0.5 * (1.0 + z))[None, :, None]
    Rm, Rp = rface[0][:, :, None], rface[1][:, :, None]        # [p, n, 1]
    Zm, Zp = zface[0][:, None, :], zface[1][:, None, :]        # [p, 1, m]
    cmm, cpm = zface[0][:, 0], zface[0][:, -1]                 # z = -1 at r = -1, +1
    cmp_, cpp = zface[1][:, 0], zface[1][:, -1]                # z = +1 at r = -1, +1
    corner = ((1 - a) * (1 - b) * cmm[:, None, None] + a * (1 - b) * cpm[:, None, None] +
              (1 - a) * b * cmp_[:, None, None] + a * b * cpp[:, None, None])
    return (1 - a) * Rm + a * Rp + (1 - b) * Zm + b * Zp - corner
