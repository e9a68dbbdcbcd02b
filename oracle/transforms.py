"""Doubled CCF grid and value <-> coefficient transforms (Section 2).

Oracle module (test infrastructure only; see the package docstring).

Array conventions (shared with the library's interface, not with its code):

* values    ``f[l, k, j]``: theta index l, z index k, r index j (r fastest),
  sampled at the grid point x_(j,k,l) of Definition "grid";
* full coefficients ``c[l, k, j]``: coefficient of T_j(r) T_k(z) e^{i w theta}
  with w = l - floor(p/2) (Definition of the CCF polynomial);
* half coefficients ``h[w, k, j]`` for w = 0..floor(p/2): the Hermitian half of
  a real field.  For even p the slot w = p/2 holds the coefficient of
  e^{-i (p/2) theta} (the paper's w = -p/2), which is the same function on the
  grid as e^{+i (p/2) theta}.

READING (normalisation and orientation of the DCT/DFT are not stated in the
paper): they are fixed by the interpolation property of Section 2 -- the
interpolant built from the coefficients takes the given values at the grid
points.  Because r_j = -cos(j pi/(m-1)) runs upwards, the DCT-I acts on the
reversed line; because theta_0 = -pi, the DFT carries the phase (-1)^w.
"""

import numpy as np
import scipy.fft as sfft


def grid(m, n, p):
    """Definition "grid": r_j, z_k, theta_l of CCF_(m,n,p)."""
    j = np.arange(m)
    k = np.arange(n)
    l = np.arange(p)
    r = np.cos((m - j - 1) * np.pi / (m - 1))
    z = np.cos((n - k - 1) * np.pi / (n - 1))
    th = (2 * l - p) * np.pi / p
    return r, z, th


def wavenumbers(p):
    """w = l - floor(p/2) for storage index l = 0..p-1 (CCF polynomial def.)."""
    return np.arange(p) - p // 2


def _cheb_fwd(f, axis):
    """Chebyshev coefficients from values at upward-ordered Lobatto points."""
    M = f.shape[axis] - 1
    g = np.flip(f, axis=axis)
    c = sfft.dct(g, type=1, axis=axis) / M
    idx0 = [slice(None)] * f.ndim
    idxM = [slice(None)] * f.ndim
    idx0[axis] = 0
    idxM[axis] = M
    c[tuple(idx0)] *= 0.5
    c[tuple(idxM)] *= 0.5
    return c


def _cheb_inv(c, axis):
    """Values at upward-ordered Lobatto points from Chebyshev coefficients."""
    M = c.shape[axis] - 1
    h = np.array(c, copy=True)
    mid = [slice(None)] * c.ndim
    mid[axis] = slice(1, M)
    h[tuple(mid)] *= 0.5
    g = sfft.dct(h, type=1, axis=axis)
    return np.flip(g, axis=axis)


def forward(f):
    """Values -> full CCF coefficients (Section 2): DCT-I in r, DCT-I in z, DFT in theta."""
    f = np.asarray(f, dtype=np.float64)
    p = f.shape[0]
    c = _cheb_fwd(f, axis=2)
    c = _cheb_fwd(c, axis=1)
    F = np.fft.fft(c, axis=0) / p
    w = wavenumbers(p)
    sign = np.where(w % 2 == 0, 1.0, -1.0)
    return sign[:, None, None] * F[w % p]


def inverse(c, real=True):
    """Full CCF coefficients -> values (the inverse of ``forward``)."""
    c = np.asarray(c)
    p = c.shape[0]
    w = wavenumbers(p)
    sign = np.where(w % 2 == 0, 1.0, -1.0)
    F = np.empty_like(c, dtype=np.complex128)
    F[w % p] = sign[:, None, None] * c
    v = np.fft.ifft(F, axis=0) * p
    v = _cheb_inv(v, axis=1)
    v = _cheb_inv(v, axis=2)
    return v.real.copy() if real else v


def evaluate(c, r, z, th):
    """Evaluate the interpolant f* of Section 2 at arbitrary points (slow, exact sum).

    Uses numpy's Chebyshev evaluation for T_j and explicit exponentials.
    """
    c = np.asarray(c)
    p, n, m = c.shape
    w = wavenumbers(p)
    Tr = np.polynomial.chebyshev.chebvander(np.asarray(r, dtype=float), m - 1)  # (P, m)
    Tz = np.polynomial.chebyshev.chebvander(np.asarray(z, dtype=float), n - 1)  # (P, n)
    E = np.exp(1j * np.outer(np.asarray(th, dtype=float), w))                  # (P, p)
    return np.einsum("lkj,Pj,Pk,Pl->P", c, Tr, Tz, E)


def to_half(c):
    """Full coefficients [p][n][m] -> Hermitian half [floor(p/2)+1][n][m]."""
    p = c.shape[0]
    h = np.empty((p // 2 + 1,) + c.shape[1:], dtype=np.complex128)
    for w in range(p // 2 + 1):
        if p % 2 == 0 and w == p // 2:
            h[w] = c[0]                      # w = -p/2 sits at storage index 0
        else:
            h[w] = c[w + p // 2]
    return h


def from_half(h, p):
    """Hermitian half -> full coefficients of the real field it describes."""
    c = np.zeros((p,) + h.shape[1:], dtype=np.complex128)
    for l, w in enumerate(wavenumbers(p)):
        if p % 2 == 0 and w == -(p // 2):
            c[l] = h[p // 2].real
        elif w == 0:
            c[l] = h[0].real
        elif w > 0:
            c[l] = h[w]
        else:
            c[l] = np.conj(h[-w])
    return c
