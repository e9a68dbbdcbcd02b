"""CPU FP64 oracle for the Chebyshev-Chebyshev-Fourier (CCF) cylinder solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library; the two
meet only through the seeded generators in ``synth`` and through arrays.

What the oracle computes (Darrow, "A Quasi-Optimal Spectral Solver for the Heat
and Poisson Equations in a Closed Cylinder", arXiv 2206.04827):

* ``operators``   -- the sparse ultraspherical operators of Section 3 (the
                     matrix equation (HelmholtzMatEqn)) and the per-wavenumber
                     tau/Dirichlet systems built from them.
* ``transforms``  -- the doubled CCF grid (Definition "grid") and the
                     DCT-I / DCT-I / DFT value<->coefficient transforms of
                     Section 2.
* ``sylvester``   -- the exact (to rounding) solution of each per-mode
                     Sylvester equation by two independent dense routes:
                     Kronecker LU and diagonalised Bartels-Stewart, plus
                     extended-precision iterative refinement.
* ``adi``         -- Algorithm 1 (ADI) with the Zolotarev shifts of Section 3,
                     written in the paper's order, with the sign and shift-role
                     corrections documented there.
* ``problems``    -- Poisson and BDF1/BDF4 heat solves on the whole cylinder.
* ``boundary``    -- the physical parity j = w (mod 2) of smooth fields on the
                     doubled grid, and a transfinite lift from boundary traces.
* ``pt``          -- the poloidal-toroidal decomposition of Section 4 through
                     two horizontal (disk) Poisson solves (eq. (ptpoisson)).

Every function cites the section, equation, definition or table it follows.
Readings of places where the paper is silent, garbled or inconsistent are
stated where they are used.
"""

from . import operators, transforms, sylvester, adi, problems, adjoint, boundary, pt  # noqa: F401
