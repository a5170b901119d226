"""FP64 CPU oracle for the robust-pseudospectral (rPS) occ-RI exchange build.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does, and
this package imports nothing from it.

Everything here is plain numpy/scipy in float64, written from the paper
(Sharma, White, Beylkin, "Fast exchange with Gaussian basis set using robust
pseudospectral method", arXiv:2207.04636).  Each function names the section or
equation it follows.  Conventions used throughout:

* Basis values are plain function values Phi[R, mu] = phi_mu(R); the paper's
  pSinc coefficients are sqrt(dV) * phi_mu(R) with dV = Omega / N_g (Sec. 2.1.2,
  2.2), so every contraction below carries one factor dV.
* The Coulomb operator on the grid is Vc f = irfftn(k * rfftn(f)) with
  k(G) = 4 pi / |G|^2 and k(0) = 0 (Sec. 2.2 Eq. 7-8, G=0 removed as in
  Sec. 4.5).

Modules
-------
grid         cell, grid points, G vectors, Coulomb kernel, Vc
basis        periodized Gaussian shells on the grid (Sec. 2.1.3)
conventional exact grid exchange by one Poisson solve per orbital pair (Sec. 2.4)
brute        dense Coulomb matrix by direct G summation (no FFT), tiny grids
rng          Philox4x32-10 counter-based generator (sketch matrices)
isdf         point selection (randomized QRCP, Voronoi ISDF), fit, V, W (Sec. 3.1, 4.1, 4.3)
rps          rPS / PS / THC exchange in occ-RI and full form (Sec. 3.2, 3.3)
coulomb      Coulomb matrix J and E_J on the grid (Sec. 2.3, steps 1-4)

Parity status: every function is pinned by a CPU test except the specific
interpolation point set produced by the randomized selection, which depends on
random numbers and ties ("parity unpinned"; its quality is pinned instead).
"""
