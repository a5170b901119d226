"""Brute-force references that use no FFT, for tiny grids.

* ``dense_coulomb``: the grid Coulomb matrix v(R - R') of Sec. 2.2 (Eq. 7-8)
  built by summing cos(G . (R - R')) k(G) over every plane wave of the grid.
* ``analytic_s_coulomb``: the Coulomb interaction of two periodized s-type
  Gaussian charges as a reciprocal-lattice sum of their analytic Fourier
  transforms (Sec. 2.1.3, Eq. 4), G = 0 removed.  The grid result converges to
  it exponentially as the mesh is refined.
"""
from __future__ import annotations

import math

import numpy as np

from . import grid as _grid


def dense_coulomb(lattice, mesh) -> np.ndarray:
    """Dense (N_g, N_g) matrix of the grid Coulomb operator,
    M[R, R'] = (1/N_g) sum_G k(G) cos(G . (R - R')), by explicit summation."""
    R = _grid.grid_points(lattice, mesh)
    G = _grid.gvectors(lattice, mesh).reshape(-1, 3)
    k = _grid.coulomb_kernel(lattice, mesh).reshape(-1)
    ph = G @ R.T                                   # (N_G, N_g)
    c, s = np.cos(ph), np.sin(ph)
    ng = R.shape[0]
    return ((c.T * k) @ c + (s.T * k) @ s) / ng


def analytic_s_coulomb(lattice, A, a, B, b, gmax_exp: float = 60.0) -> float:
    """(rho_A | rho_B) for two normalised periodized s Gaussians
    rho_X = sum_T (2x/pi)^(3/4) exp(-x |r - X - T|^2), as
    (1/Omega) sum_{G != 0} 4 pi / G^2 rho_A(G)* rho_B(G) with
    rho_X(G) = (2x/pi)^(3/4) (pi/x)^(3/2) exp(-G^2/(4x)) exp(-i G . X).
    The G sum runs over the full reciprocal lattice until the Gaussian factor
    falls below exp(-gmax_exp)."""
    lat = np.asarray(lattice, dtype=np.float64)
    Bv = _grid.reciprocal(lat)
    om = _grid.volume(lat)
    s = 0.25 / a + 0.25 / b
    gcut = math.sqrt(gmax_exp / s)
    nmax = [int(math.ceil(gcut / np.linalg.norm(Bv[i]))) + 1 for i in range(3)]
    rng = [np.arange(-m, m + 1) for m in nmax]
    Nn = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3)
    G = Nn @ Bv
    G2 = np.einsum("ij,ij->i", G, G)
    keep = G2 > 0
    G, G2 = G[keep], G2[keep]
    na = (2 * a / math.pi) ** 0.75 * (math.pi / a) ** 1.5
    nb = (2 * b / math.pi) ** 0.75 * (math.pi / b) ** 1.5
    d = np.asarray(A, dtype=np.float64) - np.asarray(B, dtype=np.float64)
    terms = 4 * math.pi / G2 * np.exp(-G2 * s) * np.cos(G @ d)
    return float(na * nb * terms.sum() / om)
