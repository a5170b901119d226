"""Madelung correction of the exchange with the G = 0 term removed (Sec. 4.5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The exchange kernel drops G = 0; Sec. 4.5 adds back nM/2 with M the Madelung
constant of the cell (n electrons).  Reading taken here (the text gives no sign
or definition of M):

* M = -phi(0), where phi is the potential at a lattice site of a unit point
  charge on every site of the lattice with a uniform neutralising background,
  its own bare 1/r removed.  By Ewald's splitting with any eta > 0,
      phi(0) = sum_{T != 0} erfc(eta |T|) / |T|
             + (4 pi / Omega) sum_{G != 0} exp(-G^2 / (4 eta^2)) / G^2
             - 2 eta / sqrt(pi) - pi / (eta^2 Omega).
  M > 0 for the cells here (2.8373 / L for a simple cubic cell of side L).
* For orthonormal occupied orbitals the divergent G = 0 part of (ij|ji) is
  replaced by M delta_ij, so
      K_occ -> K_occ + M S C,      E_x -> E_x - M tr(C^T S C) = E_x - n_occ M,
  with S the overlap; n_occ M = nM/2 for n = 2 n_occ electrons.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from . import grid as _grid


def madelung(lattice, eta: float | None = None, tol: float = 1e-16) -> float:
    """M = -phi(0) by the Ewald sum above (both sums taken until their terms
    fall below tol relative)."""
    lat = np.asarray(lattice, dtype=np.float64)
    om = _grid.volume(lat)
    if eta is None:
        eta = math.sqrt(math.pi) / om ** (1.0 / 3.0)
    # real-space images: erfc(eta r) < tol  ->  eta r > ~6
    rcut = 6.5 / eta
    nr = [int(math.ceil(rcut / np.linalg.norm(lat[i]))) + 1 for i in range(3)]
    rng = [np.arange(-m, m + 1) for m in nr]
    Tn = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3)
    T = Tn @ lat
    r = np.linalg.norm(T, axis=1)
    r = r[r > 0]
    real = float(np.sum(erfc(eta * r) / r))
    # reciprocal: exp(-G^2 / 4 eta^2) < tol  ->  G < 2 eta sqrt(-ln tol)
    B = _grid.reciprocal(lat)
    gcut = 2.0 * eta * math.sqrt(-math.log(tol))
    ng = [int(math.ceil(gcut / np.linalg.norm(B[i]))) + 1 for i in range(3)]
    rng = [np.arange(-m, m + 1) for m in ng]
    Gn = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3)
    G = Gn @ B
    G2 = np.einsum("ij,ij->i", G, G)
    G2 = G2[G2 > 0]
    recip = float(4.0 * math.pi / om * np.sum(np.exp(-G2 / (4.0 * eta * eta)) / G2))
    phi0 = real + recip - 2.0 * eta / math.sqrt(math.pi) - math.pi / (eta * eta * om)
    return -phi0


def correct(K: np.ndarray, E: float, C: np.ndarray, S: np.ndarray, M: float):
    """Exchange with the Madelung term: (K_occ + M S C, E_x - M tr(C^T S C))."""
    SC = S @ C
    return K + M * SC, E - M * float(np.trace(C.T @ SC))
