"""Coulomb matrix on the grid, Sec. 2.3 ("Coulomb matrix"), steps 1-4.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With the density matrix D = C C^T of the occupied orbitals (Sec. 2.3), the
steps in the paper's order are

    1. rho(R)      = sum_{lambda sigma} D_{lambda sigma} phi_lambda(R) phi_sigma(R)
    2. rho(G)      = forward transform of rho
    3. V_H(R)      = inverse transform of k(G) rho(G)      (together: V_H = Vc rho)
    4. J_{mu nu}   = dV sum_R phi_mu(R) phi_nu(R) V_H(R)

in the plain-value convention of the package (the paper's pSinc coefficients
carry sqrt(dV) each, and its 1/Omega with the unnormalised transforms reduces
to Vc = irfftn(k rfftn(.))).

The paper does not define a Coulomb energy.  Reported here is
    E_J = sum_{ij} (ii|jj) = tr(D J) = dV sum_R rho(R) V_H(R),
the partner of E_x = -sum_{ij} (ij|ji): with doubly occupied spatial orbitals
the closed-shell two-electron energy is 2 E_J + E_x.
"""
from __future__ import annotations

import numpy as np

from . import grid as _grid


def density(Phi: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Step 1: rho(R) = sum_{lambda sigma} D_{lambda sigma} phi_lambda(R) phi_sigma(R),
    D = C C^T.  Returns (N_g,)."""
    D = C @ C.T
    return np.einsum("rl,rl->r", Phi @ D, Phi)


def build_j(Phi: np.ndarray, C: np.ndarray, lattice, mesh):
    """Steps 1-4.  Returns (J (N, N), E_J, V_H (N_g,))."""
    dV = _grid.dvol(lattice, mesh)
    rho = density(Phi, C)
    vh = _grid.poisson(rho, lattice, mesh)            # steps 2-3
    J = dV * (Phi.T @ (vh[:, None] * Phi))            # step 4
    E = dV * float(rho @ vh)
    return J, E, vh
