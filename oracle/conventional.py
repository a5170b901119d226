"""Exact grid exchange by one Poisson solve per occupied-orbital pair.

Sec. 2.4, Eq. 9: K_{mu nu} = sum_i (mu i | i nu), evaluated by forming the pair
product on the grid, applying the Coulomb operator with an FFT, and contracting
with the other pair.  The occ-RI form (Sec. 3.3) only needs K_{mu j} =
sum_i (mu i | i j), so one Poisson solve per unordered pair (i, j) suffices:

    V_ij     = Vc(u_i u_j)                       u_i = sum_mu C_{mu i} phi_mu
    K(mu, j) = dV sum_R Phi(R, mu) sum_i u_i(R) V_ij(R)
    E_x      = -sum_ij (ij|ji) = -dV sum_ij sum_R u_i u_j V_ij

E_x is the closed-shell exchange energy with doubly occupied spatial orbitals,
E_x = -tr(C^T K_occ) (the paper does not define E_x; see the design notes).
"""
from __future__ import annotations

import numpy as np

from . import grid as _grid


def exchange_occ(Phi: np.ndarray, C: np.ndarray, lattice, mesh, batch: int = 64):
    """Conventional occ-RI exchange.  Returns (K_occ (N, n), E_x)."""
    dV = _grid.dvol(lattice, mesh)
    k = _grid.coulomb_kernel(lattice, mesh)
    U = Phi @ C                                   # (N_g, n) orbitals on the grid
    n = U.shape[1]
    Y = np.zeros_like(U)                          # Y[:, j] = sum_i u_i V_ij
    E = 0.0
    pairs = [(i, j) for i in range(n) for j in range(i, n)]
    for s in range(0, len(pairs), batch):
        chunk = pairs[s:s + batch]
        I = np.array([p[0] for p in chunk])
        J = np.array([p[1] for p in chunk])
        rho = (U[:, I] * U[:, J]).T               # (b, N_g) pair densities
        Vij = _grid.poisson(rho, lattice, mesh, k)
        for t, (i, j) in enumerate(chunk):
            Y[:, j] += U[:, i] * Vij[t]
            e = float(rho[t] @ Vij[t])
            if i != j:
                Y[:, i] += U[:, j] * Vij[t]
                E += 2.0 * e
            else:
                E += e
    K = dV * (Phi.T @ Y)
    return K, -dV * E


def exchange_full(Phi: np.ndarray, C: np.ndarray, lattice, mesh) -> np.ndarray:
    """Conventional full exchange matrix K_{mu nu} = sum_i (mu i | i nu)
    (Eq. 9) with one Poisson solve per (i, nu).  For small tests only."""
    dV = _grid.dvol(lattice, mesh)
    k = _grid.coulomb_kernel(lattice, mesh)
    U = Phi @ C
    N = Phi.shape[1]
    K = np.zeros((N, N))
    for i in range(U.shape[1]):
        rho = (U[:, i][:, None] * Phi).T          # (N, N_g): u_i phi_nu
        Vin = _grid.poisson(rho, lattice, mesh, k)
        K += dV * ((Phi * U[:, i][:, None]).T @ Vin.T)
    return K
