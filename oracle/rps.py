"""Robust pseudospectral (rPS) exchange, plus the PS and THC variants.

Sec. 3.2, Eq. 13: the rPS two-electron integral is
    fit.exact (line 1) + exact.fit (line 2) - fit.fit (line 3),
with V the potential of the fitting functions and W = V chi^T (Eq. 14).  Only
line 1 is the pseudospectral (PS) approximation; only line 3 is THC.

Sec. 3.3, Eq. 16 (occ-RI): with U = Phi C (orbitals on the grid), U_g = U at the
interpolation points, P = U_g U^T, A = V o P, P_g = U_g U_g^T, B = W o P_g
(o = elementwise product), the three lines become

    K1 = Phi^T (A^T U_g)      (grid-side basis function, Eq. 16 first line)
    K2 = Phi_g^T (A U)        (point-side basis function, second line)
    K3 = Phi_g^T (B U_g)      (fit.fit, third line)
    K_occ = dV (K1 + K2 - K3),   K_occ[mu, j] = sum_i (mu i | i j)

The contraction order of the second line (A U first, then Phi_g^T) is the one
Sec. 4.4 prefers.  The energy is E_x = -tr(C^T K_occ) = -dV (2 sum A o P -
sum B o P_g), both routes are returned.

Full matrix (Eq. 15 and its two partner terms):
    K_full = dV [Phi_g^T A Phi + (Phi_g^T A Phi)^T - Phi_g^T B Phi_g].
"""
from __future__ import annotations

import numpy as np


def _parts(Phi, points, V, W, C):
    U = Phi @ C
    Ug = U[points]
    P = Ug @ U.T
    A = V * P
    Pg = Ug @ Ug.T
    B = W * Pg
    return U, Ug, P, A, Pg, B


def build_occ(Phi, points, V, W, C, dV, return_parts=False):
    """rPS occ-RI exchange (Eq. 16).  Returns (K_occ (N, n), E_x, E_x_trace)."""
    Phi_g = Phi[points]
    U, Ug, P, A, Pg, B = _parts(Phi, points, V, W, C)
    M1T = A.T @ Ug          # (N_g, n)   line 1 intermediate
    M2 = A @ U              # (N_chi, n) line 2 intermediate (Sec. 4.4 order)
    Y = B @ Ug              # (N_chi, n) line 3 intermediate
    K1 = Phi.T @ M1T
    K2 = Phi_g.T @ M2
    K3 = Phi_g.T @ Y
    K = dV * (K1 + K2 - K3)
    e1 = float(np.sum(A * P))
    e3 = float(np.sum(B * Pg))
    E = -dV * (2.0 * e1 - e3)
    Etr = -float(np.sum(C * K))
    if return_parts:
        return K, E, Etr, dict(K1=dV * K1, K2=dV * K2, K3=dV * K3, e1=e1, e3=e3)
    return K, E, Etr


def build_full(Phi, points, V, W, C, dV):
    """rPS full exchange matrix K_{mu nu} (Eq. 15 plus partner terms)."""
    Phi_g = Phi[points]
    _, _, _, A, _, B = _parts(Phi, points, V, W, C)
    T = Phi_g.T @ (A @ Phi)
    return dV * (T + T.T - Phi_g.T @ (B @ Phi_g))


def ps_occ(Phi, points, V, W, C, dV):
    """PS (first line of Eq. 13 only) in occ-RI form: K = dV Phi_g^T (A U)."""
    Phi_g = Phi[points]
    U, _, _, A, _, _ = _parts(Phi, points, V, W, C)
    K = dV * (Phi_g.T @ (A @ U))
    return K, -float(np.sum(C * K))


def thc_occ(Phi, points, V, W, C, dV):
    """THC (third line of Eq. 13 only) in occ-RI form: K = dV Phi_g^T (B U_g)."""
    Phi_g = Phi[points]
    _, Ug, _, _, _, B = _parts(Phi, points, V, W, C)
    K = dV * (Phi_g.T @ (B @ Ug))
    return K, -float(np.sum(C * K))


def exchange_energy(C, K) -> float:
    """E_x = -tr(C^T K) for K_occ[mu, i] (closed shell, doubly occupied)."""
    return -float(np.sum(np.asarray(C) * np.asarray(K)))
