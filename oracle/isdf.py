"""ISDF set-up: interpolation points, fitting functions, potentials and W.

* Point selection, Sec. 3.1 and Sec. 4.3.  QR with column pivoting of the pair
  matrix rho_{mu nu, R} = phi_mu(R) phi_nu(R) picks the interpolation points as
  the leading pivots.  The randomized form replaces rho by the sketch
  rho_{mn, R} = (sum_mu G1_{mu m} phi_mu(R)) (sum_nu G2_{nu n} phi_nu(R)) with
  G1, G2 random N x p matrices with orthonormal columns, p = ceil(sqrt(K)) + m
  (m = 4 here).  Voronoi ISDF (v-ISDF) first picks ~c N_I + 10 points inside each
  atom's Voronoi set with the same randomized QRCP, then selects N_chi points out
  of their union with one more randomized QRCP.
* Fit, Sec. 3.1, Eq. 11: the least-squares problem is solved through the normal
  equations X chi = X_{:,R} with X = rho^T rho, using the product structure
  X_{R_g, R} = (sum_mu phi_mu(R_g) phi_mu(R))^2 and a Cholesky factorisation of
  X_{gg} (Sec. 4.3).  If the plain Cholesky fails, it is retried once with the
  diagonal shift 1e-13 * max diag(X_gg) (the paper names no regularisation).
  N_chi = N_g is the exact case: chi = identity.
* Potentials, Sec. 3.2: V[g, :] = Vc(chi_g) (the potential of each fitting
  function) and W = V chi^T (Eq. 14), symmetrised.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import grid as _grid
from . import rng as _rng

OVERSAMPLE = 4
CHOL_SHIFT = 1e-13


def sketch_size(K: int, N: int) -> int:
    """p = ceil(sqrt(K)) + m, capped at N (G1, G2 need orthonormal columns)."""
    return min(int(N), int(math.ceil(math.sqrt(K))) + OVERSAMPLE)


def orthonormal_sketch(N: int, p: int, seed: int, stream: int) -> np.ndarray:
    """N x p random matrix with orthonormal columns (Q factor of a Gaussian
    matrix from the counter-based generator)."""
    Z = _rng.sketch_normal(N, p, seed, stream)
    Q, _ = np.linalg.qr(Z)
    return Q


def randomized_qrcp(Phi_cols: np.ndarray, K: int, seed: int, streams, return_r=False):
    """Leading K pivots of QRCP on the sketch of the pair matrix.

    Phi_cols : (ncols, N) basis values at the candidate grid points.
    Returns indices into the candidate list, in pivot order."""
    ncols, N = Phi_cols.shape
    K = min(K, ncols)
    p = sketch_size(K, N)
    G1 = orthonormal_sketch(N, p, seed, streams[0])
    G2 = orthonormal_sketch(N, p, seed, streams[1])
    A = Phi_cols @ G1                       # (ncols, p)
    B = Phi_cols @ G2
    M = (A[:, :, None] * B[:, None, :]).reshape(ncols, p * p).T   # (p^2, ncols)
    R, piv = sla.qr(M, mode="r", pivoting=True)
    if return_r:
        return piv[:K], np.abs(np.diag(R))
    return piv[:K]


def qrcp_full(Phi_cols: np.ndarray, K: int) -> np.ndarray:
    """Deterministic QRCP on the full pair matrix (Sec. 3.1), small cases only."""
    ncols, N = Phi_cols.shape
    M = (Phi_cols[:, :, None] * Phi_cols[:, None, :]).reshape(ncols, N * N).T
    _, piv = sla.qr(M, mode="r", pivoting=True)
    return piv[:K]


def select_global(Phi: np.ndarray, naux: int, seed: int) -> np.ndarray:
    """Randomized ISDF over the whole grid (Sec. 4.3, first algorithm)."""
    return np.asarray(randomized_qrcp(Phi, naux, seed, (0, 1)), dtype=np.int64)


def select_voronoi(Phi: np.ndarray, owner: np.ndarray, nfunc_atom: np.ndarray,
                   naux: int, seed: int) -> np.ndarray:
    """Voronoi ISDF (Sec. 4.3, second algorithm).

    owner      : (N_g,) nearest-atom index of every grid point (Sec. 4.1)
    nfunc_atom : (natom,) number of basis functions centred on each atom, N_I
    Per atom I: K_I = min(|kappa_I|, ceil(c N_I) + 10) points with c = N_chi/N
    from the sketch restricted to kappa_I (all N functions, streams 2+2I, 3+2I).
    The union R_h (atom order, pivot order within an atom) is reduced to N_chi
    points by a second randomized QRCP (streams 0, 1).  Falls back to the global
    selection if |R_h| < N_chi."""
    N = Phi.shape[1]
    c = naux / N
    cand = []
    for I in range(len(nfunc_atom)):
        kap = np.flatnonzero(owner == I)
        if kap.size == 0:
            continue
        KI = min(kap.size, int(math.ceil(c * nfunc_atom[I] - 1e-9)) + 10)
        piv = randomized_qrcp(Phi[kap], KI, seed, (2 + 2 * I, 3 + 2 * I))
        cand.append(kap[piv])
    Rh = np.concatenate(cand) if cand else np.zeros(0, dtype=np.int64)
    if Rh.size < naux:
        return select_global(Phi, naux, seed)
    piv = randomized_qrcp(Phi[Rh], naux, seed, (0, 1))
    return np.asarray(Rh[piv], dtype=np.int64)


def fitting_metric(Phi_g: np.ndarray) -> np.ndarray:
    """X_gg = (Phi_g Phi_g^T)^2 (elementwise), Eq. 11 with the product structure."""
    S = Phi_g @ Phi_g.T
    return S * S


def cholesky_with_shift(X: np.ndarray):
    """Lower Cholesky factor of X; on failure retry once with the shift
    1e-13 * max diag(X).  Returns (L, shift)."""
    try:
        return sla.cholesky(X, lower=True), 0.0
    except np.linalg.LinAlgError:
        lam = CHOL_SHIFT * float(np.max(np.diag(X)))
        return sla.cholesky(X + lam * np.eye(X.shape[0]), lower=True), lam


def fit(Phi: np.ndarray, points: np.ndarray):
    """chi (N_chi, N_g) from X_gg chi = X_gR (Eq. 11).  Returns (chi, shift)."""
    ng = Phi.shape[0]
    if len(points) == ng and np.array_equal(np.sort(points), np.arange(ng)):
        chi = np.zeros((ng, ng))
        chi[np.arange(ng), points] = 1.0
        return chi, 0.0
    Phi_g = Phi[points]
    L, lam = cholesky_with_shift(fitting_metric(Phi_g))
    T = Phi_g @ Phi.T
    XgR = T * T
    chi = sla.cho_solve((L, True), XgR)
    return chi, lam


def potentials(chi: np.ndarray, lattice, mesh):
    """V[g, :] = Vc(chi_g) and W = V chi^T, symmetrised (Eq. 12, 14)."""
    V = _grid.poisson(chi, lattice, mesh)
    W = V @ chi.T
    W = 0.5 * (W + W.T)
    return V, W


def setup(w, Phi: np.ndarray, points: np.ndarray | None = None, mode: str = "voronoi",
          owner: np.ndarray | None = None):
    """Full ISDF set-up for workload ``w``.  Returns a dict with points,
    Phi_g, chi, V, W, shift."""
    if points is None:
        seed = w.sketch_seed()
        if mode == "voronoi":
            from . import basis as _basis
            own = _basis.voronoi(w) if owner is None else owner
            points = select_voronoi(Phi, own, w.funcs_per_atom(), w.naux, seed)
        elif mode == "global":
            points = select_global(Phi, w.naux, seed)
        else:
            raise ValueError(mode)
    points = np.asarray(points, dtype=np.int64)
    chi, lam = fit(Phi, points)
    V, W = potentials(chi, w.lattice, w.mesh)
    return dict(points=points, Phi_g=Phi[points], chi=chi, V=V, W=W, shift=lam)
