"""Periodized atom-centred Gaussian basis functions sampled on the grid.

Sec. 2.1.3: phi_P(r) = sum_T phi(r + T) over lattice vectors T, phi a Gaussian
centred on an atom.  The paper obtains grid values through reciprocal space and
an FFT (Sec. 4.1); this oracle samples the periodized functions directly in real
space by summing images, which avoids band-limiting and is the definition the
library implements as well.

Shell components and normalisation (free-space primitive normalisation):
  s : N_s exp(-a r^2),                N_s = (2a/pi)^(3/4)
  p : N_p (x, y, z) exp(-a r^2),      N_p = N_s * 2 sqrt(a)
  d : real-spherical, in the order
      xy, yz, zx   with N_s * 4a
      x^2 - y^2    with N_s * 2a
      3z^2 - r^2   with N_s * 2a / sqrt(3)
Images T are summed while a |r - A - T|^2 <= CUTOFF.
"""
from __future__ import annotations

import math

import numpy as np

from . import grid as _grid

CUTOFF = 50.0          # exponent cutoff a r^2 for the image sum (e^-50 ~ 2e-22)
NFUNC = {0: 1, 1: 3, 2: 5}


def shell_values(l: int, a: float, d: np.ndarray) -> np.ndarray:
    """Values of the normalised shell components at displacements d (npts,3).

    Returns (npts, 2l+1 or 1)."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    r2 = x * x + y * y + z * z
    ns = (2.0 * a / math.pi) ** 0.75
    e = np.exp(-a * r2)
    if l == 0:
        return (ns * e)[:, None]
    if l == 1:
        c = ns * 2.0 * math.sqrt(a)
        return np.stack([c * x * e, c * y * e, c * z * e], axis=1)
    if l == 2:
        c1 = ns * 4.0 * a
        c2 = ns * 2.0 * a
        c3 = ns * 2.0 * a / math.sqrt(3.0)
        return np.stack([c1 * x * y * e, c1 * y * z * e, c1 * z * x * e,
                         c2 * (x * x - y * y) * e, c3 * (2 * z * z - x * x - y * y) * e], axis=1)
    raise ValueError("l must be 0, 1 or 2")


def _images(lattice, center, a):
    """Lattice translations T such that the image centred at center+T can reach
    the cell within the cutoff radius (a superset; the per-point cutoff is
    applied separately)."""
    lat = np.asarray(lattice, dtype=np.float64)
    B = _grid.reciprocal(lat)
    rc = math.sqrt(CUTOFF / a)
    h = 2.0 * math.pi / np.linalg.norm(B, axis=1)          # plane spacings
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)]) @ lat
    mid = 0.5 * lat.sum(axis=0)
    rb = np.max(np.linalg.norm(corners - mid, axis=1))
    m = [int(math.ceil(rc / hk)) + 2 for hk in h]
    out = []
    for i in range(-m[0], m[0] + 1):
        for j in range(-m[1], m[1] + 1):
            for k in range(-m[2], m[2] + 1):
                T = i * lat[0] + j * lat[1] + k * lat[2]
                if np.linalg.norm(center + T - mid) <= rc + rb:
                    out.append(T)
    return out


def wrap_into_cell(lattice, r):
    lat = np.asarray(lattice, dtype=np.float64)
    f = np.asarray(r, dtype=np.float64) @ np.linalg.inv(lat)
    return (f - np.floor(f)) @ lat


def eval_basis(w, points: np.ndarray | None = None) -> np.ndarray:
    """Phi[R, mu] for the workload ``w`` at ``points`` (default: every grid
    point, linear C order).  Returns float64 (npts, N)."""
    lat = np.asarray(w.lattice, dtype=np.float64)
    if points is None:
        points = _grid.grid_points(lat, w.mesh)
    points = np.asarray(points, dtype=np.float64)
    cols = []
    for s in range(len(w.shell_l)):
        l = int(w.shell_l[s])
        a = float(w.shell_exp[s])
        A = wrap_into_cell(lat, w.atoms[int(w.shell_atom[s])])
        acc = np.zeros((points.shape[0], NFUNC[l]))
        for T in _images(lat, A, a):
            d = points - (A + T)
            r2 = np.einsum("ij,ij->i", d, d)
            sel = a * r2 <= CUTOFF
            if np.any(sel):
                acc[sel] += shell_values(l, a, d[sel])
        cols.append(acc)
    return np.concatenate(cols, axis=1)


def voronoi(w) -> np.ndarray:
    """Sec. 4.1: index of the nearest atom (over periodic images) for every
    grid point; ties go to the lower atom index.  Returns int64 (N_g,)."""
    lat = np.asarray(w.lattice, dtype=np.float64)
    pts = _grid.grid_points(lat, w.mesh)
    inv = np.linalg.inv(lat)
    best = np.full(pts.shape[0], np.inf)
    owner = np.zeros(pts.shape[0], dtype=np.int64)
    shifts = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]) @ lat
    for I, A in enumerate(np.asarray(w.atoms, dtype=np.float64)):
        f = (pts - A) @ inv
        f -= np.round(f)
        d0 = f @ lat
        dmin = np.full(pts.shape[0], np.inf)
        for s in shifts:
            d = d0 + s
            dmin = np.minimum(dmin, np.einsum("ij,ij->i", d, d))
        upd = dmin < best
        best[upd] = dmin[upd]
        owner[upd] = I
    return owner


def overlap(Phi: np.ndarray, dV: float) -> np.ndarray:
    """Grid overlap S = dV Phi^T Phi (the metric used to orthonormalise C)."""
    return dV * (Phi.T @ Phi)


def screen(Phi: np.ndarray, eps: float, dV: float) -> np.ndarray:
    """Screened basis of Sec. 4.1: per atom the stored values on its Voronoi set
    are those of the pSinc coefficients phi~ = sqrt(dV) phi above eps1 in
    magnitude; everything else is dropped.  The Voronoi sets partition the grid,
    so as a matrix this is Phi with the entries sqrt(dV) |phi| < eps set to zero
    (eps = 0 keeps everything).  The storage layout (one dense block per atom)
    does not change any value."""
    if eps <= 0.0:
        return Phi.copy()
    out = Phi.copy()
    out[np.sqrt(dV) * np.abs(Phi) < eps] = 0.0
    return out
