"""Cell, uniform grid, plane-wave vectors and the G=0-excluded Coulomb kernel.

Sec. 2.1 (plane-wave and pSinc bases): cell vectors a_i, reciprocal vectors A_j
with a_i . A_j = 2 pi delta_ij, grid points R = sum_i (n_i / N_i) a_i, and
plane waves with G = sum_i n_i A_i.  The paper's integer range for n_i is off by
one for even N_i; the numpy ``fftfreq`` range [-N/2, N/2-1] is used instead.

Sec. 2.2 (Eq. 7-8): on the grid the Coulomb operator is diagonal in G with
eigenvalue 4 pi / G^2; Sec. 4.5 drops the G = 0 term.
"""
from __future__ import annotations

import numpy as np


def volume(lattice: np.ndarray) -> float:
    """Omega = a1 . (a2 x a3), taken positive."""
    return float(abs(np.linalg.det(np.asarray(lattice, dtype=np.float64))))


def reciprocal(lattice: np.ndarray) -> np.ndarray:
    """Rows A_j with a_i . A_j = 2 pi delta_ij."""
    a = np.asarray(lattice, dtype=np.float64)
    return 2.0 * np.pi * np.linalg.inv(a).T


def grid_points(lattice: np.ndarray, mesh) -> np.ndarray:
    """(N_g, 3) cartesian grid points, linear index (i1*N2 + i2)*N3 + i3."""
    mesh = [int(m) for m in mesh]
    f = [np.arange(m) / m for m in mesh]
    F = np.stack(np.meshgrid(*f, indexing="ij"), axis=-1).reshape(-1, 3)
    return F @ np.asarray(lattice, dtype=np.float64)


def dvol(lattice, mesh) -> float:
    """Volume element dV = Omega / N_g."""
    return volume(lattice) / float(np.prod(mesh))


def gvectors(lattice, mesh) -> np.ndarray:
    """(N1, N2, N3, 3) G vectors in numpy FFT order."""
    B = reciprocal(lattice)
    n = [np.fft.fftfreq(int(m)) * int(m) for m in mesh]
    Nn = np.stack(np.meshgrid(*n, indexing="ij"), axis=-1)
    return Nn @ B


def coulomb_kernel(lattice, mesh) -> np.ndarray:
    """k(G) = 4 pi / |G|^2 with k(0) = 0, shape (N1, N2, N3), FFT order.

    For even meshes in skewed cells the Nyquist plane is ambiguous; k is
    symmetrised over G <-> -G (mod mesh) so that the operator stays real.
    For orthogonal cells this changes nothing."""
    G = gvectors(lattice, mesh)
    G2 = np.einsum("...i,...i->...", G, G)
    k = np.zeros_like(G2)
    nz = G2 > 0
    k[nz] = 4.0 * np.pi / G2[nz]
    kneg = k[tuple(np.ix_(*[(-np.arange(int(m))) % int(m) for m in mesh]))]
    return 0.5 * (k + kneg)


def poisson(f: np.ndarray, lattice, mesh, kernel=None) -> np.ndarray:
    """Vc f = irfftn(k * rfftn(f)) for real f given on the grid.

    ``f`` has shape (..., N_g) with the grid flattened in C order; the result
    has the same shape.  With plain function values this is the potential that
    appears in Eq. 9 (and, for the fitting functions, in Eq. 12) up to the
    factor conventions stated in the package docstring."""
    mesh = tuple(int(m) for m in mesh)
    k = coulomb_kernel(lattice, mesh) if kernel is None else kernel
    kh = k[..., : mesh[2] // 2 + 1]
    shp = f.shape
    F = np.fft.rfftn(f.reshape(shp[:-1] + mesh), axes=(-3, -2, -1))
    out = np.fft.irfftn(F * kh, s=mesh, axes=(-3, -2, -1))
    return out.reshape(shp)
