"""Seeded synthetic workloads for the robust-pseudospectral exchange build.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
geometry, basis-set and random-coefficient recipes only: none of the method's
arithmetic (no basis evaluation, no Coulomb kernel, no fitting).

The paper's benchmark systems (LiH and diamond crystals with GTH basis sets and
pseudopotentials, Sec. 5) need data files that are not available, so the
workloads below stand in for them with the same structure: an fcc diamond
lattice with a (1/4,1/4,1/4) basis, a conventional cubic cell of 6.74 bohr,
supercells of it, Gaussian shells on every atom, and N_aux = c*N with c around
4-6 (Sec. 5.1, Table 3; Sec. 5.4).

Seeds: every workload draws from ``numpy.random.SeedSequence([220704636, id])``
spawned into named sub-streams (positions, exponents, coefficients, sketch,
shape, perturbation), so a workload is reproducible from its id alone.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_ROOT = 220704636
NFUNC = {0: 1, 1: 3, 2: 5}   # s, p, and real-spherical d
_STREAMS = ("positions", "exponents", "coefficients", "sketch", "shape", "perturbation")


@dataclasses.dataclass
class Workload:
    """One periodic cell with a Gaussian basis, occupied count and N_aux.

    lattice : (3,3) float64, rows are the cell vectors a1, a2, a3 (bohr)
    mesh    : (3,) int, grid points along a1, a2, a3
    atoms   : (natom,3) float64 cartesian atom positions (bohr)
    shell_atom, shell_l, shell_exp : per-shell atom index, angular momentum
              (0, 1, 2) and exponent (bohr^-2); shell centre = atoms[shell_atom]
    nocc    : number of occupied orbitals (columns of C)
    naux    : number of interpolation points N_chi
    cid     : id used to derive the seeds
    """
    name: str
    lattice: np.ndarray
    mesh: np.ndarray
    atoms: np.ndarray
    shell_atom: np.ndarray
    shell_l: np.ndarray
    shell_exp: np.ndarray
    nocc: int
    naux: int
    cid: int

    @property
    def nbas(self) -> int:
        return int(sum(NFUNC[int(l)] for l in self.shell_l))

    @property
    def ngrid(self) -> int:
        return int(np.prod(self.mesh))

    @property
    def natom(self) -> int:
        return int(self.atoms.shape[0])

    @property
    def shell_center(self) -> np.ndarray:
        return self.atoms[self.shell_atom]

    @property
    def volume(self) -> float:
        return float(abs(np.linalg.det(self.lattice)))

    def funcs_per_atom(self) -> np.ndarray:
        n = np.zeros(self.natom, dtype=np.int64)
        for a, l in zip(self.shell_atom, self.shell_l):
            n[a] += NFUNC[int(l)]
        return n

    def sketch_seed(self) -> int:
        """64-bit seed for the random sketch matrices of the point selection."""
        ss = _streams(self.cid)["sketch"]
        return int(ss.generate_state(2, dtype=np.uint32).view(np.uint64)[0])

    def with_naux(self, naux: int) -> "Workload":
        return dataclasses.replace(self, naux=int(naux))


def _streams(cid: int):
    kids = np.random.SeedSequence([SEED_ROOT, int(cid)]).spawn(len(_STREAMS))
    return dict(zip(_STREAMS, kids))


def _rng(cid: int, stream: str) -> np.random.Generator:
    return np.random.default_rng(_streams(cid)[stream])


def _loguniform(rng, lo, hi, size):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------

def tiny_cell(cid: int = 1) -> Workload:
    """Cubic cell L=6.0 bohr, 24^3 grid, 2 atoms at seeded uniform positions,
    5 s + 5 p shells per atom (N=40), exponents log-uniform in [0.2, 8],
    8 occupied orbitals, N_aux = 160."""
    L = 6.0
    pos = _rng(cid, "positions").uniform(0.0, L, size=(2, 3))
    exps = _loguniform(_rng(cid, "exponents"), 0.2, 8.0, 20)
    shell_atom, shell_l = [], []
    for a in range(2):
        shell_atom += [a] * 10
        shell_l += [0] * 5 + [1] * 5
    return Workload("tiny-L6-24^3-N40-n8-Naux160", np.eye(3) * L, np.array([24, 24, 24]),
                    pos, np.array(shell_atom), np.array(shell_l), exps, 8, 160, cid)


DIAMOND_L = 6.74
# fcc translations plus the (1/4,1/4,1/4) basis, fractional coordinates
_FCC = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
DIAMOND_FRAC = np.concatenate([_FCC, _FCC + 0.25])


def diamond_supercell(rep=(1, 1, 1), mesh_per_cell: int = 48, nocc_per_atom: int = 2,
                      c: float = 6.0, cid: int = 2, strain=None, jitter: float = 0.05,
                      naux: Optional[int] = None, name: Optional[str] = None) -> Workload:
    """Diamond-like crystal: rep[0] x rep[1] x rep[2] conventional cells of
    L = 6.74 bohr (8 atoms each: fcc + (1/4,1/4,1/4)), positions jittered by
    N(0, jitter) bohr.  Every atom carries the same 'element' basis of
    2 s, 2 p and 1 real-spherical d shell (13 functions) with exponents drawn
    once, log-uniform in [0.1, 10].  ``strain`` (3,) scales the cell axes
    (orthorhombic strain).  N_aux defaults to round(c*N)."""
    rep = np.asarray(rep, dtype=np.int64)
    scale = np.ones(3) if strain is None else 1.0 + np.asarray(strain, dtype=np.float64)
    lat = np.diag(DIAMOND_L * rep * scale)
    frac = []
    for i in range(rep[0]):
        for j in range(rep[1]):
            for k in range(rep[2]):
                frac.append((DIAMOND_FRAC + np.array([i, j, k])) / rep)
    frac = np.concatenate(frac)
    pos = frac @ lat
    pos = pos + _rng(cid, "positions").normal(0.0, jitter, size=pos.shape)
    elem_exp = _loguniform(_rng(cid, "exponents"), 0.1, 10.0, 5)
    elem_l = [0, 0, 1, 1, 2]
    natom = pos.shape[0]
    shell_atom = np.repeat(np.arange(natom), 5)
    shell_l = np.tile(elem_l, natom)
    shell_exp = np.tile(elem_exp, natom)
    if np.isscalar(mesh_per_cell):
        mesh = np.asarray(rep) * int(mesh_per_cell)
    else:
        mesh = np.asarray(mesh_per_cell, dtype=np.int64)
    nbas = 13 * natom
    if naux is None:
        naux = int(round(c * nbas))
    nm = name or f"diamond-{rep[0]}x{rep[1]}x{rep[2]}-{'x'.join(map(str, mesh))}-N{nbas}-n{nocc_per_atom*natom}-Naux{naux}"
    return Workload(nm, lat, mesh, pos, shell_atom, shell_l, shell_exp,
                    nocc_per_atom * natom, int(naux), cid)


def diamond_cell(c: float = 6.0) -> Workload:
    """8-atom diamond-like cell, 48^3 grid, N=104, n_occ=16, N_aux = c*N
    (c in {4, 6, 8, 10} for the convergence sweep)."""
    return diamond_supercell((1, 1, 1), 48, 2, c=c, cid=2)


def diamond_2x2x2() -> Workload:
    """64-atom 2x2x2 supercell, 72^3 grid, N=832, n_occ=128, N_aux=6N=4992."""
    return diamond_supercell((2, 2, 2), (72, 72, 72), 2, c=6.0, cid=3)


def diamond_3x3x3() -> Workload:
    """216-atom 3x3x3 supercell, 108^3 grid, N=2808, n_occ=432, N_aux=12000."""
    return diamond_supercell((3, 3, 3), (108, 108, 108), 2, naux=12000, cid=4)


def smooth_235(n: int) -> int:
    """Smallest integer >= n whose only prime factors are 2, 3 and 5."""
    m = max(1, int(n))
    while True:
        k = m
        for p in (2, 3, 5):
            while k % p == 0:
                k //= p
        if k == 1:
            return m
        m += 1


def batch_cells(count: int = 64, cid: int = 5) -> List[Workload]:
    """Uneven batch: supercell shapes uniform over {1,2}^3, diagonal strain
    U(-5%, +5%), jitter N(0,0.05); per-axis grid = smallest 2,3,5-smooth
    N_i >= L_i/h with h ~ U[0.187, 0.215] bohr, clamped to [32, 72];
    N_aux = 6N, n_occ = 2 per atom."""
    rng = _rng(cid, "shape")
    out = []
    for b in range(count):
        rep = rng.integers(1, 3, size=3)
        strain = rng.uniform(-0.05, 0.05, size=3)
        h = rng.uniform(0.187, 0.215)
        Ls = DIAMOND_L * rep * (1 + strain)
        mesh = np.array([min(72, max(32, smooth_235(int(math.ceil(L / h))))) for L in Ls])
        out.append(diamond_supercell(rep, mesh, 2, c=6.0, cid=1000 + b, strain=strain))
    return out


def tiny_s_cell(nfunc: int = 6, mesh: int = 8, L: float = 4.0, nocc: int = 2,
                naux: int = 8, cid: int = 90, lmax: int = 0) -> Workload:
    """Very small cell for brute-force pins: ``nfunc`` shells (s only unless
    lmax > 0) at seeded positions, exponents log-uniform in [0.5, 3]."""
    rng = _rng(cid, "positions")
    pos = rng.uniform(0, L, size=(nfunc, 3))
    exps = _loguniform(_rng(cid, "exponents"), 0.5, 3.0, nfunc)
    ls = np.zeros(nfunc, dtype=np.int64)
    if lmax > 0:
        ls = np.arange(nfunc) % (lmax + 1)
    return Workload(f"tiny-s{nfunc}-{mesh}^3", np.eye(3) * L, np.array([mesh] * 3), pos,
                    np.arange(nfunc), ls, exps, nocc, naux, cid)


# ---------------------------------------------------------------------------
# Occupied coefficients
# ---------------------------------------------------------------------------

def random_coefficients(w: Workload, stream: str = "coefficients") -> np.ndarray:
    """Seeded N x n_occ matrix of standard normal entries (before orthonormalisation)."""
    return _rng(w.cid, stream).standard_normal((w.nbas, w.nocc))


def lowdin(C0: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Make the columns of C0 orthonormal in the metric S: C = C0 (C0^T S C0)^(-1/2)."""
    M = C0.T @ S @ C0
    M = 0.5 * (M + M.T)
    w, Q = np.linalg.eigh(M)
    return C0 @ (Q * (1.0 / np.sqrt(w))) @ Q.T


def perturbed(C: np.ndarray, S: np.ndarray, step: int, angle: float = 0.01,
              w: Optional[Workload] = None, cid: int = 0) -> np.ndarray:
    """Occupied-virtual rotation by a small angle, as in an SCF step: mixes C
    with a random direction from the S-orthogonal complement, then
    re-orthonormalises."""
    seed = (w.cid if w is not None else cid)
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, seed, 7, step]))
    Z = rng.standard_normal(C.shape)
    comp = Z - C @ (C.T @ (S @ Z))
    comp /= np.linalg.norm(comp)
    return lowdin(C + angle * math.sqrt(C.shape[1]) * comp, S)
