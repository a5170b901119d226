"""The batching form on the 64-cell workload: 64 independent diamond-like
cells of uneven size (supercell shapes {1,2}^3, diagonal strain +-5%, atom
jitter N(0, 0.05) bohr, 2,3,5-smooth grids 32^3 - 72^3, N_aux = 6N, n_occ = 2
per atom), all mixed-precision builds captured in one HIP graph.

Checks, per cell:
- the mixed build in the graph is within |dE_x| < 1e-6 Ha of the same cell's
  FP64 GPU build (the precision bar), and max|dK| / max|K| is reported;
- the 1x1x1 cells among the first ones are also checked against the FP64
  oracle on the library's points (|dE_x| < 1e-8 Ha, max|dK| / max|K| < 1e-7
  for the FP64 build; < 1e-6 Ha for the mixed one);
- a second replay, with eager work in between, reproduces the first bit for
  bit.
"""
import sys

import numpy as np
import pytest

import rps_inputs as ri
from oracle import basis, grid, isdf, rps

pytestmark = pytest.mark.gpu

ORACLE_CELLS = 3      # 1x1x1 cells checked against the oracle (each a few seconds of CPU)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2207_04636_amd as P
    P.load()
    return P


def test_batch_of_64_uneven_cells(lib):
    import torch
    cells = ri.batch_cells(64)
    _say(f"case: batching form, {len(cells)} cells, FP32 graph vs per-cell FP64 builds")
    pts, Cs, E64, K64 = [], [], [], []
    n_oracle = 0
    for i, w in enumerate(cells):
        with lib.Context.from_workload(w, seed=w.sketch_seed()) as ctx:
            p = ctx.points()
            C = ri.lowdin(ri.random_coefficients(w), ctx.overlap())
            K, E = ctx.build(C)
        pts.append(p)
        Cs.append(C)
        E64.append(E)
        K64.append(K)
        msg = f"  cell {i:2d} {w.name}: FP64 E_x={E:.10f}"
        if w.natom == 8 and n_oracle < ORACLE_CELLS:
            Phi = basis.eval_basis(w)
            dV = grid.dvol(w.lattice, w.mesh)
            st = isdf.setup(w, Phi, points=p)
            Kr, Er, _ = rps.build_occ(Phi, p, st["V"], st["W"], C, dV)
            dk = float(np.abs(K - Kr).max() / np.abs(Kr).max())
            msg += f"  vs oracle dE={E - Er:.2e} dK={dk:.2e}"
            assert abs(E - Er) < 1e-8 and dk < 1e-7
            n_oracle += 1
        _say(msg)
    assert n_oracle == ORACLE_CELLS
    ctxs = [lib.Context.from_workload(w, points=pts[i], precision=lib.PREC_FP32) for i, w in enumerate(cells)]
    try:
        dev = torch.device("cuda:0")
        Cd = [torch.from_numpy(C).to(dev) for C in Cs]
        Kd = [torch.full((w.nbas, w.nocc), float("nan"), dtype=torch.float64, device=dev) for w in cells]
        ex = torch.full((len(cells),), float("nan"), dtype=torch.float64, device=dev)
        with lib.Batch(ctxs, Cd, Kd, ex, autotune=True) as bat:
            inf = bat.info()
            _say(f"  graph: {inf['branches']} branches, replay {inf['replay_ms']:.2f} ms, create {inf['create_s']:.1f} s")
            bat.run()
            torch.cuda.synchronize()
            E32 = ex.cpu().numpy().copy()
            K32 = [k.cpu().numpy() for k in Kd]
            ctxs[0].build(Cd[0], torch.empty_like(Kd[0]))      # eager work between replays
            for k in Kd:
                k.fill_(float("nan"))
            bat.run()
            torch.cuda.synchronize()
            for i in range(len(cells)):
                assert np.array_equal(Kd[i].cpu().numpy(), K32[i]) and float(ex[i]) == E32[i], i
        worst = 0.0
        for i, w in enumerate(cells):
            dE = E32[i] - E64[i]
            dk = float(np.abs(K32[i] - K64[i]).max() / np.abs(K64[i]).max())
            worst = max(worst, abs(dE))
            _say(f"  cell {i:2d} mixed vs FP64: dE={dE:.3e} dK={dk:.3e}")
            assert abs(dE) < 1e-6, (i, dE)
            assert dk < 1e-4
        _say(f"  max |dE_x| over the batch: {worst:.3e}")
    finally:
        for c in ctxs:
            c.close()
