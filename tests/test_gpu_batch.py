"""GPU tests of the batching form (rps_batch_*) and the autotuner.

A batch of uneven cells (fast-path and general-path sizes, the GEMM form,
FP64, FP32 and split-BF16, dense and screened basis) is captured into one HIP
graph.  Every replay must reproduce, bit for
bit, the eager builds of the same contexts (same tuned launch parameters, no
atomics anywhere), also with eager work and synchronisations between replays;
the config-1 cell is also checked against the FP64 oracle."""
import dataclasses
import sys

import numpy as np
import pytest

import rps_inputs as ri
from oracle import basis, grid, isdf, rps

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2207_04636_amd as P
    P.load()
    return P


def _cells():
    """(workload, precision 0 FP64 / 1 FP32 / 2 split-BF16, eps1 of the screened basis)"""
    cfg1 = ri.tiny_cell()
    c2 = ri.diamond_cell(4.0)
    g1 = ri.diamond_supercell(rep=(2, 1, 1), mesh_per_cell=20, nocc_per_atom=2, c=4.0, cid=61)
    g2 = ri.diamond_supercell(rep=(1, 1, 2), mesh_per_cell=16, nocc_per_atom=3, c=3.0, cid=64)
    # n = 150 (padded 160): the GEMM form inside the graph
    g3 = dataclasses.replace(ri.diamond_supercell(rep=(2, 1, 1), mesh_per_cell=20, nocc_per_atom=2, c=4.0,
                                                  cid=65), nocc=150)
    return [(cfg1, 0, 0.0), (cfg1, 1, 0.0), (c2, 0, 0.0), (c2, 1, 0.0), (g1, 0, 0.0), (g1, 1, 0.0),
            (g2, 0, 0.0), (g1, 2, 1e-4), (g3, 1, 1e-8)]


@pytest.fixture(scope="module")
def batch_setup(lib):
    import torch
    cells = _cells()
    ctxs, Cs, refs = [], [], []
    pts1 = None
    for w, prec, eps in cells:
        kw = dict(precision=[lib.PREC_FP64, lib.PREC_FP32, lib.PREC_BF16X3][prec], basis_eps=eps)
        if w.name == cells[0][0].name:
            if pts1 is None:
                Phi = basis.eval_basis(w)
                pts1 = isdf.setup(w, Phi)["points"]
            kw["points"] = pts1
        else:
            kw["seed"] = w.sketch_seed()
        ctx = lib.Context.from_workload(w, **kw)
        S = ctx.overlap()
        C = ri.lowdin(ri.random_coefficients(w), S)
        ctxs.append(ctx)
        Cs.append(torch.from_numpy(C).cuda())
        refs.append(C)
    Ks = [torch.empty((w.nbas, w.nocc), dtype=torch.float64, device="cuda") for w, _, _ in cells]
    ex = torch.zeros(len(cells), dtype=torch.float64, device="cuda")
    yield dict(cells=cells, ctxs=ctxs, Cs=Cs, Ks=Ks, ex=ex, Chost=refs, pts1=pts1)
    for c in ctxs:
        c.close()


def test_batch_replays_match_eager(lib, batch_setup):
    import torch
    b = batch_setup
    _say(f"case: batch of {len(b['cells'])} cells, autotuned, graph replays vs eager builds")
    with lib.Batch(b["ctxs"], b["Cs"], b["Ks"], b["ex"], autotune=True) as bat:
        inf = bat.info()
        _say(f"  branches={inf['branches']} create={inf['create_s']:.2f}s replay={inf['replay_ms']:.3f}ms")
        # eager reference with the tuned parameters, into separate buffers
        Ke, Ee = [], []
        for ctx, C in zip(b["ctxs"], b["Cs"]):
            K = torch.empty_like(b["Ks"][len(Ke)])
            e = torch.zeros(1, dtype=torch.float64, device="cuda")
            ctx.build(C, K, e)
            Ke.append(K)
            Ee.append(e)
        torch.cuda.synchronize()
        for rep in range(3):
            for K in b["Ks"]:
                K.fill_(float("nan"))
            b["ex"].fill_(float("nan"))
            bat.run()
            torch.cuda.synchronize()
            for i in range(len(b["cells"])):
                assert torch.equal(b["Ks"][i], Ke[i]), (rep, i)
                assert float(b["ex"][i]) == float(Ee[i][0]), (rep, i)
            # eager work between replays
            b["ctxs"][0].build(b["Cs"][0], Ke[0].clone(), None)
            torch.cuda.synchronize()


def test_batch_cell_against_oracle(lib, batch_setup):
    import torch
    b = batch_setup
    _say("case: batch cell 0 (config 1) against the FP64 oracle")
    w = b["cells"][0][0]
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    st = isdf.setup(w, Phi)
    C = b["Chost"][0]
    Kref, Eref, _ = rps.build_occ(Phi, st["points"], st["V"], st["W"], C, dV)
    with lib.Batch(b["ctxs"][:2], b["Cs"][:2], b["Ks"][:2], b["ex"][:2], autotune=False, branches=2) as bat:
        assert bat.info()["branches"] == 2
        bat.run()
        torch.cuda.synchronize()
    K = b["Ks"][0].cpu().numpy()
    E = float(b["ex"][0])
    assert abs(E - Eref) < 1e-8
    assert np.abs(K - Kref).max() / np.abs(Kref).max() < 1e-7
    E32 = float(b["ex"][1])
    assert abs(E32 - Eref) < 1e-6


def test_autotune_keeps_results(lib):
    """Tuning changes launch shapes, not results beyond rounding."""
    import torch
    _say("case: autotune on config 2 (c = 4)")
    w = ri.diamond_cell(4.0)
    with lib.Context.from_workload(w, seed=w.sketch_seed()) as ctx:
        C = torch.from_numpy(ri.lowdin(ri.random_coefficients(w), ctx.overlap())).cuda()
        K0, _ = ctx.build(C)
        K = torch.empty_like(K0)
        ms = ctx.autotune(C, K)
        K1, _ = ctx.build(C)
        torch.cuda.synchronize()
        _say(f"  tuned build {ms:.3f} ms")
        assert ms > 0
        d = float((K1 - K0).abs().max() / K0.abs().max())
        assert d < 1e-12
