"""The no-allocation build (rps_build_exchange_occRI_noalloc) against the
regular build (rps_build_exchange_occRI) on the same contexts, through the C
ABI with device pointers.

Calls in a row on one device share the library's static scratch, each later
call with a smaller input than the one before it in each precision (the 48^3
cell, then the 24^3 cell), FP64 and FP32 contexts.  Each result must meet the
oracle bar against the regular build (FP64: |dE_x| < 1e-8 Ha, max|dK|/max|K|
< 1e-7; FP32 context: the same, since both run the same kernels) and is in
fact identical to it (same plan, same kernels, fixed summation order).  A
context that never built (no workspace of its own) is built with it and device
free memory must not change.  Sizes beyond the scratch, and contexts off the
fused path, are refused on the host before any launch.
"""
import dataclasses
import os
import sys

import numpy as np
import pytest

import rps_inputs as ri
from oracle import basis, grid, isdf, rps

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2207_04636_amd as P
    P.load()
    return P


@pytest.fixture(scope="module")
def cells():
    """(workload, points, C, K_oracle, E_oracle): the 48^3 cell at c = 6 (stored
    oracle results), the 24^3 config-1 cell (live oracle)."""
    g = np.load(os.path.join(GOLDEN, "diamond1x1x1_c6.npz"))
    w2 = ri.diamond_cell(6.0)
    w1 = ri.tiny_cell()
    Phi = basis.eval_basis(w1)
    dV = grid.dvol(w1.lattice, w1.mesh)
    C1 = ri.lowdin(ri.random_coefficients(w1), basis.overlap(Phi, dV))
    st = isdf.setup(w1, Phi, owner=basis.voronoi(w1))
    K1, E1, _ = rps.build_occ(Phi, st["points"], st["V"], st["W"], C1, dV)
    return [(w2, g["points"], g["C"], g["K"], float(g["E"])), (w1, st["points"], C1, K1, E1)]


def _kerr(K, Kref):
    return float(np.abs(K - Kref).max() / np.abs(Kref).max())


def _raw_noalloc(lib, ctx, Cd, Kd, exd):
    import torch
    L = lib.load()
    st = L.rps_build_exchange_occRI_noalloc(ctx._h, int(Cd.shape[1]), Cd.data_ptr(), Kd.data_ptr(),
                                            exd.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return st, L.rps_last_error().decode()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_regular_build(lib, cells, prec):
    import torch
    p = lib.PREC_FP64 if prec == "fp64" else lib.PREC_FP32
    bar_e = 1e-8 if prec == "fp64" else 1e-6
    for w, pts, C, Kref, Eref in cells:              # larger cell first, then the smaller one
        _say(f"case: no-allocation build, {prec}, {w.name}")
        Cd = torch.from_numpy(np.ascontiguousarray(C)).cuda()
        Kn = torch.full((w.nbas, w.nocc), float("nan"), dtype=torch.float64, device="cuda")
        exn = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        with lib.Context.from_workload(w, points=pts, precision=p) as warm:
            st, msg = _raw_noalloc(lib, warm, Cd, Kn, exn)      # loads the kernels' code on first use
            assert st == 0, msg
        with lib.Context.from_workload(w, points=pts, precision=p) as ctx:
            # a context without any workspace of its own: device free memory must not move
            # (a regular first build would allocate its workspace, megabytes at these sizes)
            Kn.fill_(float("nan"))
            exn.fill_(float("nan"))
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            st, msg = _raw_noalloc(lib, ctx, Cd, Kn, exn)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            assert st == 0, msg
            assert free0 - free1 < (1 << 20), (free0, free1)
            # the regular entry point on the same context
            Kr = torch.full_like(Kn, float("nan"))
            exr = torch.full_like(exn, float("nan"))
            ctx.build(Cd, Kr, exr)
            torch.cuda.synchronize()
            Kn_h, Kr_h = Kn.cpu().numpy(), Kr.cpu().numpy()
            En, Er = float(exn.item()), float(exr.item())
            _say(f"  noalloc vs regular: dE={En - Er:.3e} dK={_kerr(Kn_h, Kr_h):.3e}; "
                 f"vs oracle dE={En - Eref:.3e} dK={_kerr(Kn_h, Kref):.3e}; free memory change {free0 - free1} B")
            assert abs(En - Er) < bar_e and _kerr(Kn_h, Kr_h) < 1e-7
            assert np.array_equal(Kn_h, Kr_h) and En == Er
            assert abs(En - Eref) < bar_e
            # a second no-allocation call on the same context after the regular one
            Kn.fill_(float("nan"))
            st, msg = _raw_noalloc(lib, ctx, Cd, Kn, exn)
            torch.cuda.synchronize()
            assert st == 0, msg
            assert torch.equal(Kn, Kr) and float(exn.item()) == Er


def test_noalloc_refuses_what_it_cannot_hold(lib, cells):
    import torch
    w2 = cells[0][0]
    # n = 64 on the 48^3 cell: the fused path, but its workspace is above the static maximum
    big = dataclasses.replace(w2, nocc=64)
    _say("case: no-allocation build refuses a workspace above its maximum and the general path")
    with lib.Context.from_workload(big, points=cells[0][1]) as ctx:
        C = torch.from_numpy(ri.lowdin(ri.random_coefficients(big), ctx.overlap())).cuda()
        K = torch.full((big.nbas, big.nocc), float("nan"), dtype=torch.float64, device="cuda")
        ex = torch.zeros(1, dtype=torch.float64, device="cuda")
        st, msg = _raw_noalloc(lib, ctx, C, K, ex)
        _say(f"  {msg}")
        assert st == lib.RPS_ERR_SHAPE and "scratch" in msg
        assert torch.isnan(K).all()                   # outputs untouched
    # n = 32 in the FP32 form runs the general (streaming) path: refused
    mid = dataclasses.replace(w2, nocc=32)
    with lib.Context.from_workload(mid, points=cells[0][1], precision=lib.PREC_FP32) as ctx:
        C = torch.zeros((mid.nbas, mid.nocc), dtype=torch.float64, device="cuda")
        K = torch.full((mid.nbas, mid.nocc), float("nan"), dtype=torch.float64, device="cuda")
        ex = torch.zeros(1, dtype=torch.float64, device="cuda")
        st, msg = _raw_noalloc(lib, ctx, C, K, ex)
        _say(f"  {msg}")
        assert st == lib.RPS_ERR_SHAPE and "fused path" in msg
        assert torch.isnan(K).all()
