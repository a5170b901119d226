"""GPU parity of the general-size build against the FP64 oracle.

The general path covers any N and n: the streaming form (two passes over V,
one per output of Eq. 16 lines 1-2, plus the fit-fit line on W) for padded
n <= 128, and the GEMM form (A = V o P materialised in chunks) above it.  The
cases below are diamond-like supercells on coarse grids, sized so the oracle
finishes in seconds while the GPU kernels see several workgroups, ragged x
blocks (N_aux and N_g not multiples of the 128-row block), ragged n (padding
to 16), every orbital block count used by configs 3 and 5, and n above the
streaming form's limit (the GEMM form of config 4).

Bars with shared interpolation points: FP64 |dE_x| < 1e-8 Ha and
max|dK|/max|K| < 1e-7; FP32 form |dE_x| < 1e-6 Ha with the K error reported
(bounded at 1e-4)."""
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


CASES = {
    # N = 208, n = 32 (two 16-column blocks), N_g = 40 x 20 x 20
    "2x1x1-n32": dict(rep=(2, 1, 1), mesh_per_cell=20, nocc_per_atom=2, c=4.0, cid=61),
    # N = 208, n = 40 (padded to 48), N_aux = 5N
    "2x1x1-n40": dict(rep=(2, 1, 1), mesh_per_cell=20, nocc_per_atom=2, c=5.0, cid=62, nocc=40),
    # N = 416, n = 128 (eight blocks, the config-3 shape), N_g = 32 x 32 x 16
    "2x2x1-n128": dict(rep=(2, 2, 1), mesh_per_cell=16, nocc_per_atom=4, c=4.0, cid=63),
    # N = 208, n = 150 (padded to 160, above the streaming form: the GEMM form, as config 4)
    "2x1x1-n150": dict(rep=(2, 1, 1), mesh_per_cell=20, nocc_per_atom=2, c=4.0, cid=64, nocc=150),
}


def _workload(name):
    kw = dict(CASES[name])
    nocc = kw.pop("nocc", None)
    w = ri.diamond_supercell(**kw)
    if nocc is not None:
        w = dataclasses.replace(w, nocc=nocc)
    return w


_cache = {}


def _case(name):
    if name not in _cache:
        w = _workload(name)
        Phi = basis.eval_basis(w)
        dV = grid.dvol(w.lattice, w.mesh)
        C = ri.lowdin(ri.random_coefficients(w), basis.overlap(Phi, dV))
        st = isdf.setup(w, Phi)
        K, E, _ = rps.build_occ(Phi, st["points"], st["V"], st["W"], C, dV)
        args = (Phi, st["points"], st["V"], st["W"], C, dV)
        _cache[name] = dict(w=w, C=C, points=st["points"], K=K, E=E, args=args)
    return _cache[name]


@pytest.fixture(scope="module")
def lib():
    import paper_2207_04636_amd as P
    P.load()
    return P


def _kerr(K, Kref):
    return float(np.abs(K - Kref).max() / np.abs(Kref).max())


@pytest.mark.parametrize("name", list(CASES))
def test_general_fp64(lib, name):
    _say(f"case: general FP64 {name}")
    cs = _case(name)
    w = cs["w"]
    with lib.Context.from_workload(w, points=cs["points"]) as ctx:
        K, E = ctx.build(cs["C"])
        K2, E2 = ctx.build(cs["C"])
    dk = _kerr(K, cs["K"])
    _say(f"  N={w.nbas} n={w.nocc} Ng={w.ngrid} Naux={w.naux}: dE={E - cs['E']:.3e} dK={dk:.3e}")
    assert abs(E - cs["E"]) < 1e-8
    assert dk < 1e-7
    assert np.array_equal(K, K2) and E == E2
    CK = cs["C"].T @ K
    assert np.abs(CK - CK.T).max() < 1e-10 * np.abs(CK).max()


@pytest.mark.parametrize("name", list(CASES))
def test_general_fp32(lib, name):
    _say(f"case: general FP32 form {name}")
    cs = _case(name)
    with lib.Context.from_workload(cs["w"], points=cs["points"], precision=lib.PREC_FP32) as ctx:
        K, E = ctx.build(cs["C"])
    dk = _kerr(K, cs["K"])
    _say(f"  FP32 form: dE={E - cs['E']:.3e} max|dK|/max|K|={dk:.3e}")
    assert abs(E - cs["E"]) < 1e-6
    assert dk < 1e-4


@pytest.mark.parametrize("name", list(CASES))
def test_general_bf16x3(lib, name):
    """Split-BF16 products (a_hi b_hi + a_hi b_lo + a_lo b_hi, FP32 accumulation
    within a tile, FP64 across tiles) on the streaming passes."""
    _say(f"case: general split-BF16 form {name}")
    cs = _case(name)
    with lib.Context.from_workload(cs["w"], points=cs["points"], precision=lib.PREC_BF16X3) as ctx:
        K, E = ctx.build(cs["C"])
        assert ctx.info()["precision"] == lib.PREC_BF16X3
    dk = _kerr(K, cs["K"])
    _say(f"  BF16x3 form: dE={E - cs['E']:.3e} max|dK|/max|K|={dk:.3e}")
    assert abs(E - cs["E"]) < 1e-6
    assert dk < 1e-4


@pytest.mark.parametrize("variant", ["ps", "thc"])
def test_general_variants(lib, variant):
    _say(f"case: general {variant} 2x1x1-n40")
    cs = _case("2x1x1-n40")
    Kref, Eref = rps.ps_occ(*cs["args"]) if variant == "ps" else rps.thc_occ(*cs["args"])
    v = lib.VARIANT_PS if variant == "ps" else lib.VARIANT_THC
    with lib.Context.from_workload(cs["w"], points=cs["points"]) as ctx:
        K, E = ctx.build(cs["C"], variant=v)
    assert abs(E - Eref) < 1e-8
    assert _kerr(K, Kref) < 1e-7


def test_full_exchange_general(lib):
    """Full K_{mu nu} for N = 208 (N > 128) against the oracle; K_full C = K_occ."""
    _say("case: full exchange matrix 2x1x1-n32")
    cs = _case("2x1x1-n32")
    Kref = rps.build_full(*cs["args"])
    with lib.Context.from_workload(cs["w"], points=cs["points"]) as ctx:
        Kf = ctx.build_full(cs["C"])
        Ko, _ = ctx.build(cs["C"])
    assert _kerr(Kf, Kref) < 1e-7
    assert np.abs(Kf - Kf.T).max() < 1e-12 * np.abs(Kf).max()
    assert _kerr(Kf @ cs["C"], Ko) < 1e-10


@pytest.mark.parametrize("name,prec,rchunk", [
    ("2x1x1-n32", "fp64", None), ("2x1x1-n32", "fp32", None), ("2x1x1-n32", "bf16x3", None),
    ("2x1x1-n40", "fp64", 1000), ("2x1x1-n40", "fp32", 1000), ("2x1x1-n150", "fp32", 3333),
])
def test_gemm_form(lib, monkeypatch, name, prec, rchunk):
    """The GEMM form (used for padded n > 128) forced onto smaller n, and with
    grid chunks that do not divide N_g (rchunk columns, last chunk ragged).  The
    precision forms run its three chunk products on the FP32 matrix cores."""
    _say(f"case: general GEMM form {name} {prec} chunk={rchunk}")
    monkeypatch.setenv("RPS_GENERAL_GEMM", "1")
    if rchunk is not None:
        monkeypatch.setenv("RPS_GEMM_RCHUNK", str(rchunk))
    cs = _case(name)
    p = {"fp64": lib.PREC_FP64, "fp32": lib.PREC_FP32, "bf16x3": lib.PREC_BF16X3}[prec]
    with lib.Context.from_workload(cs["w"], points=cs["points"], precision=p) as ctx:
        K, E = ctx.build(cs["C"])
        K2, E2 = ctx.build(cs["C"])
    tol_e, tol_k = (1e-8, 1e-7) if prec == "fp64" else (1e-6, 1e-4)
    _say(f"  dE={E - cs['E']:.3e} dK={_kerr(K, cs['K']):.3e}")
    assert abs(E - cs["E"]) < tol_e
    assert _kerr(K, cs["K"]) < tol_k
    assert np.array_equal(K, K2) and E == E2


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stream_form_on_small_cell(lib, monkeypatch, prec):
    """Config 1 (n = 8, one orbital block) forced onto the general path."""
    _say(f"case: config-1 on the general path, {prec}")
    monkeypatch.setenv("RPS_BUILD_PATH", "general")
    w = ri.tiny_cell()
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    C = ri.lowdin(ri.random_coefficients(w), basis.overlap(Phi, dV))
    st = isdf.setup(w, Phi)
    Kref, Eref, _ = rps.build_occ(Phi, st["points"], st["V"], st["W"], C, dV)
    p = lib.PREC_FP64 if prec == "fp64" else lib.PREC_FP32
    with lib.Context.from_workload(w, points=st["points"], precision=p) as ctx:
        K, E = ctx.build(C)
    tol_e, tol_k = (1e-8, 1e-7) if prec == "fp64" else (1e-6, 1e-4)
    _say(f"  dE={E - Eref:.3e} dK={_kerr(K, Kref):.3e}")
    assert abs(E - Eref) < tol_e
    assert _kerr(K, Kref) < tol_k
