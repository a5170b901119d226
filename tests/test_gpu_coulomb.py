"""GPU parity of the Coulomb matrix build (rps_build_coulomb) and of the
Madelung term of the exchange (rps_madelung_correct, Sec. 4.5) against the FP64
oracle (Sec. 2.3, steps 1-4).

Every step runs in FP64 on both sides; they differ only in summation order
(the oracle's FFT against the library's direct per-axis transforms, numpy's
products against the matrix cores), so the bar is max|dJ|/max|J| < 1e-11
and |dE_J| < 1e-11 |E_J|.  Cases span one to several output tiles, ragged
N (not a multiple of the 128-wide tile), ragged n (padding to 16), n = 1,
and the precision form of the context (J stays FP64 there)."""
import dataclasses
import sys

import numpy as np
import pytest

import rps_inputs as ri
from oracle import basis, coulomb, grid, madelung

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2207_04636_amd as P
    P.load()
    return P


def _cases():
    return {
        "config1": (ri.tiny_cell(), None),
        "config2-c4": (ri.diamond_cell(4.0), None),
        "config2-n5": (ri.diamond_cell(4.0), 5),
        "config2-n1": (ri.diamond_cell(4.0), 1),
        "2x1x1-n40": (ri.diamond_supercell(rep=(2, 1, 1), mesh_per_cell=20, nocc_per_atom=2, c=4.0, cid=62), 40),
        "2x2x1-n128": (ri.diamond_supercell(rep=(2, 2, 1), mesh_per_cell=16, nocc_per_atom=4, c=4.0, cid=63), None),
    }


def _rel(J, Jref):
    return float(np.abs(J - Jref).max() / np.abs(Jref).max())


@pytest.mark.parametrize("name", list(_cases()) + ["config2-c4-gemm"])
def test_coulomb_against_oracle(lib, name, monkeypatch):
    """Bases with N <= 128 and n <= 64 take the one-pass small-basis kernels; the
    others (and "-gemm", forced) the chunked GEMM path."""
    if name.endswith("-gemm"):
        monkeypatch.setenv("RPS_COULOMB_GEMM", "1")
        name = name[: -len("-gemm")]
    w, nocc = _cases()[name]
    if nocc is not None:
        w = dataclasses.replace(w, nocc=nocc)
    _say(f"case: Coulomb {name} N={w.nbas} n={w.nocc} Ng={w.ngrid}")
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    C = ri.lowdin(ri.random_coefficients(w), basis.overlap(Phi, dV))
    Jref, Eref, _ = coulomb.build_j(Phi, C, w.lattice, w.mesh)
    with lib.Context.from_workload(w, seed=w.sketch_seed()) as ctx:
        J, E = ctx.build_coulomb(C)
        J2, E2 = ctx.build_coulomb(C)
    _say(f"  dE_J={E - Eref:.3e} (E_J={Eref:.8f}) max|dJ|/max|J|={_rel(J, Jref):.3e}")
    assert _rel(J, Jref) < 1e-11
    assert abs(E - Eref) < 1e-11 * abs(Eref)
    assert np.array_equal(J, J.T)
    assert np.array_equal(J, J2) and E == E2


def test_coulomb_device_pointers_and_precision_form(lib):
    """Device-pointer calls equal host calls bit for bit; a context in the
    FP32 precision form gives the same J (J does not read V)."""
    import torch
    w = ri.diamond_cell(4.0)
    _say("case: Coulomb config 2, device pointers and FP32 context")
    with lib.Context.from_workload(w, seed=w.sketch_seed()) as ctx:
        C = ri.lowdin(ri.random_coefficients(w), ctx.overlap())
        Jh, Eh = ctx.build_coulomb(C)
        Cd = torch.from_numpy(C).cuda()
        Jd = torch.full((w.nbas, w.nbas), float("nan"), dtype=torch.float64, device="cuda")
        ed = torch.zeros(1, dtype=torch.float64, device="cuda")
        ctx.build_coulomb(Cd, Jd, ed)
        ctx.build_coulomb(Cd, Jd, None)
        torch.cuda.synchronize()
        assert np.array_equal(Jd.cpu().numpy(), Jh) and float(ed[0]) == Eh
        pts = ctx.points()
    with lib.Context.from_workload(w, points=pts, precision=lib.PREC_FP32) as ctx:
        J32, E32 = ctx.build_coulomb(C)
    assert np.array_equal(J32, Jh) and E32 == Eh


@pytest.mark.parametrize("name", ["config1", "config2-c4"])
def test_madelung_correction_against_oracle(lib, name):
    """K + M S C and E - M tr(C^T S C) on the library's exchange outputs, against
    the oracle's correction of the same K and E with its own S and M."""
    import torch
    w, _ = _cases()[name]
    _say(f"case: Madelung term {name}")
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    S = basis.overlap(Phi, dV)
    C = ri.lowdin(ri.random_coefficients(w), S)
    M = madelung.madelung(w.lattice)
    with lib.Context.from_workload(w, seed=w.sketch_seed()) as ctx:
        assert abs(ctx.info()["madelung"] - M) < 1e-13 * M
        K, E = ctx.build(C)
        Kc, Ec = ctx.madelung_correct(C, K, E)
        Kref, Eref = madelung.correct(K, E, C, S, M)
        # a second call, device pointers, in place (the overlap formed by the first is kept)
        Cd = torch.from_numpy(C).cuda()
        Kd = torch.from_numpy(K).cuda()
        ed = torch.tensor([E], dtype=torch.float64, device="cuda")
        ctx.madelung_correct(Cd, Kd, ed)
        torch.cuda.synchronize()
        Kd1, ed1 = Kd.cpu().numpy(), float(ed[0])
    _say(f"  M={M:.10f} dE={Ec - Eref:.3e} dK={np.abs(Kc - Kref).max() / np.abs(Kref).max():.3e}")
    assert abs(Ec - Eref) < 1e-12 * abs(Eref)
    assert np.abs(Kc - Kref).max() < 1e-12 * np.abs(Kref).max()
    assert abs((E - Ec) - C.shape[1] * M) < 1e-10
    assert np.array_equal(Kd1, Kc) and ed1 == Ec

