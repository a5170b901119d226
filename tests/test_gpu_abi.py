"""GPU tests of the named C-ABI entry points, called directly through ctypes
with live contexts, and of the set-up's error and retry paths.

- rps_setup_isdf + rps_build_exchange_occRI (host and device pointers) and
  rps_build_exchange_occRI_batched against the FP64 oracle on the config-1
  cell (live oracle) and the config-2 cell at c = 4 (stored oracle results),
  with the oracle's points given to the library: |dE_x| < 1e-8 Ha and
  max|dK| / max|K| < 1e-7.
- The fitting-metric Cholesky retry (Sec. 4.3 names a Cholesky factorisation;
  the shift rule is our reading): more points than the pair-space rank makes
  X_gg singular; library and oracle record the same shift.
- A metric that stays singular after the shift gives RPS_ERR_NOT_PD.
- A captured batch refuses to replay after a context's workspace changed.
- rps_info.build_arith names the arithmetic a build ran.
"""
import ctypes as ct
import os
import sys

import numpy as np
import pytest

import rps_inputs as ri
from oracle import basis, conventional, grid, isdf, rps

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


def _kerr(K, Kref):
    return float(np.abs(K - Kref).max() / np.abs(Kref).max())


class _Raw:
    """Keeps the host arrays of one rps_cell / rps_basis alive for a call."""

    def __init__(self, B, w):
        self.cell = B.Cell()
        self.cell.lattice[:] = list(np.asarray(w.lattice, dtype=np.float64).reshape(9))
        self.cell.mesh[:] = [int(m) for m in w.mesh]
        self.atoms = np.ascontiguousarray(w.atoms, dtype=np.float64)
        self.sa = np.ascontiguousarray(w.shell_atom, dtype=np.int32)
        self.sl = np.ascontiguousarray(w.shell_l, dtype=np.int32)
        self.se = np.ascontiguousarray(w.shell_exp, dtype=np.float64)
        self.basis = B.Basis(int(self.atoms.shape[0]), int(self.sl.shape[0]),
                             self.atoms.ctypes.data_as(ct.POINTER(ct.c_double)),
                             self.sa.ctypes.data_as(ct.POINTER(ct.c_int32)),
                             self.sl.ctypes.data_as(ct.POINTER(ct.c_int32)),
                             self.se.ctypes.data_as(ct.POINTER(ct.c_double)))


def _setup(lib, w, points, precision=0):
    """rps_setup_isdf called directly; returns the raw context handle."""
    B = lib.binding
    raw = _Raw(B, w)
    pts = np.ascontiguousarray(points, dtype=np.int64)
    h = ct.c_void_p()
    st = lib.load().rps_setup_isdf(ct.byref(raw.cell), ct.byref(raw.basis), len(pts), 0, 0, precision,
                                   pts.ctypes.data_as(ct.POINTER(ct.c_int64)), None, ct.byref(h))
    assert st == 0, lib.load().rps_last_error().decode()
    return h


def _info(lib, h):
    inf = lib.binding.Info()
    assert lib.load().rps_get_info(h, ct.byref(inf)) == 0
    return inf.as_dict()


@pytest.fixture(scope="module")
def refs():
    """(workload, points, C, K_ref, E_ref) for the config-1 cell (live oracle)
    and the config-2 cell at c = 4 (stored oracle results)."""
    w1 = ri.tiny_cell()
    Phi = basis.eval_basis(w1)
    dV = grid.dvol(w1.lattice, w1.mesh)
    C1 = ri.lowdin(ri.random_coefficients(w1), basis.overlap(Phi, dV))
    st = isdf.setup(w1, Phi, owner=basis.voronoi(w1))
    K1, E1, _ = rps.build_occ(Phi, st["points"], st["V"], st["W"], C1, dV)
    g = np.load(os.path.join(GOLDEN, "diamond1x1x1_c4.npz"))
    w2 = ri.diamond_cell(4.0)
    return [(w1, st["points"], C1, K1, E1), (w2, g["points"], g["C"], g["K"], float(g["E"]))]


def test_named_setup_and_build_host_and_device(lib, refs):
    import torch
    L = lib.load()
    for w, pts, C, Kref, Eref in refs:
        _say(f"case: rps_setup_isdf + rps_build_exchange_occRI on {w.name}")
        h = _setup(lib, w, pts)
        try:
            out = np.empty((w.nbas, w.nocc))
            pts_back = np.empty(len(pts), dtype=np.int64)
            assert L.rps_get_points(h, pts_back.ctypes.data) == 0
            assert np.array_equal(pts_back, pts)
            Cc = np.ascontiguousarray(C)
            e = ct.c_double(0.0)
            assert L.rps_build_exchange_occRI(h, w.nocc, Cc.ctypes.data, out.ctypes.data, ct.addressof(e),
                                              lib.PTRS_HOST, None) == 0
            _say(f"  host: dE={e.value - Eref:.3e} dK={_kerr(out, Kref):.3e}")
            assert abs(e.value - Eref) < 1e-8 and _kerr(out, Kref) < 1e-7
            assert _info(lib, h)["build_arith"] == lib.PREC_FP64
            Cd = torch.from_numpy(Cc).cuda()
            Kd = torch.full((w.nbas, w.nocc), float("nan"), dtype=torch.float64, device="cuda")
            exd = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
            stream = torch.cuda.current_stream().cuda_stream
            assert L.rps_build_exchange_occRI(h, w.nocc, Cd.data_ptr(), Kd.data_ptr(), exd.data_ptr(),
                                              lib.PTRS_DEVICE, stream) == 0
            torch.cuda.synchronize()
            assert np.array_equal(Kd.cpu().numpy(), out) and float(exd.item()) == e.value
            eh = ct.c_double(0.0)
            assert L.rps_exchange_energy(w.nbas, w.nocc, Cc.ctypes.data, out.ctypes.data, ct.byref(eh)) == 0
            assert abs(eh.value - e.value) < 1e-10
        finally:
            L.rps_destroy(h)


def test_batched_entry_point(lib, refs):
    """rps_build_exchange_occRI_batched over two cells of different sizes, with
    host pointers and with device pointers, each cell against the oracle."""
    import torch
    L = lib.load()
    _say("case: rps_build_exchange_occRI_batched, config 1 + config 2 (c = 4)")
    hs = [_setup(lib, w, pts) for w, pts, _, _, _ in refs]
    try:
        nb = len(refs)
        H = (ct.c_void_p * nb)(*[h.value for h in hs])
        nocc = (ct.c_int32 * nb)(*[w.nocc for w, *_ in refs])
        Ch = [np.ascontiguousarray(r[2]) for r in refs]
        Kh = [np.empty((w.nbas, w.nocc)) for w, *_ in refs]
        exh = np.full(nb, np.nan)
        st = L.rps_build_exchange_occRI_batched(H, nb, nocc, (ct.c_void_p * nb)(*[c.ctypes.data for c in Ch]),
                                                (ct.c_void_p * nb)(*[k.ctypes.data for k in Kh]),
                                                exh.ctypes.data, lib.PTRS_HOST, None)
        assert st == 0, L.rps_last_error().decode()
        for (w, _, _, Kref, Eref), K, E in zip(refs, Kh, exh):
            _say(f"  host {w.name}: dE={E - Eref:.3e} dK={_kerr(K, Kref):.3e}")
            assert abs(E - Eref) < 1e-8 and _kerr(K, Kref) < 1e-7
        Cd = [torch.from_numpy(c).cuda() for c in Ch]
        Kd = [torch.full(k.shape, float("nan"), dtype=torch.float64, device="cuda") for k in Kh]
        exd = torch.full((nb,), float("nan"), dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        st = L.rps_build_exchange_occRI_batched(H, nb, nocc, (ct.c_void_p * nb)(*[c.data_ptr() for c in Cd]),
                                                (ct.c_void_p * nb)(*[k.data_ptr() for k in Kd]),
                                                exd.data_ptr(), lib.PTRS_DEVICE, stream)
        assert st == 0, L.rps_last_error().decode()
        torch.cuda.synchronize()
        for i in range(nb):
            assert np.array_equal(Kd[i].cpu().numpy(), Kh[i])
            assert float(exd[i]) == exh[i]
    finally:
        for h in hs:
            L.rps_destroy(h)


def test_cholesky_shift_retry(lib):
    """24 points for 3 s functions (pair-space rank 6): X_gg is singular, the
    plain factorisation fails and the retry with 1e-13 max diag(X_gg) runs in
    both library and oracle.  The fit then reproduces every pair product, so
    rPS equals exact exchange; the build must match the oracle."""
    _say("case: fitting-metric Cholesky retry (24 points, pair rank 6)")
    w = ri.tiny_s_cell(3, 8, 4.0, 2, 24, cid=91)
    Phi = basis.eval_basis(w)
    dV = grid.dvol(w.lattice, w.mesh)
    C = ri.lowdin(ri.random_coefficients(w), basis.overlap(Phi, dV))
    pts = np.random.default_rng(3).choice(w.ngrid, 24, replace=False)
    st = isdf.setup(w, Phi, points=pts)
    Kref, Eref, _ = rps.build_occ(Phi, pts, st["V"], st["W"], C, dV)
    Kc, Ec = conventional.exchange_occ(Phi, C, w.lattice, w.mesh)
    assert st["shift"] > 0
    with lib.Context.from_workload(w, points=pts) as ctx:
        shift = ctx.info()["chol_shift"]
        K, E = ctx.build(C)
    _say(f"  shift lib {shift:.6e} oracle {st['shift']:.6e}; dE={E - Eref:.3e} dK={_kerr(K, Kref):.3e} "
         f"E-E_conv={E - Ec:.3e}")
    assert shift > 0 and abs(shift - st["shift"]) < 1e-10 * st["shift"]
    assert abs(E - Eref) < 1e-8 and _kerr(K, Kref) < 1e-7


def test_not_positive_definite_error(lib):
    """Screening every basis value away (eps1 far above any pSinc coefficient)
    leaves X_gg = 0: its largest diagonal is 0, so the shift is 0 and the
    retry fails too.  The set-up returns RPS_ERR_NOT_PD and no context."""
    _say("case: RPS_ERR_NOT_PD from a vanishing fitting metric")
    w = ri.tiny_s_cell(3, 8, 4.0, 2, 10, cid=91)
    with pytest.raises(lib.RpsError) as ei:
        lib.Context.from_workload(w, points=np.arange(0, 500, 50), basis_eps=1e30)
    assert ei.value.status == lib.RPS_ERR_NOT_PD
    _say(f"  {ei.value}")


def test_batch_refuses_stale_workspace(lib):
    """A batch graph holds each context's workspace addresses.  After
    rps_autotune reallocates a context's workspace, rps_batch_run returns
    RPS_ERR_STATE (checked on the host, nothing is launched); a new batch over
    the same contexts replays again and matches an eager build."""
    import torch
    _say("case: batch replay after a context's workspace changed")
    w = ri.tiny_cell()
    with lib.Context.from_workload(w, seed=w.sketch_seed()) as ctx:
        C = torch.from_numpy(ri.lowdin(ri.random_coefficients(w), ctx.overlap())).cuda()
        K = torch.empty((w.nbas, w.nocc), dtype=torch.float64, device="cuda")
        ex = torch.zeros(1, dtype=torch.float64, device="cuda")
        with lib.Batch([ctx], [C], [K], ex, autotune=False, branches=1) as bat:
            bat.run()
            torch.cuda.synchronize()
            ctx.autotune(C, torch.empty_like(K))
            with pytest.raises(lib.RpsError) as ei:
                bat.run()
            assert ei.value.status == lib.RPS_ERR_STATE
            _say(f"  {ei.value}")
        Ke = torch.empty_like(K)
        ctx.build(C, Ke)
        with lib.Batch([ctx], [C], [K], ex, autotune=False, branches=1) as bat:
            K.fill_(float("nan"))
            bat.run()
            torch.cuda.synchronize()
        assert torch.equal(K, Ke)


def test_build_arith_reported(lib, refs):
    """A split-BF16 context on the config-1 cell (n = 8) runs the FP32 fused
    kernel; rps_info says so."""
    w, pts, C, Kref, Eref = refs[0]
    _say("case: build_arith of a split-BF16 context on the fused path")
    with lib.Context.from_workload(w, points=pts, precision=lib.PREC_BF16X3) as ctx:
        assert ctx.info()["build_arith"] == -1
        K, E = ctx.build(C)
        assert ctx.info()["build_arith"] == lib.PREC_FP32
    assert abs(E - Eref) < 1e-6


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_setup_from_potentials_matches_setup(lib, refs, prec):
    """rps_setup_isdf_from_potentials given the V and W a regular set-up made
    (host arrays, then device tensors) builds exactly what that set-up builds;
    the FP32 form is given V rounded to FP32 as its store holds it."""
    import torch
    w, pts, C, Kref, Eref = refs[0]
    p = lib.PREC_FP64 if prec == "fp64" else lib.PREC_FP32
    _say(f"case: set-up from given potentials, {prec}, {w.name}")
    with lib.Context.from_workload(w, points=pts) as c64:
        V = c64.array(1)
        W = c64.array(2)
    with lib.Context.from_workload(w, points=pts, precision=p) as ref:
        K0, E0 = ref.build(C)
    Vg = V if p == lib.PREC_FP64 else V.astype(np.float32)
    for dev in (False, True):
        Vin = torch.from_numpy(Vg).cuda() if dev else Vg
        Win = torch.from_numpy(W).cuda() if dev else W
        with lib.Context.from_potentials(w, pts, Vin, Win, precision=p) as ctx:
            assert np.array_equal(ctx.points(), pts)
            K1, E1 = ctx.build(C)
        _say(f"  {'device' if dev else 'host'} inputs: dE={E1 - E0:.3e} dK={_kerr(K1, K0):.3e}")
        assert np.array_equal(K1, K0) and E1 == E0
    assert abs(E0 - Eref) < (1e-8 if p == lib.PREC_FP64 else 1e-6)
