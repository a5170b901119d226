"""CPU checks of the C ABI library: it loads, exports every function that
include/rps.h declares, and rejects bad arguments before touching a device."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import paper_2207_04636_amd as P
from paper_2207_04636_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rps.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rps_\w+)\s*\(", txt)))


def test_header_and_exports_agree():
    decl = _declared()
    assert "rps_setup_isdf" in decl and "rps_build_exchange_occRI" in decl and "rps_exchange_energy" in decl
    assert sorted(P.EXPORTS) == decl
    lib = P.load()
    for name in decl:
        assert hasattr(lib, name), name
        # every entry point that takes arguments has them declared (ctypes would
        # otherwise pass 64-bit pointers as 32-bit ints)
        if name not in ("rps_abi_version", "rps_last_error"):
            assert getattr(lib, name).argtypes, name
    assert lib.rps_abi_version() == 1


def test_exchange_energy_host():
    rg = np.random.default_rng(0)
    C = rg.standard_normal((7, 3))
    K = rg.standard_normal((7, 3))
    assert abs(P.exchange_energy(C, K) + np.sum(C * K)) < 1e-14


def _setup_status(**over):
    lib = P.load()
    cell = B.Cell()
    cell.lattice[:] = list(np.eye(3).reshape(9) * 5.0)
    cell.mesh[:] = [8, 8, 8]
    atoms = np.array([[0.0, 0, 0], [2.0, 2, 2]])
    sa = np.array([0, 1], dtype=np.int32)
    sl = np.array([0, 1], dtype=np.int32)
    se = np.array([1.0, 0.7])
    for k, v in over.items():
        if k == "lattice":
            cell.lattice[:] = list(np.asarray(v, float).reshape(9))
        elif k == "mesh":
            cell.mesh[:] = v
        elif k == "sl":
            sl = np.asarray(v, dtype=np.int32)
        elif k == "se":
            se = np.asarray(v, float)
        elif k == "sa":
            sa = np.asarray(v, dtype=np.int32)
    b = B.Basis(2, len(sl), atoms.ctypes.data_as(ct.POINTER(ct.c_double)), sa.ctypes.data_as(ct.POINTER(ct.c_int32)),
                sl.ctypes.data_as(ct.POINTER(ct.c_int32)), se.ctypes.data_as(ct.POINTER(ct.c_double)))
    naux = over.get("naux", 10)
    pts = over.get("points")
    pp = None
    if pts is not None:
        pts = np.asarray(pts, dtype=np.int64)
        pp = pts.ctypes.data_as(ct.POINTER(ct.c_int64))
    h = ct.c_void_p()
    if "eps" in over:
        st = lib.rps_setup_isdf_screened(ct.byref(cell), ct.byref(b), naux, 1, over.get("mode", 0),
                                         over.get("prec", 0), pp, over["eps"], None, ct.byref(h))
    else:
        st = lib.rps_setup_isdf(ct.byref(cell), ct.byref(b), naux, 1, over.get("mode", 0), over.get("prec", 0), pp,
                                None, ct.byref(h))
    return st, lib.rps_last_error().decode(), h


@pytest.mark.parametrize("over,status", [
    (dict(lattice=np.zeros((3, 3))), B.RPS_ERR_ARG),
    (dict(mesh=[8, 1, 8]), B.RPS_ERR_SHAPE),
    (dict(mesh=[8, 8, 257]), B.RPS_ERR_SHAPE),
    (dict(sl=[0, 3]), B.RPS_ERR_ARG),
    (dict(se=[1.0, -1.0]), B.RPS_ERR_ARG),
    (dict(sa=[0, 5]), B.RPS_ERR_ARG),
    (dict(naux=0), B.RPS_ERR_SHAPE),
    (dict(naux=513), B.RPS_ERR_SHAPE),
    (dict(naux=3, points=[1, 2, 1]), B.RPS_ERR_SHAPE),
    (dict(naux=3, points=[1, 2, 512]), B.RPS_ERR_SHAPE),
    (dict(prec=7), B.RPS_ERR_ARG),
    (dict(mode=5), B.RPS_ERR_ARG),
    (dict(eps=-1e-8), B.RPS_ERR_ARG),
    (dict(eps=float("nan")), B.RPS_ERR_ARG),
    (dict(eps=float("inf")), B.RPS_ERR_ARG),
])
def test_setup_rejects_bad_arguments(over, status):
    st, msg, h = _setup_status(**over)
    assert st == status, msg
    assert msg and h.value is None


def test_calls_without_context_fail_cleanly():
    lib = P.load()
    K = np.zeros((2, 2))
    C = np.zeros((2, 2))
    assert lib.rps_build_exchange_occRI(None, 2, C.ctypes.data, K.ctypes.data, None, 0, None) == B.RPS_ERR_ARG
    assert "ctx" in lib.rps_last_error().decode()
    assert lib.rps_get_points(None, None) == B.RPS_ERR_ARG
    assert lib.rps_build_coulomb(None, 2, C.ctypes.data, K.ctypes.data, None, 0, None) == B.RPS_ERR_ARG
    assert "ctx" in lib.rps_last_error().decode()
    lib.rps_destroy(None)


def test_batch_and_tuner_argument_errors():
    """The batching form and the autotuner reject bad arguments before any
    device work (no GPU is touched on these paths)."""
    import ctypes as ct
    lib = P.load()
    C = np.zeros((2, 2))
    assert lib.rps_autotune(None, 2, C.ctypes.data, C.ctypes.data, None, None, None) == B.RPS_ERR_ARG
    out = ct.c_void_p(123)
    H = (ct.c_void_p * 1)(None)
    nocc = (ct.c_int32 * 1)(2)
    Cp = (ct.c_void_p * 1)(C.ctypes.data)
    Kp = (ct.c_void_p * 1)(C.ctypes.data)
    assert lib.rps_batch_create(H, 1, nocc, Cp, Kp, None, 0, None, ct.byref(out)) == B.RPS_ERR_ARG
    assert out.value is None                       # cleared on failure
    assert "NULL" in lib.rps_last_error().decode()
    assert lib.rps_batch_create(H, 0, nocc, Cp, Kp, None, 0, None, ct.byref(out)) == B.RPS_ERR_ARG
    assert lib.rps_batch_create(H, 1, nocc, Cp, Kp, None, 1 << 20, None, ct.byref(out)) == B.RPS_ERR_ARG
    assert lib.rps_batch_run(None, None) == B.RPS_ERR_ARG
    assert lib.rps_batch_info(None, None, None) == B.RPS_ERR_ARG
    lib.rps_batch_destroy(None)


def test_python_errors_are_loud():
    with pytest.raises(P.RpsError):
        P.Context(np.eye(3) * 5, [8, 8, 8], [[0, 0, 0]], [0], [0], [1.0], naux=0)


def test_madelung_constant_host():
    """The library's host Ewald sum (its own implementation) against the oracle's."""
    from oracle import madelung as om
    for lat in (np.eye(3) * 6.74, np.array([[0, .5, .5], [.5, 0, .5], [.5, .5, 0]]) * 3.1,
                np.array([[6.0, 0, 0], [0.8, 5.5, 0], [0.3, 0.2, 6.2]])):
        assert abs(P.madelung_constant(lat) - om.madelung(lat)) < 1e-13 * om.madelung(lat)
    with pytest.raises(P.RpsError):
        P.madelung_constant(np.array([[1.0, 0, 0], [2.0, 0, 0], [0, 0, 1.0]]))



class _NoLib:
    """Stands in for the library: any call into it fails the test, so the
    binding's argument checks must raise first."""
    def __getattr__(self, name):
        raise AssertionError(f"library function {name} called with invalid arguments")


def _fake_context(nbas=5):
    ctx = object.__new__(B.Context)
    ctx._lib = _NoLib()
    ctx._h = ct.c_void_p(0)
    ctx.nbas, ctx.naux, ctx.ngrid, ctx.dvol = nbas, 10, 512, 0.1
    return ctx


@pytest.mark.parametrize("C", [np.zeros((4, 2)), np.zeros((6, 2)), np.zeros((5, 0)), np.zeros(5),
                               np.zeros((5, 2, 1))])
def test_binding_rejects_bad_coefficient_shapes(C):
    """The library reads N x n_occ doubles from C through a raw pointer: a C
    with another number of rows would be read out of bounds, so the binding
    refuses it before any library call."""
    ctx = _fake_context(5)
    with pytest.raises(ValueError):
        ctx.build(C)
    with pytest.raises(ValueError):
        ctx.build_coulomb(C)
    with pytest.raises(ValueError):
        ctx.build_full(C)


def test_binding_rejects_bad_outputs_and_batches():
    ctx = _fake_context(5)
    C = np.zeros((5, 2))
    with pytest.raises(ValueError):
        ctx.madelung_correct(C, np.zeros((5, 3)))
    with pytest.raises(ValueError):
        ctx.autotune(C, np.zeros((5, 2)))             # host arrays: the tuner takes device tensors
    with pytest.raises(ValueError):
        P.exchange_energy(np.zeros((5, 2)), np.zeros((5, 3)))
    other = _fake_context(7)
    with pytest.raises(ValueError):                   # C[1] has the rows of the first context
        B.build_batched([ctx, other], [C, C], [C, np.zeros((7, 2))])
    with pytest.raises(ValueError):                   # lists of different lengths
        B.build_batched([ctx, other], [C], [C])
    with pytest.raises(ValueError):                   # ex too short for two cells
        B.build_batched([ctx, ctx], [C, C], [np.zeros((5, 2)), np.zeros((5, 2))], ex=np.zeros(1))
    with pytest.raises(ValueError):                   # integer K
        B.build_batched([ctx], [C], [np.zeros((5, 2), dtype=np.int64)])
    with pytest.raises(ValueError):                   # the graph-captured batch takes device tensors
        B.Batch([ctx], [C], [np.zeros((5, 2))])


def test_binding_checks_torch_tensors():
    torch = pytest.importorskip("torch")
    ctx = _fake_context(5)
    K = np.zeros((5, 2))
    with pytest.raises(ValueError):                   # non-contiguous
        B._check_array(torch.zeros((2, 5), dtype=torch.float64).t(), (5, 2), "C")
    with pytest.raises(ValueError):                   # float32
        B._check_array(torch.zeros((5, 2), dtype=torch.float32), (5, 2), "C")
    with pytest.raises(ValueError):                   # wrong shape
        B._check_array(torch.zeros((5, 3), dtype=torch.float64), (5, 2), "K")
    B._check_array(torch.zeros((5, 2), dtype=torch.float64), (5, 2), "C")
    with pytest.raises(ValueError):                   # a host array where a device tensor is needed
        B._check_array(K, (5, 2), "K", torch.device("cpu"))


def _from_pot_status(naux=10, points=True, ldv=None, ldw=None, V=True, W=True, flags=0, exact=False):
    lib = P.load()
    cell = B.Cell()
    cell.lattice[:] = list(np.eye(3).reshape(9) * 5.0)
    cell.mesh[:] = [8, 8, 8]
    atoms = np.array([[0.0, 0, 0], [2.0, 2, 2]])
    sa = np.array([0, 1], dtype=np.int32)
    sl = np.array([0, 1], dtype=np.int32)
    se = np.array([1.0, 0.7])
    b = B.Basis(2, 2, atoms.ctypes.data_as(ct.POINTER(ct.c_double)), sa.ctypes.data_as(ct.POINTER(ct.c_int32)),
                sl.ctypes.data_as(ct.POINTER(ct.c_int32)), se.ctypes.data_as(ct.POINTER(ct.c_double)))
    if exact:
        naux = 512
    pts = np.arange(naux, dtype=np.int64)
    Vh = np.zeros((naux, 512))
    Wh = np.zeros((naux, naux))
    h = ct.c_void_p()
    st = lib.rps_setup_isdf_from_potentials(ct.byref(cell), ct.byref(b), naux,
                                            pts.ctypes.data_as(ct.POINTER(ct.c_int64)) if points else None, 0,
                                            Vh.ctypes.data if V else None, 512 if ldv is None else ldv,
                                            Wh.ctypes.data if W else None, naux if ldw is None else ldw, flags, None,
                                            ct.byref(h))
    return st, lib.rps_last_error().decode(), h


@pytest.mark.parametrize("kw,status", [
    (dict(points=False), B.RPS_ERR_ARG),
    (dict(V=False), B.RPS_ERR_ARG),
    (dict(W=False), B.RPS_ERR_ARG),
    (dict(ldv=511), B.RPS_ERR_SHAPE),
    (dict(ldw=9), B.RPS_ERR_SHAPE),
    (dict(flags=5), B.RPS_ERR_ARG),
    (dict(exact=True), B.RPS_ERR_SHAPE),
])
def test_setup_from_potentials_rejects_bad_arguments(kw, status):
    """The set-up from given potentials checks its arguments before any device call."""
    st, msg, h = _from_pot_status(**kw)
    assert st == status, msg
    assert msg and h.value is None
