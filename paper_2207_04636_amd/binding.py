"""ctypes binding of librps.so (include/rps.h).  Argument marshalling only:
every step of the set-up and of the exchange build runs in the HIP library.

Host arrays are numpy float64 / int64; device arrays are torch CUDA (HIP)
tensors, in which case the calls are ordered on the given (or current) torch
stream and are asynchronous.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librps.so")

RPS_OK, RPS_ERR_ARG, RPS_ERR_SHAPE, RPS_ERR_NOMEM, RPS_ERR_NOT_PD, RPS_ERR_DEVICE, RPS_ERR_STATE = range(7)
PREC_FP64, PREC_FP32, PREC_BF16X3 = 0, 1, 2
SELECT_VORONOI, SELECT_GLOBAL = 0, 1
VARIANT_RPS, VARIANT_PS, VARIANT_THC = 0, 1, 2
PTRS_HOST, PTRS_DEVICE = 0, 1
STATUS_NAMES = {0: "RPS_OK", 1: "RPS_ERR_ARG", 2: "RPS_ERR_SHAPE", 3: "RPS_ERR_NOMEM",
                4: "RPS_ERR_NOT_PD", 5: "RPS_ERR_DEVICE", 6: "RPS_ERR_STATE"}

# every symbol declared in include/rps.h
EXPORTS = ("rps_setup_isdf", "rps_setup_isdf_screened", "rps_setup_isdf_from_potentials",
           "rps_build_exchange_occRI", "rps_build_exchange_variant",
           "rps_build_exchange_occRI_noalloc",
           "rps_build_exchange_full", "rps_build_coulomb", "rps_madelung_constant", "rps_madelung_correct",
           "rps_build_exchange_occRI_batched",
           "rps_exchange_energy",
           "rps_overlap", "rps_get_points", "rps_get_info", "rps_get_array", "rps_destroy",
           "rps_last_error", "rps_abi_version", "rps_set_profiling", "rps_get_profile", "rps_autotune",
           "rps_batch_create", "rps_batch_run", "rps_batch_info", "rps_batch_destroy")
BATCH_AUTOTUNE = 1


def BATCH_BRANCHES(k: int) -> int:
    return (int(k) & 15) << 8


class RpsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Cell(ct.Structure):
    _fields_ = [("lattice", ct.c_double * 9), ("mesh", ct.c_int32 * 3)]


class Basis(ct.Structure):
    _fields_ = [("natom", ct.c_int32), ("nshell", ct.c_int32),
                ("atom_xyz", ct.POINTER(ct.c_double)), ("shell_atom", ct.POINTER(ct.c_int32)),
                ("shell_l", ct.POINTER(ct.c_int32)), ("shell_exp", ct.POINTER(ct.c_double))]


class Info(ct.Structure):
    _fields_ = [("ngrid", ct.c_int64), ("nbas", ct.c_int64), ("naux", ct.c_int64),
                ("ngrid_pad", ct.c_int64), ("nbas_pad", ct.c_int64), ("naux_pad", ct.c_int64),
                ("n_candidates", ct.c_int64), ("dvol", ct.c_double), ("chol_shift", ct.c_double),
                ("setup_seconds", ct.c_double), ("device_bytes", ct.c_int64),
                ("precision", ct.c_int32), ("exact", ct.c_int32), ("madelung", ct.c_double),
                ("basis_fill", ct.c_double), ("basis_pair_fill", ct.c_double),
                ("build_arith", ct.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load librps.so; raises if it is not built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2207_04636_amd.build (no CPU fallback exists)")
    # Load the HIP runtime by soname first, globally: if torch (or anything else)
    # already loaded a libamdhip64.so.7 this returns that same instance, so the
    # library and torch share one runtime.  Letting it arrive only as a private
    # dependency of librps.so left the device undiscovered on the MI355X hosts.
    try:
        ct.CDLL("libamdhip64.so.7", mode=ct.RTLD_GLOBAL)
    except OSError:
        pass
    lib = ct.CDLL(path)
    P, I32, I64, U64, D = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_uint64, ct.c_double
    lib.rps_setup_isdf.argtypes = [ct.POINTER(Cell), ct.POINTER(Basis), I64, U64, I32, I32,
                                   ct.POINTER(ct.c_int64), P, ct.POINTER(P)]
    lib.rps_setup_isdf_screened.argtypes = [ct.POINTER(Cell), ct.POINTER(Basis), I64, U64, I32, I32,
                                            ct.POINTER(ct.c_int64), D, P, ct.POINTER(P)]
    lib.rps_setup_isdf_from_potentials.argtypes = [ct.POINTER(Cell), ct.POINTER(Basis), I64, ct.POINTER(ct.c_int64),
                                                   I32, P, I64, P, I64, I32, P, ct.POINTER(P)]
    lib.rps_build_exchange_occRI.argtypes = [P, I32, P, P, P, I32, P]
    lib.rps_build_exchange_variant.argtypes = [P, I32, I32, P, P, P, I32, P]
    lib.rps_build_exchange_occRI_noalloc.argtypes = [P, I32, P, P, P, P]
    lib.rps_build_exchange_full.argtypes = [P, I32, P, P, I32, P]
    lib.rps_build_coulomb.argtypes = [P, I32, P, P, P, I32, P]
    lib.rps_madelung_constant.argtypes = [P, ct.POINTER(D)]
    lib.rps_madelung_correct.argtypes = [P, I32, P, P, P, I32, P]
    lib.rps_build_exchange_occRI_batched.argtypes = [ct.POINTER(P), I32, ct.POINTER(I32), ct.POINTER(P),
                                                     ct.POINTER(P), P, I32, P]
    lib.rps_exchange_energy.argtypes = [I32, I32, P, P, ct.POINTER(D)]
    lib.rps_overlap.argtypes = [P, P]
    lib.rps_get_points.argtypes = [P, P]
    lib.rps_get_info.argtypes = [P, ct.POINTER(Info)]
    lib.rps_get_array.argtypes = [P, I32, I64, I64, P]
    lib.rps_set_profiling.argtypes = [P, I32]
    lib.rps_get_profile.argtypes = [P, P]
    lib.rps_autotune.argtypes = [P, I32, P, P, P, P, ct.POINTER(D)]
    lib.rps_batch_create.argtypes = [ct.POINTER(P), I32, ct.POINTER(I32), ct.POINTER(P), ct.POINTER(P), P, I32, P,
                                     ct.POINTER(P)]
    lib.rps_batch_run.argtypes = [P, P]
    lib.rps_batch_info.argtypes = [P, ct.POINTER(I32), P]
    lib.rps_batch_destroy.argtypes = [P]
    lib.rps_batch_destroy.restype = None
    lib.rps_destroy.argtypes = [P]
    lib.rps_destroy.restype = None
    lib.rps_last_error.restype = ct.c_char_p
    for name in EXPORTS:
        if name not in ("rps_destroy", "rps_last_error", "rps_batch_destroy"):
            getattr(lib, name).restype = ct.c_int32
    _lib = lib
    return lib


def _check(st: int):
    if st != RPS_OK:
        raise RpsError(st, _lib.rps_last_error().decode())


def madelung_constant(lattice) -> float:
    """Madelung constant of the lattice (rows a1, a2, a3 in bohr); host only."""
    lib = load()
    lat = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(9))
    m = ct.c_double(0.0)
    _check(lib.rps_madelung_constant(lat.ctypes.data, ct.byref(m)))
    return m.value


def _ptr(x) -> int:
    """Address of a numpy array or torch tensor."""
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return int(x.data_ptr())


def _is_device(x) -> bool:
    return not isinstance(x, np.ndarray) and getattr(x, "is_cuda", False)


def _check_array(x, shape, name, device=None):
    """Raise ValueError unless x is a C-contiguous float64 array of the given
    shape (a numpy array, or a torch tensor on `device` when that is given).
    The library reads and writes exactly these extents through raw pointers,
    so a wrong shape would mean out-of-bounds accesses there."""
    shape = tuple(int(s) for s in shape)
    if isinstance(x, np.ndarray):
        if device is not None:
            raise ValueError(f"{name} must be a device tensor like the other operands, got a numpy array")
        ok = x.dtype == np.float64 and x.flags.c_contiguous
        dtype = x.dtype
    else:
        if not hasattr(x, "data_ptr"):
            raise ValueError(f"{name} must be a numpy array or a torch tensor, got {type(x).__name__}")
        import torch
        ok = x.dtype == torch.float64 and x.is_contiguous()
        dtype = x.dtype
        if device is not None and x.device != device:
            raise ValueError(f"{name} is on {x.device}, expected {device}")
        if device is None and getattr(x, "is_cuda", False):
            raise ValueError(f"{name} is a device tensor but the other operands are host arrays")
    if not ok:
        raise ValueError(f"{name} must be a C-contiguous float64 array (got dtype {dtype})")
    if tuple(x.shape) != shape:
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {shape}")


def _check_scalar_out(x, name, device, count=1):
    """ex / ej outputs of device calls: a float64 tensor of >= count elements on device."""
    if x is None:
        return
    import torch
    if not hasattr(x, "data_ptr") or x.dtype != torch.float64 or not x.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 tensor")
    if x.device != device:
        raise ValueError(f"{name} is on {x.device}, expected {device}")
    if x.numel() < count:
        raise ValueError(f"{name} needs at least {count} element(s), has {x.numel()}")


def _coef_cols(C, nbas, name="C") -> int:
    """Number of occupied orbitals of a coefficient matrix with nbas rows."""
    if getattr(C, "ndim", None) != 2 or int(C.shape[0]) != int(nbas) or int(C.shape[1]) < 1:
        raise ValueError(f"{name} must have shape ({nbas}, n_occ) with n_occ >= 1, got {tuple(getattr(C, 'shape', ()))}")
    return int(C.shape[1])


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                return int(torch.cuda.current_stream().cuda_stream)
        except Exception:
            return None
        return None
    return int(getattr(stream, "cuda_stream", stream))


class Context:
    """An rPS set-up (points, V, W on the device) for one cell and basis."""

    def _marshal(self, lattice, mesh, atoms, shell_atom, shell_l, shell_exp):
        cell = Cell()
        lat = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(9))
        cell.lattice[:] = list(lat)
        cell.mesh[:] = [int(m) for m in mesh]
        self._atoms = np.ascontiguousarray(np.asarray(atoms, dtype=np.float64).reshape(-1, 3))
        self._sa = np.ascontiguousarray(np.asarray(shell_atom, dtype=np.int32))
        self._sl = np.ascontiguousarray(np.asarray(shell_l, dtype=np.int32))
        self._se = np.ascontiguousarray(np.asarray(shell_exp, dtype=np.float64))
        b = Basis(int(self._atoms.shape[0]), int(self._sl.shape[0]),
                  self._atoms.ctypes.data_as(ct.POINTER(ct.c_double)),
                  self._sa.ctypes.data_as(ct.POINTER(ct.c_int32)),
                  self._sl.ctypes.data_as(ct.POINTER(ct.c_int32)),
                  self._se.ctypes.data_as(ct.POINTER(ct.c_double)))
        return cell, b

    def _finish(self, h):
        self._h = h
        inf = self.info()
        self.nbas, self.naux, self.ngrid = int(inf["nbas"]), int(inf["naux"]), int(inf["ngrid"])
        self.dvol = float(inf["dvol"])

    def __init__(self, lattice, mesh, atoms, shell_atom, shell_l, shell_exp, naux: int,
                 seed: int = 0, select: int = SELECT_VORONOI, precision: int = PREC_FP64,
                 points=None, stream=None, basis_eps: float = 0.0):
        lib = load()
        self._lib = lib
        cell, b = self._marshal(lattice, mesh, atoms, shell_atom, shell_l, shell_exp)
        pts = None
        if points is not None:
            self._pts_in = np.ascontiguousarray(np.asarray(points, dtype=np.int64))
            pts = self._pts_in.ctypes.data_as(ct.POINTER(ct.c_int64))
        h = ct.c_void_p()
        _check(lib.rps_setup_isdf_screened(ct.byref(cell), ct.byref(b), int(naux),
                                           ct.c_uint64(int(seed) & (2**64 - 1)), int(select), int(precision),
                                           pts, float(basis_eps), _stream_handle(stream), ct.byref(h)))
        self._finish(h)

    @classmethod
    def from_potentials(cls, w, points, V, W, precision: int = PREC_FP64, stream=None):
        """rps_setup_isdf_from_potentials: a context for workload w whose points,
        V [N_aux x N_g] (float64 for FP64, float32 for the precision forms) and
        W [N_aux x N_aux] (float64) are given (numpy arrays, or torch device tensors)."""
        self = object.__new__(cls)
        self._lib = load()
        cell, b = self._marshal(w.lattice, w.mesh, w.atoms, w.shell_atom, w.shell_l, w.shell_exp)
        self._pts_in = np.ascontiguousarray(np.asarray(points, dtype=np.int64))
        naux, ng = len(self._pts_in), int(np.prod(w.mesh))
        vdt = "float64" if precision == PREC_FP64 else "float32"
        dev = _is_device(V)
        for x, shape, name, dt in ((V, (naux, ng), "V", vdt), (W, (naux, naux), "W", "float64")):
            if tuple(x.shape) != shape or str(x.dtype).split(".")[-1] != dt:
                raise ValueError(f"{name} must be {dt} of shape {shape}, got {x.dtype} {tuple(x.shape)}")
            if _is_device(x) != dev or not (x.flags.c_contiguous if isinstance(x, np.ndarray) else x.is_contiguous()):
                raise ValueError(f"V and W must both be contiguous host arrays or both device tensors")
        h = ct.c_void_p()
        _check(self._lib.rps_setup_isdf_from_potentials(
            ct.byref(cell), ct.byref(b), naux, self._pts_in.ctypes.data_as(ct.POINTER(ct.c_int64)), int(precision),
            _ptr(V), ng, _ptr(W), naux, PTRS_DEVICE if dev else PTRS_HOST, _stream_handle(stream), ct.byref(h)))
        self._finish(h)
        return self

    @classmethod
    def from_workload(cls, w, **kw):
        """Convenience: any object with lattice, mesh, atoms, shell_atom,
        shell_l, shell_exp and naux attributes."""
        kw.setdefault("naux", w.naux)
        return cls(w.lattice, w.mesh, w.atoms, w.shell_atom, w.shell_l, w.shell_exp, **kw)

    # ---------------------------------------------------------------- builds
    def build(self, C, K=None, ex=None, variant: int = VARIANT_RPS, stream=None):
        """K_occ (N x n) and E_x.  numpy C -> synchronous host call returning
        (K, E); torch CUDA C -> stream-ordered call writing K (and ex, a
        1-element float64 tensor) and returning them."""
        if _is_device(C):
            import torch
            n = _coef_cols(C, self.nbas)
            _check_array(C, (self.nbas, n), "C", C.device)
            if K is None:
                K = torch.empty((self.nbas, n), dtype=torch.float64, device=C.device)
            _check_array(K, (self.nbas, n), "K", C.device)
            _check_scalar_out(ex, "ex", C.device)
            exp_ = 0 if ex is None else _ptr(ex)
            _check(self._lib.rps_build_exchange_variant(self._h, int(variant), n, _ptr(C), _ptr(K), exp_ or None,
                                                        PTRS_DEVICE, _stream_handle(stream)))
            return K, ex
        C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
        n = _coef_cols(C, self.nbas)
        Kh = np.empty((self.nbas, n))
        e = ct.c_double(0.0)
        _check(self._lib.rps_build_exchange_variant(self._h, int(variant), n, C.ctypes.data, Kh.ctypes.data,
                                                    ct.addressof(e), PTRS_HOST, None))
        return Kh, e.value

    def build_noalloc(self, C, K, ex=None, stream=None):
        """rps_build_exchange_occRI_noalloc: the build on the library's static
        device scratch (no device allocation); C, K (and ex) device tensors."""
        if not _is_device(C):
            raise ValueError("the no-allocation build takes device tensors")
        n = _coef_cols(C, self.nbas)
        _check_array(C, (self.nbas, n), "C", C.device)
        _check_array(K, (self.nbas, n), "K", C.device)
        _check_scalar_out(ex, "ex", C.device)
        _check(self._lib.rps_build_exchange_occRI_noalloc(self._h, n, _ptr(C), _ptr(K),
                                                          None if ex is None else _ptr(ex), _stream_handle(stream)))
        return K, ex

    def build_full(self, C):
        C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
        _coef_cols(C, self.nbas)
        Kh = np.empty((self.nbas, self.nbas))
        _check(self._lib.rps_build_exchange_full(self._h, int(C.shape[1]), C.ctypes.data, Kh.ctypes.data,
                                                 PTRS_HOST, None))
        return Kh

    def build_coulomb(self, C, J=None, ej=None, stream=None):
        """Coulomb matrix J (N x N) and E_J (rps_build_coulomb).  numpy C ->
        synchronous host call returning (J, E_J); torch CUDA C -> stream-ordered
        call writing J (and ej, a 1-element float64 tensor) and returning them."""
        if _is_device(C):
            import torch
            n = _coef_cols(C, self.nbas)
            _check_array(C, (self.nbas, n), "C", C.device)
            if J is None:
                J = torch.empty((self.nbas, self.nbas), dtype=torch.float64, device=C.device)
            _check_array(J, (self.nbas, self.nbas), "J", C.device)
            _check_scalar_out(ej, "ej", C.device)
            _check(self._lib.rps_build_coulomb(self._h, int(C.shape[1]), _ptr(C), _ptr(J),
                                               None if ej is None else _ptr(ej), PTRS_DEVICE,
                                               _stream_handle(stream)))
            return J, ej
        C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
        _coef_cols(C, self.nbas)
        Jh = np.empty((self.nbas, self.nbas))
        e = ct.c_double(0.0)
        _check(self._lib.rps_build_coulomb(self._h, int(C.shape[1]), C.ctypes.data, Jh.ctypes.data,
                                           ct.addressof(e), PTRS_HOST, None))
        return Jh, e.value

    def madelung_correct(self, C, K, ex=None, stream=None):
        """Madelung term in place (rps_madelung_correct).  numpy C, K: returns
        (K + M S C, E - M tr(C^T S C)) with E = ex (a float, or None); torch
        CUDA C, K (and ex, a 1-element float64 tensor): stream-ordered, returns (K, ex)."""
        if _is_device(C):
            n = _coef_cols(C, self.nbas)
            _check_array(C, (self.nbas, n), "C", C.device)
            _check_array(K, (self.nbas, n), "K", C.device)
            _check_scalar_out(ex, "ex", C.device)
            _check(self._lib.rps_madelung_correct(self._h, int(C.shape[1]), _ptr(C), _ptr(K),
                                                  None if ex is None else _ptr(ex), PTRS_DEVICE,
                                                  _stream_handle(stream)))
            return K, ex
        C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
        n = _coef_cols(C, self.nbas)
        Kh = np.array(K, dtype=np.float64, order="C", copy=True)
        _check_array(Kh, (self.nbas, n), "K")
        e = ct.c_double(0.0 if ex is None else float(ex))
        _check(self._lib.rps_madelung_correct(self._h, int(C.shape[1]), C.ctypes.data, Kh.ctypes.data,
                                              None if ex is None else ct.addressof(e), PTRS_HOST, None))
        return Kh, (None if ex is None else e.value)

    # ---------------------------------------------------------------- inspection
    def points(self) -> np.ndarray:
        out = np.empty(self.naux, dtype=np.int64)
        _check(self._lib.rps_get_points(self._h, out.ctypes.data))
        return out

    def info(self) -> dict:
        inf = Info()
        _check(self._lib.rps_get_info(self._h, ct.byref(inf)))
        return inf.as_dict()

    def overlap(self) -> np.ndarray:
        S = np.empty((self.nbas, self.nbas))
        _check(self._lib.rps_overlap(self._h, S.ctypes.data))
        return S

    def array(self, which: int, row0: int = 0, nrows: Optional[int] = None) -> np.ndarray:
        """0: Phi rows (N_g x N), 1: V rows (N_chi x N_g), 2: W (N_chi x N_chi),
        3: Voronoi owner per grid point."""
        total = {0: self.ngrid, 1: self.naux, 2: self.naux, 3: self.ngrid}[which]
        ncol = {0: self.nbas, 1: self.ngrid, 2: self.naux, 3: 1}[which]
        nrows = total - row0 if nrows is None else nrows
        out = np.empty((nrows, ncol)) if which != 3 else np.empty(nrows)
        _check(self._lib.rps_get_array(self._h, int(which), int(row0), int(nrows), out.ctypes.data))
        return out

    def autotune(self, C, K, ex=None, stream=None) -> float:
        """Tune this context's launch parameters on device tensors C, K (and ex);
        returns the best mean build time in ms (see rps_autotune)."""
        if not _is_device(C):
            raise ValueError("autotune takes device tensors C, K (and ex)")
        n = _coef_cols(C, self.nbas)
        _check_array(C, (self.nbas, n), "C", C.device)
        _check_array(K, (self.nbas, n), "K", C.device)
        _check_scalar_out(ex, "ex", C.device)
        best = ct.c_double(0.0)
        _check(self._lib.rps_autotune(self._h, int(C.shape[1]), _ptr(C), _ptr(K), None if ex is None else _ptr(ex),
                                      _stream_handle(stream), ct.byref(best)))
        return best.value

    def set_profiling(self, enable: bool = True):
        _check(self._lib.rps_set_profiling(self._h, 1 if enable else 0))

    def profile(self) -> dict:
        """Kernel timings recorded since the last read (see rps_get_profile)."""
        out = np.zeros(4)
        _check(self._lib.rps_get_profile(self._h, out.ctypes.data))
        return dict(builds=int(out[0]), fused_ms=float(out[1]), line3_ms=float(out[2]), build_ms=float(out[3]))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.rps_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def exchange_energy(C: np.ndarray, K: np.ndarray) -> float:
    """E_x = -tr(C^T K) through the library's host routine."""
    lib = load()
    C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    K = np.ascontiguousarray(np.asarray(K, dtype=np.float64))
    if C.ndim != 2 or K.shape != C.shape:
        raise ValueError(f"C and K must be 2-D arrays of one shape, got {C.shape} and {K.shape}")
    e = ct.c_double(0.0)
    _check(lib.rps_exchange_energy(int(C.shape[0]), int(C.shape[1]), C.ctypes.data, K.ctypes.data, ct.byref(e)))
    return e.value


def _check_batch(ctxs, Cs, Ks, ex, device_only):
    """Per-cell checks of a batch: C[b], K[b] of shape (N_b, n_b), all host
    arrays or all device tensors on one device; ex of >= len(ctxs) elements."""
    nb = len(ctxs)
    if len(Cs) != nb or len(Ks) != nb:
        raise ValueError(f"{nb} contexts need {nb} C and K arrays, got {len(Cs)} and {len(Ks)}")
    if nb == 0:
        return False
    dev = _is_device(Cs[0])
    if device_only and not dev:
        raise ValueError("the batching form takes device tensors")
    device = Cs[0].device if dev else None
    for b, (c, C, K) in enumerate(zip(ctxs, Cs, Ks)):
        n = _coef_cols(C, c.nbas, f"C[{b}]")
        _check_array(C, (c.nbas, n), f"C[{b}]", device)
        _check_array(K, (c.nbas, n), f"K[{b}]", device)
    if ex is not None:
        if dev:
            _check_scalar_out(ex, "ex", device, nb)
        elif not (isinstance(ex, np.ndarray) and ex.dtype == np.float64 and ex.flags.c_contiguous
                  and ex.size >= nb):
            raise ValueError(f"ex must be a contiguous float64 array of >= {nb} elements")
    return dev


def build_batched(ctxs, Cs, Ks, ex=None, stream=None):
    """Batched builds over several contexts (all host arrays or all device
    tensors; rps_build_exchange_occRI_batched).  ex: float64 array of
    len(ctxs) elements or None."""
    lib = load()
    dev = _check_batch(ctxs, Cs, Ks, ex, device_only=False)
    nb = len(ctxs)
    H = (ct.c_void_p * nb)(*[c._h.value for c in ctxs])
    nocc = (ct.c_int32 * nb)(*[int(C.shape[1]) for C in Cs])
    Cp = (ct.c_void_p * nb)(*[_ptr(C) for C in Cs])
    Kp = (ct.c_void_p * nb)(*[_ptr(K) for K in Ks])
    _check(lib.rps_build_exchange_occRI_batched(H, nb, nocc, Cp, Kp, None if ex is None else _ptr(ex),
                                                PTRS_DEVICE if dev else PTRS_HOST, _stream_handle(stream)))


class Batch:
    """Batching form: the builds of many contexts captured into one HIP graph
    (rps_batch_create); run() replays it with one launch.  Cs, Ks are device
    tensors (their addresses are baked into the graph), ex a device float64
    tensor of len(ctxs) elements or None."""

    def __init__(self, ctxs, Cs, Ks, ex=None, autotune: bool = True, branches: int = 0, stream=None):
        lib = load()
        self._lib = lib
        _check_batch(ctxs, Cs, Ks, ex, device_only=True)
        self._keep = (list(ctxs), list(Cs), list(Ks), ex)
        nb = len(ctxs)
        H = (ct.c_void_p * nb)(*[c._h.value for c in ctxs])
        nocc = (ct.c_int32 * nb)(*[int(C.shape[1]) for C in Cs])
        Cp = (ct.c_void_p * nb)(*[_ptr(C) for C in Cs])
        Kp = (ct.c_void_p * nb)(*[_ptr(K) for K in Ks])
        flags = (BATCH_AUTOTUNE if autotune else 0) | (BATCH_BRANCHES(branches) if branches else 0)
        h = ct.c_void_p()
        _check(lib.rps_batch_create(H, nb, nocc, Cp, Kp, None if ex is None else _ptr(ex), flags,
                                    _stream_handle(stream), ct.byref(h)))
        self._h = h

    def run(self, stream=None):
        _check(self._lib.rps_batch_run(self._h, _stream_handle(stream)))

    def info(self) -> dict:
        nbr = ct.c_int32(0)
        sec = np.zeros(3)
        _check(self._lib.rps_batch_info(self._h, ct.byref(nbr), sec.ctypes.data))
        return dict(branches=int(nbr.value), create_s=float(sec[0]), capture_s=float(sec[1]),
                    replay_ms=float(sec[2]) * 1e3)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.rps_batch_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
