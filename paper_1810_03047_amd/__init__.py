"""Python binding of libqtm.so, the MI355X quantum-trajectories engine.

Argument marshalling only: every step of the method runs in the library's HIP
kernels (see include/qtm.h for the semantics of each call).  PyTorch is used
only to hand the library the current HIP stream.  Importing works without a
GPU; creating a context needs the built library and a gfx950 device, and any
missing piece raises QtmError instead of falling back to anything else.

Operators are any objects with attributes ``fmt`` ("dense" | "csr" | "diag"),
``dim``, ``val`` (complex array), and for CSR ``row_ptr``/``col_ind``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqtm.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_STEP, E_STATE = 0, -1, -2, -3, -4, -5
PREC_FP64, PREC_FP32 = 0, 1
FORM_LEARNED, FORM_BATCHED = 1, 2
INT_DOPRI5, INT_EXPO = 0, 1       # integrators: adaptive Dormand-Prince 5(4); exact propagator (stiff)
MLP_NPARAM, MLP_NTOTAL = 5443, 5475
SEG_REC = 20
NOALLOC_SCRATCH_MB = 32          # QTM_NOALLOC_SCRATCH_MB of include/qtm.h

_FMT = {"dense": 0, "csr": 1, "diag": 2}
_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int32)


class QtmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libqtm error {code}: {msg}")
        self.code = code


class _Op(C.Structure):
    _fields_ = [("fmt", C.c_int32), ("dim", C.c_int32), ("nnz", C.c_int64), ("val", _dp),
                ("row_ptr", _ip), ("col_ind", _ip)]


class _Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("precision", C.c_int32), ("form", C.c_uint32),
                ("max_steps", C.c_int64), ("device", C.c_int32), ("record_jumps", C.c_int32),
                ("stream", C.c_void_p), ("keep_traj", C.c_int32), ("seg_cap", C.c_int32),
                ("tile_cols", C.c_int32), ("team_waves", C.c_int32), ("integrator", C.c_int32),
                ("expo_substeps", C.c_int32), ("class_waves", C.c_int32 * 3), ("chunk_traj", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("ntraj", C.c_int64), ("accepted", C.c_int64), ("rejected", C.c_int64), ("segments", C.c_int64),
                ("jumps", C.c_int64), ("rhs_evals", C.c_int64), ("passes", C.c_int64), ("failed_traj", C.c_int64),
                ("kernel_ms", C.c_double), ("elapsed_ms", C.c_double), ("blocks", C.c_int32),
                ("threads", C.c_int32), ("tile_cols", C.c_int32), ("lds_bytes", C.c_int32),
                ("max_team_passes", C.c_int64), ("root_evals", C.c_int64),
                ("team_shape", C.c_int32), ("reserved_stats", C.c_int32)]


class _Drive(C.Structure):
    _fields_ = [("c", C.c_double), ("a", C.c_double), ("b", C.c_double), ("omega", C.c_double)]


class _System(C.Structure):
    _fields_ = [("H", C.POINTER(_Op)), ("c_ops", C.POINTER(_Op)), ("n_c", C.c_int32), ("psi0", _dp),
                ("tlist", _dp), ("n_t", C.c_int32), ("e_ops", C.POINTER(_Op)), ("n_e", C.c_int32)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "qtm_opts_default": (None, [C.POINTER(_Opts)]),
    "qtm_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(_Op), C.POINTER(_Op), C.c_int32, _dp, _dp, C.c_int32,
                             C.POINTER(_Op), C.c_int32, C.POINTER(_Opts)]),
    "qtm_create_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(_System), C.POINTER(_Opts)]),
    "qtm_create_td": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(_Op), C.POINTER(_Op), C.POINTER(_Drive), C.c_int32,
                                C.POINTER(_Op), C.c_int32, _dp, _dp, C.c_int32, C.POINTER(_Op), C.c_int32,
                                C.POINTER(_Opts)]),
    "qtm_run": (C.c_int, [C.c_void_p, C.c_int64, C.c_uint64]),
    "qtm_run_range": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_uint64]),
    "qtm_run_range_noalloc": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_uint64, _dp, _dp]),
    "qtm_expect": (C.c_int, [C.c_void_p, _dp, _dp]),
    "qtm_expect_system": (C.c_int, [C.c_void_p, C.c_int32, _dp, _dp]),
    "qtm_sums": (C.c_int, [C.c_void_p, C.c_int32, _dp, _dp, C.POINTER(C.c_int64)]),
    "qtm_traj_expect": (C.c_int, [C.c_void_p, C.c_int32, _dp]),
    "qtm_jumps": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int32, _dp, _ip, _ip]),
    "qtm_traj_stats": (C.c_int, [C.c_void_p, C.c_int32, _ip]),
    "qtm_stats": (C.c_int, [C.c_void_p, C.POINTER(_Stats)]),
    "qtm_set_proposal": (C.c_int, [C.c_void_p, _fp, C.c_int32, C.POINTER(_Op), C.c_int32]),
    "qtm_get_proposal": (C.c_int, [C.c_void_p, _fp, C.c_int32]),
    "qtm_segments": (C.c_int, [C.c_void_p, _fp]),
    "qtm_train_proposal": (C.c_int, [C.c_void_p, _fp, _fp, C.c_int64, C.c_int32, C.c_int32, C.c_float, C.c_uint64, _fp]),
    "qtm_proposal_grad": (C.c_int, [C.c_void_p, _fp, _fp, C.c_int64, _fp, _fp]),
    "qtm_tile_candidates": (C.c_int, [C.c_int32, _ip, C.c_int32]),
    "qtm_batch_tile_candidates": (C.c_int, [C.c_int32, _ip, C.c_int32]),
    "qtm_last_error": (C.c_char_p, []),
    "qtm_destroy": (None, [C.c_void_p]),
}


def tile_candidates(d: int):
    """Team sizes the small dense kernel offers for dimension d (first = default)."""
    w = np.zeros(8, dtype=np.int32)
    n = load().qtm_tile_candidates(int(d), _ptr(w, _ip), 8)
    return [int(x) for x in w[:n]]


def batch_tile_candidates(cls: int):
    """Team sizes the batched tile-class launch offers for class cls (d <= 64, 128, 256)."""
    w = np.zeros(8, dtype=np.int32)
    n = load().qtm_batch_tile_candidates(int(cls), _ptr(w, _ip), 8)
    return [int(x) for x in w[:n]]


def tile_class(d: int) -> int:
    """Tile class of a dense system of dimension d in a batch (-1 above 256)."""
    rt = 2 * ((d + 7) // 8 * 8) // 16
    return 0 if rt <= 8 else 1 if rt <= 16 else 2 if rt <= 32 else -1


def exported_names():
    return sorted(_SIGS)


def load(path: Optional[str] = None) -> C.CDLL:
    """Loads libqtm.so (raises QtmError if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise QtmError(E_DEVICE, f"{p} is missing: run `python -m paper_1810_03047_amd.build`")
    try:
        # torch first, so that the library binds to the HIP runtime torch has loaded
        # (one runtime per process; a second copy loaded later sees no device)
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover
        pass
    L = C.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = L
    return L


def last_error() -> str:
    return load().qtm_last_error().decode()


def _check(rc: int):
    if rc != OK:
        raise QtmError(rc, last_error())


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


class _OpHold:
    def __init__(self, op, d=None):
        fmt = _FMT[op.fmt]
        self.val = np.ascontiguousarray(np.asarray(op.val, dtype=np.complex128).ravel()).view(np.float64)
        self.rp = None if op.row_ptr is None else np.ascontiguousarray(op.row_ptr, dtype=np.int32)
        self.ci = None if op.col_ind is None else np.ascontiguousarray(op.col_ind, dtype=np.int32)
        nnz = len(self.ci) if self.ci is not None else 0
        self.s = _Op(fmt, int(op.dim), nnz, _ptr(self.val), _ptr(self.rp, _ip), _ptr(self.ci, _ip))


def _ops(ops):
    holds = [_OpHold(o) for o in ops]
    arr = (_Op * max(1, len(holds)))(*[h.s for h in holds])
    return holds, arr


@dataclass
class Opts:
    rtol: float = 1e-6
    atol: float = 1e-8
    precision: int = PREC_FP64
    form: int = 0
    max_steps: int = 1_000_000
    device: int = 0
    record_jumps: int = 0
    keep_traj: int = 0
    seg_cap: int = 0
    tile_cols: int = 0
    team_waves: int = 0
    integrator: int = INT_DOPRI5
    expo_substeps: int = 0
    class_waves: tuple = (0, 0, 0)     # batched tile classes d <= 64, 128, 256: waves per team (0: default)
    chunk_traj: int = 0                # runs keeping no per-trajectory data: trajectories per chunk (0: budget)
    stream: Optional[int] = None      # raw hipStream_t; None: torch's current stream when available

    def _c(self) -> _Opts:
        o = _Opts()
        load().qtm_opts_default(C.byref(o))
        o.rtol, o.atol, o.precision, o.form = self.rtol, self.atol, self.precision, self.form
        o.max_steps, o.device, o.record_jumps = self.max_steps, self.device, self.record_jumps
        o.keep_traj, o.seg_cap, o.tile_cols = self.keep_traj, self.seg_cap, self.tile_cols
        o.team_waves = self.team_waves
        o.integrator, o.expo_substeps = self.integrator, self.expo_substeps
        for k in range(3):
            o.class_waves[k] = int(self.class_waves[k])
        o.chunk_traj = int(self.chunk_traj)
        st = self.stream
        if st is None:
            try:
                import torch
                if torch.cuda.is_available():
                    st = torch.cuda.current_stream(self.device).cuda_stream
            except Exception:
                st = None
        o.stream = st
        return o


class Context:
    """A qtm_ctx: one system (or a batch) uploaded to the device."""

    def __init__(self, handle: C.c_void_p, dims, opts: Opts):
        self._h = handle
        # the library's destroy entry point is held by the context itself, so that a
        # context still alive when the interpreter shuts down (module globals already
        # cleared) is freed all the same
        self._destroy_fn = load().qtm_destroy
        self.dims = dims            # list of (d, n_e, n_t) per system
        self.opts = opts
        self.last_count = 0

    def __del__(self):
        self.destroy()

    def destroy(self):
        h = getattr(self, "_h", None)
        fn = getattr(self, "_destroy_fn", None)
        if h and fn is not None:
            fn(h)
        self._h = None

    # -------------------------------------------------------------- runs
    def run(self, ntraj: int, seed: int = 0):
        _check(load().qtm_run(self._h, int(ntraj), int(seed)))
        self.last_count = int(ntraj)
        return self

    def run_range(self, begin: int, count: int, seed: int = 0):
        _check(load().qtm_run_range(self._h, int(begin), int(count), int(seed)))
        self.last_count = int(count)
        return self

    def run_range_noalloc(self, begin: int, count: int, seed: int = 0):
        """qtm_run_range_noalloc: (sum [n_e, n_t] complex, sumsq [n_e, n_t]) of the
        trajectories [begin, begin + count), computed without any device allocation."""
        _, n_e, n_t = self.dims[0]
        s = np.zeros((n_e, n_t), dtype=np.complex128)
        s2 = np.zeros((n_e, n_t))
        _check(load().qtm_run_range_noalloc(self._h, int(begin), int(count), int(seed),
                                            _ptr(s.view(np.float64)), _ptr(s2)))
        self.last_count = 0
        return s, s2

    def expect(self, system: int = 0):
        """(mean [n_e, n_t] complex, var [n_e, n_t])."""
        _, n_e, n_t = self.dims[system]
        mean = np.zeros((n_e, n_t), dtype=np.complex128)
        var = np.zeros((n_e, n_t))
        _check(load().qtm_expect_system(self._h, system, _ptr(mean.view(np.float64)), _ptr(var)))
        return mean, var

    def sums(self, system: int = 0):
        _, n_e, n_t = self.dims[system]
        s = np.zeros((n_e, n_t), dtype=np.complex128)
        s2 = np.zeros((n_e, n_t))
        n = C.c_int64(0)
        _check(load().qtm_sums(self._h, system, _ptr(s.view(np.float64)), _ptr(s2), C.byref(n)))
        return s, s2, int(n.value)

    def traj_expect(self, system: int = 0):
        _, n_e, n_t = self.dims[system]
        X = np.zeros((self.last_count, n_e, n_t), dtype=np.complex128)
        _check(load().qtm_traj_expect(self._h, system, _ptr(X.view(np.float64))))
        return X

    def jumps(self, traj: int, system: int = 0, cap: Optional[int] = None):
        cap = cap or max(1, self.opts.record_jumps)
        t = np.zeros(cap)
        ch = np.zeros(cap, dtype=np.int32)
        n = C.c_int32(0)
        _check(load().qtm_jumps(self._h, system, int(traj), cap, _ptr(t), _ptr(ch, _ip), C.byref(n)))
        m = min(int(n.value), cap)
        return t[:m], ch[:m], int(n.value)

    def traj_stats(self, system: int = 0):
        st = np.zeros((self.last_count, 4), dtype=np.int32)
        _check(load().qtm_traj_stats(self._h, system, _ptr(st, _ip)))
        return st

    def stats(self) -> dict:
        s = _Stats()
        _check(load().qtm_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in _Stats._fields_}

    # ------------------------------------------------------ proposal MLP
    def set_proposal(self, params: np.ndarray, f_ops: Sequence = ()):
        p = np.ascontiguousarray(params, dtype=np.float32)
        holds, arr = _ops(f_ops)
        _check(load().qtm_set_proposal(self._h, _ptr(p, _fp), len(p), arr, len(f_ops)))

    def get_proposal(self) -> np.ndarray:
        p = np.zeros(MLP_NTOTAL, dtype=np.float32)
        _check(load().qtm_get_proposal(self._h, _ptr(p, _fp), MLP_NTOTAL))
        return p

    def segments(self) -> np.ndarray:
        out = np.zeros((self.last_count, self.opts.seg_cap, SEG_REC), dtype=np.float32)
        _check(load().qtm_segments(self._h, _ptr(out, _fp)))
        return out

    def train_proposal(self, feat, tgt, epochs: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0):
        f = np.ascontiguousarray(feat, dtype=np.float32)
        t = np.ascontiguousarray(tgt, dtype=np.float32)
        losses = np.zeros(epochs, dtype=np.float32)
        _check(load().qtm_train_proposal(self._h, _ptr(f, _fp), _ptr(t, _fp), len(f), epochs, batch, lr, seed,
                                         _ptr(losses, _fp)))
        return losses

    def proposal_grad(self, feat, tgt):
        f = np.ascontiguousarray(feat, dtype=np.float32)
        t = np.ascontiguousarray(tgt, dtype=np.float32)
        g = np.zeros(MLP_NPARAM, dtype=np.float32)
        L = np.zeros(1, dtype=np.float32)
        _check(load().qtm_proposal_grad(self._h, _ptr(f, _fp), _ptr(t, _fp), len(f), _ptr(L, _fp), _ptr(g, _fp)))
        return float(L[0]), g


def create(H, c_ops, psi0, tlist, e_ops, opts: Optional[Opts] = None) -> Context:
    """qtm_create: one system."""
    opts = opts or Opts()
    L = load()
    hh, harr = _ops([H])
    ch, carr = _ops(c_ops)
    eh, earr = _ops(e_ops)
    psi = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128)).view(np.float64)
    tl = np.ascontiguousarray(tlist, dtype=np.float64)
    h = C.c_void_p()
    o = opts._c()
    _check(L.qtm_create(C.byref(h), harr, carr, len(c_ops), _ptr(psi), _ptr(tl), len(tl), earr, len(e_ops),
                        C.byref(o)))
    return Context(h, [(int(H.dim), len(e_ops), len(tl))], opts)


def create_td(H0, td, c_ops, psi0, tlist, e_ops, opts: Optional[Opts] = None) -> Context:
    """qtm_create_td: H(t) = H0 + sum_k f_k(t) H_k, td = [(H_k, (c, a, b, omega)), ...] with
    f_k(t) = c + a cos(omega t) + b sin(omega t)."""
    opts = opts or Opts()
    L = load()
    hh, harr = _ops([H0])
    th, tarr = _ops([op for op, _ in td])
    drv = (_Drive * max(1, len(td)))(*[_Drive(*[float(x) for x in cf]) for _, cf in td])
    ch, carr = _ops(c_ops)
    eh, earr = _ops(e_ops)
    psi = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128)).view(np.float64)
    tl = np.ascontiguousarray(tlist, dtype=np.float64)
    h = C.c_void_p()
    o = opts._c()
    _check(L.qtm_create_td(C.byref(h), harr, tarr, drv, len(td), carr, len(c_ops), _ptr(psi), _ptr(tl), len(tl),
                           earr, len(e_ops), C.byref(o)))
    return Context(h, [(int(H0.dim), len(e_ops), len(tl))], opts)


def create_system(system, opts: Optional[Opts] = None) -> Context:
    """qtm_create (or qtm_create_td when the system has time-dependent terms ``td``) from an
    object with H, c_ops, psi0, tlist, e_ops attributes."""
    td = getattr(system, "td", None)
    if td:
        return create_td(system.H, td, system.c_ops, system.psi0, system.tlist, system.e_ops, opts)
    return create(system.H, system.c_ops, system.psi0, system.tlist, system.e_ops, opts)


def create_batch(systems, opts: Optional[Opts] = None) -> Context:
    """qtm_create_batch: systems of mixed dimension in one context."""
    opts = opts or Opts()
    L = load()
    keep = []
    arr = (_System * len(systems))()
    dims = []
    for i, s in enumerate(systems):
        hh, harr = _ops([s.H])
        ch, carr = _ops(s.c_ops)
        eh, earr = _ops(s.e_ops)
        psi = np.ascontiguousarray(np.asarray(s.psi0, dtype=np.complex128)).view(np.float64)
        tl = np.ascontiguousarray(s.tlist, dtype=np.float64)
        keep += [hh, harr, ch, carr, eh, earr, psi, tl]
        arr[i] = _System(harr, carr, len(s.c_ops), _ptr(psi), _ptr(tl), len(tl), earr, len(s.e_ops))
        dims.append((int(s.H.dim), len(s.e_ops), len(tl)))
    h = C.c_void_p()
    o = opts._c()
    _check(L.qtm_create_batch(C.byref(h), len(systems), arr, C.byref(o)))
    return Context(h, dims, opts)
