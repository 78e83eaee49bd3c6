"""CPU oracle for the quantum trajectories method -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
library.  Contents:

* ``liboracle.so`` (``qtm_oracle.cpp``): FP64 trajectory solver following the
  paper's Algorithm 1 (Sec. 2.2) with the Dormand-Prince 5(4) integrator,
  Philox4x64-10 random streams, FP64 averaging and the learned-proposal MLP;
* ``lindblad``: brute-force density-matrix integration of the Lindblad
  equation (Sec. 2.2, the master equation the trajectory average converges to);
* ``closed_forms``: analytic solutions used to pin the above.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import build as _build

_lib = None
_lib_fast = None


class _Op(C.Structure):
    _fields_ = [("fmt", C.c_int32), ("dim", C.c_int32), ("nnz", C.c_int64),
                ("val", C.POINTER(C.c_double)), ("row_ptr", C.POINTER(C.c_int32)),
                ("col_ind", C.POINTER(C.c_int32))]


_FMT = {"dense": 0, "csr": 1, "diag": 2}
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


def lib(fast: bool = False):
    """The parity build, or (fast=True) the -O3 AVX2/FMA build used only to time the
    oracle as a CPU baseline."""
    global _lib, _lib_fast
    if (_lib_fast if fast else _lib) is None:
        path = _build.ensure_built(fast)
        L = C.CDLL(path)
        L.qtmref_philox4x64_10.argtypes = [C.POINTER(C.c_uint64)] * 3
        L.qtmref_uniform53.argtypes = [C.c_uint64]
        L.qtmref_uniform53.restype = C.c_double
        L.qtmref_build_M.argtypes = [C.POINTER(_Op), C.POINTER(_Op), C.c_int, _dp]
        L.qtmref_dopri_step.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                        _dp, _dp, _dp, C.c_int, _dp, _dp]
        L.qtmref_integrate_nojump.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                              C.c_double, C.c_int, _dp, _ip, _dp, _dp, C.c_double, _ip]
        L.qtmref_run.argtypes = [C.POINTER(_Op), C.POINTER(_Op), C.c_int, _dp, _dp, C.c_int,
                                 C.POINTER(_Op), C.c_int, C.c_double, C.c_double, C.c_int64,
                                 C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, C.c_int,
                                 _dp, C.POINTER(_Op), C.c_int,
                                 _dp, C.c_int, _dp, _ip, _ip, _lp, C.c_int, _dp, _lp,
                                 C.POINTER(_Op), _dp, C.c_int]
        L.qtmref_average.argtypes = [_dp, C.c_int64, C.c_int, C.c_int, _dp, _dp]
        L.qtmref_mlp_nparam.restype = C.c_int
        L.qtmref_mlp_ntotal.restype = C.c_int
        L.qtmref_mlp_forward.argtypes = [_dp, _dp, C.c_int64, _dp]
        L.qtmref_mlp_loss_grad.argtypes = [_dp, _dp, _dp, C.c_int64, _dp]
        L.qtmref_mlp_loss_grad.restype = C.c_double
        L.qtmref_tableau.argtypes = [_dp] * 5
        L.qtmref_snap_step.argtypes = [C.c_double]
        L.qtmref_snap_step.restype = C.c_double
        if fast:
            _lib_fast = L
        else:
            _lib = L
    return _lib_fast if fast else _lib


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


def _cplx(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).view(np.float64)


class _OpHolder:
    """Keeps the numpy buffers behind a ctypes operator record alive."""

    def __init__(self, op):
        self.val = _cplx(np.asarray(op.val).ravel())
        self.rp = None if op.row_ptr is None else np.ascontiguousarray(op.row_ptr, dtype=np.int32)
        self.ci = None if op.col_ind is None else np.ascontiguousarray(op.col_ind, dtype=np.int32)
        self.s = _Op(_FMT[op.fmt], op.dim, len(self.ci) if self.ci is not None else 0,
                     _ptr(self.val), _ptr(self.rp, _ip), _ptr(self.ci, _ip))


def _op_array(ops):
    holders = [_OpHolder(o) for o in ops]
    arr = (_Op * max(1, len(holders)))(*[h.s for h in holders]) if holders else (_Op * 1)()
    return holders, arr


# --------------------------------------------------------------- Philox
def philox4x64_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.array(ctr, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().qtmref_philox4x64_10(c.ctypes.data_as(C.POINTER(C.c_uint64)),
                               k.ctypes.data_as(C.POINTER(C.c_uint64)),
                               out.ctypes.data_as(C.POINTER(C.c_uint64)))
    return out


def uniform53(x: int) -> float:
    return lib().qtmref_uniform53(C.c_uint64(int(x)))


# ------------------------------------------------------------ building M
def build_M(H, c_ops) -> np.ndarray:
    """Dense copy of the oracle's right-hand-side matrix M = -i H_eff."""
    hh, harr = _op_array([H])
    ch, carr = _op_array(c_ops)
    out = np.zeros((H.dim, H.dim), dtype=np.complex128)
    lib().qtmref_build_M(harr, carr, len(c_ops), _ptr(out.view(np.float64)))
    return out


def dopri_step(M: np.ndarray, y: np.ndarray, h: float, rtol: float = 1e-6, atol: float = 1e-8,
               thetas: Sequence[float] = ()):
    d = M.shape[0]
    Mr, yr = _cplx(M), _cplx(y)
    ynew = np.zeros(d, dtype=np.complex128)
    ev = np.zeros(d, dtype=np.complex128)
    en = np.zeros(1)
    th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64))
    u = np.zeros((max(1, len(th)), d), dtype=np.complex128)
    lib().qtmref_dopri_step(d, _ptr(Mr), _ptr(yr), h, rtol, atol, _ptr(ynew.view(np.float64)),
                            _ptr(ev.view(np.float64)), _ptr(en), len(th), _ptr(th) if len(th) else None,
                            _ptr(u.view(np.float64)))
    return ynew, ev, float(en[0]), u[:len(th)]


def integrate_nojump(M: np.ndarray, y0: np.ndarray, t0: float, t_end: float, rtol: float = 1e-6,
                     atol: float = 1e-8, cap: int = 100000, first_step: float = 0.0,
                     with_rejections: bool = False):
    """Jump-free integration of psi' = M psi; returns the accepted times, the end
    state and the first step (and the number of rejected attempts when asked).
    ``first_step`` > 0 replaces the starting-step rule."""
    d = M.shape[0]
    ts = np.zeros(cap)
    n = np.zeros(1, dtype=np.int32)
    nrej = np.zeros(1, dtype=np.int32)
    yend = np.zeros(d, dtype=np.complex128)
    h0 = np.zeros(1)
    lib().qtmref_integrate_nojump(d, _ptr(_cplx(M)), _ptr(_cplx(y0)), t0, t_end, rtol, atol, cap,
                                  _ptr(ts), _ptr(n, _ip), _ptr(yend.view(np.float64)), _ptr(h0),
                                  float(first_step), _ptr(nrej, _ip))
    out = (ts[:min(cap, int(n[0]))], yend, float(h0[0]))
    return out + (int(nrej[0]),) if with_rejections else out


# ---------------------------------------------------------- trajectories
NF = 16


def run(system, ntraj: int, seed: int = 0, sys_id: int = 0, traj_begin: int = 0,
        rtol: float = 1e-6, atol: float = 1e-8, max_steps: int = 10_000_000, nthreads: int = 0,
        mlp: Optional[np.ndarray] = None, f_ops=None, jcap: int = 64, seg_cap: int = 0,
        fast: bool = False) -> dict:
    """Runs trajectories [traj_begin, traj_begin + ntraj) of ``system`` in FP64.

    Returns per-trajectory outputs ``X`` [ntraj, n_e, n_t] (complex), the
    index-ordered average ``mean`` [n_e, n_t] (complex) and ``var`` (of the
    real part), the jump log, per-trajectory stats (accepted, rejected, rhs,
    segments, jumps), optional segment records and the status.  A system with a ``td``
    attribute (a list of (H_k, (c, a, b, w)) pairs) has the time-dependent Hamiltonian
    H0 + sum_k (c + a cos(w t) + b sin(w t)) H_k.  ``fast`` runs the
    -O3 AVX2/FMA timing build instead of the parity build.
    """
    s = system
    n_e, n_t = len(s.e_ops), len(s.tlist)
    hh, harr = _op_array([s.H])
    ch, carr = _op_array(s.c_ops)
    eh, earr = _op_array(s.e_ops)
    fh, farr = _op_array(f_ops or [])
    # time-dependent terms H_k with coefficients f_k(t) = c + a cos(w t) + b sin(w t)
    td = getattr(s, "td", None) or []
    th, tarr = _op_array([op for op, _ in td])
    tcoef = np.ascontiguousarray([list(cf) for _, cf in td], dtype=np.float64).reshape(-1) if td else np.zeros(4)
    X = np.zeros((ntraj, n_e, n_t), dtype=np.complex128)
    jt = np.zeros((ntraj, max(1, jcap)))
    jc = np.zeros((ntraj, max(1, jcap)), dtype=np.int32)
    jn = np.zeros(ntraj, dtype=np.int32)
    stats = np.zeros((ntraj, 5), dtype=np.int64)
    segs = np.zeros((ntraj, max(1, seg_cap), NF + 4)) if seg_cap > 0 else None
    fail = np.zeros(1, dtype=np.int64)
    psi = _cplx(s.psi0)
    tl = np.ascontiguousarray(s.tlist, dtype=np.float64)
    mp = None if mlp is None else np.ascontiguousarray(mlp, dtype=np.float64)
    st = lib(fast).qtmref_run(harr, carr, len(s.c_ops), _ptr(psi), _ptr(tl), n_t, earr, n_e,
                          rtol, atol, max_steps, seed, sys_id, traj_begin, ntraj, nthreads,
                          _ptr(mp), farr, len(f_ops or []),
                          _ptr(X.view(np.float64)), jcap, _ptr(jt), _ptr(jc, _ip), _ptr(jn, _ip),
                          _ptr(stats, _lp), seg_cap, _ptr(segs), _ptr(fail, _lp),
                          tarr, _ptr(tcoef), len(td))
    mean = np.zeros((n_e, n_t), dtype=np.complex128)
    var = np.zeros((n_e, n_t))
    lib().qtmref_average(_ptr(X.view(np.float64)), ntraj, n_e, n_t, _ptr(mean.view(np.float64)), _ptr(var))
    return dict(status=int(st), fail_traj=int(fail[0]), X=X, mean=mean, var=var,
                jump_times=jt[:, :jcap], jump_channels=jc[:, :jcap], jump_counts=jn,
                stats=stats, segs=segs)


# ------------------------------------------------------------------ MLP
def mlp_nparam() -> int:
    return lib().qtmref_mlp_nparam()


def mlp_ntotal() -> int:
    return lib().qtmref_mlp_ntotal()


def mlp_forward(params: np.ndarray, feat: np.ndarray) -> np.ndarray:
    p = np.ascontiguousarray(params, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.float64).reshape(-1, NF)
    out = np.zeros((f.shape[0], 3))
    lib().qtmref_mlp_forward(_ptr(p), _ptr(f), f.shape[0], _ptr(out))
    return out


def mlp_loss_grad(params: np.ndarray, feat: np.ndarray, tgt: np.ndarray, want_grad: bool = True):
    p = np.ascontiguousarray(params, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.float64).reshape(-1, NF)
    t = np.ascontiguousarray(tgt, dtype=np.float64).reshape(-1, 3)
    g = np.zeros(mlp_nparam()) if want_grad else None
    L = lib().qtmref_mlp_loss_grad(_ptr(p), _ptr(f), _ptr(t), f.shape[0], _ptr(g))
    return L, g


def tableau():
    c, a, b, bs, dd = np.zeros(7), np.zeros((7, 6)), np.zeros(7), np.zeros(7), np.zeros(7)
    lib().qtmref_tableau(_ptr(c), _ptr(a), _ptr(b), _ptr(bs), _ptr(dd))
    return dict(c=c, a=a, b=b, bs=bs, dd=dd)


def snap_step(log_h: float) -> float:
    return lib().qtmref_snap_step(log_h)
