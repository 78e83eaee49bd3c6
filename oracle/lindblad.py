"""Brute-force Lindblad integration (test infrastructure).

The trajectory average converges to Tr(O rho(t)) where rho solves the
Lindblad master equation of the paper's Sec. 2.2 (hbar = 1):

    rho' = -i [H, rho] + sum_n ( C_n rho C_n^dag - 1/2 {C_n^dag C_n, rho} ).

Two independent routes:
* ``expect_expm``: the Liouvillian superoperator (column-stacking vec,
  vec(A rho B) = (B^T kron A) vec(rho)) exponentiated with scipy.linalg.expm,
  for d up to about 40;
* ``expect_ode``: the matrix equation integrated with scipy's DOP853 at tight
  tolerance using sparse operators, for larger d, and for time-dependent
  Hamiltonians H(t) = H + sum_k f_k(t) H_k (a system's ``td`` list).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.integrate import solve_ivp


def _dense(op) -> np.ndarray:
    return op.to_dense()


def _sparse(op):
    if op.fmt == "csr":
        return sp.csr_matrix((op.val, op.col_ind, op.row_ptr), shape=(op.dim, op.dim))
    if op.fmt == "diag":
        return sp.diags(op.val).tocsr()
    return sp.csr_matrix(op.val)


def liouvillian(system) -> np.ndarray:
    d = system.dim
    I = np.eye(d, dtype=np.complex128)
    H = _dense(system.H)
    L = -1j * (np.kron(I, H) - np.kron(H.T, I))
    for c in system.c_ops:
        Cm = _dense(c)
        CdC = Cm.conj().T @ Cm
        L += np.kron(Cm.conj(), Cm) - 0.5 * np.kron(I, CdC) - 0.5 * np.kron(CdC.T, I)
    return L


def expect_expm(system) -> np.ndarray:
    """Tr(O_e rho(t_k)) for every e, k by exact exponentiation; returns [n_e, n_t] complex."""
    d = system.dim
    L = liouvillian(system)
    rho0 = np.outer(system.psi0, system.psi0.conj())
    v = rho0.reshape(-1, order="F")
    out = np.zeros((len(system.e_ops), len(system.tlist)), dtype=np.complex128)
    O = [_dense(o) for o in system.e_ops]
    t_prev = system.tlist[0]
    props = {}   # one propagator per distinct time step (uniform grids need one)
    for k, t in enumerate(system.tlist):
        if t != t_prev:
            dt = t - t_prev
            key = round(dt, 12)
            if key not in props:
                props[key] = sla.expm(L * dt)
            v = props[key] @ v
            t_prev = t
        rho = v.reshape(d, d, order="F")
        for e, Om in enumerate(O):
            out[e, k] = np.trace(Om @ rho)
    return out


def expect_ode(system, rtol: float = 1e-10, atol: float = 1e-12) -> np.ndarray:
    """Same quantity from the matrix equation rho' = M rho + rho M^dag + sum C rho C^dag,
    M = -i H - 1/2 sum C^dag C, integrated with DOP853; returns [n_e, n_t] complex."""
    d = system.dim
    H = _sparse(system.H)
    Cs = [_sparse(c) for c in system.c_ops]
    Mx = (-1j * H).tocsr()
    for Cm in Cs:
        Mx = (Mx - 0.5 * (Cm.conj().T @ Cm)).tocsr()

    # time-dependent terms H_k with coefficients f_k(t) = c + a cos(w t) + b sin(w t)
    td = [(_sparse(op), cf) for op, cf in (getattr(system, "td", None) or [])]

    def rhs(t, y):
        rho = y.reshape(d, d)
        Mt = Mx
        for Hk, (c, a, b, w) in td:
            Mt = Mt - 1j * (c + a * np.cos(w * t) + b * np.sin(w * t)) * Hk
        # rho M^dag = (M rho^dag)^dag and C rho C^dag = C (C rho^dag)^dag
        out = Mt @ rho + (Mt @ rho.conj().T).conj().T
        for Cm in Cs:
            out = out + Cm @ (Cm @ rho.conj().T).conj().T
        return out.reshape(-1)

    rho0 = np.outer(system.psi0, system.psi0.conj()).astype(np.complex128)
    sol = solve_ivp(rhs, (system.tlist[0], system.tlist[-1]), rho0.reshape(-1), method="DOP853",
                    t_eval=system.tlist, rtol=rtol, atol=atol)
    Os = [_sparse(o) for o in system.e_ops]
    out = np.zeros((len(system.e_ops), len(system.tlist)), dtype=np.complex128)
    for k in range(len(system.tlist)):
        rho = sol.y[:, k].reshape(d, d)
        for e, Om in enumerate(Os):
            out[e, k] = (Om @ rho).diagonal().sum()
    return out
