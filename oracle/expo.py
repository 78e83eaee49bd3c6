"""Oracle of the exact-propagator (stiff) form -- TEST INFRASTRUCTURE ONLY.

For a time-independent effective Hamiltonian the no-jump evolution of Algorithm 1
(Sec. 2.2) has the closed form psi(t) = exp((t - t_s) M) psi_s, M = -i H_eff, from
the segment start (t_s, psi_s): its stiffness (the paper's reason for offering BDF,
Sec. 2.1) then costs nothing.  This module writes the method out with that exact
solution, using scipy's matrix exponential as a library primitive:

* the squared norm n(t) = ||psi(t)||^2 is non-increasing (d n/dt = -sum_n ||C_n psi||^2),
  so the jump time of a segment with threshold r is the unique first t with
  n(t) = r, found by bisection to 1e-13 after bracketing it between the output
  times (the first output time whose norm is below r);
* the channel choice, the jump and the random streams follow the DOPRI5 oracle
  (qtm_oracle.cpp): Philox4x64-10 with key (seed, system) and counter
  (trajectory, segment, 0, 0), word 0 -> r, word 1 -> channel uniform; smallest
  channel whose cumulative probability reaches u times the total;
* outputs <psi|O|psi>/<psi|psi> at the output times, t_k == t* from the
  post-jump state.
The output times must be uniformly spaced (the library's form steps on that grid).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import build_M, philox4x64_10, uniform53


def _expect(O, psi):
    nn = np.vdot(psi, psi).real
    return np.array([np.vdot(psi, o @ psi) / nn for o in O])


def run_expo(system, ntraj: int, seed: int = 0, sys_id: int = 0, traj_begin: int = 0, jcap: int = 32) -> dict:
    s = system
    M = build_M(s.H, s.c_ops)
    C = [c.to_dense() for c in s.c_ops]
    O = [o.to_dense() for o in s.e_ops]
    tl = np.asarray(s.tlist, dtype=np.float64)
    n_t, n_e = len(tl), len(O)
    dt = (tl[-1] - tl[0]) / (n_t - 1)
    E = sla.expm(dt * M)                        # propagator over one output interval
    X = np.zeros((ntraj, n_e, n_t), dtype=np.complex128)
    jt = np.zeros((ntraj, jcap))
    jc = np.zeros((ntraj, jcap), dtype=np.int32)
    jn = np.zeros(ntraj, dtype=np.int64)
    for q in range(ntraj):
        traj = traj_begin + q
        seg = 0

        def draw(j):
            w = philox4x64_10([traj, j, 0, 0], [seed, sys_id])
            return uniform53(int(w[0])), uniform53(int(w[1]))

        r, u = draw(seg)
        psi = np.array(s.psi0, dtype=np.complex128)
        t_a, psi_a = tl[0], psi.copy()          # last known point of the current segment
        X[q, :, 0] = _expect(O, psi)
        k = 0
        while k < n_t - 1:
            # the state at the next output time
            if t_a == tl[k]:
                psi_b = E @ psi_a
            else:
                psi_b = sla.expm((tl[k + 1] - t_a) * M) @ psi_a
            if np.vdot(psi_b, psi_b).real >= r:
                k += 1
                t_a, psi_a = tl[k], psi_b
                X[q, :, k] = _expect(O, psi_a)
                continue
            # jump inside (t_a, t_{k+1}): bisection on the exact norm
            lo, hi = t_a, tl[k + 1]
            while hi - lo > 1e-13:
                mid = 0.5 * (lo + hi)
                p = sla.expm((mid - t_a) * M) @ psi_a
                if np.vdot(p, p).real < r:
                    hi = mid
                else:
                    lo = mid
            ts = 0.5 * (lo + hi)
            star = sla.expm((ts - t_a) * M) @ psi_a
            pn = np.array([np.vdot(c @ star, c @ star).real for c in C])
            tot = pn.sum()
            ch = -1
            if tot > 0.0:
                cum = np.cumsum(pn)
                for n in range(len(C)):
                    if pn[n] > 0.0 and cum[n] >= u * tot:
                        ch = n
                        break
                if ch < 0:
                    ch = int(np.nonzero(pn > 0.0)[0][-1])
            if ch >= 0:
                new = (C[ch] @ star) / np.sqrt(pn[ch])
            else:
                new = star / np.sqrt(np.vdot(star, star).real)
            if jn[q] < jcap:
                jt[q, jn[q]], jc[q, jn[q]] = ts, ch
            jn[q] += 1
            seg += 1
            r, u = draw(seg)
            t_a, psi_a = ts, new
            if tl[k + 1] == ts:              # output at the jump time: the post-jump state
                k += 1
                X[q, :, k] = _expect(O, psi_a)
    mean = X.mean(axis=0)
    var = np.maximum((X.real ** 2).mean(axis=0) - mean.real ** 2, 0.0)
    return dict(X=X, mean=mean, var=var, jump_times=jt, jump_channels=jc, jump_counts=jn)
