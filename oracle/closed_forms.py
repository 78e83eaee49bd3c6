"""Closed-form solutions that pin the oracle (test infrastructure).

Each function states the model it solves; all use hbar = 1 and the
Lindblad master equation of the paper's Sec. 2.2.
"""
from __future__ import annotations

from math import factorial

import numpy as np


def two_level_sz(t, Omega: float = 1.0, gamma: float = 0.5):
    """<sigma_z>(t) of the resonantly driven decaying two-level atom
    (H = (Omega/2) sigma_x, C = sqrt(gamma) sigma_-), starting in |g>
    (Torrey's solution of the optical Bloch equations).

    Bloch equations: u' = 0, v' = -(gamma/2) v - Omega w, w' = Omega v - gamma (w + 1)
    with w = <sigma_z>.  The steady state is w_ss = -gamma^2/(gamma^2 + 2 Omega^2) and
    the transient decays as exp(-3 gamma t/4) with frequency mu = sqrt(Omega^2 - gamma^2/16).
    """
    t = np.asarray(t, dtype=np.float64)
    g, W = gamma, Omega
    mu = np.sqrt(W * W - g * g / 16.0)
    wss = -g * g / (g * g + 2 * W * W)
    return wss - (1.0 + wss) * np.exp(-0.75 * g * t) * (np.cos(mu * t) + (0.75 * g / mu) * np.sin(mu * t))


def two_level_nojump_survival(tau, Omega: float = 1.0, gamma: float = 0.5):
    """No-jump probability ||exp(M tau)|g>||^2 for the driven two-level atom,
    M = -i (Omega/2) sigma_x - (gamma/2) |e><e|."""
    tau = np.asarray(tau, dtype=np.float64)
    W, g = Omega, gamma
    mu = np.sqrt(W * W / 4.0 - g * g / 16.0)
    return np.exp(-g * tau / 2) * ((W * W / (4 * mu * mu)) * np.sin(mu * tau) ** 2
                                   + (np.cos(mu * tau) + (g / (4 * mu)) * np.sin(mu * tau)) ** 2)


def unitary_example_sz(t, c_scale: float = 0.05):
    """The paper's Sec. 4.1 model: H = (2 pi/10) sigma_x, C = c sigma_x, psi0 = |0>.
    Both terms conserve <sigma_x>; (y, z) rotate at 2 omega = 0.4 pi and decay at 2 c^2:
    <sigma_z>(t) = exp(-2 c^2 t) cos(0.4 pi t)."""
    t = np.asarray(t, dtype=np.float64)
    return np.exp(-2 * c_scale ** 2 * t) * np.cos(0.4 * np.pi * t)


def unitary_example_nojump_norm(t, c_scale: float = 0.05):
    """||psi(t)||^2 without jumps: C^dag C = c^2 I, so the norm is exp(-c^2 t)."""
    return np.exp(-c_scale ** 2 * np.asarray(t, dtype=np.float64))


def jcm_excited_population(t, N: int = 20, alpha: float = 2.0, g: float = 1.0):
    """Closed Jaynes-Cummings model (no decay, zero detuning), atom excited,
    cavity in the truncated coherent state: P_e(t) = sum_n p_n cos^2(g sqrt(n+1) t)
    on the Fock cutoff N (the top level n = N-1 does not couple and keeps P_e = 1)."""
    t = np.asarray(t, dtype=np.float64)
    amp = np.array([np.exp(-alpha ** 2 / 2) * alpha ** n / np.sqrt(float(factorial(n))) for n in range(N)])
    p = amp ** 2 / np.sum(amp ** 2)
    out = np.zeros_like(t)
    for n in range(N):
        out += p[n] * (np.cos(g * np.sqrt(n + 1) * t) ** 2 if n < N - 1 else 1.0)
    return out


def photon_number(t, kappa: float = 1.0 / 0.129, n_th: float = 0.063):
    """Thermal damping of one photon (Sec. 4.4 model, untruncated):
    <n>(t) = n_th + (1 - n_th) exp(-kappa t)."""
    t = np.asarray(t, dtype=np.float64)
    return n_th + (1.0 - n_th) * np.exp(-kappa * t)


def identity_channel_jumps(r_seq, u_seq, a: float, b: float, t_end: float):
    """Jumps for C1 = sqrt(a) sigma_x, C2 = sqrt(b) sigma_z (both C^dag C ~ I):
    every segment decays as exp(-(a+b) t), so segment j ends after -ln(r_j)/(a+b)
    and channel 0 is taken iff u_j <= a/(a+b).  Returns (times, channels)."""
    times, chans, t = [], [], 0.0
    for r, u in zip(r_seq, u_seq):
        t = t - np.log(r) / (a + b)
        if t >= t_end:
            break
        times.append(t)
        chans.append(0 if u * (a + b) <= a else 1)
    return np.array(times), np.array(chans, dtype=np.int32)
