"""Seeded synthetic inputs for the quantum-trajectory engine and its oracle.

This module only builds the *inputs* of the method: the system Hamiltonian H,
the collapse operators C_n, the initial state psi0, the output times and the
expectation operators O_k.  It holds none of the method's arithmetic (no
effective Hamiltonian, no integration, no averaging); both the HIP library and
the CPU oracle form everything else themselves from these arrays.

Operators are returned as ``Op`` records in one of three storage formats:

* ``"dense"``: ``val`` is a complex128 array of shape (d, d), row-major;
* ``"csr"``:   ``val`` (nnz,) complex128, ``row_ptr`` (d+1,) int32,
  ``col_ind`` (nnz,) int32 (compressed sparse rows, the storage the paper
  uses for band-structured operators, Sec. 2.2 and the trilinear example
  of Sec. 4.2);
* ``"diag"``:  ``val`` (d,) complex128, the diagonal of a diagonal operator.

Workloads (names follow the paper's examples and the benchmark configs):

* ``two_level``       driven decaying two-level atom, H = (Omega/2) sigma_x,
                      C = sqrt(gamma) sigma_-;
* ``unitary_example`` the paper's unitary-Hamiltonian example (Sec. 4.1):
                      H = (2 pi/10) sigma_x, C0 = 0.05 sigma_x, E0 = sigma_z;
* ``jaynes_cummings`` cavity (Fock cutoff N) times a two-level atom (Sec. 4.3);
* ``tfim``            transverse-field Ising chain with per-site decay (CSR);
* ``hetero_batch``    random systems of mixed dimension;
* ``photon_birth_death`` the thermal cavity of Sec. 4.4;
* ``trilinear``       the optical parametric amplifier of Sec. 4.2 (CSR).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import factorial, sqrt
from typing import List, Optional

import numpy as np


@dataclass
class Op:
    fmt: str                      # "dense" | "csr" | "diag"
    dim: int
    val: np.ndarray               # complex128
    row_ptr: Optional[np.ndarray] = None   # int32, csr only
    col_ind: Optional[np.ndarray] = None   # int32, csr only

    def to_dense(self) -> np.ndarray:
        if self.fmt == "dense":
            return np.array(self.val, dtype=np.complex128)
        if self.fmt == "diag":
            return np.diag(np.asarray(self.val, dtype=np.complex128))
        out = np.zeros((self.dim, self.dim), dtype=np.complex128)
        for i in range(self.dim):
            for p in range(self.row_ptr[i], self.row_ptr[i + 1]):
                out[i, self.col_ind[p]] += self.val[p]
        return out

    @property
    def nnz(self) -> int:
        if self.fmt == "dense":
            return self.dim * self.dim
        return int(len(self.val))


@dataclass
class System:
    name: str
    H: Op
    c_ops: List[Op]
    psi0: np.ndarray              # complex128 (d,)
    tlist: np.ndarray             # float64 (n_t,), tlist[0] = t0
    e_ops: List[Op]
    meta: dict = field(default_factory=dict)
    # time-dependent terms: H(t) = H + sum_k f_k(t) H_k with f_k(t) = c + a cos(w t) + b sin(w t),
    # given as (H_k, (c, a, b, w)) pairs (the right-hand side of the paper's Sec. 3 takes t)
    td: list = field(default_factory=list)

    @property
    def dim(self) -> int:
        return self.H.dim


# ----------------------------------------------------------------- helpers
def dense(a) -> Op:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    assert a.ndim == 2 and a.shape[0] == a.shape[1]
    return Op("dense", a.shape[0], a)


def diag(v) -> Op:
    v = np.ascontiguousarray(np.asarray(v, dtype=np.complex128))
    return Op("diag", v.shape[0], v)


def csr_from_dense(a, drop_zeros: bool = True) -> Op:
    a = np.asarray(a, dtype=np.complex128)
    d = a.shape[0]
    rp = [0]
    ci: list = []
    vv: list = []
    for i in range(d):
        for j in range(d):
            if (not drop_zeros) or a[i, j] != 0:
                ci.append(j)
                vv.append(a[i, j])
        rp.append(len(ci))
    return Op("csr", d, np.array(vv, dtype=np.complex128),
              np.array(rp, dtype=np.int32), np.array(ci, dtype=np.int32))


def csr_from_triplets(d: int, rows, cols, vals) -> Op:
    """CSR from (row, col, value) triplets; duplicates are summed, columns sorted."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.complex128)
    key = rows * d + cols
    order = np.argsort(key, kind="stable")
    key, vals = key[order], vals[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, start) if len(vals) else vals
    r = (uniq // d).astype(np.int64)
    c = (uniq % d).astype(np.int32)
    rp = np.zeros(d + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return Op("csr", d, np.ascontiguousarray(summed), rp, np.ascontiguousarray(c))


def destroy(n: int) -> np.ndarray:
    """Bosonic lowering operator on the Fock cutoff {0..n-1}: a|k> = sqrt(k)|k-1>."""
    a = np.zeros((n, n), dtype=np.complex128)
    for k in range(1, n):
        a[k - 1, k] = sqrt(k)
    return a


def coherent_amplitudes(n: int, alpha: complex) -> np.ndarray:
    """Truncated Poisson amplitudes e^{-|a|^2/2} a^k/sqrt(k!), renormalised."""
    v = np.array([np.exp(-abs(alpha) ** 2 / 2) * alpha ** k / sqrt(factorial(k))
                  for k in range(n)], dtype=np.complex128)
    return v / np.linalg.norm(v)


SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


# --------------------------------------------------------------- workloads
def two_level(Omega: float = 1.0, gamma: float = 0.5, t_end: float = 10.0,
              n_t: int = 101) -> System:
    """Resonantly driven, decaying two-level atom.

    Basis |e> = (1, 0), |g> = (0, 1); sigma_- = |g><e|; psi0 = |g>;
    observable sigma_z = diag(1, -1).
    """
    sm = np.array([[0, 0], [1, 0]], dtype=np.complex128)
    H = dense(0.5 * Omega * SX)
    C = dense(sqrt(gamma) * sm)
    psi0 = np.array([0, 1], dtype=np.complex128)
    return System("two_level", H, [C], psi0, np.linspace(0.0, t_end, n_t),
                  [diag([1.0, -1.0])], dict(Omega=Omega, gamma=gamma))


def unitary_example(n_t: int = 101, c_scale: float = 0.05, t_end: float = 10.0) -> System:
    """The paper's first example (Sec. 4.1): H = (2 pi/10) sigma_x, psi0 = |0>,
    C0 = c_scale * sigma_x (0.05 in the paper), E0 = sigma_z, t in [0, 10]."""
    H = dense((2 * np.pi / 10) * SX)
    C = dense(c_scale * SX)
    return System("unitary_example", H, [C], np.array([1, 0], dtype=np.complex128),
                  np.linspace(0.0, t_end, n_t), [dense(SZ)], dict(c_scale=c_scale))


def two_channel_identity(a: float, b: float, t_end: float = 10.0, n_t: int = 11) -> System:
    """Two collapse operators whose C^dagger C are multiples of the identity:
    C1 = sqrt(a) sigma_x, C2 = sqrt(b) sigma_z, H = 0.3 sigma_y + 0.2 sigma_z.
    Every state then decays as exp(-(a+b) t) and channel 1 is chosen with
    probability a/(a+b) independently of the state."""
    H = dense(0.3 * SY + 0.2 * SZ)
    return System("two_channel_identity", H, [dense(sqrt(a) * SX), dense(sqrt(b) * SZ)],
                  np.array([1, 0], dtype=np.complex128), np.linspace(0.0, t_end, n_t),
                  [dense(SZ), dense(SX)], dict(a=a, b=b))


def jaynes_cummings(N: int = 20, g: float = 1.0, delta: float = 0.0, kappa: float = 0.1,
                    gamma_a: float = 0.05, alpha: complex = 2.0, t_end: float = 50.0,
                    n_t: int = 501, atom_excited: bool = True, fmt: str = "dense") -> System:
    """Cavity with Fock cutoff N times a two-level atom (paper Sec. 4.3).

    a = destroy(N) (x) I_2, sigma_- = I_N (x) destroy(2) (basis index 1 of the
    atom is the excited state), H = delta a^dag a + g (a^dag sigma_- + a sigma_+),
    C = {sqrt(kappa) a, sqrt(gamma_a) sigma_-} (each dropped when its rate is 0),
    psi0 = coherent(alpha) (x) |excited>.  Basis index = 2 n + s.
    Observables (diagonal): <a^dag a>, <sigma_+ sigma_->.
    """
    I2 = np.eye(2, dtype=np.complex128)
    IN = np.eye(N, dtype=np.complex128)
    a = np.kron(destroy(N), I2)
    sm = np.kron(IN, destroy(2))
    Hm = delta * a.conj().T @ a + g * (a.conj().T @ sm + a @ sm.conj().T)
    cops = []
    if kappa > 0:
        cops.append(np.sqrt(kappa) * a)
    if gamma_a > 0:
        cops.append(np.sqrt(gamma_a) * sm)
    atom = np.array([0, 1] if atom_excited else [1, 0], dtype=np.complex128)
    psi0 = np.kron(coherent_amplitudes(N, alpha), atom)
    n_diag = np.repeat(np.arange(N, dtype=np.float64), 2)
    e_diag = np.tile(np.array([0.0, 1.0]), N)
    mk = dense if fmt == "dense" else csr_from_dense
    return System("jaynes_cummings", mk(Hm), [mk(c) for c in cops], psi0,
                  np.linspace(0.0, t_end, n_t), [diag(n_diag), diag(e_diag)],
                  dict(N=N, g=g, delta=delta, kappa=kappa, gamma_a=gamma_a, alpha=alpha))


def tfim(L: int = 10, J: float = 1.0, h: float = 0.8, gamma: float = 0.05,
         t_end: float = 20.0, n_t: int = 201) -> System:
    """Open transverse-field Ising chain with per-site decay, in CSR.

    H = -J sum_{i<L-1} sz_i sz_{i+1} - h sum_i sx_i; C_i = sqrt(gamma) sigma_-^i
    (up -> down).  Site i is bit (L-1-i) of the basis index (site 0 is the most
    significant factor of the tensor product); bit value 0 = up (sz = +1).
    psi0 = all up = index 0.  Observables: <sz_i>, i = 0..L-1 (diagonal).
    """
    d = 1 << L
    idx = np.arange(d)
    bits = [((idx >> (L - 1 - i)) & 1) for i in range(L)]
    sz = [1 - 2 * b for b in bits]
    zz = np.zeros(d)
    for i in range(L - 1):
        zz += sz[i] * sz[i + 1]
    rows, cols, vals = [idx], [idx], [-J * zz]
    for i in range(L):
        rows.append(idx)
        cols.append(idx ^ (1 << (L - 1 - i)))
        vals.append(np.full(d, -h))
    H = csr_from_triplets(d, np.concatenate(rows), np.concatenate(cols),
                          np.concatenate(vals).astype(np.complex128))
    cops = []
    for i in range(L):
        up = idx[bits[i] == 0]
        cops.append(csr_from_triplets(d, up | (1 << (L - 1 - i)), up,
                                      np.full(len(up), sqrt(gamma), dtype=np.complex128)))
    psi0 = np.zeros(d, dtype=np.complex128)
    psi0[0] = 1.0
    e_ops = [diag(s.astype(np.float64)) for s in sz]
    return System("tfim", H, cops, psi0, np.linspace(0.0, t_end, n_t), e_ops,
                  dict(L=L, J=J, h=h, gamma=gamma))


def random_system(rng: np.random.Generator, d: int, n_c: int, t_end: float = 20.0,
                  n_t: int = 101, c_norm: float = 0.1) -> System:
    """One random system: H = (A + A^dag)/(2 sqrt(d)) with A complex Gaussian
    (unit variance per complex entry), C = c_norm * B/||B||_2 (spectral norm),
    psi0 = e_0, observables <H> (dense) and |0><0| (diagonal)."""
    A = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2)
    Hm = (A + A.conj().T) / (2 * np.sqrt(d))
    cops = []
    for _ in range(n_c):
        B = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2)
        cops.append(dense(c_norm * B / np.linalg.norm(B, 2)))
    psi0 = np.zeros(d, dtype=np.complex128)
    psi0[0] = 1.0
    p0 = np.zeros(d)
    p0[0] = 1.0
    return System(f"random_d{d}", dense(Hm), cops, psi0, np.linspace(0.0, t_end, n_t),
                  [dense(Hm), diag(p0)], dict(d=d, n_c=n_c))


def hetero_batch(n_sys: int = 64, d_min: int = 8, d_max: int = 256, key: int = 0,
                 t_end: float = 20.0, n_t: int = 101) -> List[System]:
    """Heterogeneous batch: n_sys random systems, d ~ U{d_min..d_max},
    n_c ~ U{1..4}, drawn from numpy Generator(Philox(key))."""
    rng = np.random.Generator(np.random.Philox(key=key))
    out = []
    for _ in range(n_sys):
        d = int(rng.integers(d_min, d_max + 1))
        n_c = int(rng.integers(1, 5))
        out.append(random_system(rng, d, n_c, t_end, n_t))
    return out


def photon_birth_death(N: int = 5, kappa: float = 1.0 / 0.129, n_th: float = 0.063,
                       t_end: float = 1.0, n_t: int = 101) -> System:
    """Thermal cavity of the paper's Sec. 4.4: H = a^dag a, psi0 = |1>,
    c0 = sqrt(kappa (1 + n_th)) a, c1 = sqrt(kappa n_th) a^dag, observable a^dag a."""
    a = destroy(N)
    psi0 = np.zeros(N, dtype=np.complex128)
    psi0[1] = 1.0
    return System("photon_birth_death", dense(a.conj().T @ a),
                  [dense(np.sqrt(kappa * (1 + n_th)) * a), dense(np.sqrt(kappa * n_th) * a.conj().T)],
                  psi0, np.linspace(0.0, t_end, n_t), [diag(np.arange(N, dtype=np.float64))],
                  dict(N=N, kappa=kappa, n_th=n_th))


def trilinear(N: int = 8, K: float = 1.0, gammas=(0.1, 0.1, 0.4), alpha: float = sqrt(3.0),
              t_end: float = 4.0, n_t: int = 100) -> System:
    """Optical parametric amplifier of the paper's Sec. 4.2 in CSR:
    H = i K (a b^dag c^dag - a^dag b c), psi0 = |alpha>|0>|0>,
    c_i = sqrt(2 gamma_i) a_i, observables n_i = a_i^dag a_i."""
    d1 = destroy(N)
    I = np.eye(N, dtype=np.complex128)
    a0 = np.kron(np.kron(d1, I), I)
    a1 = np.kron(np.kron(I, d1), I)
    a2 = np.kron(np.kron(I, I), d1)
    Hm = 1j * K * (a0 @ a1.conj().T @ a2.conj().T - a0.conj().T @ a1 @ a2)
    vac = np.zeros(N, dtype=np.complex128)
    vac[0] = 1
    psi0 = np.kron(np.kron(coherent_amplitudes(N, alpha), vac), vac)
    cops = [csr_from_dense(np.sqrt(2 * g) * a) for g, a in zip(gammas, (a0, a1, a2))]
    e_ops = [diag(np.real(np.diag(a.conj().T @ a))) for a in (a0, a1, a2)]
    return System("trilinear", csr_from_dense(Hm), cops, psi0, np.linspace(0.0, t_end, n_t),
                  e_ops, dict(N=N, K=K, gammas=gammas, alpha=alpha))


def driven_two_level(Delta: float = 1.0, Omega: float = 2.0, omega: float = 1.0, gamma: float = 0.5,
                     t_end: float = 10.0, n_t: int = 101) -> System:
    """Two-level atom driven by a classical field without the rotating-wave
    approximation: H(t) = (Delta/2) sigma_z + Omega cos(omega t) sigma_x,
    C = sqrt(gamma) sigma_-, psi0 = |g>, observables sigma_z and sigma_x."""
    sm = np.array([[0, 0], [1, 0]], dtype=np.complex128)
    s = System("driven_two_level", dense(0.5 * Delta * SZ), [dense(sqrt(gamma) * sm)],
               np.array([0, 1], dtype=np.complex128), np.linspace(0.0, t_end, n_t),
               [diag([1.0, -1.0]), dense(SX)], dict(Delta=Delta, Omega=Omega, omega=omega, gamma=gamma))
    s.td = [(dense(SX), (0.0, Omega, 0.0, omega))]
    return s


def commuting_drive(c: float = 0.3, a: float = 0.8, b: float = -0.4, w: float = 1.7, gamma: float = 0.2,
                    t_end: float = 6.0, n_t: int = 61) -> System:
    """H(t) = f(t) sigma_x with f(t) = c + a cos(w t) + b sin(w t) and C = sqrt(gamma) I:
    the no-jump state is exp(-i F(t) sigma_x) psi0 e^(-gamma t / 2) with F the integral
    of f, jumps leave the normalised state unchanged, so <sigma_z>(t) = cos(2 F(t))
    on every trajectory for psi0 = |e>."""
    s = System("commuting_drive", dense(np.zeros((2, 2), dtype=np.complex128)),
               [dense(sqrt(gamma) * np.eye(2, dtype=np.complex128))], np.array([1, 0], dtype=np.complex128),
               np.linspace(0.0, t_end, n_t), [diag([1.0, -1.0])], dict(c=c, a=a, b=b, w=w, gamma=gamma))
    s.td = [(dense(SX), (c, a, b, w))]
    return s


def driven_jaynes_cummings(N: int = 20, eps: float = 0.3, omega_d: float = 1.0, t_end: float = 20.0,
                           n_t: int = 201, **kw) -> System:
    """The Jaynes-Cummings system of jaynes_cummings() with the cavity driven by a
    classical field: H(t) = H_JC + eps cos(omega_d t) (a + a^dag) (d = 2 N, dense)."""
    s = jaynes_cummings(N=N, t_end=t_end, n_t=n_t, **kw)
    a = np.kron(destroy(N), np.eye(2, dtype=np.complex128))
    s.name = "driven_jaynes_cummings"
    s.td = [(dense(a + a.conj().T), (0.0, eps, 0.0, omega_d))]
    s.meta.update(eps=eps, omega_d=omega_d)
    return s


def by_name(name: str, **kw) -> System:
    return {"two_level": two_level, "unitary_example": unitary_example,
            "jaynes_cummings": jaynes_cummings, "tfim": tfim,
            "photon_birth_death": photon_birth_death, "trilinear": trilinear}[name](**kw)
