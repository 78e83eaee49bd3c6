"""Pins of the CPU oracle against things other than itself (no GPU).

* Philox4x64-10 against numpy's independent implementation.
* The Dormand-Prince tableau and its dense output against exact rational
  order conditions (sympy), and the oracle's coefficient table against those
  rationals; the oracle's step against the matrix exponential (convergence
  order), and its whole step sequence against scipy's RK45.
* M = -i H_eff against the values the paper prints for its first example.
* Jump times and channels against a closed form; the failure path.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import sympy as sy
from scipy.integrate import RK45

import oracle
import workloads as w
from oracle import closed_forms as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox
def _numpy_block(ctr, key):
    """numpy's Philox pre-increments the 256-bit counter before each block."""
    c = int(ctr[0]) | (int(ctr[1]) << 64) | (int(ctr[2]) << 128) | (int(ctr[3]) << 192)
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    g = np.random.Philox(counter=np.array(words, dtype=np.uint64),
                         key=np.array([int(key[0]), int(key[1])], dtype=np.uint64))
    return g.random_raw(4)


@pytest.mark.parametrize("ctr,key", [((0, 0, 0, 0), (0, 0)), ((1, 0, 0, 0), (5, 7)),
                                     ((12345, 7, 0, 0), (0, 3)), ((2**64 - 1, 2, 9, 1), (2**63 + 11, 42)),
                                     ((0, 1, 0, 0), (2**64 - 1, 2**64 - 1))])
def test_philox_matches_numpy(ctr, key):
    assert np.array_equal(oracle.philox4x64_10(ctr, key), _numpy_block(ctr, key))


def test_uniform53_range_and_mapping():
    assert oracle.uniform53(0) == 0.5 * 2.0 ** -53
    assert oracle.uniform53(2**64 - 1) == 1.0 - 0.5 * 2.0 ** -53
    assert oracle.uniform53(1 << 63) == 0.5 + 0.5 * 2.0 ** -53


# --------------------------------------------------------------- tableau
R = sy.Rational
C_EX = [R(0), R(1, 5), R(3, 10), R(4, 5), R(8, 9), R(1), R(1)]
A_EX = [[],
        [R(1, 5)],
        [R(3, 40), R(9, 40)],
        [R(44, 45), R(-56, 15), R(32, 9)],
        [R(19372, 6561), R(-25360, 2187), R(64448, 6561), R(-212, 729)],
        [R(9017, 3168), R(-355, 33), R(46732, 5247), R(49, 176), R(-5103, 18656)],
        [R(35, 384), R(0), R(500, 1113), R(125, 192), R(-2187, 6784), R(11, 84)]]
B_EX = [R(35, 384), R(0), R(500, 1113), R(125, 192), R(-2187, 6784), R(11, 84), R(0)]
BS_EX = [R(5179, 57600), R(0), R(7571, 16695), R(393, 640), R(-92097, 339200), R(187, 2100), R(1, 40)]
D_EX = [R(-12715105075, 11282082432), R(0), R(87487479700, 32700410799), R(-10690763975, 1880347072),
        R(701980252875, 199316789632), R(-1453857185, 822651844), R(69997945, 29380423)]


def _amat():
    A = sy.zeros(7, 7)
    for s in range(7):
        for j, v in enumerate(A_EX[s]):
            A[s, j] = v
    return A


def _conditions(bvec, order, scale=lambda k: 1):
    """Butcher order conditions up to ``order``; returns list of (lhs, rhs)."""
    A = _amat()
    c = sy.Matrix(C_EX)
    b = sy.Matrix(bvec).T
    one = sy.ones(7, 1)
    cp = lambda k: c.applyfunc(lambda x: x ** k)
    had = lambda u, v: sy.Matrix([u[i] * v[i] for i in range(7)])
    conds = [(b * one, 1, 1)]
    if order >= 2:
        conds += [(b * c, R(1, 2), 2)]
    if order >= 3:
        conds += [(b * cp(2), R(1, 3), 3), (b * A * c, R(1, 6), 3)]
    if order >= 4:
        conds += [(b * cp(3), R(1, 4), 4), (b * had(c, A * c), R(1, 8), 4), (b * A * cp(2), R(1, 12), 4),
                  (b * A * A * c, R(1, 24), 4)]
    if order >= 5:
        Ac = A * c
        conds += [(b * cp(4), R(1, 5), 5), (b * had(cp(2), Ac), R(1, 10), 5), (b * had(c, A * cp(2)), R(1, 15), 5),
                  (b * had(c, A * Ac), R(1, 30), 5), (b * had(Ac, Ac), R(1, 20), 5), (b * A * cp(3), R(1, 20), 5),
                  (b * A * had(c, Ac), R(1, 40), 5), (b * A * A * cp(2), R(1, 60), 5), (b * A * A * Ac, R(1, 120), 5)]
    return [(lhs[0, 0], rhs * scale(p)) for lhs, rhs, p in conds]


def test_tableau_row_sums():
    for s in range(7):
        assert sum(A_EX[s], R(0)) == C_EX[s]
    assert A_EX[6] == B_EX[:6]


def test_tableau_order_conditions():
    c5 = _conditions(B_EX, 5)
    assert len(c5) == 17
    for lhs, rhs in c5:
        assert sy.simplify(lhs - rhs) == 0
    for lhs, rhs in _conditions(BS_EX, 4):
        assert sy.simplify(lhs - rhs) == 0
    # the embedded 4th-order weights are not 5th order (otherwise no error estimate)
    assert any(sy.simplify(l - r) != 0 for l, r in _conditions(BS_EX, 5)[8:])


def test_dense_output_order_conditions():
    th = sy.Symbol("theta")
    b = sy.Matrix(B_EX)
    e1 = sy.Matrix([1, 0, 0, 0, 0, 0, 0])
    e7 = sy.Matrix([0, 0, 0, 0, 0, 0, 1])
    dd = sy.Matrix(D_EX)
    # u(th) = y + th (Delta + (1-th)(B + th (R4 + (1-th) R5)))  with
    # Delta = h b.k, B = h k1 - Delta, R4 = Delta - h k7 - B, R5 = h d.k
    bt = th * (b + (1 - th) * ((e1 - b) + th * ((b - e7 - (e1 - b)) + (1 - th) * dd)))
    bt = bt.applyfunc(sy.expand)
    for lhs, rhs in _conditions(list(bt), 4, scale=lambda p: th ** p):
        assert sy.expand(lhs - rhs) == 0
    assert (bt.subs(th, 1) - b).applyfunc(sy.simplify) == sy.zeros(7, 1)
    # derivative at theta = 0 is k1 and at theta = 1 is k7
    dbt = bt.diff(th)
    assert (dbt.subs(th, 0) - e1).applyfunc(sy.simplify) == sy.zeros(7, 1)
    assert (dbt.subs(th, 1) - e7).applyfunc(sy.simplify) == sy.zeros(7, 1)


def test_oracle_table_equals_rationals():
    t = oracle.tableau()
    f = lambda v: float(v)
    assert np.array_equal(t["c"], [f(v) for v in C_EX])
    for s in range(7):
        for j in range(6):
            ex = f(A_EX[s][j]) if j < len(A_EX[s]) else 0.0
            assert t["a"][s, j] == ex, (s, j)
    assert np.array_equal(t["b"], [f(v) for v in B_EX])
    assert np.array_equal(t["bs"], [f(v) for v in BS_EX])
    assert np.array_equal(t["dd"], [f(v) for v in D_EX])


def test_step_convergence_orders():
    """Local error of y_new ~ h^6, of the error estimate ~ h^5 and of the dense
    output ~ h^5 on a linear system, against scipy's matrix exponential."""
    rng = np.random.default_rng(3)
    d = 5
    M = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) * 0.5
    y0 = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    hs = [0.2, 0.1, 0.05]
    th = 0.37
    ey, ee, eu = [], [], []
    for h in hs:
        ynew, evec, _, u = oracle.dopri_step(M, y0, h, thetas=[th])
        ey.append(np.linalg.norm(ynew - sla.expm(M * h) @ y0))
        ee.append(np.linalg.norm(evec))
        eu.append(np.linalg.norm(u[0] - sla.expm(M * th * h) @ y0))
    for errs, order in ((ey, 6), (ee, 5), (eu, 5)):
        slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
        assert all(abs(s - order) < 0.6 for s in slopes), (order, slopes)


def test_dense_output_endpoints():
    rng = np.random.default_rng(4)
    d = 3
    M = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    y0 = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    ynew, _, _, u = oracle.dopri_step(M, y0, 0.1, thetas=[0.0, 1.0])
    assert np.allclose(u[0], y0, atol=0, rtol=1e-15)
    assert np.allclose(u[1], ynew, atol=1e-15, rtol=1e-14)


# ------------------------------------------------------------- H_eff / M
def test_M_matches_paper_printed_example():
    rows = np.loadtxt(os.path.join(GOLDEN, "unitary_example_rhs.txt"))
    s = w.unitary_example()
    M = oracle.build_M(s.H, s.c_ops)
    for r, c, re, im in rows:
        assert abs(M[int(r), int(c)] - (re + 1j * im)) < 5e-9


def test_M_sparse_equals_dense_and_definition():
    """CSR assembly equals the dense one, and both equal -iH - 1/2 sum C^dag C
    written with numpy (photon model: a and a^dag catch a transposed product)."""
    s = w.photon_birth_death()
    Md = oracle.build_M(s.H, s.c_ops)
    Hs = w.csr_from_dense(s.H.to_dense())
    Cs = [w.csr_from_dense(c.to_dense()) for c in s.c_ops]
    Ms = oracle.build_M(Hs, Cs)
    ref = -1j * s.H.to_dense() - 0.5 * sum(c.to_dense().conj().T @ c.to_dense() for c in s.c_ops)
    assert np.allclose(Md, ref, atol=1e-14)
    assert np.allclose(Ms, ref, atol=1e-14)
    # C^dag C != C C^dag here, so the order of the product matters
    a = s.c_ops[0].to_dense()
    assert not np.allclose(a.conj().T @ a, a @ a.conj().T)


# ----------------------------------------------------- stepper vs scipy
@pytest.mark.parametrize("make", [lambda: w.jaynes_cummings(N=10, t_end=5.0),
                                  lambda: w.two_level(),
                                  lambda: w.photon_birth_death()])
def test_step_sequence_matches_scipy_rk45(make):
    s = make()
    M = oracle.build_M(s.H, s.c_ops)
    t0, t1 = s.tlist[0], s.tlist[-1]
    ts, yend, h0 = oracle.integrate_nojump(M, s.psi0, t0, t1, 1e-6, 1e-8)
    solver = RK45(lambda t, y: M @ y, t0, s.psi0.astype(np.complex128), t1, rtol=1e-6, atol=1e-8)
    ref = []
    while solver.status == "running":
        solver.step()
        ref.append(solver.t)
    assert len(ts) == len(ref)
    assert np.max(np.abs(ts - np.array(ref))) < 1e-9
    assert np.allclose(yend, solver.y, rtol=0, atol=1e-10)


# ----------------------------------------------------------- jump times
def _uniforms(traj, n, seed=0, sys_id=0):
    r, u = [], []
    for j in range(n):
        x = _numpy_block((traj, j, 0, 0), (seed, sys_id))
        r.append(((int(x[0]) >> 11) + 0.5) * 2.0 ** -53)
        u.append(((int(x[1]) >> 11) + 0.5) * 2.0 ** -53)
    return r, u


@pytest.mark.parametrize("rtol,tol", [(1e-6, 2e-5), (1e-10, 1e-8)])
def test_jump_times_and_channels_closed_form(rtol, tol):
    a, b = 0.3, 0.2
    s = w.two_channel_identity(a, b, t_end=10.0)
    res = oracle.run(s, 40, seed=11, rtol=rtol, atol=rtol * 1e-2)
    assert res["status"] == 0
    total = 0
    for i in range(40):
        r, u = _uniforms(i, 40, seed=11)
        t_ex, c_ex = cf.identity_channel_jumps(r, u, a, b, 10.0)
        n = res["jump_counts"][i]
        assert n == len(t_ex), i
        assert np.all(np.abs(res["jump_times"][i, :n] - t_ex) < tol * (1 + np.arange(n)))
        assert np.array_equal(res["jump_channels"][i, :n], c_ex)
        total += n
    assert total > 100   # the closed form is exercised with many jumps


def test_first_jump_time_unitary_example():
    """Sec. 4.1 model with the decay scaled up: ||psi||^2 = exp(-c^2 t) exactly,
    so the first jump is at -ln(r_0)/c^2."""
    c = 0.5
    s = w.unitary_example(c_scale=c, t_end=10.0, n_t=11)
    res = oracle.run(s, 30, seed=5, rtol=1e-9, atol=1e-11)
    for i in range(30):
        r, _ = _uniforms(i, 1, seed=5)
        t1 = -np.log(r[0]) / c ** 2
        if t1 < 10.0:
            assert res["jump_counts"][i] >= 1
            assert abs(res["jump_times"][i, 0] - t1) < 1e-7
        else:
            assert res["jump_counts"][i] == 0


def test_counter_layout_trajectory_offset():
    """Trajectory i uses counter (i, segment): running [k, N) alone equals the
    tail of one [0, N) run, so ranges can be merged (sharding property)."""
    s = w.two_level()
    full = oracle.run(s, 60, seed=3)
    tail = oracle.run(s, 20, seed=3, traj_begin=40)
    assert np.array_equal(full["X"][40:], tail["X"])
    head = oracle.run(s, 40, seed=3)
    merged = (head["mean"] * 40 + tail["mean"] * 20) / 60
    assert np.allclose(merged, full["mean"], atol=1e-13)


def test_failure_path_max_steps():
    s = w.two_level()
    res = oracle.run(s, 5, seed=0, traj_begin=7, max_steps=3)
    assert res["status"] == -4
    assert res["fail_traj"] == 7


# ------------------------------------------------- rejection branch vs scipy
@pytest.mark.parametrize("make,scale", [(lambda: w.jaynes_cummings(N=10, t_end=5.0), 40.0),
                                        (lambda: w.two_level(), 60.0),
                                        (lambda: w.photon_birth_death(), 30.0)])
def test_rejection_branch_matches_scipy_rk45(make, scale):
    """A first step far above the starting-step rule's forces rejected attempts.
    scipy's RK45 (same pair, same standard controller: shrink by
    max(0.2, 0.9 err^-1/5) on rejection, no growth on the step after a rejection)
    given the same first step takes the same accepted times and the same number of
    rejections.  scipy's attempts are counted from its right-hand-side evaluations:
    one for f(t0), then six per attempted step (FSAL)."""
    s = make()
    M = oracle.build_M(s.H, s.c_ops)
    t0, t1 = s.tlist[0], s.tlist[-1]
    _, _, h_rule = oracle.integrate_nojump(M, s.psi0, t0, t1, 1e-6, 1e-8)
    h_first = min(scale * h_rule, 0.5 * (t1 - t0))
    ts, yend, h0, nrej = oracle.integrate_nojump(M, s.psi0, t0, t1, 1e-6, 1e-8, first_step=h_first,
                                                 with_rejections=True)
    assert h0 == h_first
    solver = RK45(lambda t, y: M @ y, t0, s.psi0.astype(np.complex128), t1, rtol=1e-6, atol=1e-8,
                  first_step=h_first)
    ref = []
    while solver.status == "running":
        solver.step()
        ref.append(solver.t)
    attempts = (solver.nfev - 1) // 6
    assert (solver.nfev - 1) % 6 == 0
    scipy_rej = attempts - len(ref)
    print(f"accepted {len(ref)}, rejected {scipy_rej} (oracle {nrej})")
    assert scipy_rej >= 1                      # the rejection branch is exercised
    assert nrej == scipy_rej
    assert len(ts) == len(ref)
    assert np.max(np.abs(ts - np.array(ref))) < 1e-9
    assert np.allclose(yend, solver.y, rtol=0, atol=1e-10)


# --------------------------------------------- segment-start features at t0
def test_features_at_t0_closed_form():
    """The learned form's 16 segment-start features of the first segment, for the
    Jaynes-Cummings workload: the atom starts excited (population 1); the cavity
    populations are the truncated, renormalised Poisson weights of the coherent
    state, e^-|a|^2 |a|^2n / n!; <C_1^dag C_1> = kappa <n>; <C_2^dag C_2> = gamma_a
    (excited atom); log r of the segment's Philox threshold; elapsed fraction 0."""
    from math import factorial
    N, alpha, kappa, gamma_a = 20, 2.0, 0.1, 0.05
    s = w.jaynes_cummings(N=N, alpha=alpha, kappa=kappa, gamma_a=gamma_a, t_end=2.0, n_t=21)
    d = s.dim
    f_ops = [w.diag(np.tile([0.0, 1.0], N))]
    for n in range(11):
        v = np.zeros(d)
        v[2 * n:2 * n + 2] = 1.0
        f_ops.append(w.diag(v))
    res = oracle.run(s, 5, seed=4, f_ops=f_ops, seg_cap=2)
    p = np.array([np.exp(-alpha ** 2) * alpha ** (2 * n) / factorial(n) for n in range(N)])
    p /= p.sum()
    n_mean = float(np.sum(np.arange(N) * p))
    for i in range(5):
        f = res["segs"][i, 0, :16]
        r, _ = _uniforms(i, 1, seed=4)
        ref = np.concatenate([[1.0], p[:11], [kappa * n_mean, gamma_a, np.log(r[0]), 0.0]])
        assert np.max(np.abs(f - ref)) < 1e-12, (i, f - ref)
        assert res["segs"][i, 0, 19] == 1.0


# ------------------------------------------------------ step-size underflow
def test_failure_path_step_underflow():
    """H = 1e12 sigma_x on [1e6, 1e6 + 1]: the accepted steps grow until the first
    rejection, whose reduced step lies below 16 eps |t| (the analogue of the
    paper's solver reporting an error level): the trajectory fails with -4, long
    before max_steps, after exactly one rejection."""
    s = w.two_level()
    s.H = w.dense(1e12 * w.systems.SX)
    s.tlist = np.array([1e6, 1e6 + 1.0])
    res = oracle.run(s, 3, seed=0, traj_begin=5, max_steps=1_000_000)
    assert res["status"] == -4
    assert res["fail_traj"] == 5
    acc, rej = res["stats"][0, 0], res["stats"][0, 1]
    assert rej == 1 and 0 < acc < 100, (acc, rej)


# -------------------------------------------------- proposal step limits
def test_snap_limits_extreme_proposals():
    """The snapped proposal is 2^(k/4) with log2 h limited to [-40, 10]; a
    non-finite proposal takes the lower end."""
    assert oracle.snap_step(-1e4) == 2.0 ** -40
    assert oracle.snap_step(1e30) == 2.0 ** 10
    assert oracle.snap_step(float("nan")) == 2.0 ** -40
    assert oracle.snap_step(float("-inf")) == 2.0 ** -40
    assert oracle.snap_step(float("inf")) == 2.0 ** 10
    assert oracle.snap_step(np.log(2.0) * -40.0) == 2.0 ** -40


def test_learned_run_with_out_of_range_proposal_completes():
    """A proposal network whose output bias is -1e4 (h = e^-10000) would otherwise
    give h = 0 and spend max_steps attempts; with the limit the controller grows the
    first step from 2^-40 and every trajectory completes with ordinary step counts."""
    s = w.two_level()
    p = np.zeros(oracle.mlp_ntotal())
    p[-16:] = 1.0
    nparam = oracle.mlp_nparam()
    p[nparam - 3] = -1e4
    res = oracle.run(s, 16, seed=2, mlp=p, max_steps=5000)
    assert res["status"] == 0
    plain = oracle.run(s, 16, seed=2)
    assert np.array_equal(res["jump_counts"], plain["jump_counts"])
    assert res["stats"][:, 0].max() < 3 * plain["stats"][:, 0].max()
