"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.  FP64 forms: identical jump counts per trajectory,
jump times within 1e-8, per-trajectory expectation values within 1e-8 and
averages within 3 sigma/sqrt(N) + 1e-6 (in practice far tighter)."""
import numpy as np
import pytest

import oracle
import paper_1810_03047_amd as qtm
import workloads as w

pytestmark = pytest.mark.gpu

JT_TOL = 1e-8      # jump times (FP64 forms)
X_TOL = 1e-8       # per-trajectory expectation values (FP64 forms)


def gpu_run(system, ntraj, seed=0, begin=0, jcap=32, **kw):
    print(f"[gpu] {system.name} d={system.dim} ntraj={ntraj} seed={seed} opts={kw}", flush=True)
    o = qtm.Opts(record_jumps=jcap, keep_traj=1, **kw)
    ctx = qtm.create_system(system, o)
    ctx.run_range(begin, ntraj, seed)
    mean, var = ctx.expect()
    jt = np.zeros((ntraj, jcap))
    jc = np.full((ntraj, jcap), -9, dtype=np.int32)
    jn = np.zeros(ntraj, dtype=np.int64)
    for i in range(ntraj):
        t, c, n = ctx.jumps(i)
        jt[i, :len(t)] = t
        jc[i, :len(c)] = c
        jn[i] = n
    out = dict(X=ctx.traj_expect(), mean=mean, var=var, jt=jt, jc=jc, jn=jn, stats=ctx.stats(),
               tstats=ctx.traj_stats())
    ctx.destroy()
    return out


def compare_exact(g, r, ntraj, jcap=32):
    assert np.array_equal(g["jn"], r["jump_counts"]), np.nonzero(g["jn"] != r["jump_counts"])
    worst = 0.0
    for i in range(ntraj):
        n = min(int(r["jump_counts"][i]), jcap)
        if n:
            worst = max(worst, np.max(np.abs(g["jt"][i, :n] - r["jump_times"][i, :n])))
            assert np.array_equal(g["jc"][i, :n], r["jump_channels"][i, :n]), i
    assert worst <= JT_TOL, worst
    dx = np.max(np.abs(g["X"] - r["X"]))
    assert dx <= X_TOL, dx
    # accepted/rejected steps and segments agree too
    assert np.array_equal(g["tstats"][:, 0], r["stats"][:, 0])
    assert np.array_equal(g["tstats"][:, 1], r["stats"][:, 1])
    return worst, dx


def test_two_level_fp64_exact():
    s = w.two_level()
    n = 500
    g = gpu_run(s, n, seed=0)
    r = oracle.run(s, n, seed=0, jcap=32)
    worst, dx = compare_exact(g, r, n)
    print(f"two_level: max |dt_jump| = {worst:.3e}, max |dX| = {dx:.3e}")
    assert np.max(np.abs(g["mean"] - r["mean"])) < 1e-10
    assert np.allclose(g["var"], r["var"], atol=1e-10)


def test_jaynes_cummings_fp64_exact_small():
    s = w.jaynes_cummings(t_end=10.0, n_t=101)
    n = 333                    # ragged: not a multiple of the 16-column tile
    g = gpu_run(s, n, seed=3)
    r = oracle.run(s, n, seed=3, jcap=32)
    worst, dx = compare_exact(g, r, n)
    print(f"jcm small: max |dt_jump| = {worst:.3e}, max |dX| = {dx:.3e}")


def test_two_channel_identity_closed_form_and_oracle():
    s = w.two_channel_identity(0.3, 0.2, t_end=10.0)
    n = 64
    g = gpu_run(s, n, seed=11)
    r = oracle.run(s, n, seed=11, jcap=32)
    compare_exact(g, r, n)


def test_photon_birth_death_two_channels():
    s = w.photon_birth_death()
    n = 200
    g = gpu_run(s, n, seed=2)
    r = oracle.run(s, n, seed=2, jcap=32)
    compare_exact(g, r, n)


def test_no_collapse_operators():
    s = w.jaynes_cummings(kappa=0.0, gamma_a=0.0, t_end=5.0, n_t=51)
    g = gpu_run(s, 17, seed=0)
    r = oracle.run(s, 17, seed=0)
    assert g["jn"].sum() == 0
    compare_exact(g, r, 17)


def test_traj_range_offset():
    s = w.two_level()
    g = gpu_run(s, 40, seed=5, begin=1000)
    r = oracle.run(s, 40, seed=5, traj_begin=1000, jcap=32)
    compare_exact(g, r, 40)


def test_batched_persistent_equals_plain():
    s = w.jaynes_cummings(t_end=5.0, n_t=51)
    a = gpu_run(s, 100, seed=1)
    b = gpu_run(s, 100, seed=1, form=qtm.FORM_BATCHED)
    assert np.array_equal(a["jn"], b["jn"])
    assert np.array_equal(a["X"], b["X"])


@pytest.mark.parametrize("form", [0, qtm.FORM_BATCHED])
def test_chunked_run_equals_single_run(form):
    """A run that keeps no per-trajectory data goes chunk by chunk when it holds more
    trajectories than a chunk: the same trajectories (same statistics) and the same
    sums up to the order of the FP64 additions.  In the batched form the full chunks
    replay one captured graph and the last, smaller one takes another."""
    s = w.jaynes_cummings(N=6, t_end=4.0, n_t=41)
    n = 100
    print(f"[gpu] chunked run jcm N=6 n={n} form={form}", flush=True)
    res = {}
    for chunk in (0, 7, 33):
        ctx = qtm.create_system(s, qtm.Opts(chunk_traj=chunk, form=form))
        ctx.run(n, 5)
        st = ctx.stats()
        sums = ctx.sums()
        mean, var = ctx.expect()
        ctx.destroy()
        res[chunk] = (st, sums, mean, var)
    st0, (s0, q0, c0), m0, v0 = res[0]
    for chunk in (7, 33):
        st, (s1, q1, c1), m1, v1 = res[chunk]
        assert c1 == c0 == n
        for k in ("accepted", "rejected", "segments", "jumps"):       # per-trajectory statistics
            assert st[k] == st0[k], (chunk, k)
        assert st["ntraj"] == n and st["failed_traj"] == -1
        assert np.allclose(s1, s0, rtol=1e-13, atol=1e-13), chunk
        assert np.allclose(q1, q0, rtol=1e-13, atol=1e-13), chunk
        assert np.allclose(m1, m0, rtol=1e-13, atol=1e-13), chunk
    # a context that keeps per-trajectory data never chunks
    ctx = qtm.create_system(s, qtm.Opts(chunk_traj=7, keep_traj=1, form=form))
    ctx.run(n, 5)
    assert ctx.traj_expect().shape[0] == n
    ctx.destroy()


def test_failure_path_max_steps():
    s = w.two_level()
    ctx = qtm.create_system(s, qtm.Opts(max_steps=3))
    with pytest.raises(qtm.QtmError) as e:
        ctx.run_range(7, 5, 0)
    assert e.value.code == qtm.E_STEP
    assert ctx.stats()["failed_traj"] == 7
    with pytest.raises(qtm.QtmError) as e2:
        ctx.expect()
    assert e2.value.code == qtm.E_STATE


def test_invalid_inputs_rejected():
    s = w.two_level()
    bad = s.psi0 * 1.1
    with pytest.raises(qtm.QtmError) as e:
        qtm.create(s.H, s.c_ops, bad, s.tlist, s.e_ops)
    assert e.value.code == qtm.E_INVAL
    with pytest.raises(qtm.QtmError):
        qtm.create(s.H, s.c_ops, s.psi0, s.tlist[::-1].copy(), s.e_ops)
    Hn = w.dense(np.array([[np.nan, 0], [0, 1]]))
    with pytest.raises(qtm.QtmError):
        qtm.create(Hn, s.c_ops, s.psi0, s.tlist, s.e_ops)


def test_batched_graph_replays_match_eager():
    """The batched form captures its run into a graph and replays it; every replay
    (new seed, new trajectory range, eager runs in between) equals an eager run of
    the plain form on the same trajectories, and a new count re-captures."""
    s = w.jaynes_cummings(t_end=5.0, n_t=51)
    g = qtm.create_system(s, qtm.Opts(form=qtm.FORM_BATCHED, record_jumps=16, keep_traj=1))
    e = qtm.create_system(s, qtm.Opts(form=0, record_jumps=16, keep_traj=1))
    for rep, (begin, count, seed) in enumerate([(0, 96, 1), (96, 96, 1), (0, 96, 7), (5, 40, 3), (0, 96, 2)]):
        print(f"[gpu] replay {rep}: begin={begin} count={count} seed={seed}", flush=True)
        g.run_range(begin, count, seed)
        Xg = g.traj_expect()
        mg, _ = g.expect()
        jg = [g.jumps(i)[2] for i in range(count)]
        e.run_range(begin, count, seed)
        Xe = e.traj_expect()
        me, _ = e.expect()
        je = [e.jumps(i)[2] for i in range(count)]
        assert jg == je, rep
        assert np.max(np.abs(Xg - Xe)) <= 1e-10, rep
        assert np.max(np.abs(mg - me)) <= 1e-12, rep
