"""GPU parity of the sparse, mixed-precision, batched and learned forms against
the FP64 oracle, and of the proposal network's device gradients."""
import numpy as np
import pytest

import oracle
import paper_1810_03047_amd as qtm
import workloads as w

pytestmark = pytest.mark.gpu

JT_TOL = 1e-8


def _gpu(system, ntraj, seed=0, begin=0, jcap=32, **kw):
    print(f"[gpu] {system.name} d={system.dim} ntraj={ntraj} seed={seed} begin={begin} opts={kw}", flush=True)
    ctx = qtm.create_system(system, qtm.Opts(record_jumps=jcap, keep_traj=1, **kw))
    ctx.run_range(begin, ntraj, seed)
    return ctx


def _jumps(ctx, n, jcap=32):
    jt = np.zeros((n, jcap))
    jc = np.full((n, jcap), -9, dtype=np.int32)
    jn = np.zeros(n, dtype=np.int64)
    for i in range(n):
        t, c, cnt = ctx.jumps(i)
        jt[i, :len(t)], jc[i, :len(c)], jn[i] = t, c, cnt
    return jt, jc, jn


def _exact(ctx, r, n, xtol=1e-8):
    jt, jc, jn = _jumps(ctx, n)
    assert np.array_equal(jn, r["jump_counts"]), np.nonzero(jn != r["jump_counts"])
    worst = 0.0
    for i in range(n):
        m = min(int(jn[i]), 32)
        if m:
            worst = max(worst, float(np.max(np.abs(jt[i, :m] - r["jump_times"][i, :m]))))
            assert np.array_equal(jc[i, :m], r["jump_channels"][i, :m])
    assert worst <= JT_TOL, worst
    dx = float(np.max(np.abs(ctx.traj_expect() - r["X"])))
    assert dx <= xtol, dx
    return worst, dx


def _stat(mean, var, ref, n, k=3.0, floor=1e-6):
    bound = k * np.sqrt(np.maximum(var, 0.0) / n) + floor
    dev = np.abs(mean - ref)
    return bool(np.all(dev <= bound)), float(np.max(dev / bound))


# ------------------------------------------------------------------ sparse
def test_sparse_tfim_fp64_exact_small():
    s = w.tfim(L=6, t_end=5.0, n_t=26)
    n = 97
    ctx = _gpu(s, n, seed=4)
    r = oracle.run(s, n, seed=4, jcap=32)
    print("tfim L=6:", _exact(ctx, r, n))


def test_sparse_tfim_full_size_sampled():
    """L = 10 (d = 1024, CSR, 10 channels, t in [0, 20]): 512 GPU trajectories,
    24 of them recomputed one by one by the oracle."""
    s = w.tfim()
    n = 512
    ctx = _gpu(s, n, seed=0)
    X = ctx.traj_expect()
    jt, jc, jn = _jumps(ctx, n)
    for i in range(0, n, n // 24):
        r = oracle.run(s, 1, seed=0, traj_begin=i, jcap=32)
        assert jn[i] == r["jump_counts"][0], i
        m = min(int(jn[i]), 32)
        assert np.array_equal(jc[i, :m], r["jump_channels"][0, :m])
        assert np.all(np.abs(jt[i, :m] - r["jump_times"][0, :m]) <= JT_TOL)
        assert np.max(np.abs(X[i] - r["X"][0])) <= 1e-8


@pytest.mark.parametrize("cols", [1, 2])
def test_sparse_wide_blocks_fp64_exact(cols):
    """512 < d <= 1024 runs on 512-thread blocks (two rows per thread, two waves per
    SIMD); one and two trajectories per block, trajectory by trajectory against the
    oracle (Ising chain L = 10, d = 1024)."""
    s = w.tfim(t_end=4.0, n_t=41)
    n = 40
    ctx = _gpu(s, n, seed=6, tile_cols=cols)
    st = ctx.stats()
    assert st["threads"] == 512 and st["tile_cols"] == cols, st
    r = oracle.run(s, n, seed=6, jcap=32)
    print(f"tfim L=10 wide blocks, {cols} trajectories per block:", _exact(ctx, r, n))


def test_sparse_small_blocks_fp64_exact():
    """d <= 512 with enough trajectories to occupy small blocks: 64 threads of four rows
    each at d = 256 (Ising chain L = 8), 4,096 trajectories in the batched form; sampled
    trajectories recomputed one by one by the oracle."""
    s = w.tfim(L=8, t_end=4.0, n_t=41)
    n = 4096
    ctx = _gpu(s, n, seed=9, form=qtm.FORM_BATCHED)
    st = ctx.stats()
    assert st["threads"] == 64, st
    X = ctx.traj_expect()
    jt, jc, jn = _jumps(ctx, n)
    worst = 0.0
    for i in range(0, n, n // 16):
        r = oracle.run(s, 1, seed=9, traj_begin=i, jcap=32)
        assert jn[i] == r["jump_counts"][0], i
        m = min(int(jn[i]), 32)
        assert np.array_equal(jc[i, :m], r["jump_channels"][0, :m])
        if m:
            worst = max(worst, float(np.max(np.abs(jt[i, :m] - r["jump_times"][0, :m]))))
        assert np.max(np.abs(X[i] - r["X"][0])) <= 1e-8
    assert worst <= JT_TOL, worst
    print(f"tfim L=8, 64-thread blocks: worst jump-time difference {worst:.2e}")


def test_sparse_fp32_products_statistical():
    s = w.tfim(L=6, t_end=5.0, n_t=26)
    n = 3000
    ctx = _gpu(s, n, seed=1, precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED)
    mean, var = ctx.expect()
    r = oracle.run(s, n, seed=1)
    ok, worst = _stat(mean.real, r["var"], r["mean"].real, n)
    print("sparse fp32 worst deviation / bound:", worst)
    assert ok, worst


def _embed(s, d):
    """The system s in a space of dimension d > s.dim: the extra rows and columns of
    every operator are empty, so the sliced ELL has slices without entries."""
    def csr(op):
        m = op.to_dense()
        r, c = np.nonzero(m)
        return w.csr_from_triplets(d, r, c, m[r, c])
    psi0 = np.zeros(d, dtype=np.complex128)
    psi0[:s.dim] = s.psi0
    e_ops = [w.diag(np.concatenate([np.asarray(e.to_dense().diagonal()), np.zeros(d - s.dim)])) for e in s.e_ops]
    return w.System(s.name + "_embedded", csr(s.H), [csr(c) for c in s.c_ops], psi0, s.tlist, e_ops)


def test_sparse_empty_slices():
    """Ising chain L = 6 embedded in d = 320 (rows 64..319 empty; two rows per
    thread): FP64 exact against the oracle, FP32 (two-row groups, ELL in LDS)
    statistical."""
    s = _embed(w.tfim(L=6, t_end=3.0, n_t=16), 320)
    n = 64
    ctx = _gpu(s, n, seed=5)
    r = oracle.run(s, n, seed=5, jcap=32)
    print("embedded tfim fp64:", _exact(ctx, r, n))
    n32 = 1000
    ctx32 = _gpu(s, n32, seed=6, precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED)
    mean, var = ctx32.expect()
    r32 = oracle.run(s, n32, seed=6)
    ok, worst = _stat(mean.real, r32["var"], r32["mean"].real, n32)
    print("embedded tfim fp32 worst deviation / bound:", worst)
    assert ok, worst


# ------------------------------------------------------------------ mixed precision (dense)
def test_dense_fp32_products_statistical_and_close():
    s = w.jaynes_cummings(t_end=10.0, n_t=101)
    n = 2000
    ctx = _gpu(s, n, seed=7, precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED)
    mean, var = ctx.expect()
    r = oracle.run(s, n, seed=7)
    ok, worst = _stat(mean.real, r["var"], r["mean"].real, n)
    print("dense fp32 worst deviation / bound:", worst)
    assert ok, worst
    # the same random streams: most trajectories take the same jumps
    _, _, jn = _jumps(ctx, n)
    assert np.mean(jn == r["jump_counts"]) > 0.95


@pytest.mark.parametrize("waves", [0, 1, 2])
def test_team_shapes_agree(waves):
    """Every team shape offered for d = 40 gives the oracle's FP64 trajectories."""
    s = w.jaynes_cummings(t_end=4.0, n_t=41)
    cands = qtm.tile_candidates(s.dim)
    tw = 0 if waves == 0 else cands[min(waves, len(cands) - 1)]
    n = 48
    ctx = _gpu(s, n, seed=9, team_waves=tw, form=qtm.FORM_BATCHED)
    r = oracle.run(s, n, seed=9, jcap=32)
    _exact(ctx, r, n)


@pytest.mark.parametrize("d", [16, 24, 32, 48, 56, 64])
@pytest.mark.parametrize("prec", [0, 1])
def test_team_dimensions(d, prec):
    """Default team shape for every tile count (d = 16 .. 64): FP64 exact, FP32 close."""
    s = w.jaynes_cummings(N=d // 2, t_end=4.0, n_t=41)
    n = 32
    ctx = _gpu(s, n, seed=d, precision=prec, form=qtm.FORM_BATCHED)
    r = oracle.run(s, n, seed=d, jcap=32)
    if prec == 0:
        _exact(ctx, r, n)
    else:
        _, _, jn = _jumps(ctx, n)
        assert np.mean(jn == r["jump_counts"]) > 0.9
        assert np.max(np.abs(ctx.traj_expect() - r["X"])) < 1e-3


# ------------------------------------------------------------------ batch of mixed dimension
def test_batch_mixed_dimension_fp64_exact():
    rng = np.random.Generator(np.random.Philox(key=3))
    dims = [8, 24, 40, 70, 150]
    systems = [w.random_system(rng, d, 1 + i % 3, t_end=6.0, n_t=31, c_norm=0.3) for i, d in enumerate(dims)]
    n = 40
    print(f"[gpu] batch dims={dims} ntraj={n}", flush=True)
    ctx = qtm.create_batch(systems, qtm.Opts(record_jumps=32, keep_traj=1))
    ctx.run(n, 5)
    for sidx, s in enumerate(systems):
        r = oracle.run(s, n, seed=5, sys_id=sidx, jcap=32)
        jn = np.array([ctx.jumps(i, system=sidx)[2] for i in range(n)])
        assert np.array_equal(jn, r["jump_counts"]), (sidx, np.nonzero(jn != r["jump_counts"]))
        X = ctx.traj_expect(sidx)
        assert np.max(np.abs(X - r["X"])) <= 1e-8, sidx
        mean, _ = ctx.expect(sidx)
        assert np.max(np.abs(mean - r["mean"])) <= 1e-9, sidx


@pytest.mark.parametrize("form", [0, 2])
def test_hetero_batch_one_launch_and_fanout(form):
    """Heterogeneous batch (random systems, d = 8 .. 200, 1-4 dense collapse operators):
    form 2 runs every system in one persistent launch, form 0 one launch per system
    over side streams; both give the oracle's FP64 trajectories for every system."""
    systems = w.hetero_batch(n_sys=6, d_min=8, d_max=200, key=5, t_end=5.0, n_t=26)
    n = 24
    print(f"[gpu] hetero batch dims={[x.dim for x in systems]} form={form} ntraj={n}", flush=True)
    ctx = qtm.create_batch(systems, qtm.Opts(record_jumps=32, keep_traj=1, form=form))
    ctx.run(n, 8)
    for sidx, s in enumerate(systems):
        r = oracle.run(s, n, seed=8, sys_id=sidx, jcap=32)
        jn = np.array([ctx.jumps(i, system=sidx)[2] for i in range(n)])
        assert np.array_equal(jn, r["jump_counts"]), (sidx, np.nonzero(jn != r["jump_counts"]))
        X = ctx.traj_expect(sidx)
        assert np.max(np.abs(X - r["X"])) <= 1e-8, sidx


# ------------------------------------------------------------------ learned proposal
def _bf16(x):
    a = np.asarray(x, dtype=np.float32).copy()
    u = a.view(np.uint32)
    u += np.uint32(0x7FFF) + ((u >> 16) & 1)
    u &= np.uint32(0xFFFF0000)
    return u.view(np.float32)


def _working_params(p32):
    """The values the device uses: BF16-rounded weights, FP32 biases and standardisation."""
    p = np.asarray(p32, dtype=np.float32).copy()
    nf, nh, no = 16, 64, 3
    oW1, ob1 = 0, nh * nf
    oW2 = ob1 + nh
    ob2 = oW2 + nh * nh
    oW3 = ob2 + nh
    for a, n in ((oW1, nh * nf), (oW2, nh * nh), (oW3, no * nh)):
        p[a:a + n] = _bf16(p[a:a + n])
    return p.astype(np.float64)


def _random_proposal(rng, log_h=np.log(0.05)):
    p = np.zeros(qtm.MLP_NTOTAL, dtype=np.float32)
    nf, nh = 16, 64
    p[0:nh * nf] = rng.standard_normal(nh * nf) * 0.2
    p[nh * nf + nh:nh * nf + nh + nh * nh] = rng.standard_normal(nh * nh) * 0.1
    o3 = nh * nf + nh + nh * nh + nh
    p[o3:o3 + 3 * nh] = rng.standard_normal(3 * nh) * 0.05
    p[o3 + 3 * nh:o3 + 3 * nh + 3] = [log_h, 0.0, 1.0]
    p[-16:] = 1.0            # scales; means stay 0
    return p


def _jcm_feature_ops(N):
    d = 2 * N
    ops = [w.diag(np.tile([0.0, 1.0], N))]
    for k in range(11):
        v = np.zeros(d)
        if 2 * k + 2 <= d:
            v[2 * k:2 * k + 2] = 1.0
        ops.append(w.diag(v))
    return ops


def test_proposal_gradient_matches_oracle():
    rng = np.random.default_rng(0)
    s = w.two_level()
    ctx = qtm.create_system(s, qtm.Opts())
    p = _random_proposal(rng)
    ctx.set_proposal(p, [])
    n = 777
    feat = rng.standard_normal((n, 16)).astype(np.float32)
    tgt = np.stack([rng.standard_normal(n), rng.standard_normal(n), (rng.random(n) < 0.3)], 1).astype(np.float32)
    L, g = ctx.proposal_grad(feat, tgt)
    Lr, gr = oracle.mlp_loss_grad(_working_params(p), feat.astype(np.float64), tgt.astype(np.float64))
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    print(f"device loss {L:.6f} oracle {Lr:.6f}; gradient relative error {rel:.2e}")
    assert abs(L - Lr) <= 1e-4 * abs(Lr) + 1e-6
    assert rel <= 1e-4


def test_training_reduces_loss():
    rng = np.random.default_rng(1)
    s = w.two_level()
    ctx = qtm.create_system(s, qtm.Opts())
    n = 20000
    feat = rng.standard_normal((n, 16)).astype(np.float32)
    # targets with a learnable structure
    lh = (0.5 * feat[:, 0] - 0.3 * feat[:, 3] - 2.0).astype(np.float32)
    lt = (0.2 * feat[:, 1] + 0.5 + 0.1 * rng.standard_normal(n)).astype(np.float32)
    tgt = np.stack([lh, lt, (rng.random(n) < 0.2).astype(np.float32)], 1)
    losses = ctx.train_proposal(feat, tgt, epochs=6, batch=1024, lr=2e-3, seed=0)
    print("losses", losses)
    assert losses[-1] < 0.5 * losses[0]


def test_learned_form_matches_oracle_with_same_weights():
    rng = np.random.default_rng(2)
    s = w.jaynes_cummings(N=10, t_end=8.0, n_t=81)
    f_ops = _jcm_feature_ops(10)
    p = _random_proposal(rng, log_h=np.log(0.08))
    n = 64
    print(f"[gpu] learned form jcm N=10 ntraj={n}", flush=True)
    ctx = qtm.create_system(s, qtm.Opts(form=qtm.FORM_LEARNED | qtm.FORM_BATCHED, record_jumps=32, keep_traj=1))
    ctx.set_proposal(p, f_ops)
    ctx.run(n, 3)
    r = oracle.run(s, n, seed=3, jcap=32, mlp=_working_params(p), f_ops=f_ops)
    _exact(ctx, r, n)
    # the proposal replaced the starting-step rule: fewer product evaluations per segment
    plain = oracle.run(s, n, seed=3)
    print("attempted steps learned", r["stats"][:, :2].sum(), "plain", plain["stats"][:, :2].sum())


def test_learned_form_fp64_exact_on_the_headline_instance():
    """The learned + batched form at d = 40 (Jaynes-Cummings N = 20) on the banded single-
    wave team (the headline's instance, here with FP64 products): with the same BF16
    weights the oracle takes the same steps, jumps and outputs, trajectory by trajectory."""
    rng = np.random.default_rng(5)
    s = w.jaynes_cummings(N=20, t_end=6.0, n_t=61)
    f_ops = _jcm_feature_ops(20)
    p = _random_proposal(rng, log_h=np.log(0.06))
    n = 64
    print(f"[gpu] learned form jcm N=20 ntraj={n} team_waves=1", flush=True)
    ctx = qtm.create_system(s, qtm.Opts(form=qtm.FORM_LEARNED | qtm.FORM_BATCHED, team_waves=1, record_jumps=32,
                                        keep_traj=1))
    ctx.set_proposal(p, f_ops)
    ctx.run(n, 11)
    assert ctx.stats()["team_shape"] == 1501, ctx.stats()["team_shape"]      # banded, 5 row tiles, 1 wave
    r = oracle.run(s, n, seed=11, jcap=32, mlp=_working_params(p), f_ops=f_ops)
    print("learned jcm N=20:", _exact(ctx, r, n))
    st = ctx.stats()
    assert st["accepted"] == int(r["stats"][:, 0].sum()) and st["rejected"] == int(r["stats"][:, 1].sum())


def test_segment_records_for_training():
    s = w.jaynes_cummings(N=10, t_end=8.0, n_t=81)
    f_ops = _jcm_feature_ops(10)
    n = 32
    ctx = qtm.create_system(s, qtm.Opts(seg_cap=8, form=qtm.FORM_BATCHED))
    ctx.set_proposal(_random_proposal(np.random.default_rng(0)), f_ops)
    ctx.run(n, 0)
    seg = ctx.segments()
    r = oracle.run(s, n, seed=0, f_ops=f_ops, seg_cap=8)
    for i in range(n):
        for z in range(8):
            if r["segs"][i, z, 19] == 0:
                assert seg[i, z, 19] == 0
                continue
            assert seg[i, z, 19] == 1
            assert np.allclose(seg[i, z, :16], r["segs"][i, z, :16], rtol=1e-5, atol=1e-6)
            assert seg[i, z, 18] == r["segs"][i, z, 18]
            if r["segs"][i, z, 18] == 0:
                assert abs(seg[i, z, 16] - r["segs"][i, z, 16]) <= 1e-5 * (1 + abs(r["segs"][i, z, 16]))
            assert abs(seg[i, z, 17] - r["segs"][i, z, 17]) <= 1e-5 * abs(r["segs"][i, z, 17])


def test_trained_proposal_gains_over_starting_step_rule():
    """The proposal trained on the device from segment records of the plain solver
    takes fewer attempted steps per trajectory and a shorter critical path (most
    product passes of one 16-trajectory team) than the starting-step rule, on the
    same trajectories.  Measured, not pinned: the size of the gain is reported."""
    s = w.jaynes_cummings(t_end=20.0, n_t=201)
    f_ops = _jcm_feature_ops(20)
    gen = qtm.create_system(s, qtm.Opts(seg_cap=16, form=qtm.FORM_BATCHED))
    p0 = np.zeros(qtm.MLP_NTOTAL, dtype=np.float32)
    p0[-16:] = 1.0
    gen.set_proposal(p0, f_ops)
    gen.run_range(0, 20000, 11)
    seg = gen.segments().reshape(-1, qtm.SEG_REC)
    seg = seg[(seg[:, 19] > 0) & (seg[:, 17] > 0)]
    tau = np.where(seg[:, 18] > 0, 1.0, seg[:, 16])
    F = seg[:, :16].astype(np.float32)
    T = np.stack([np.log(seg[:, 17]), np.log(np.maximum(tau, 1e-12)), seg[:, 18]], 1).astype(np.float32)
    gen.destroy()
    trainer = qtm.create_system(s, qtm.Opts())      # starts from the library's initialisation
    losses = trainer.train_proposal(F, T, epochs=8, batch=4096, lr=2e-3, seed=0)
    prop = trainer.get_proposal()
    trainer.destroy()
    res = {}
    for name, form in (("rule", qtm.FORM_BATCHED), ("learned", qtm.FORM_BATCHED | qtm.FORM_LEARNED)):
        ctx = qtm.create_system(s, qtm.Opts(form=form))
        if form & qtm.FORM_LEARNED:
            ctx.set_proposal(prop, f_ops)
        ctx.run(4000, 3)
        st = ctx.stats()
        res[name] = (st["accepted"] + st["rejected"], st["max_team_passes"], st["passes"])
        ctx.destroy()
    print(f"training loss {losses[0]:.4f} -> {losses[-1]:.4f} on {len(F)} samples; "
          f"attempted steps rule {res['rule'][0]} learned {res['learned'][0]}; "
          f"critical path rule {res['rule'][1]} learned {res['learned'][1]} passes; "
          f"total passes rule {res['rule'][2]} learned {res['learned'][2]}")
    assert losses[-1] < losses[0]
    assert res["learned"][0] < res["rule"][0]
    assert res["learned"][2] < res["rule"][2]


@pytest.mark.parametrize("class_waves", [(0, 0, 0), (8, 8, 4), (4, 4, 16)])
def test_batch_tile_class_shapes_fp64_exact(class_waves):
    """Every team shape offered for the three tile classes of a batch (d <= 64, 128, 256)
    gives the oracle's FP64 trajectories; the systems run in cost order."""
    rng = np.random.Generator(np.random.Philox(key=12))
    dims = [16, 56, 72, 120, 136, 250]
    systems = [w.random_system(rng, d, 1 + i % 3, t_end=3.0, n_t=16, c_norm=0.3) for i, d in enumerate(dims)]
    n = 32
    print(f"[gpu] batch tile classes dims={dims} class_waves={class_waves} ntraj={n}", flush=True)
    ctx = qtm.create_batch(systems, qtm.Opts(form=qtm.FORM_BATCHED, record_jumps=32, keep_traj=1,
                                             class_waves=class_waves))
    ctx.run(n, 13)
    for sidx, s in enumerate(systems):
        r = oracle.run(s, n, seed=13, sys_id=sidx, jcap=32)
        jn = np.array([ctx.jumps(i, system=sidx)[2] for i in range(n)])
        assert np.array_equal(jn, r["jump_counts"]), (sidx, np.nonzero(jn != r["jump_counts"]))
        X = ctx.traj_expect(sidx)
        assert np.max(np.abs(X - r["X"])) <= 1e-8, sidx


def test_batch_tile_class_shape_rejected():
    rng = np.random.Generator(np.random.Philox(key=12))
    systems = [w.random_system(rng, d, 1, t_end=1.0, n_t=3) for d in (16, 24)]
    with pytest.raises(qtm.QtmError):
        qtm.create_batch(systems, qtm.Opts(form=qtm.FORM_BATCHED, class_waves=(5, 0, 0)))
    assert qtm.batch_tile_candidates(2) == [8, 4, 16]


def test_batch_tile_class_on_spmm_kernel_fp64_exact():
    """class_waves = -1 runs a tile class on the sliced-ELL SpMM kernel inside the batched
    launch: the oracle's FP64 trajectories as well."""
    rng = np.random.Generator(np.random.Philox(key=14))
    dims = [20, 48, 90, 110, 180, 230]
    systems = [w.random_system(rng, d, 1 + i % 3, t_end=3.0, n_t=16, c_norm=0.3) for i, d in enumerate(dims)]
    n = 32
    print(f"[gpu] batch tile classes on SpMM dims={dims} ntraj={n}", flush=True)
    ctx = qtm.create_batch(systems, qtm.Opts(form=qtm.FORM_BATCHED, record_jumps=32, keep_traj=1,
                                             class_waves=(-1, -1, -1)))
    ctx.run(n, 15)
    for sidx, s in enumerate(systems):
        r = oracle.run(s, n, seed=15, sys_id=sidx, jcap=32)
        jn = np.array([ctx.jumps(i, system=sidx)[2] for i in range(n)])
        assert np.array_equal(jn, r["jump_counts"]), (sidx, np.nonzero(jn != r["jump_counts"]))
        assert np.max(np.abs(ctx.traj_expect(sidx) - r["X"])) <= 1e-8, sidx
