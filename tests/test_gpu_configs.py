"""GPU parity of the benchmarked FP32 configurations against the FP64 oracle, on
the same trajectories and random streams, with the stated statistical bound
3 sigma/sqrt(N) + 1e-6 on every average (sigma from the oracle's trajectories):

* the headline form exactly as bench.py times it: Jaynes-Cummings (d = 40),
  proposal trained on the device from plain-solver segment records, batched,
  FP32 products, single-wave teams with the banded-operator instance;
* the heterogeneous batch in its tile-class launches with FP32 products (all
  three classes, d <= 64, 128, 256);
* the dense block kernel (64 < d <= 128) with FP32 products.

Each test prints its worst deviation in units of the bound."""
import numpy as np
import pytest

import bench
import oracle
import paper_1810_03047_amd as qtm
import workloads as w

pytestmark = pytest.mark.gpu


def _bound_check(mean_gpu, r_mean, r_var, n):
    sig = np.sqrt(np.maximum(r_var, 0.0) / n)
    bound = 3.0 * sig + 1e-6
    dev = np.abs(mean_gpu.real - r_mean.real)
    return bool(np.all(dev <= bound)), float(np.max(dev / bound))


def _jump_counts(ctx, n, system=0):
    return np.array([ctx.jumps(i, system=system)[2] for i in range(n)])


def test_headline_learned_batched_fp32_jcm_d40():
    """The exact headline configuration: 10,000 trajectories of the d = 40 Jaynes-Cummings
    workload with the proposal trained the way bench.py trains it, against the oracle
    running the same BF16-rounded weights (FP64 activations) on the same trajectories."""
    s = w.jaynes_cummings()
    print("[gpu] headline: training data + proposal training", flush=True)
    F, T, f_ops = bench.training_data(qtm, s)
    trainer = qtm.create_system(s, qtm.Opts())
    trainer.train_proposal(F, T, epochs=8, batch=4096, lr=2e-3, seed=0)
    params = trainer.get_proposal()
    trainer.destroy()
    n = 10_000
    print(f"[gpu] headline: learned+batched+FP32 n={n}", flush=True)
    ctx = qtm.create_system(s, qtm.Opts(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED | qtm.FORM_LEARNED,
                                        record_jumps=32, keep_traj=1))
    ctx.set_proposal(params, f_ops)
    ctx.run(n, 0)
    st = ctx.stats()
    assert st["team_shape"] == 1501, st["team_shape"]      # 5 row tiles, one wave, banded instance
    mean, _ = ctx.expect()
    jn = _jump_counts(ctx, n)
    r = oracle.run(s, n, seed=0, jcap=32, mlp=bench._working_params(params), f_ops=f_ops)
    ok, worst = _bound_check(mean, r["mean"], r["var"], n)
    same = float(np.mean(jn == r["jump_counts"]))
    print(f"headline: worst deviation / bound {worst:.3f}; identical jump counts {same:.4f}")
    assert ok, worst
    assert same > 0.95, same


@pytest.mark.timeout(600)
def test_hetero_tile_classes_fp32():
    """64 systems (d 8..256) x 500 trajectories in the three tile-class launches with FP32
    products, every system's averages against the oracle's average of the same 500
    trajectories.  (Systems whose jump rate is low have jump times that are ill
    conditioned in FP32 -- the norm decays slowly -- so a small trajectory subset can
    be dominated by one trajectory whose jump moved across an output time; all 500
    are compared.)"""
    systems = w.hetero_batch()
    classes = {0: 0, 1: 0, 2: 0}
    for s in systems:
        classes[0 if s.dim <= 64 else 1 if s.dim <= 128 else 2] += 1
    assert all(v > 0 for v in classes.values()), classes
    n = 500
    print(f"[gpu] hetero tile classes FP32 n={n} x {len(systems)}", flush=True)
    ctx = qtm.create_batch(systems, qtm.Opts(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED, record_jumps=32))
    ctx.run(n, 0)
    worst, same, tot = 0.0, 0, 0
    for sidx, s in enumerate(systems):
        mean, _ = ctx.expect(sidx)
        r = oracle.run(s, n, seed=0, sys_id=sidx, jcap=32)
        ok, wv = _bound_check(mean, r["mean"], r["var"], n)
        worst = max(worst, wv)
        assert ok, (sidx, s.dim, wv)
        jn = _jump_counts(ctx, n, system=sidx)
        same += int(np.sum(jn == r["jump_counts"]))
        tot += n
    print(f"hetero FP32: worst deviation / bound {worst:.3f}; identical jump counts {same / tot:.4f}")
    assert same / tot > 0.95


def test_dense_block_kernel_fp32():
    """A random dense system with d = 100 (the block kernel's range 64 < d <= 128), FP32
    products, batched: 2,000 trajectories against the oracle."""
    rng = np.random.Generator(np.random.Philox(key=41))
    s = w.random_system(rng, 100, 3, t_end=8.0, n_t=41, c_norm=0.3)
    n = 2000
    print(f"[gpu] dense block kernel FP32 d={s.dim} n={n}", flush=True)
    ctx = qtm.create_system(s, qtm.Opts(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED, record_jumps=32))
    ctx.run(n, 12)
    assert ctx.stats()["team_shape"] == 0        # not the small dense kernel
    mean, _ = ctx.expect()
    r = oracle.run(s, n, seed=12, jcap=32)
    ok, worst = _bound_check(mean, r["mean"], r["var"], n)
    same = float(np.mean(_jump_counts(ctx, n) == r["jump_counts"]))
    print(f"dense block FP32: worst deviation / bound {worst:.3f}; identical jump counts {same:.4f}")
    assert ok, worst
    assert same > 0.95, same


def test_root_evaluations_counted():
    """Every jump-time root find costs the scan up to the first sign change (1..32
    evaluations) plus 39 bisection halvings of a 1/32-wide bracket down to 1e-13 (44 of
    the whole interval when rounding leaves no scan point below the threshold)."""
    s = w.jaynes_cummings(t_end=10.0, n_t=101)
    ctx = qtm.create_system(s, qtm.Opts(form=qtm.FORM_BATCHED))
    ctx.run(512, 1)
    st = ctx.stats()
    assert st["jumps"] > 0
    assert 40 * st["jumps"] <= st["root_evals"] <= 76 * st["jumps"], (st["jumps"], st["root_evals"])
