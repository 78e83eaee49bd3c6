"""GPU parity at the full sizes of the benchmark workloads, in the launch
configurations bench.py times, on trajectories the oracle recomputes one by one
(FP64 forms) and on the averages over all trajectories (FP32 forms); plus the
largest supported system (d = 2048, 16 jump operators, 16 observables)."""
import numpy as np
import pytest

import oracle
import paper_1810_03047_amd as qtm
import workloads as w

pytestmark = pytest.mark.gpu
JT_TOL = 1e-8


def _check_sampled(ctx, system, n, seed, picks, sys_id=0, sidx=0, jcap=32):
    X = ctx.traj_expect(sidx)
    for i in picks:
        r = oracle.run(system, 1, seed=seed, sys_id=sys_id, traj_begin=int(i), jcap=jcap)
        t, c, cnt = ctx.jumps(int(i), system=sidx)
        assert cnt == r["jump_counts"][0], (sidx, i, cnt, r["jump_counts"][0])
        m = min(cnt, jcap)
        assert np.array_equal(c[:m], r["jump_channels"][0, :m]), (sidx, i)
        assert np.all(np.abs(t[:m] - r["jump_times"][0, :m]) <= JT_TOL), (sidx, i)
        assert np.max(np.abs(X[i] - r["X"][0])) <= 1e-8, (sidx, i)


def test_jaynes_cummings_full_plain_fp64_every_trajectory():
    """10,000 trajectories, t in [0, 50], 501 outputs, FP64 products, default team shape:
    every trajectory against the oracle (jump counts, channels, jump times, outputs)."""
    s = w.jaynes_cummings()
    n = 10_000
    print(f"[gpu] jcm full size plain FP64 n={n}", flush=True)
    ctx = qtm.create_system(s, qtm.Opts(record_jumps=32, keep_traj=1))
    ctx.run(n, 0)
    r = oracle.run(s, n, seed=0, jcap=32)
    X = ctx.traj_expect()
    worst_t = 0.0
    for i in range(n):
        t, c, cnt = ctx.jumps(i)
        assert cnt == r["jump_counts"][i], (i, cnt, r["jump_counts"][i])
        m = min(cnt, 32)
        assert np.array_equal(c[:m], r["jump_channels"][i, :m]), i
        if m:
            worst_t = max(worst_t, float(np.max(np.abs(t[:m] - r["jump_times"][i, :m]))))
    dx = float(np.max(np.abs(X - r["X"])))
    print(f"jcm full FP64: worst jump-time difference {worst_t:.2e}, worst output difference {dx:.2e}")
    assert worst_t <= JT_TOL
    assert dx <= 1e-8


def test_jaynes_cummings_full_batched_fp32_averages():
    """The headline launch configuration (batched, FP32 products, graph replay):
    averages over all 10,000 trajectories within 3 sigma/sqrt(N) + 1e-6 of the
    oracle's average of the same trajectories."""
    s = w.jaynes_cummings()
    n = 10_000
    print(f"[gpu] jcm full size batched FP32 n={n}", flush=True)
    ctx = qtm.create_system(s, qtm.Opts(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED))
    ctx.run(n, 2)
    ctx.run(n, 3)            # a graph replay
    mean, var = ctx.expect()
    r = oracle.run(s, n, seed=3)
    bound = 3.0 * np.sqrt(np.maximum(r["var"], 0.0) / n) + 1e-6
    dev = np.abs(mean.real - r["mean"].real)
    print("jcm full FP32: worst deviation / bound", float(np.max(dev / bound)))
    assert np.all(dev <= bound)


def test_tfim_full_plain_fp64_sampled():
    """Ising chain L = 10, 20,000 trajectories, t in [0, 20], FP64 products."""
    s = w.tfim()
    n = 20_000
    print(f"[gpu] tfim full size plain FP64 n={n}", flush=True)
    ctx = qtm.create_system(s, qtm.Opts(record_jumps=32, keep_traj=1))
    ctx.run(n, 0)
    _check_sampled(ctx, s, n, 0, np.linspace(0, n - 1, 12).astype(int))


def test_tfim_full_batched_fp32_lds_ell():
    """The benchmarked Ising configuration (batched, FP32 products, 20,000 trajectories):
    the sliced ELL (123 KB) is resident in LDS.  The average of trajectories 0..1999
    against the oracle's average of the same trajectories, and the average of all
    20,000 against the FP64 run of the same trajectories (itself checked against the
    oracle above), both within 3 sigma/sqrt(N) + 1e-6."""
    s = w.tfim()
    n, m = 20_000, 2000
    print(f"[gpu] tfim full size batched FP32 n={n}", flush=True)
    ctx = qtm.create_system(s, qtm.Opts(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED, keep_traj=1))
    ctx.run(n, 4)
    st = ctx.stats()
    assert st["lds_bytes"] > 120_000, st["lds_bytes"]      # staging + resident ELL
    mean32, _ = ctx.expect()
    sub = ctx.traj_expect()[:m].mean(axis=0)
    print(f"[gpu] tfim oracle subset n={m}", flush=True)
    r = oracle.run(s, m, seed=4)
    bound = 3.0 * np.sqrt(np.maximum(r["var"], 0.0) / m) + 1e-6
    dev = np.abs(sub.real - r["mean"].real)
    print("tfim FP32 vs oracle (2,000): worst deviation / bound", float(np.max(dev / bound)))
    assert np.all(dev <= bound)
    ref = qtm.create_system(s, qtm.Opts())
    ref.run(n, 4)
    mean64, var64 = ref.expect()
    bound = 3.0 * np.sqrt(np.maximum(var64, 0.0) / n) + 1e-6
    dev = np.abs(mean32.real - mean64.real)
    print("tfim FP32 vs FP64 (20,000): worst deviation / bound", float(np.max(dev / bound)))
    assert np.all(dev <= bound)


def test_hetero_full_batched_fp64_sampled():
    """64 systems x 500 trajectories in the batched tile-class launches, FP64
    products: sampled trajectories of 16 systems recomputed by the oracle."""
    systems = w.hetero_batch()
    n = 500
    print(f"[gpu] hetero full size batched FP64 n={n} x {len(systems)}", flush=True)
    ctx = qtm.create_batch(systems, qtm.Opts(form=qtm.FORM_BATCHED, record_jumps=32, keep_traj=1))
    ctx.run(n, 0)
    for sidx in range(0, len(systems), 4):
        _check_sampled(ctx, systems[sidx], n, 0, [int(sidx * 7) % n], sys_id=sidx, sidx=sidx)


def test_largest_system_sparse():
    """d = 2048 (the largest supported), banded random H in CSR, 16 jump operators,
    16 observables: FP64 parity on every trajectory."""
    rng = np.random.Generator(np.random.Philox(key=17))
    d, nc, ne = 2048, 16, 16
    rows, cols, vals = [], [], []
    for off in (0, 1, 3, 17):
        i = np.arange(d - off)
        v = (rng.standard_normal(d - off) + (1j * rng.standard_normal(d - off) if off else 0)) * 0.3
        rows += [i, i + off] if off else [i]
        cols += [i + off, i] if off else [i]
        vals += [v, np.conj(v)] if off else [v.real.astype(np.complex128)]
    H = w.csr_from_triplets(d, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))
    cops = []
    for k in range(nc):
        i = np.arange(d - 1 - k)
        cops.append(w.csr_from_triplets(d, i, i + 1 + k, np.full(len(i), 0.05, dtype=np.complex128)))
    e_ops = [w.diag((np.arange(d) % (k + 2) == 0).astype(float)) for k in range(ne)]
    psi0 = np.zeros(d, dtype=np.complex128)
    psi0[d // 2] = 1.0
    s = w.System("large_sparse", H, cops, psi0, np.linspace(0.0, 2.0, 11), e_ops, {})
    n = 12
    print(f"[gpu] largest sparse d={d} n_c={nc} n_e={ne} ntraj={n}", flush=True)
    ctx = qtm.create_system(s, qtm.Opts(record_jumps=32, keep_traj=1))
    ctx.run(n, 4)
    _check_sampled(ctx, s, n, 4, range(n))
