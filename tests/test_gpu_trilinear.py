"""GPU parity on the paper's trilinear Hamiltonian (Sec. 4.2): the optical parametric
amplifier H = iK(a b^dag c^dag - a^dag b c) with three damped modes, Fock cutoff 8 per
mode (d = 512, CSR), coherent pump alpha = sqrt(3), t in [0, 4] with 100 outputs.

* FP64 products: every trajectory of a 256-trajectory run against the oracle (jump
  counts, channels, jump times within 1e-8, outputs within 1e-8);
* the benchmarked configuration (20,000 trajectories, batched, FP32 products): the
  averages within 3 sigma/sqrt(N) + 1e-6 of the oracle's average of the same
  trajectories, and the FP64 batched run on sampled trajectories."""
import numpy as np
import pytest

import oracle
import paper_1810_03047_amd as qtm
import workloads as w

pytestmark = pytest.mark.gpu
JT_TOL = 1e-8


def _jumps(ctx, n, jcap=32):
    jt = np.zeros((n, jcap))
    jc = np.full((n, jcap), -9, dtype=np.int32)
    jn = np.zeros(n, dtype=np.int64)
    for i in range(n):
        t, c, cnt = ctx.jumps(i)
        jt[i, :len(t)], jc[i, :len(c)], jn[i] = t, c, cnt
    return jt, jc, jn


def test_trilinear_fp64_every_trajectory():
    s = w.trilinear()
    n = 256
    print(f"[gpu] trilinear FP64 d={s.dim} n={n}", flush=True)
    ctx = qtm.create_system(s, qtm.Opts(record_jumps=32, keep_traj=1))
    ctx.run(n, 1)
    r = oracle.run(s, n, seed=1, jcap=32)
    jt, jc, jn = _jumps(ctx, n)
    assert np.array_equal(jn, r["jump_counts"]), np.nonzero(jn != r["jump_counts"])
    worst = 0.0
    for i in range(n):
        m = min(int(jn[i]), 32)
        if m:
            assert np.array_equal(jc[i, :m], r["jump_channels"][i, :m]), i
            worst = max(worst, float(np.max(np.abs(jt[i, :m] - r["jump_times"][i, :m]))))
    dx = float(np.max(np.abs(ctx.traj_expect() - r["X"])))
    print(f"trilinear FP64: worst jump-time difference {worst:.2e}, worst output difference {dx:.2e}, "
          f"{jn.sum()} jumps")
    assert worst <= JT_TOL and dx <= 1e-8


def test_trilinear_full_size_batched():
    s = w.trilinear()
    n = 20_000
    print(f"[gpu] trilinear batched FP32 n={n}", flush=True)
    ctx = qtm.create_system(s, qtm.Opts(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED, record_jumps=32))
    ctx.run(n, 0)
    mean, _ = ctx.expect()
    _, _, jn = _jumps(ctx, n)
    r = oracle.run(s, n, seed=0, jcap=32)
    bound = 3.0 * np.sqrt(np.maximum(r["var"], 0.0) / n) + 1e-6
    dev = np.abs(mean.real - r["mean"].real)
    same = float(np.mean(jn == r["jump_counts"]))
    print(f"trilinear FP32: worst deviation / bound {float(np.max(dev / bound)):.3f}; "
          f"identical jump counts {same:.4f}")
    assert np.all(dev <= bound)
    assert same > 0.95
    print(f"[gpu] trilinear batched FP64 n={n}", flush=True)
    c64 = qtm.create_system(s, qtm.Opts(form=qtm.FORM_BATCHED, record_jumps=32, keep_traj=1))
    c64.run(n, 0)
    X = c64.traj_expect()
    for i in np.linspace(0, n - 1, 16).astype(int):
        t, c, cnt = c64.jumps(int(i))
        assert cnt == r["jump_counts"][i], i
        m = min(cnt, 32)
        assert np.array_equal(c[:m], r["jump_channels"][i, :m])
        assert np.all(np.abs(t[:m] - r["jump_times"][i, :m]) <= JT_TOL)
        assert np.max(np.abs(X[i] - r["X"][i])) <= 1e-8
