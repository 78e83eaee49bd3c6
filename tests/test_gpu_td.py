"""GPU parity of time-dependent Hamiltonians H(t) = H0 + sum_k f_k(t) H_k,
f_k(t) = c + a cos(w t) + b sin(w t) (qtm_create_td; the small dense kernel's
time-dependent instances), against the FP64 oracle on the same trajectories:

* FP64 products: identical jump counts and channels, jump times and outputs within
  1e-8, for single-wave teams (d = 2, 40) and multi-wave teams (d = 56, 64), with
  the terms' fragments in LDS and (two terms at d = 40 in FP64) in global memory;
* FP32 products, batched: averages within 3 sigma/sqrt(N) + 1e-6;
* the closed form of a drive commuting with the decay: <sigma_z> = cos(2 F(t));
* invalid inputs."""
import numpy as np
import pytest

import oracle
import paper_1810_03047_amd as qtm
import workloads as w

pytestmark = pytest.mark.gpu
JT_TOL = 1e-8


def _exact(system, n, seed, **kw):
    print(f"[gpu] td {system.name} d={system.dim} terms={len(system.td)} n={n} seed={seed} {kw}", flush=True)
    ctx = qtm.create_system(system, qtm.Opts(record_jumps=32, keep_traj=1, **kw))
    ctx.run(n, seed)
    r = oracle.run(system, n, seed=seed, jcap=32)
    worst = 0.0
    for i in range(n):
        t, c, cnt = ctx.jumps(i)
        assert cnt == r["jump_counts"][i], (i, cnt, r["jump_counts"][i])
        m = min(cnt, 32)
        assert np.array_equal(c[:m], r["jump_channels"][i, :m]), i
        if m:
            worst = max(worst, float(np.max(np.abs(t[:m] - r["jump_times"][i, :m]))))
    dx = float(np.max(np.abs(ctx.traj_expect() - r["X"])))
    st = ctx.stats()
    print(f"td {system.name}: worst jump-time difference {worst:.2e}, worst output difference {dx:.2e}, "
          f"{int(r['jump_counts'].sum())} jumps, team shape {st['team_shape']}, LDS {st['lds_bytes']}")
    assert worst <= JT_TOL and dx <= 1e-8
    return ctx, st


def test_td_driven_two_level_fp64():
    _exact(w.driven_two_level(), 500, 3)


@pytest.mark.parametrize("form", [0, qtm.FORM_BATCHED])
def test_td_driven_jaynes_cummings_fp64(form):
    s = w.driven_jaynes_cummings(t_end=10.0, n_t=101)
    _, st = _exact(s, 160, 4, form=form)
    assert st["team_shape"] == 501          # five row tiles, one wave, no banded instance


@pytest.mark.parametrize("N,shape", [(28, 402), (32, 204)])
def test_td_multi_wave_teams_fp64(N, shape):
    s = w.driven_jaynes_cummings(N=N, t_end=4.0, n_t=41)
    _, st = _exact(s, 48, 5, form=qtm.FORM_BATCHED)
    assert st["team_shape"] == shape


def test_td_two_terms_fragments_in_global_memory():
    """Two time-dependent terms at d = 40 in FP64: the three operators' fragments (153 KB)
    leave no LDS for the teams, so the terms are read from global memory."""
    s = w.driven_jaynes_cummings(t_end=6.0, n_t=61)
    a = np.kron(w.destroy(20), np.eye(2, dtype=np.complex128))
    sz = np.kron(np.eye(20), np.diag([-1.0, 1.0]))
    s.td = [s.td[0], (w.dense(0.5 * (a.conj().T @ a) + 0.2 * sz), (0.1, 0.0, 0.3, 0.7))]
    _, st = _exact(s, 64, 6, form=qtm.FORM_BATCHED)
    assert st["lds_bytes"] < 2 * (80 * 80 * 8), st["lds_bytes"]


def test_td_fp32_batched_statistical():
    s = w.driven_jaynes_cummings(t_end=10.0, n_t=101)
    n = 4000
    print(f"[gpu] td driven jcm FP32 batched n={n}", flush=True)
    ctx = qtm.create_system(s, qtm.Opts(precision=qtm.PREC_FP32, form=qtm.FORM_BATCHED, record_jumps=32))
    ctx.run(n, 7)
    mean, _ = ctx.expect()
    r = oracle.run(s, n, seed=7, jcap=32)
    bound = 3.0 * np.sqrt(np.maximum(r["var"], 0.0) / n) + 1e-6
    dev = np.abs(mean.real - r["mean"].real)
    same = float(np.mean(np.array([ctx.jumps(i)[2] for i in range(n)]) == r["jump_counts"]))
    print(f"td FP32: worst deviation / bound {float(np.max(dev / bound)):.3f}; identical jump counts {same:.4f}")
    assert np.all(dev <= bound)
    assert same > 0.95


def test_td_commuting_drive_closed_form_on_gpu():
    s = w.commuting_drive()
    c, a, b, om = (s.meta[k] for k in ("c", "a", "b", "w"))
    t = s.tlist
    F = c * t + (a / om) * np.sin(om * t) + (b / om) * (1.0 - np.cos(om * t))
    ctx = qtm.create_system(s, qtm.Opts(rtol=1e-9, atol=1e-12, keep_traj=1))
    ctx.run(64, 2)
    X = ctx.traj_expect()
    err = float(np.max(np.abs(X[:, 0, :].real - np.cos(2.0 * F))))
    print(f"td closed form: worst |<sigma_z> - cos 2F| {err:.2e}")
    assert err < 1e-7


def test_td_invalid_inputs():
    s = w.driven_jaynes_cummings(N=40, t_end=1.0, n_t=3)          # d = 80 > 64
    with pytest.raises(qtm.QtmError) as e:
        qtm.create_system(s)
    assert e.value.code == qtm.E_INVAL
    s = w.driven_two_level()
    s.td = s.td * 5
    with pytest.raises(qtm.QtmError) as e:
        qtm.create_system(s)
    assert e.value.code == qtm.E_INVAL
    s = w.driven_two_level()
    s.td = [(s.td[0][0], (0.0, np.nan, 0.0, 1.0))]
    with pytest.raises(qtm.QtmError) as e:
        qtm.create_system(s)
    assert e.value.code == qtm.E_INVAL
