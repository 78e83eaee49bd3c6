"""GPU parity of the exact-propagator integrator (QTM_INT_EXPO, the stiff form)
against its oracle (oracle/expo.py: scipy's matrix exponential and bisection on the
exact norm) on the same random streams: identical jump counts and channels, jump
times within 1e-8, outputs within 1e-8; a stiff cavity also against the Lindblad
equation; and the inputs the integrator refuses."""
import numpy as np
import pytest

import paper_1810_03047_amd as qtm
import workloads as w
from oracle import expo, lindblad

pytestmark = pytest.mark.gpu
JT_TOL = 1e-8


def _exact(system, n, seed, **kw):
    print(f"[gpu] expo {system.name} d={system.dim} n={n} seed={seed} {kw}", flush=True)
    ctx = qtm.create_system(system, qtm.Opts(integrator=qtm.INT_EXPO, record_jumps=32, keep_traj=1, **kw))
    ctx.run(n, seed)
    r = expo.run_expo(system, n, seed=seed)
    worst = 0.0
    for i in range(n):
        t, c, cnt = ctx.jumps(i)
        assert cnt == r["jump_counts"][i], (i, cnt, r["jump_counts"][i])
        m = min(cnt, 32)
        assert np.array_equal(c[:m], r["jump_channels"][i, :m]), i
        if m:
            worst = max(worst, float(np.max(np.abs(t[:m] - r["jump_times"][i, :m]))))
    X = ctx.traj_expect()
    dx = float(np.max(np.abs(X - r["X"])))
    st = ctx.stats()
    print(f"expo {system.name}: worst jump-time difference {worst:.2e}, worst output difference {dx:.2e}, "
          f"{int(r['jump_counts'].sum())} jumps, {st['passes']} products")
    assert worst <= JT_TOL and dx <= 1e-8
    return ctx, r


@pytest.mark.parametrize("form", [0, qtm.FORM_BATCHED])
def test_expo_small_jcm(form):
    _exact(w.jaynes_cummings(N=6, t_end=8.0, n_t=81), 64, 3, form=form)


def test_expo_jcm_d40():
    _exact(w.jaynes_cummings(t_end=6.0, n_t=61), 48, 4, form=qtm.FORM_BATCHED)


def test_expo_substeps_agree():
    s = w.jaynes_cummings(N=6, t_end=8.0, n_t=41)
    _exact(s, 48, 5, expo_substeps=4)


def test_expo_stiff_cavity():
    """Cavity decay 40 (the cavity relaxes 40 times faster than the coupling acts):
    exact against the oracle, and the average against the Lindblad equation."""
    s = w.jaynes_cummings(N=6, kappa=40.0, gamma_a=0.05, alpha=1.0, t_end=4.0, n_t=41)
    _exact(s, 128, 6, form=qtm.FORM_BATCHED)
    n = 20000
    ctx = qtm.create_system(s, qtm.Opts(integrator=qtm.INT_EXPO, form=qtm.FORM_BATCHED))
    ctx.run(n, 7)
    mean, var = ctx.expect()
    ref = lindblad.expect_expm(s)
    bound = 3.0 * np.sqrt(var / n) + 1e-6
    dev = np.abs(mean.real - ref.real)
    print(f"expo stiff cavity vs Lindblad: worst deviation / bound {float(np.max(dev / bound)):.3f}")
    assert np.all(dev <= bound)


def test_expo_refuses():
    s = w.jaynes_cummings(N=6, t_end=2.0, n_t=21)
    for kw in (dict(precision=qtm.PREC_FP32), dict(form=qtm.FORM_LEARNED)):
        with pytest.raises(qtm.QtmError) as e:
            qtm.create_system(s, qtm.Opts(integrator=qtm.INT_EXPO, **kw))
        assert e.value.code == qtm.E_INVAL
    s2 = w.jaynes_cummings(N=6, t_end=2.0, n_t=21)
    s2.tlist = np.concatenate([s2.tlist[:10], s2.tlist[10:] + 0.01])
    s2.tlist[-1] = 2.0 + 0.01
    with pytest.raises(qtm.QtmError):
        qtm.create_system(s2, qtm.Opts(integrator=qtm.INT_EXPO))
    with pytest.raises(qtm.QtmError):
        qtm.create_system(w.jaynes_cummings(N=24, t_end=1.0, n_t=3), qtm.Opts(integrator=qtm.INT_EXPO))
    with pytest.raises(qtm.QtmError):
        qtm.create_system(w.driven_two_level(), qtm.Opts(integrator=qtm.INT_EXPO))
