"""qtm_run_range_noalloc (the entry point for callers that cannot allocate) against
qtm_run_range on the same context, trajectories and seed: FP64 products give the
same trajectories, so the sums agree up to the summation order (relative 1e-12);
FP32 products with the persistent form likewise (the same kernel runs).  Two calls in
a row, the second on a smaller range, exercise the shared scratch array (the first
call spans several chunks of it)."""
import numpy as np
import pytest

import paper_1810_03047_amd as qtm
import workloads as w

pytestmark = pytest.mark.gpu


def _close(a, b, count):
    scale = np.abs(b) + count
    return float(np.max(np.abs(a - b) / scale))


@pytest.mark.parametrize("prec,form", [(qtm.PREC_FP64, 0), (qtm.PREC_FP32, qtm.FORM_BATCHED)])
def test_noalloc_matches_run_range(prec, form):
    s = w.jaynes_cummings()
    m = len(s.e_ops) * len(s.tlist)
    chunk = (qtm.NOALLOC_SCRATCH_MB << 20) // (16 * m + 20)
    ctx = qtm.create_system(s, qtm.Opts(precision=prec, form=form))
    for begin, count in ((0, 5000), (300, 700)):
        print(f"[gpu] noalloc prec={prec} form={form} range=({begin}, {count}) chunks~{-(-count // chunk)}", flush=True)
        s1, q1 = ctx.run_range_noalloc(begin, count, seed=5)
        st = ctx.stats()
        assert st["ntraj"] == count and st["accepted"] > 0
        with pytest.raises(qtm.QtmError):      # read-back calls refer to qtm_run only
            ctx.expect()
        ctx.run_range(begin, count, seed=5)
        s2, q2, n2 = ctx.sums()
        assert n2 == count
        d1, d2 = _close(s1, s2, count), _close(q1, q2, count)
        print(f"noalloc vs run_range: relative difference of sums {d1:.2e}, of squares {d2:.2e}")
        assert d1 <= 1e-12 and d2 <= 1e-12
    ctx.destroy()


def test_noalloc_rejects_what_it_cannot_hold():
    # several systems in one context
    rng = np.random.Generator(np.random.Philox(key=2))
    systems = [w.random_system(rng, d, 1, t_end=1.0, n_t=5) for d in (8, 16)]
    b = qtm.create_batch(systems, qtm.Opts())
    with pytest.raises(qtm.QtmError) as e:
        b.run_range_noalloc(0, 4)
    assert e.value.code == qtm.E_INVAL
    b.destroy()
    # one trajectory's outputs larger than the scratch array
    n_t = ((qtm.NOALLOC_SCRATCH_MB << 20) // 16) // 2 + 10
    s = w.two_level(t_end=1.0, n_t=n_t)
    c = qtm.create_system(s, qtm.Opts())
    with pytest.raises(qtm.QtmError) as e:
        c.run_range_noalloc(0, 2)
    assert e.value.code == qtm.E_INVAL
    c.destroy()
