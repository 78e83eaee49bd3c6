"""Pins of the oracle's learned-proposal MLP (16 -> 64 -> 64 -> 3, GELU)."""
import numpy as np
from scipy.stats import norm as normal

import oracle

NF, NH, NO = 16, 64, 3


def _unpack(p):
    o = 0
    out = {}
    for name, shape in (("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
                        ("W3", (NO, NH)), ("b3", (NO,)), ("mu", (NF,)), ("sd", (NF,))):
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def _random_params(rng):
    p = np.zeros(oracle.mlp_ntotal())
    q = _unpack(p)
    q["W1"][:] = rng.standard_normal((NH, NF)) / 4
    q["b1"][:] = rng.standard_normal(NH) * 0.1
    q["W2"][:] = rng.standard_normal((NH, NH)) / 8
    q["b2"][:] = rng.standard_normal(NH) * 0.1
    q["W3"][:] = rng.standard_normal((NO, NH)) / 8
    q["b3"][:] = rng.standard_normal(NO) * 0.1
    q["mu"][:] = rng.standard_normal(NF)
    q["sd"][:] = 0.5 + rng.random(NF)
    return p


def test_param_count():
    assert oracle.mlp_nparam() == NH * NF + NH + NH * NH + NH + NO * NH + NO
    assert oracle.mlp_ntotal() == oracle.mlp_nparam() + 2 * NF


def test_gelu_special_case():
    """With W2 = 0 the output is b3 + W3 gelu(b2), gelu(x) = x Phi(x) (normal CDF)."""
    rng = np.random.default_rng(0)
    p = _random_params(rng)
    q = _unpack(p)
    q["W2"][:] = 0.0
    out = oracle.mlp_forward(p, rng.standard_normal((3, NF)))
    b2 = q["b2"]
    ref = q["b3"] + q["W3"] @ (b2 * normal.cdf(b2))
    assert np.allclose(out, ref[None, :], atol=1e-14)


def test_affine_special_case():
    """Large positive pre-activations make GELU the identity, so the network is the
    affine map W3 (W2 (W1 x' + b1) + b2) + b3 with x' = (x - mu)/sd."""
    rng = np.random.default_rng(1)
    p = _random_params(rng)
    q = _unpack(p)
    q["b1"][:] = 60.0
    q["b2"][:] = 0.0
    q["W2"][:] = np.abs(q["W2"]) * 0.01
    q["b2"][:] = 60.0
    x = rng.standard_normal((4, NF)) * 0.1
    xs = (x - q["mu"]) / q["sd"]
    h1 = xs @ q["W1"].T + q["b1"]
    h2 = h1 @ q["W2"].T + q["b2"]
    ref = h2 @ q["W3"].T + q["b3"]
    assert np.allclose(oracle.mlp_forward(p, x), ref, rtol=1e-12, atol=1e-10)


def test_gradient_vs_central_differences():
    rng = np.random.default_rng(2)
    p = _random_params(rng)
    n = 32
    x = rng.standard_normal((n, NF))
    tgt = np.stack([rng.standard_normal(n), rng.standard_normal(n), (rng.random(n) < 0.3).astype(float)], 1)
    L, g = oracle.mlp_loss_grad(p, x, tgt)
    idx = rng.choice(oracle.mlp_nparam(), 120, replace=False)
    eps = 1e-6
    num = np.zeros(len(idx))
    for m, i in enumerate(idx):
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        num[m] = (oracle.mlp_loss_grad(pp, x, tgt, False)[0] - oracle.mlp_loss_grad(pm, x, tgt, False)[0]) / (2 * eps)
    rel = np.linalg.norm(num - g[idx]) / np.linalg.norm(num)
    assert rel < 1e-6, rel


def test_snap_grid():
    for lh in (-3.0, -0.1, 0.0, 0.7, 2.3):
        h = oracle.snap_step(lh)
        k = 4 * np.log2(h)
        assert abs(k - round(k)) < 1e-12
        assert abs(np.log2(h) - lh / np.log(2)) <= 0.125 + 1e-12
