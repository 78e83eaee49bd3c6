"""Pins of the exact-propagator oracle (oracle/expo.py, the stiff form's oracle), no GPU:

* against the independent DOPRI5 oracle at a tight tolerance on the same random
  streams (same jumps, jump times and outputs to the DOPRI5 accuracy);
* a closed form: C proportional to I gives jump times sum_j -ln(r_j)/gamma and the
  unitary expectation values;
* a stiff system (cavity decay 40 times the coupling) against the Lindblad equation."""
import numpy as np

import oracle
import workloads as w
from oracle import expo, lindblad


def test_expo_oracle_matches_dopri5_oracle():
    s = w.jaynes_cummings(N=6, t_end=6.0, n_t=61)
    n = 24
    a = expo.run_expo(s, n, seed=3)
    b = oracle.run(s, n, seed=3, rtol=1e-11, atol=1e-13, jcap=32)
    assert np.array_equal(a["jump_counts"], b["jump_counts"])
    for q in range(n):
        m = int(min(a["jump_counts"][q], 32))
        assert np.array_equal(a["jump_channels"][q, :m], b["jump_channels"][q, :m])
        assert np.max(np.abs(a["jump_times"][q, :m] - b["jump_times"][q, :m]), initial=0.0) < 1e-8
    assert np.max(np.abs(a["X"] - b["X"])) < 1e-7


def test_expo_oracle_closed_form_identity_channels():
    s = w.two_channel_identity(0.3, 0.2, t_end=10.0, n_t=41)
    n = 16
    res = expo.run_expo(s, n, seed=1)
    g = 0.3 + 0.2
    for q in range(n):
        tj = 0.0
        for j in range(int(res["jump_counts"][q])):
            r = oracle.uniform53(int(oracle.philox4x64_10([q, j, 0, 0], [1, 0])[0]))
            tj += -np.log(r) / g
            assert abs(res["jump_times"][q, j] - tj) < 1e-11 * (1.0 + tj)


def test_expo_oracle_stiff_cavity_vs_lindblad():
    """Jaynes-Cummings with cavity decay 40 (40 times g): the cavity relaxes in 0.025
    while the dynamics of interest take units of time."""
    s = w.jaynes_cummings(N=6, kappa=40.0, gamma_a=0.05, alpha=1.0, t_end=4.0, n_t=41)
    n = 3000
    res = expo.run_expo(s, n, seed=5)
    ref = lindblad.expect_expm(s)
    for e in range(2):
        bound = 3.0 * np.sqrt(res["var"][e] / n) + 1e-6
        dev = np.abs(res["mean"][e].real - ref[e].real)
        assert np.all(dev <= bound), (e, float(np.max(dev / bound)))
