"""Oracle trajectory averages against the Lindblad master equation and closed
forms, plus invariants of the method (no GPU)."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import workloads as w
from oracle import closed_forms as cf
from oracle import lindblad


def _within(mean, var, ref, n, k=3.0, floor=1e-6):
    """|mean - ref| <= k sigma/sqrt(n) + floor at every point."""
    bound = k * np.sqrt(var / n) + floor
    return np.all(np.abs(mean - ref) <= bound), np.max(np.abs(mean - ref) / bound)


def _within_many(mean, var, ref, n, floor=1e-6):
    """For many time points of one independent sample: none beyond 4 sigma/sqrt(n) +
    floor (chance 6e-5 per point) and at most 5% of the points beyond 3 sigma/sqrt(n) +
    floor.  0.27% of independent points lie beyond 3 sigma by chance; consecutive
    output times of one sample are correlated, so a single excursion of the average
    covers several of them."""
    z = np.abs(mean - ref) / (np.sqrt(var / n) + floor / 3.0)
    return (np.mean(z > 3.0) <= 0.05 and np.all(z <= 4.0)), float(np.max(z))


def test_lindblad_routes_agree_with_closed_forms():
    s = w.two_level()
    assert np.max(np.abs(lindblad.expect_expm(s)[0] - cf.two_level_sz(s.tlist))) < 1e-13
    assert np.max(np.abs(lindblad.expect_ode(s)[0] - cf.two_level_sz(s.tlist))) < 1e-8
    s = w.unitary_example()
    assert np.max(np.abs(lindblad.expect_expm(s)[0] - cf.unitary_example_sz(s.tlist))) < 1e-13
    s = w.photon_birth_death()
    # the Fock cutoff N = 5 changes <n> by at most 2e-5
    assert np.max(np.abs(lindblad.expect_expm(s)[0] - cf.photon_number(s.tlist))) < 2.5e-5
    s = w.jaynes_cummings(kappa=0.0, gamma_a=0.0)
    assert np.max(np.abs(lindblad.expect_expm(s)[1] - cf.jcm_excited_population(s.tlist))) < 1e-12


def test_two_level_average_vs_torrey():
    s = w.two_level()
    n = 20000
    res = oracle.run(s, n, seed=0)
    assert res["status"] == 0
    ok, worst = _within(res["mean"][0].real, res["var"][0], cf.two_level_sz(s.tlist), n)
    assert ok, worst
    # expected number of jumps on [0, 10] is about 2.07
    assert abs(res["jump_counts"].mean() - 2.07) < 0.05


def test_unitary_example_average_vs_closed_form():
    s = w.unitary_example(c_scale=0.3)
    n = 8000
    res = oracle.run(s, n, seed=1)
    ok, worst = _within(res["mean"][0].real, res["var"][0], cf.unitary_example_sz(s.tlist, 0.3), n)
    assert ok, worst


def test_photon_birth_death_two_channels():
    """Two channels, one of them a creation operator: the channel statistics
    enter <n>; checked against the exact truncated Lindblad solution."""
    s = w.photon_birth_death()
    n = 20000
    res = oracle.run(s, n, seed=2)
    ref = lindblad.expect_expm(s)[0].real
    ok, worst = _within(res["mean"][0].real, res["var"][0], ref, n)
    assert ok, worst
    assert set(np.unique(res["jump_channels"][res["jump_counts"] > 0, 0])) <= {0, 1}


def test_jaynes_cummings_vs_lindblad():
    s = w.jaynes_cummings(t_end=10.0, n_t=101)
    n = 3000
    res = oracle.run(s, n, seed=0)
    ref = lindblad.expect_expm(s)
    for e in range(2):
        ok, worst = _within(res["mean"][e].real, res["var"][e], ref[e].real, n)
        assert ok, (e, worst)


def test_small_tfim_vs_lindblad():
    s = w.tfim(L=4, t_end=5.0, n_t=26)
    n = 6000
    res = oracle.run(s, n, seed=4)
    ref = lindblad.expect_expm(s)
    for e in range(4):
        ok, worst = _within(res["mean"][e].real, res["var"][e], ref[e].real, n)
        assert ok, (e, worst)


def test_random_system_vs_lindblad():
    rng = np.random.Generator(np.random.Philox(key=9))
    s = w.random_system(rng, 12, 3, t_end=20.0, n_t=41, c_norm=0.3)
    n = 6000
    res = oracle.run(s, n, seed=6)
    ref = lindblad.expect_ode(s)
    for e in range(2):
        ok, worst = _within(res["mean"][e].real, res["var"][e], ref[e].real, n)
        assert ok, (e, worst)


def test_trilinear_small_cutoff_vs_lindblad():
    """The optical parametric amplifier of Sec. 4.2 (H = iK(a b^dag c^dag - a^dag b c),
    three damped modes, coherent pump) at Fock cutoff 5 per mode (d = 125, CSR).
    20,000 trajectories: at early times the signal and idler averages rest on the few
    trajectories that have jumped (before any jump every trajectory has n_b = n_c), and
    fewer trajectories leave that tail too thin for the sample variance to describe."""
    s = w.trilinear(N=5)
    n = 20000
    res = oracle.run(s, n, seed=3)
    ref = lindblad.expect_ode(s, rtol=1e-8, atol=1e-10)
    for e in range(3):
        ok, worst = _within(res["mean"][e].real, res["var"][e], ref[e].real, n)
        assert ok, (e, worst)


@pytest.mark.slow
def test_trilinear_full_size_vs_lindblad():
    """The paper's size: cutoff 8 per mode (d = 512, CSR), t in [0, 4], 100 outputs;
    brute-force Lindblad by DOP853 on the 512 x 512 density matrix.  300 points of one
    independent sample are compared, so the 3-sigma bound is applied as a rate."""
    s = w.trilinear()
    assert s.dim == 512
    n = 20000
    res = oracle.run(s, n, seed=5)
    ref = lindblad.expect_ode(s, rtol=1e-7, atol=1e-9)
    ok, worst = _within_many(res["mean"].real, res["var"], ref.real, n)
    assert ok, worst


def test_trilinear_closed_system_conservation():
    """Without damping, H moves one quantum from the pump into the signal and idler
    pair: n_a + n_b, n_a + n_c and hence n_b - n_c are conserved on every trajectory
    (no jumps), at the tolerance of the integration."""
    s = w.trilinear(gammas=(0.0, 0.0, 0.0))
    s.c_ops = []
    res = oracle.run(s, 2, seed=0, rtol=1e-9, atol=1e-11)
    assert res["jump_counts"].sum() == 0
    X = res["X"].real
    n0 = X[0, 0, 0]
    assert np.max(np.abs(X[:, 0] + X[:, 1] - n0)) < 1e-6
    assert np.max(np.abs(X[:, 1] - X[:, 2])) < 1e-6
    assert np.max(X[:, 1]) > 0.5          # the signal mode is actually populated


# ------------------------------------------------------------ invariants
def test_identity_observable_and_hermitian_imaginary_part():
    s = w.jaynes_cummings(N=8, t_end=10.0, n_t=51)
    s.e_ops = [w.diag(np.ones(s.dim)), s.e_ops[0], w.dense(s.H.to_dense())]
    res = oracle.run(s, 200, seed=0)
    assert np.max(np.abs(res["X"][:, 0] - 1.0)) < 1e-13
    assert np.max(np.abs(res["X"][:, 1:].imag)) < 1e-13


def test_no_collapse_operators_is_unitary_evolution():
    s = w.jaynes_cummings(kappa=0.0, gamma_a=0.0, t_end=10.0, n_t=51)
    res = oracle.run(s, 3, seed=0, rtol=1e-10, atol=1e-12)
    assert res["jump_counts"].sum() == 0
    H = s.H.to_dense()
    for k, t in enumerate(s.tlist):
        psi = sla.expm(-1j * H * t) @ s.psi0
        for e, op in enumerate(s.e_ops):
            ex = np.vdot(psi, op.to_dense() @ psi).real
            assert np.all(np.abs(res["X"][:, e, k].real - ex) < 1e-7)
    assert np.max(np.abs(res["X"][:, 1].real - cf.jcm_excited_population(s.tlist))) < 1e-7


def test_norm_non_increasing_between_jumps():
    s = w.jaynes_cummings(N=10)
    M = oracle.build_M(s.H, s.c_ops)
    norms = []
    for t1 in np.linspace(0.5, 10.0, 20):
        _, y, _ = oracle.integrate_nojump(M, s.psi0, 0.0, t1)
        norms.append(np.vdot(y, y).real)
    norms = np.array(norms)
    # exact: d||psi||^2/dt = -sum ||C psi||^2 <= 0; numerically within rtol
    assert np.all(np.diff(norms) <= 1e-6 * norms[1:])
    assert norms[-1] < norms[0]


def test_expected_jumps_jcm():
    s = w.jaynes_cummings()
    res = oracle.run(s, 400, seed=0)
    assert abs(res["jump_counts"].mean() - 4.92) < 0.35
    st = res["stats"]
    assert np.all(st[:, 3] == st[:, 4] + 1)  # segments = jumps + 1


# ------------------------------------------------------------ time-dependent Hamiltonians
def test_td_commuting_drive_closed_form():
    """H(t) = f(t) sigma_x with C = sqrt(gamma) I: every trajectory's <sigma_z>(t) equals
    cos(2 F(t)), F the integral of f, and the jump times are the cumulative sums of
    -ln(r_j)/gamma with the oracle's own threshold draws."""
    s = w.commuting_drive()
    c, a, b, om, g = (s.meta[k] for k in ("c", "a", "b", "w", "gamma"))
    t = s.tlist
    F = c * t + (a / om) * np.sin(om * t) + (b / om) * (1.0 - np.cos(om * t))
    n = 40
    res = oracle.run(s, n, seed=2, rtol=1e-9, atol=1e-12, jcap=32)
    assert np.max(np.abs(res["X"][:, 0, :].real - np.cos(2.0 * F))) < 1e-7
    for q in range(n):
        tj = 0.0
        for j in range(int(res["jump_counts"][q])):
            r = oracle.uniform53(int(oracle.philox4x64_10([q, j, 0, 0], [2, 0])[0]))
            tj += -np.log(r) / g
            assert abs(res["jump_times"][q, j] - tj) < 1e-7 * (1.0 + tj)


def test_td_closed_system_vs_schroedinger():
    """The driven two-level atom without decay: the stage times of every right-hand-side
    evaluation matter; the oracle's states agree with a tight DOP853 integration of
    psi' = -i H(t) psi."""
    from scipy.integrate import solve_ivp
    s = w.driven_two_level(gamma=0.0)
    s.c_ops = []
    res = oracle.run(s, 1, seed=0, rtol=1e-10, atol=1e-12)
    H0 = s.H.to_dense()
    H1, (c, a, b, om) = s.td[0][0].to_dense(), s.td[0][1]

    def f(t, y):
        return -1j * ((H0 + (c + a * np.cos(om * t) + b * np.sin(om * t)) * H1) @ y)

    sol = solve_ivp(f, (s.tlist[0], s.tlist[-1]), s.psi0, method="DOP853", t_eval=s.tlist, rtol=1e-12, atol=1e-14)
    for e, op in enumerate(s.e_ops):
        O = op.to_dense()
        ex = np.array([np.vdot(sol.y[:, k], O @ sol.y[:, k]).real for k in range(len(s.tlist))])
        assert np.max(np.abs(res["X"][0, e].real - ex)) < 1e-7, e


def test_td_driven_atom_vs_lindblad():
    """The driven, decaying two-level atom without the rotating-wave approximation
    against the time-dependent Lindblad equation."""
    s = w.driven_two_level()
    n = 20000
    res = oracle.run(s, n, seed=8)
    ref = lindblad.expect_ode(s)
    for e in range(2):
        ok, worst = _within(res["mean"][e].real, res["var"][e], ref[e].real, n)
        assert ok, (e, worst)


def test_td_driven_jaynes_cummings_vs_lindblad():
    """The cavity of the Jaynes-Cummings system driven by eps cos(omega_d t)(a + a^dag)
    (cutoff 8, d = 16, t in [0, 8])."""
    s = w.driven_jaynes_cummings(N=8, eps=0.4, t_end=8.0, n_t=81, alpha=1.0)
    n = 8000
    res = oracle.run(s, n, seed=9)
    ref = lindblad.expect_ode(s)
    ok, worst = _within_many(res["mean"].real, res["var"], ref.real, n)
    assert ok, worst
