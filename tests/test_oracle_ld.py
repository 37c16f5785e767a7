"""Pins for the oracle's Langevin integrator, observables and adjoint (CPU only)."""
import math

import numpy as np
import pytest
from scipy import linalg

import oracle as orc
from oracle import moments as mom

P1 = dict(m=1.0, k=1.0, gamma=1.0, kT=1.0, dt=0.01)


def _mat(p):
    return mom.scheme_matrices(p["m"], p["k"], p["gamma"], p["kT"], p["dt"])


# ---------------------------------------------------------------------------------------------
# integrator given the noise: the scheme is linear, z_n = A^n z_0 + sum_i A^(n-1-i) B g_i

@pytest.mark.parametrize("kind", ["taus", "ran2", "lf"])
def test_ld_matches_exact_linear_solution(kind):
    p = dict(m=1.3, k=0.7, gamma=2.1, kT=0.9, dt=0.02)
    N, T = 37, 60
    rng = np.random.default_rng(3)
    x0, v0 = rng.normal(size=(3, N)), rng.normal(size=(3, N))
    ll, sl = (2281, 1252) if kind == "lf" else (0, 0)
    st_run = orc.lf_seed(5, ll) if kind == "lf" else orc.seed_states(kind, 5, np.arange(N))
    st_g = st_run.copy()
    x, v, _ = orc.ld_run(kind, st_run, N, T, p, x0, v0, ll=ll, sl=sl)
    g = orc.ld_forces(kind, st_g, N, T, ll=ll, sl=sl)
    A, B = _mat(p)
    for d in range(3):
        z = np.stack([x0[d], v0[d]])
        for n in range(T):
            z = A @ z + B @ g[n, d][None, :]
        np.testing.assert_allclose(x[d], z[0], rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(v[d], z[1], rtol=1e-11, atol=1e-11)


def test_ld_noise_free_is_matrix_power():
    p = dict(P1, kT=0.0)
    N, T = 5, 333
    rng = np.random.default_rng(4)
    x0, v0 = rng.normal(size=(3, N)), rng.normal(size=(3, N))
    x, v, _ = orc.ld_run("taus", orc.taus_seed(1, np.arange(N)), N, T, p, x0, v0)
    AT = np.linalg.matrix_power(_mat(p)[0], T)
    for d in range(3):
        z = AT @ np.stack([x0[d], v0[d]])
        np.testing.assert_allclose(x[d], z[0], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(v[d], z[1], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("kind", ["taus", "lf"])
def test_overdamped_matches_eq5_given_the_noise(kind):
    """Overdamped scheme (Eq. 5): x_{n+1} = x_n - (k h / xi) x_n + sqrt(2 kT h / xi) g_n, v untouched."""
    p = dict(m=1.3, k=0.7, gamma=2.1, kT=0.9, dt=0.02)
    xi = p["m"] * p["gamma"]
    N, T = 23, 50
    rng = np.random.default_rng(11)
    x0, v0 = rng.normal(size=(3, N)), rng.normal(size=(3, N))
    ll, sl = (2281, 1252) if kind == "lf" else (0, 0)
    st_run = orc.lf_seed(5, ll) if kind == "lf" else orc.seed_states(kind, 5, np.arange(N))
    st_g = st_run.copy()
    x, v, _ = orc.ld_run(kind, st_run, N, T, p, x0, v0, ll=ll, sl=sl, scheme=1)
    g = orc.ld_forces(kind, st_g, N, T, ll=ll, sl=sl)
    z = x0.copy()
    for n in range(T):
        z = z - p["k"] * p["dt"] / xi * z + math.sqrt(2 * p["kT"] * p["dt"] / xi) * g[n]
    np.testing.assert_allclose(x, z, rtol=1e-11, atol=1e-11)
    np.testing.assert_array_equal(v, v0)


def test_overdamped_noise_free_decay_and_closed_forms():
    """Noise-free overdamped decay is x0 a^n; the discrete closed forms tend to the continuous
    Brownian-oscillator forms of Sec. IV as h -> 0, and the variance recursion matches them."""
    p = dict(m=1.0, k=0.5, gamma=2.0, kT=0.0, dt=0.01)
    N, T = 4, 700
    x0 = np.full((3, N), 10.0)
    x, _, _ = orc.ld_run("taus", orc.taus_seed(1, np.arange(N)), N, T, p, x0, np.zeros((3, N)), scheme=1)
    a = 1.0 - p["k"] * p["dt"] / (p["m"] * p["gamma"])
    np.testing.assert_allclose(x, 10.0 * a**T, rtol=1e-12)
    # recursion var_{n+1} = a^2 var_n + b^2 against the closed form
    q = dict(m=1.0, k=1.0, gamma=1.0, kT=1.3, dt=0.01)
    mean, var = mom.overdamped_transient(**q, n_steps=400, x0=10.0)
    a, b2 = 1.0 - q["dt"], 2 * q["kT"] * q["dt"]
    v_rec, m_rec = 0.0, 10.0
    for n in range(400):
        v_rec, m_rec = a * a * v_rec + b2, a * m_rec
    assert abs(v_rec - var[400]) < 1e-12 and abs(m_rec - mean[400]) < 1e-12
    assert abs(mom.overdamped_stationary(**q) - var[400] / (1 - a ** 800)) < 1e-12
    # h -> 0: discrete mean and equilibrium correlation approach R0 exp(-t/tau), (kT/k) exp(-t/tau)
    t = 2.0
    for h, tol in ((1e-3, 2e-3), (1e-4, 2e-4)):
        n = int(round(t / h))
        qh = dict(q, dt=h)
        mean_h, _ = mom.overdamped_transient(**qh, n_steps=n, x0=10.0)
        c_h = mom.overdamped_stationary(**qh) * (1 - h) ** n
        m_c, c_c = mom.overdamped_continuous(q["k"], 1.0, q["kT"], t, 10.0)
        assert abs(mean_h[-1] - m_c) / m_c < tol and abs(c_h - c_c) / c_c < tol


def _fig4_check(obs, N, T, stride, t0, p, x0):
    """Ensemble mean decay and equilibrium autocorrelation against the exact discrete forms, each
    within 4.5 standard errors (3N independent coordinates)."""
    n = 3 * N
    steps = np.arange(0, T + 1, stride)
    mean, var = mom.overdamped_transient(**p, n_steps=T, x0=x0)
    z_mean = np.abs(obs[:, 3] - mean[steps]) / np.sqrt(np.maximum(var[steps], 1e-300) / n)
    after = steps >= t0
    taus = steps[after] - t0
    c = mom.overdamped_cross(**p, t0=t0, taus=taus, x0=x0)
    s = var[steps[after]] + mean[steps[after]] ** 2
    se_c = np.sqrt((s * s[0] + c**2) / n)  # Isserlis, means negligible after equilibration
    z_c = np.abs(obs[after, 4] - c) / se_c
    return float(np.max(z_mean[1:])), float(np.max(z_c))


@pytest.mark.parametrize("kind", ["taus", "ran2", "lf", "lcg"])
def test_fig4_overdamped_statistics_oracle(kind):
    """Sec. IV / Fig. 4 test in reduced units on the oracle: x0 = 10, xi = 2, tau = xi/k = 100 steps."""
    p = dict(m=1.0, k=2.0, gamma=2.0, kT=1.0, dt=0.01)
    N, T, stride, t0 = 3000, 1200, 20, 800
    ll, sl = (132049, 54454) if kind == "lf" else (0, 0)
    st = orc.lf_seed(1234, ll) if kind == "lf" else orc.seed_states(kind, 1234, np.arange(N))
    x0 = np.full((3, N), 10.0)
    _, _, obs = orc.ld_run(kind, st, N, T, p, x0, np.zeros((3, N)), stride=stride, t0=t0, ll=ll, sl=sl, scheme=1)
    zm, zc = _fig4_check(obs, N, T, stride, t0, p, 10.0)
    assert zm < 4.5 and zc < 4.5, (zm, zc)


def test_forces_use_four_words_per_oscillator_step():
    """(g_x, g_y) from words (w0, w1) and g_z the cosine branch of (w2, w3) (Table II caption)."""
    N, T = 3, 4
    st_w, st_g = orc.taus_seed(8, np.arange(N)), orc.taus_seed(8, np.arange(N))
    w = orc.uniform_streams("taus", st_w, 4 * T)        # [4T, N]
    g = orc.ld_forces("taus", st_g, N, T)
    for s in range(T):
        for i in range(N):
            gx, gy = orc.box_muller(int(w[4 * s, i]), int(w[4 * s + 1, i]))
            gz, _ = orc.box_muller(int(w[4 * s + 2, i]), int(w[4 * s + 3, i]))
            assert (g[s, 0, i], g[s, 1, i], g[s, 2, i]) == (gx, gy, gz)


def test_lf_forces_consume_the_shared_sequence_in_thread_order():
    """Thread j at step t takes y_{(j + N t) RNS + r} (Alg. 3's offset, RNS = 4)."""
    ll, sl, N, T = 2281, 1252, 10, 3
    win_w, win_g = orc.lf_seed(2, ll), orc.lf_seed(2, ll)
    y = orc.lf_generate(ll, sl, win_w, 4 * N * T)
    g = orc.ld_forces("lf", win_g, N, T, ll=ll, sl=sl)
    for t in range(T):
        for j in range(N):
            base = (j + N * t) * 4
            gx, gy = orc.box_muller(int(y[base]), int(y[base + 1]))
            gz, _ = orc.box_muller(int(y[base + 2]), int(y[base + 3]))
            assert (g[t, 0, j], g[t, 1, j], g[t, 2, j]) == (gx, gy, gz)


@pytest.mark.parametrize("N,T,scheme", [(3000, 60, 0), (1, 500, 0), (257, 40, 1)])
def test_lf_sampled_run_equals_the_full_run(N, T, scheme):
    """The sampled lagged-Fibonacci run follows its oscillators exactly as the full run does
    (same words, same order, same arithmetic), and leaves the sequence at the same place."""
    ll, sl = 2281, 1252
    p = dict(m=1.0, k=1.3, gamma=0.7, kT=0.9, dt=0.01)
    rng = np.random.Generator(np.random.PCG64(5))
    ids = np.unique(np.concatenate([[0, N - 1], rng.integers(0, N, 20)]))
    win_s, win_f = orc.lf_seed(8, ll), orc.lf_seed(8, ll)
    xs, vs = orc.ld_run_lf_sampled(win_s, ll, sl, N, T, p, ids, scheme=scheme)
    xf, vf, _ = orc.ld_run("lf", win_f, N, T, p, ll=ll, sl=sl, scheme=scheme)
    assert np.array_equal(xs, xf[:, ids]) and np.array_equal(vs, vf[:, ids])
    assert np.array_equal(win_s, win_f)


def test_lf_sampled_run_rejects_bad_ids():
    with pytest.raises(RuntimeError):
        orc.ld_run_lf_sampled(orc.lf_seed(1, 2281), 2281, 1252, 10, 2, P1, [3, 3])
    with pytest.raises(RuntimeError):
        orc.ld_run_lf_sampled(orc.lf_seed(1, 2281), 2281, 1252, 10, 2, P1, [10])


# ---------------------------------------------------------------------------------------------
# exact discrete moments

@pytest.mark.parametrize("p", [P1, dict(P1, dt=0.005), dict(m=1.0, k=2.0, gamma=10.0, kT=2.0, dt=0.01),
                               dict(m=1.0, k=0.5, gamma=0.1, kT=0.5, dt=0.01), dict(m=2.5, k=0.3, gamma=4.0, kT=1.7, dt=0.03)])
def test_stationary_closed_form_solves_lyapunov(p):
    A, B = _mat(p)
    S = linalg.solve_discrete_lyapunov(A, B @ B.T)
    x2, v2, xv = mom.stationary_closed_form(**p)
    np.testing.assert_allclose([S[0, 0], S[1, 1], S[0, 1]], [x2, v2, xv], rtol=1e-10)


def test_stationary_tends_to_equipartition():
    for h in (1e-2, 1e-3, 1e-4):
        x2, v2, _ = mom.stationary_closed_form(1.0, 2.0, 1.5, 0.8, h)
        assert abs(x2 - 0.8 / 2.0) < 2 * h and abs(v2 - 0.8) < 2 * h


def test_config1_discrete_values():
    x2, v2, _ = mom.stationary_closed_form(**P1)
    assert abs(x2 - 1.0000251) < 1e-7 and abs(v2 - 1.0050504) < 1e-7


def test_discrete_autocorrelation_tends_to_continuous_ou():
    p = dict(m=1.0, k=1.0, gamma=1.0, kT=1.0, dt=1e-3)
    taus = np.arange(0, 5001, 500)
    cxx, cvv = mom.cross_moments(**p, t0=20000, taus=taus)
    ref_x, ref_v = mom.continuous_ou(1.0, 1.0, 1.0, 1.0, taus * p["dt"])
    assert np.max(np.abs(cxx - ref_x)) < 5e-3 and np.max(np.abs(cvv - ref_v)) < 5e-3


# ---------------------------------------------------------------------------------------------
# statistical test against the exact discrete moments (the paper's randomness test, Sec. IV)

def _z(est, exact, se):
    return np.abs(est - exact) / se


@pytest.mark.parametrize("kind", ["taus", "ran2", "lf"])
def test_config1_ensemble_statistics(kind):
    """Config-1 workload: N = 1e4 3-D oscillators, 1000 steps of h = 0.01 from rest."""
    N, T, stride, t0 = 10_000, 1000, 10, 500
    ll, sl = (132049, 54454) if kind == "lf" else (0, 0)
    st = orc.lf_seed(1234, ll) if kind == "lf" else orc.seed_states(kind, 1234, np.arange(N))
    x, v, obs = orc.ld_run(kind, st, N, T, P1, stride=stride, t0=t0, ll=ll, sl=sl)
    steps = np.arange(0, T + 1, stride)
    ex2, ev2, exv, _ = mom.second_moments(**P1, n_steps=T)
    n = 3 * N
    ok = steps > 0
    sx = ex2[steps][ok]
    sv = ev2[steps][ok]
    # Var(x^2) = 2 E[x^2]^2 for a centred Gaussian
    assert np.max(_z(obs[ok, 0], sx, sx * math.sqrt(2.0 / n))) < 4.5
    assert np.max(_z(obs[ok, 1], sv, sv * math.sqrt(2.0 / n))) < 4.5
    # autocorrelation after t0; Var(x_t x_t0) = s_t s_t0 + C^2 (Isserlis)
    after = steps >= t0
    taus = steps[after] - t0
    cxx, cvv = mom.cross_moments(**P1, t0=t0, taus=taus)
    se_x = np.sqrt((ex2[steps[after]] * ex2[t0] + cxx**2) / n)
    se_v = np.sqrt((ev2[steps[after]] * ev2[t0] + cvv**2) / n)
    assert np.max(_z(obs[after, 4], cxx, se_x)) < 4.5
    assert np.max(_z(obs[after, 5], cvv, se_v)) < 4.5


def test_observables_are_means_over_coordinates():
    N, T = 50, 30
    st = orc.taus_seed(9, np.arange(N))
    st2 = st.copy()
    _, _, obs = orc.ld_run("taus", st, N, T, P1, stride=10, t0=10)
    x10, v10, _ = orc.ld_run("taus", st2, N, 10, P1)
    x20, v20, _ = orc.ld_run("taus", st2, N, 10, P1, x10, v10)
    np.testing.assert_allclose(obs[1, 0], np.mean(x10**2), rtol=1e-13)
    np.testing.assert_allclose(obs[1, 2], np.mean(x10 * v10), rtol=1e-13)
    np.testing.assert_allclose(obs[2, 4], np.mean(x20 * x10), rtol=1e-13)
    np.testing.assert_allclose(obs[2, 5], np.mean(v20 * v10), rtol=1e-13)
    assert obs[0, 4] == 0.0 and obs[0, 0] == 0.0


def test_run_is_resumable():
    N = 20
    st_a, st_b = orc.taus_seed(3, np.arange(N)), orc.taus_seed(3, np.arange(N))
    xa, va, _ = orc.ld_run("taus", st_a, N, 100, P1)
    xb, vb, _ = orc.ld_run("taus", st_b, N, 40, P1)
    xb, vb, _ = orc.ld_run("taus", st_b, N, 60, P1, xb, vb)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(st_a, st_b)


# ---------------------------------------------------------------------------------------------
# adjoint

PADJ = dict(m=1.0, k=1.0, gamma=1.0, kT=1.0, dt=0.01)


def test_adjoint_dkT_equals_L_over_kT():
    """From rest the path is proportional to sqrt(kT) for a fixed noise path, so dL/dkT = L/kT."""
    p = dict(m=1.0, k=1.4, gamma=0.6, kT=1.7, dt=0.02)
    N = 40
    L, g = orc.ld_adjoint("taus", orc.taus_seed(5, np.arange(N)), N, 300, p, 151, 300)
    assert abs(g[2] - L / p["kT"]) < 1e-12 * abs(L)


@pytest.mark.parametrize("kind", ["taus", "ran2"])
def test_adjoint_matches_crn_central_differences(kind):
    p = dict(m=1.0, k=1.2, gamma=0.8, kT=1.1, dt=0.01)
    N, T, tb, te = 30, 400, 201, 400
    rng = np.random.default_rng(1)
    x0, v0 = rng.normal(size=(3, N)), rng.normal(size=(3, N))
    seed = 77
    L, g = orc.ld_adjoint(kind, orc.seed_states(kind, seed, np.arange(N)), N, T, p, tb, te, x0, v0)
    for i, name in enumerate(("k", "gamma", "kT")):
        d = 1e-4 * p[name]
        hi, lo = dict(p), dict(p)
        hi[name] += d
        lo[name] -= d
        Lh = orc.ld_loss(kind, orc.seed_states(kind, seed, np.arange(N)), N, T, hi, tb, te, x0, v0)
        Ll = orc.ld_loss(kind, orc.seed_states(kind, seed, np.arange(N)), N, T, lo, tb, te, x0, v0)
        fd = (Lh - Ll) / (2 * d)
        assert abs(fd - g[i]) < 1e-6 * max(1.0, abs(g[i])), (name, fd, g[i])
    L2 = orc.ld_loss(kind, orc.seed_states(kind, seed, np.arange(N)), N, T, p, tb, te, x0, v0)
    assert abs(L - L2) < 1e-12 * abs(L)


def test_adjoint_expectation_matches_moment_recursion():
    """Config-5 shape at reduced N: the pathwise gradient averaged over oscillators estimates
    d E[L]/d theta, which the deterministic covariance recursion gives exactly."""
    N, T, tb, te = 2000, 2000, 1001, 2000
    states = orc.taus_seed(1234, np.arange(N))
    per = np.zeros((N, 3))
    for i in range(N):
        _, g = orc.ld_adjoint("taus", states[i:i + 1].copy(), 1, T, PADJ, tb, te)
        per[i] = g
    est = per.mean(axis=0)
    se = per.std(axis=0, ddof=1) / math.sqrt(N)
    exact = mom.expected_loss_grad(**PADJ, n_steps=T, t_begin=tb, t_end=te)
    assert np.all(np.abs(est - exact) < 4.5 * se + 1e-9), (est, exact, se)


def test_stationary_gradient_closed_form():
    p = dict(m=1.0, k=1.0, gamma=1.0, kT=1.0, dt=0.01)
    # a window far beyond the relaxation time is stationary
    g_rec = mom.expected_loss_grad(**p, n_steps=6000, t_begin=3001, t_end=6000, rel=1e-4)
    g_cf = mom.stationary_x2_grad(**p)
    np.testing.assert_allclose(g_rec[[0, 2]], g_cf[[0, 2]], rtol=1e-4)
    assert abs(g_rec[1] - g_cf[1]) < 1e-5


def test_fig4_lcg_correlated_seeding_fails_the_test():
    """Negative control (Fig. 4b): LCG streams seeded as windows of one sequence, four values
    apart, hand each oscillator its neighbour's noise one step later.  The ensemble mean then
    carries the neighbours' shared noise and fails the same z test that independently seeded
    streams pass; neighbouring oscillators end up almost fully correlated (about a = 1 - kh/xi)."""
    p = dict(m=1.0, k=1.0, gamma=1.0, kT=1.0, dt=0.01)
    N, T, stride, t0 = 3000, 4000, 20, 800
    x0 = np.full((3, N), 10.0)
    res = {}
    for leap in (0, 4):
        st = orc.seed_states("lcg", 1234, np.arange(N), leap=leap)
        x, _, obs = orc.ld_run("lcg", st, N, T, p, x0, np.zeros((3, N)), stride=stride, t0=t0, scheme=1)
        zm, zc = _fig4_check(obs, N, T, stride, t0, p, 10.0)
        corr = np.mean([np.corrcoef(x[d, :-1], x[d, 1:])[0, 1] for d in range(3)])
        res[leap] = (zm, zc, corr)
    assert res[0][0] < 4.5 and res[0][1] < 4.5 and abs(res[0][2]) < 0.1, res
    assert max(res[4][0], res[4][1]) > 10 and res[4][2] > 0.9, res
