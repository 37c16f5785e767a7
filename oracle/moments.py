"""Exact moments of the discrete Langevin schemes used by the oracle (FP64, numpy).

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle/``).

The paper's randomness test (Sec. IV) compares simulated <R(t)> and <R(t)R(0)> of harmonic
oscillators with the exact Ornstein-Uhlenbeck results.  A finite time step biases those continuous
results by O(h), which at the sizes used here is comparable to the sampling error, so the tests
compare against the *discrete* scheme's exact moments instead; the continuous forms are kept as a
second, O(h)-biased check.

Underdamped semi-implicit Euler-Maruyama step (per Cartesian component), z = (x, v):
    v' = c v - kap x + sig g,   x' = x + h v'
  => z' = A z + B g,  A = [[1 - h kap, h c], [-kap, c]],  B = sig [h, 1]^T,
  c = 1 - gamma h, kap = k h / m, sig = sqrt(2 gamma kT h / m).
Overdamped step (Eq. 5, random displacement sqrt(2 kT h / xi) g, xi = m gamma):
    x' = a x + b g,  a = 1 - k h / xi,  b = sqrt(2 kT h / xi).
"""
from __future__ import annotations

import math

import numpy as np


def scheme_matrices(m, k, gamma, kT, dt):
    h = float(dt)
    c = 1.0 - gamma * h
    kap = k * h / m
    sig = math.sqrt(2.0 * gamma * kT * h / m)
    A = np.array([[1.0 - h * kap, h * c], [-kap, c]])
    B = sig * np.array([[h], [1.0]])
    return A, B


def stationary_closed_form(m, k, gamma, kT, dt):
    """(<x^2>, <v^2>, <x v>) of the stationary law of the underdamped scheme.

    Solving Sigma = A Sigma A^T + B B^T by hand gives, with D = 1 - gamma h / 2 - k h^2 / (4 m):
    <v^2> = (kT/m)/D,  <x^2> = (kT/k)(1 - gamma h/2)/D,  <x v> = h <v^2> / 2.
    As h -> 0 these tend to equipartition, kT/k and kT/m.
    """
    h = float(dt)
    D = 1.0 - gamma * h / 2.0 - k * h * h / (4.0 * m)
    v2 = (kT / m) / D
    x2 = (kT / k) * (1.0 - gamma * h / 2.0) / D
    return x2, v2, h * v2 / 2.0


def overdamped_stationary(m, k, gamma, kT, dt):
    xi = m * gamma
    a = 1.0 - k * dt / xi
    b2 = 2.0 * kT * dt / xi
    return b2 / (1.0 - a * a)


def overdamped_transient(m, k, gamma, kT, dt, n_steps, x0=0.0):
    """Mean and variance of one coordinate of the overdamped scheme (Eq. 5),
    x_{n+1} = a x_n + b g_n with a = 1 - k h / xi, b^2 = 2 kT h / xi, xi = m gamma, from x_0 = x0:
    mean_n = x0 a^n, var_n = b^2 (1 - a^(2n)) / (1 - a^2).  Arrays over n = 0..n_steps."""
    xi = m * gamma
    a = 1.0 - k * dt / xi
    b2 = 2.0 * kT * dt / xi
    n = np.arange(n_steps + 1, dtype=float)
    return x0 * a**n, b2 * (1.0 - a ** (2 * n)) / (1.0 - a * a)


def overdamped_cross(m, k, gamma, kT, dt, t0, taus, x0=0.0):
    """E[x(t0 + tau) x(t0)] = a^tau E[x(t0)^2] (the noise after t0 is independent of x(t0))."""
    xi = m * gamma
    a = 1.0 - k * dt / xi
    mean, var = overdamped_transient(m, k, gamma, kT, dt, t0, x0)
    return a ** np.asarray(taus, dtype=float) * (var[t0] + mean[t0] ** 2)


def overdamped_continuous(k, xi, kT, t, x0):
    """Sec. IV's exact Brownian-oscillator forms: <R(t)> = R0 exp(-t/tau) and the equilibrium
    <R(t)R(0)> = (kT/k) exp(-t/tau), tau = xi/k."""
    e = np.exp(-np.asarray(t, dtype=float) * k / xi)
    return x0 * e, (kT / k) * e


def transient(m, k, gamma, kT, dt, n_steps, z0=(0.0, 0.0)):
    """Mean and covariance after n = 0..n_steps steps from the deterministic state z0.

    Returns (mean[n_steps+1, 2], cov[n_steps+1, 2, 2]) with
    mean_{n+1} = A mean_n and cov_{n+1} = A cov_n A^T + B B^T, cov_0 = 0.
    """
    A, B = scheme_matrices(m, k, gamma, kT, dt)
    BB = B @ B.T
    mean = np.zeros((n_steps + 1, 2))
    cov = np.zeros((n_steps + 1, 2, 2))
    mean[0] = z0
    for n in range(n_steps):
        mean[n + 1] = A @ mean[n]
        cov[n + 1] = A @ cov[n] @ A.T + BB
    return mean, cov


def second_moments(m, k, gamma, kT, dt, n_steps, z0=(0.0, 0.0)):
    """E[x^2], E[v^2], E[x v], E[x] for n = 0..n_steps (per component)."""
    mean, cov = transient(m, k, gamma, kT, dt, n_steps, z0)
    x2 = cov[:, 0, 0] + mean[:, 0] ** 2
    v2 = cov[:, 1, 1] + mean[:, 1] ** 2
    xv = cov[:, 0, 1] + mean[:, 0] * mean[:, 1]
    return x2, v2, xv, mean[:, 0]


def cross_moments(m, k, gamma, kT, dt, t0, taus, z0=(0.0, 0.0)):
    """E[x(t0+tau) x(t0)] and E[v(t0+tau) v(t0)] for each tau.

    E[z_{t0+tau} z_{t0}^T] = A^tau E[z_{t0} z_{t0}^T] (the noise after t0 is independent of z_{t0}).
    """
    A, _ = scheme_matrices(m, k, gamma, kT, dt)
    mean, cov = transient(m, k, gamma, kT, dt, t0, z0)
    S = cov[t0] + np.outer(mean[t0], mean[t0])
    cxx, cvv = [], []
    for tau in taus:
        M = np.linalg.matrix_power(A, int(tau)) @ S
        cxx.append(M[0, 0])
        cvv.append(M[1, 1])
    return np.array(cxx), np.array(cvv)


def expected_loss(m, k, gamma, kT, dt, n_steps, t_begin, t_end, z0=(0.0, 0.0)):
    """E[L] for L = mean over steps t_begin..t_end of the per-component <x^2>."""
    x2, _, _, _ = second_moments(m, k, gamma, kT, dt, n_steps, z0)
    return float(np.mean(x2[t_begin:t_end + 1]))


def expected_loss_grad(m, k, gamma, kT, dt, n_steps, t_begin, t_end, rel=1e-5):
    """d E[L] / d(k, gamma, kT) by central differences of the deterministic moment recursion."""
    base = dict(m=m, k=k, gamma=gamma, kT=kT, dt=dt)
    out = []
    for name in ("k", "gamma", "kT"):
        hi, lo = dict(base), dict(base)
        d = rel * base[name]
        hi[name] += d
        lo[name] -= d
        f = lambda p: expected_loss(p["m"], p["k"], p["gamma"], p["kT"], p["dt"], n_steps, t_begin, t_end)
        out.append((f(hi) - f(lo)) / (2 * d))
    return np.array(out)


def stationary_x2_grad(m, k, gamma, kT, dt):
    """Closed-form derivatives of the stationary <x^2> w.r.t. (k, gamma, kT)."""
    h = float(dt)
    D = 1.0 - gamma * h / 2.0 - k * h * h / (4.0 * m)
    x2 = (kT / k) * (1.0 - gamma * h / 2.0) / D
    d_k = x2 * (-1.0 / k + h * h / (4.0 * m * D))
    d_gamma = (kT / k) * (h / 2.0) * (k * h * h / (4.0 * m)) / (D * D)
    d_kT = x2 / kT
    return np.array([d_k, d_gamma, d_kT])


def continuous_ou(m, k, gamma, kT, tau):
    """Textbook underdamped OU autocorrelations (kT/k) phi_x(tau), (kT/m) phi_v(tau)."""
    tau = np.asarray(tau, dtype=np.float64)
    w0sq = k / m
    disc = w0sq - gamma * gamma / 4.0
    e = np.exp(-gamma * tau / 2.0)
    if disc > 0:
        w1 = math.sqrt(disc)
        cx = e * (np.cos(w1 * tau) + gamma / (2 * w1) * np.sin(w1 * tau))
        cv = e * (np.cos(w1 * tau) - gamma / (2 * w1) * np.sin(w1 * tau))
    else:
        w1 = math.sqrt(-disc)
        cx = e * (np.cosh(w1 * tau) + gamma / (2 * w1) * np.sinh(w1 * tau))
        cv = e * (np.cosh(w1 * tau) - gamma / (2 * w1) * np.sinh(w1 * tau))
    return (kT / k) * cx, (kT / m) * cv
