"""Seeded synthetic workloads: the five configurations, Table I lags and batched-ensemble draws.

This module holds inputs only -- sizes, parameters, seeds, sampled indices -- and none of the
method's arithmetic (no generator, transform or integrator).  Tests feed the same inputs to the
GPU path and to the CPU oracle; the benchmark uses them to build its workload.  Draws that are not
part of the method (ensemble parameters, sampled stream ids, random initial states) use numpy's
PCG64, so they share nothing with the generators under test.
"""
from __future__ import annotations

import dataclasses

import numpy as np

# Table I (Appendix): (sl, ll) by system size; row (23209, 12470) read as (23209, 13470), since
# x^23209 + x^12470 + 1 is reducible and 13470 gives a primitive trinomial.
TABLE1 = [(1252, 2281), (3004, 4423), (5502, 9689), (10095, 19937), (13470, 23209), (23463, 44497),
          (54454, 132049), (279695, 756839), (288477, 859433), (1010202, 3021377)]


def lf_lags_for(numbers_per_step: int):
    """Smallest Table I row whose short lag exceeds the numbers drawn per step (Alg. 3 text asks
    for sl > RNS*N); beyond the table, its last row."""
    for sl, ll in TABLE1:
        if sl > numbers_per_step:
            return ll, sl
    return TABLE1[-1][1], TABLE1[-1][0]


@dataclasses.dataclass(frozen=True)
class LDParams:
    m: float = 1.0
    k: float = 1.0
    gamma: float = 1.0
    kT: float = 1.0
    dt: float = 0.01

    def as_f32(self) -> "LDParams":
        """The values a float32 parameter block carries (both sides start from these)."""
        f = lambda a: float(np.float32(a))
        return LDParams(f(self.m), f(self.k), f(self.gamma), f(self.kT), f(self.dt))

    def asdict(self):
        return dataclasses.asdict(self)


# config 1: correctness (Hybrid Taus, N = 1e4, 1000 steps, h = 0.01, from rest)
C1 = dict(kind="taus", seed=1234, N=10_000, steps=1000, params=LDParams(dt=0.01), stride=10, t0=500)
# config 2: throughput (all three generators, N = 1e6, 1e4 steps, h = 0.005)
C2 = dict(seed=1234, N=1_000_000, steps=10_000, params=LDParams(dt=0.005), lf_lags=(3021377, 1010202))
# config 3: bare generators (2^20 streams x 1024 values; LF: one stream of 2^30)
C3 = dict(seed=1234, streams=2**20, per_stream=1024, lf_count=2**30, lf_lags=(3021377, 1010202))
# config 4: batched (512 ensembles from seed 7, Hybrid Taus, 5000 steps, h = 0.01)
C4 = dict(n_ens=512, draw_seed=7, base_seed=1234, steps=5000, dt=0.01)
# config 5: adjoint (N = 1e5, Hybrid Taus, 2000 steps, loss over steps 1001..2000, K = 100)
C5 = dict(seed=1234, N=100_000, steps=2000, params=LDParams(dt=0.01), t_begin=1001, t_end=2000, K=100)


@dataclasses.dataclass(frozen=True)
class Ensemble:
    n: int
    params: LDParams
    seed: int


def batched_ensembles(n_ens: int = 512, draw_seed: int = 7, base_seed: int = 1234, dt: float = 0.01,
                      n_lo: float = 1e3, n_hi: float = 1e6):
    """Ensemble e: N log-uniform in [n_lo, n_hi], k ~ U[0.5, 2], gamma ~ U[0.1, 10], kT ~ U[0.5, 2],
    m = 1, generator seed base_seed + e.  Parameters are rounded to float32."""
    rng = np.random.Generator(np.random.PCG64(draw_seed))
    u = rng.random((n_ens, 4))
    out = []
    for e in range(n_ens):
        n = int(np.clip(np.rint(10 ** (np.log10(n_lo) + (np.log10(n_hi) - np.log10(n_lo)) * u[e, 0])), n_lo, n_hi))
        p = LDParams(m=1.0, k=0.5 + 1.5 * u[e, 1], gamma=0.1 + 9.9 * u[e, 2], kT=0.5 + 1.5 * u[e, 3], dt=dt).as_f32()
        out.append(Ensemble(n=n, params=p, seed=base_seed + e))
    return out


def sampled_streams(n_streams: int = 2**20, n_sample: int = 64, seed: int = 99):
    """Stream ids for sampled bit-exact checks: 0, 1, the last one and the rest drawn from seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fixed = [0, 1, n_streams - 1]
    rest = rng.choice(np.arange(2, n_streams - 1), size=max(n_sample - 3, 0), replace=False)
    return np.array(sorted(set(fixed) | set(int(r) for r in rest)), dtype=np.int64)[:n_sample]


def initial_state(N: int, seed: int | None = None, scale: float = 1.0):
    """x0, v0 as [3, N] float32: zeros, or N(0, scale^2) draws from PCG64(seed)."""
    if seed is None:
        return np.zeros((3, N), np.float32), np.zeros((3, N), np.float32)
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.normal(0, scale, (3, N)).astype(np.float32), rng.normal(0, scale, (3, N)).astype(np.float32))
