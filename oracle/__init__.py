"""Plain CPU reference ("oracle") for the on-the-fly RNG + Langevin-dynamics path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``.  The product package never imports it and shares no code with
it.  The arithmetic lives in ``rngld_oracle.c`` (double precision, sequential, written from the
paper's definitions); this module only marshals numpy arrays through ctypes.  Closed-form moments
of the integrator are in :mod:`oracle.moments`.

Generators follow Zhmurov et al., arXiv:1003.1123: Hybrid Taus (Sec. II.D, Appendix A Alg. 1),
Ran2 (Sec. II.C, Alg. 2), additive lagged Fibonacci (Sec. II.E Eq. 3, Alg. 3, Table I) and the
per-stream Quick-and-Dirty LCG (Sec. II.B Eq. 1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rngld_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

TAUS, RAN2, LF, LCG = 0, 1, 2, 3
KIND_NAMES = {"taus": TAUS, "ran2": RAN2, "lf": LF, "lcg": LCG}
STATE_WORDS = {TAUS: 4, RAN2: 35, LCG: 1}
NOBS = 6
OBS_NAMES = ("x2", "v2", "xv", "x", "cxx", "cvv")


def build(force: bool = False) -> str:
    """Compile rngld_oracle.c into liboracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off", "-Wall",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB)
            u32, u64, i32, dbl, vp = C.c_uint32, C.c_uint64, C.c_int32, C.c_double, C.c_void_p
            sig = {
                "orc_splitmix64_mix": (u64, [u64]),
                "orc_seed_word": (u32, [u64, u64, u32]),
                "orc_lcg_next": (u32, [u32]),
                "orc_lcg_advance": (u32, [u32, u64]),
                "orc_lcg_period": (u64, [u32, u64]),
                "orc_lcg_seed": (None, [u64, u64, u64, vp]),
                "orc_taus_component": (u32, [u32, C.c_int]),
                "orc_taus_component_period": (u64, [u32, C.c_int, u64]),
                "orc_taus_seed": (None, [u64, u64, vp]),
                "orc_taus_lift": (None, [vp]),
                "orc_find_small_seed_word": (u64, [u64, u32, u32, u64, u64]),
                "orc_taus_next": (u32, [vp]),
                "orc_ran2_lcg1": (i32, [i32]),
                "orc_ran2_lcg2": (i32, [i32]),
                "orc_ran2_seed": (None, [u64, u64, vp]),
                "orc_ran2_next": (i32, [vp]),
                "orc_lf_seed": (None, [u64, u32, vp]),
                "orc_lf_generate": (C.c_int, [u32, u32, vp, u64, vp]),
                "orc_lf_seed_discard": (C.c_int, [u64, u32, u32, u64, vp]),
                "orc_trinomial_irreducible": (C.c_int, [u32, u32]),
                "orc_lfsr_period": (u64, [u32, u32, u64]),
                "orc_u_open": (dbl, [u32]),
                "orc_u_half": (dbl, [u32]),
                "orc_bm_radius": (dbl, [u32]),
                "orc_box_muller": (None, [u32, u32, vp, vp]),
                "orc_box_muller_many": (None, [vp, u64, vp]),
                "orc_uniform_streams": (C.c_int, [C.c_int, vp, u64, u64, vp]),
                "orc_gaussian_streams": (C.c_int, [C.c_int, vp, u64, u64, vp]),
                "orc_lf_gaussian": (C.c_int, [u32, u32, vp, u64, vp]),
                "orc_ld_run": (C.c_int, [C.c_int, vp, u32, u32, u64, u32, dbl, dbl, dbl, dbl, dbl, C.c_int,
                                          vp, vp, u32, u32, vp]),
                "orc_ld_forces": (C.c_int, [C.c_int, vp, u32, u32, u64, u32, vp]),
                "orc_ld_run_lf_sampled": (C.c_int, [u32, u32, vp, u64, u32, dbl, dbl, dbl, dbl, dbl, C.c_int, vp,
                                                     u64, vp, vp]),
                "orc_ld_adjoint": (C.c_int, [C.c_int, vp, u64, u32, dbl, dbl, dbl, dbl, dbl, vp, vp, u32, u32,
                                              vp, vp]),
                "orc_ld_adjoint_coef": (C.c_int, [C.c_int, vp, u64, u32, vp, vp, vp, vp, u32, u32, vp, vp]),
                "orc_ld_loss": (C.c_int, [C.c_int, vp, u64, u32, dbl, dbl, dbl, dbl, dbl, vp, vp, u32, u32, vp]),
            }
            for name, (res, args) in sig.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def _kind(kind) -> int:
    return KIND_NAMES[kind] if isinstance(kind, str) else int(kind)


# ---------------------------------------------------------------------------------------------
# scalar helpers

def splitmix64_mix(z: int) -> int:
    return int(lib().orc_splitmix64_mix(z & (2**64 - 1)))


def seed_word(seed: int, stream: int, i: int) -> int:
    return int(lib().orc_seed_word(seed, stream, i))


def lcg_next(x: int) -> int:
    return int(lib().orc_lcg_next(x))


def lcg_advance(x: int, n: int) -> int:
    return int(lib().orc_lcg_advance(x, n))


def lcg_period(x0: int, limit: int) -> int:
    return int(lib().orc_lcg_period(x0, limit))


def taus_component(z: int, which: int) -> int:
    return int(lib().orc_taus_component(z, which))


def taus_component_period(z0: int, which: int, limit: int) -> int:
    return int(lib().orc_taus_component_period(z0, which, limit))


def ran2_lcg1(x: int) -> int:
    return int(lib().orc_ran2_lcg1(x))


def ran2_lcg2(x: int) -> int:
    return int(lib().orc_ran2_lcg2(x))


def trinomial_irreducible(ll: int, sl: int) -> bool:
    r = lib().orc_trinomial_irreducible(ll, sl)
    if r < 0:
        raise ValueError("bad trinomial (%d, %d)" % (ll, sl))
    return bool(r)


def lfsr_period(ll: int, sl: int, limit: int) -> int:
    return int(lib().orc_lfsr_period(ll, sl, limit))


def u_open(w: int) -> float:
    return float(lib().orc_u_open(w))


def u_half(w: int) -> float:
    return float(lib().orc_u_half(w))


def bm_radius(w: int) -> float:
    return float(lib().orc_bm_radius(w))


def box_muller(w0: int, w1: int):
    g0, g1 = C.c_double(), C.c_double()
    lib().orc_box_muller(w0, w1, C.byref(g0), C.byref(g1))
    return g0.value, g1.value


def box_muller_many(words: np.ndarray) -> np.ndarray:
    """Box-Muller pairs of consecutive words, FP64."""
    words = np.ascontiguousarray(words, dtype=np.uint32)
    out = np.zeros(max(words.size, 1))
    lib().orc_box_muller_many(_p(words), words.size // 2, _p(out))
    return out[:words.size]


# ---------------------------------------------------------------------------------------------
# generator states

def taus_seed(seed: int, streams) -> np.ndarray:
    """[S, 4] uint32 Hybrid Taus states for the given global stream indices."""
    streams = np.atleast_1d(np.asarray(streams, dtype=np.uint64))
    st = np.zeros((len(streams), 4), dtype=np.uint32)
    L = lib()
    for n, j in enumerate(streams):
        L.orc_taus_seed(seed, int(j), _p(st[n]))
    return st


def lcg_seed(seed: int, streams, leap: int = 0) -> np.ndarray:
    """[S, 1] uint32 per-stream LCG states (leap 0: independent seed words; leap > 0: stream j is
    the stream-0 seed word advanced j * leap steps)."""
    streams = np.atleast_1d(np.asarray(streams, dtype=np.uint64))
    st = np.zeros((len(streams), 1), dtype=np.uint32)
    L = lib()
    for n, j in enumerate(streams):
        L.orc_lcg_seed(seed, int(j), leap, _p(st[n]))
    return st


def ran2_seed(seed: int, streams) -> np.ndarray:
    """[S, 35] int32 Ran2 states (idum, idum2, iy, iv[32])."""
    streams = np.atleast_1d(np.asarray(streams, dtype=np.uint64))
    st = np.zeros((len(streams), 35), dtype=np.int32)
    L = lib()
    for n, j in enumerate(streams):
        L.orc_ran2_seed(seed, int(j), _p(st[n]))
    return st


def taus_lift(words) -> np.ndarray:
    z = np.array(words, dtype=np.uint32)
    lib().orc_taus_lift(_p(z))
    return z


def find_small_seed_word(seed: int, i: int, floor_val: int, start: int = 0, limit: int = 2**40) -> int:
    return int(lib().orc_find_small_seed_word(seed, i, floor_val, start, limit))


def seed_states(kind, seed: int, streams, leap: int = 0) -> np.ndarray:
    kind = _kind(kind)
    if kind == LCG:
        return lcg_seed(seed, streams, leap)
    return taus_seed(seed, streams) if kind == TAUS else ran2_seed(seed, streams)


def lf_seed(seed: int, ll: int, sl: int = 0, discard: int = 0) -> np.ndarray:
    """Window [ll] uint32: y_{-ll} .. y_{-1}; with a discard D (needs sl), the window after the
    first D values of the sequence are generated and dropped: y_{D-ll} .. y_{D-1}."""
    win = np.zeros(ll, dtype=np.uint32)
    if discard:
        rc = lib().orc_lf_seed_discard(seed, ll, sl, discard, _p(win))
        if rc:
            raise RuntimeError("orc_lf_seed_discard failed: %d" % rc)
    else:
        lib().orc_lf_seed(seed, ll, _p(win))
    return win


def lf_generate(ll: int, sl: int, win: np.ndarray, count: int, keep: bool = True):
    """Next `count` values of the sequence; `win` is advanced in place. Returns the values."""
    out = np.zeros(max(count, 1), dtype=np.uint32) if keep else None
    rc = lib().orc_lf_generate(ll, sl, _p(win), count, _p(out) if keep else None)
    if rc:
        raise RuntimeError("orc_lf_generate failed: %d" % rc)
    return out[:count] if keep else None


def uniform_streams(kind, states: np.ndarray, per_stream: int) -> np.ndarray:
    """[per_stream, S] uint32 (Ran2: iy); `states` advanced in place."""
    kind = _kind(kind)
    S = states.shape[0]
    out = np.zeros((per_stream, S), dtype=np.uint32)
    rc = lib().orc_uniform_streams(kind, _p(states), S, per_stream, _p(out))
    if rc:
        raise RuntimeError("orc_uniform_streams failed: %d" % rc)
    return out


def gaussian_streams(kind, states: np.ndarray, per_stream: int) -> np.ndarray:
    kind = _kind(kind)
    S = states.shape[0]
    out = np.zeros((per_stream, S), dtype=np.float64)
    rc = lib().orc_gaussian_streams(kind, _p(states), S, per_stream, _p(out))
    if rc:
        raise RuntimeError("orc_gaussian_streams failed: %d" % rc)
    return out


def lf_gaussian(ll: int, sl: int, win: np.ndarray, count: int) -> np.ndarray:
    out = np.zeros(max(count, 1), dtype=np.float64)
    rc = lib().orc_lf_gaussian(ll, sl, _p(win), count, _p(out))
    if rc:
        raise RuntimeError("orc_lf_gaussian failed: %d" % rc)
    return out[:count]


# ---------------------------------------------------------------------------------------------
# Langevin dynamics

def _params(p):
    """p: dict or tuple (m, k, gamma, kT, dt) -- values are taken as given (float64)."""
    if isinstance(p, dict):
        return (float(p["m"]), float(p["k"]), float(p["gamma"]), float(p["kT"]), float(p["dt"]))
    return tuple(float(a) for a in p)


def ld_run(kind, states: np.ndarray, N: int, n_steps: int, params, x=None, v=None, stride: int = 0,
           t0: int = 0, ll: int = 0, sl: int = 0, scheme: int = 0):
    """Run the FP64 reference.  Returns (x[3,N], v[3,N], obs[P,6] or None); states advance in place."""
    kind = _kind(kind)
    m, k, g, kT, dt = _params(params)
    x = np.zeros((3, N)) if x is None else np.array(x, dtype=np.float64, order="C", copy=True)
    v = np.zeros((3, N)) if v is None else np.array(v, dtype=np.float64, order="C", copy=True)
    P = (n_steps // stride + 1) if stride else 0
    obs = np.zeros((max(P, 1), NOBS))
    rc = lib().orc_ld_run(kind, _p(states), ll, sl, N, n_steps, m, k, g, kT, dt, scheme, _p(x), _p(v),
                          stride, t0, _p(obs) if P else None)
    if rc:
        raise RuntimeError("orc_ld_run failed: %d" % rc)
    return x, v, (obs[:P] if P else None)


def ld_run_lf_sampled(win: np.ndarray, ll: int, sl: int, N: int, n_steps: int, params, ids, scheme: int = 0):
    """The lagged-Fibonacci run of N oscillators from rest, following only oscillators `ids`
    (ascending): returns (x[3, n], v[3, n]) of those; `win` advances by 4 N n_steps positions."""
    m, k, g, kT, dt = _params(params)
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    n = ids.size
    x = np.zeros((3, max(n, 1)))
    v = np.zeros((3, max(n, 1)))
    rc = lib().orc_ld_run_lf_sampled(ll, sl, _p(win), N, n_steps, m, k, g, kT, dt, scheme, _p(ids), n, _p(x), _p(v))
    if rc:
        raise RuntimeError("orc_ld_run_lf_sampled failed: %d" % rc)
    return x[:, :n], v[:, :n]


def ld_forces(kind, states: np.ndarray, N: int, n_steps: int, ll: int = 0, sl: int = 0) -> np.ndarray:
    """[n_steps, 3, N] Gaussian forces in the order an LD run consumes them."""
    kind = _kind(kind)
    g = np.zeros((max(n_steps, 1), 3, N))
    rc = lib().orc_ld_forces(kind, _p(states), ll, sl, N, n_steps, _p(g))
    if rc:
        raise RuntimeError("orc_ld_forces failed: %d" % rc)
    return g[:n_steps]


def ld_adjoint(kind, states: np.ndarray, N: int, n_steps: int, params, t_begin: int, t_end: int, x0=None, v0=None,
               coef=None):
    """(L, [dL/dk, dL/dgamma, dL/dkT]) by the FP64 reverse sweep; states advance in place.
    coef: None (the step's coefficients and their partials follow from `params` in FP64), or
    8 numbers (c, kap, sig, h, dkap/dk, dc/dgamma, dsig/dgamma, dsig/dkT) used as given."""
    kind = _kind(kind)
    x0 = np.zeros((3, N)) if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    v0 = np.zeros((3, N)) if v0 is None else np.ascontiguousarray(v0, dtype=np.float64)
    loss = C.c_double()
    grad = np.zeros(3)
    if coef is not None:
        q = np.ascontiguousarray(coef, dtype=np.float64)
        assert q.shape == (8,)
        cq, dq = np.ascontiguousarray(q[:4]), np.ascontiguousarray(q[4:])
        rc = lib().orc_ld_adjoint_coef(kind, _p(states), N, n_steps, _p(cq), _p(dq), _p(x0), _p(v0), t_begin, t_end,
                                       C.byref(loss), _p(grad))
        if rc:
            raise RuntimeError("orc_ld_adjoint_coef failed: %d" % rc)
        return loss.value, grad
    m, k, g, kT, dt = _params(params)
    rc = lib().orc_ld_adjoint(kind, _p(states), N, n_steps, m, k, g, kT, dt, _p(x0), _p(v0), t_begin, t_end,
                              C.byref(loss), _p(grad))
    if rc:
        raise RuntimeError("orc_ld_adjoint failed: %d" % rc)
    return loss.value, grad


def ld_loss(kind, states: np.ndarray, N: int, n_steps: int, params, t_begin: int, t_end: int, x0=None, v0=None):
    kind = _kind(kind)
    m, k, g, kT, dt = _params(params)
    x0 = np.zeros((3, N)) if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    v0 = np.zeros((3, N)) if v0 is None else np.ascontiguousarray(v0, dtype=np.float64)
    loss = C.c_double()
    rc = lib().orc_ld_loss(kind, _p(states), N, n_steps, m, k, g, kT, dt, _p(x0), _p(v0), t_begin, t_end,
                           C.byref(loss))
    if rc:
        raise RuntimeError("orc_ld_loss failed: %d" % rc)
    return loss.value


# ---------------------------------------------------------------------------------------------
# the adjoint over many oscillators on several processes

def _adjoint_slice(args):
    kind, seed, lo, hi, n_steps, params, t_begin, t_end, coef = args
    L, g = ld_adjoint(kind, seed_states(kind, seed, np.arange(lo, hi)), hi - lo, n_steps, params, t_begin, t_end,
                      coef=coef)
    return hi - lo, L, g


def ld_adjoint_split(kind, seed: int, N: int, n_steps: int, params, t_begin: int, t_end: int, workers: int = 0,
                     coef=None):
    """ld_adjoint of oscillators 0..N-1 of `seed` from rest, the oscillators split into contiguous
    slices run by separate processes.  Every oscillator has its own stream and the loss and its
    gradient are means over oscillators, so the split changes only the order of the final sum:
    the result is the size-weighted mean of the slices' results.  workers = 0: one per available
    core, at most 16."""
    import concurrent.futures as cf
    import multiprocessing as mp

    if workers <= 0:
        try:
            workers = len(os.sched_getaffinity(0))
        except AttributeError:
            workers = os.cpu_count() or 1
        workers = max(1, min(workers, 16))
    bounds = np.linspace(0, N, workers + 1).astype(np.int64)
    coef = None if coef is None else [float(c) for c in coef]
    jobs = [(kind, seed, int(bounds[i]), int(bounds[i + 1]), n_steps, params, t_begin, t_end, coef)
            for i in range(workers) if bounds[i + 1] > bounds[i]]
    build()
    # an executor (not a pool) so that a worker that dies raises instead of being replaced
    with cf.ProcessPoolExecutor(max_workers=len(jobs), mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_adjoint_slice, jobs))
    L = sum(n * Lp for n, Lp, _ in parts) / N
    g = sum(n * gp for n, _, gp in parts) / N
    return L, g
