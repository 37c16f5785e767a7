"""GPU parity of the fused RNG + Langevin-dynamics path against the CPU oracle (C ABI path).

Trajectory tolerance (1e-4 relative after 1000 steps, made well defined at zero crossings):
|x_gpu - x_ref| <= 1e-4 (|x_ref| + sqrt(kT/k)) per element, and the same for v with sqrt(kT/m).
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as orc
from oracle import moments as mom
from paper_1003_1123_amd import workloads as W

pytestmark = pytest.mark.gpu
R = pytest.importorskip("paper_1003_1123_amd._lib")

REL = 1e-4


def _say(*a):
    print("[gpu-ld]", *a, flush=True)
    sys.stdout.flush()


def _close(gpu, ref, scale):
    err = np.abs(gpu.astype(np.float64) - ref)
    bound = REL * (np.abs(ref) + scale)
    return bool(np.all(err <= bound)), float(np.max(err / bound))


def _params(p: W.LDParams, scheme=0):
    return R.make_params(p.m, p.k, p.gamma, p.kT, p.dt, scheme)


def _lf_lags(n):
    return W.lf_lags_for(4 * n)


def _setup(kind, N, seed=1234, n_total=None, ll=0, sl=0, x0=None, v0=None, leap=0):
    n_total = N if n_total is None else n_total
    cfg = R.make_cfg(kind, seed=seed, n_streams=n_total, ll=ll, sl=sl, leap=leap)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    x = torch.zeros(3 * n_total, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(x)
    if x0 is not None:
        x.copy_(torch.as_tensor(x0.reshape(-1)))
        v.copy_(torch.as_tensor(v0.reshape(-1)))
    return cfg, st, x, v


def _lf_state(st):
    """The meaningful part of a lagged-Fibonacci state: the header's position and the last ll
    values in sequence order (the rest of the ring is stale by definition)."""
    b = st.cpu().numpy()
    pos = int(b[:8].view(np.uint64)[0])
    slot, ll, sl, R = (int(v) for v in b[8:24].view(np.uint32))
    ring = b[64:64 + 4 * R].view(np.uint32)
    return pos, slot, ring[(slot - ll + np.arange(ll)) % R]


def _same_state(kind, a, b):
    """Generator states equal: every byte for per-thread kinds, the position and the last ll values
    for the lagged Fibonacci ring; the no-noise kind has none."""
    if kind == "none":
        return True
    if kind != "lf":
        return torch.equal(a, b)
    sa, sb = _lf_state(a), _lf_state(b)
    return sa[0] == sb[0] and np.array_equal(sa[2], sb[2])


def _oracle_states(kind, seed, ids, ll=0):
    return orc.lf_seed(seed, ll) if kind == "lf" else orc.seed_states(kind, seed, ids)


# ---------------------------------------------------------------------------------------------
# config 1: N = 1e4, 1000 steps, observables every 10 steps, C_xx from t0 = 500

@pytest.mark.parametrize("kind", ["taus", "ran2", "lf", "lcg"])
def test_config1_trajectory_and_observables(kind):
    N, T, stride, t0 = W.C1["N"], W.C1["steps"], W.C1["stride"], W.C1["t0"]
    p = W.C1["params"].as_f32()
    ll, sl = _lf_lags(N) if kind == "lf" else (0, 0)
    _say("config1", kind, N, T, ll, sl)
    cfg, st, x, v = _setup(kind, N, ll=ll, sl=sl)
    ens, n_ens = R.make_ensembles([(0, N, _params(p), 0)])
    obs = R.Obs(stride, t0)
    P = T // stride + 1
    out_obs = torch.zeros(P * R.NOBS, dtype=torch.float64, device="cuda")
    R.ld_run(cfg, st, ens, n_ens, N, T, x, v, obs, out_obs)
    torch.cuda.synchronize()
    xr, vr, obr = orc.ld_run(kind, _oracle_states(kind, 1234, np.arange(N), ll), N, T, p.asdict(), stride=stride,
                             t0=t0, ll=ll, sl=sl)
    okx, wx = _close(x.cpu().numpy().reshape(3, N), xr, math.sqrt(p.kT / p.k))
    okv, wv = _close(v.cpu().numpy().reshape(3, N), vr, math.sqrt(p.kT / p.m))
    _say(kind, "worst x/v error relative to bound", wx, wv)
    assert okx and okv
    g_obs = out_obs.cpu().numpy().reshape(P, R.NOBS)
    scale = np.array([p.kT / p.k, p.kT / p.m, math.sqrt(p.kT / p.k * p.kT / p.m), math.sqrt(p.kT / p.k),
                      p.kT / p.k, p.kT / p.m])
    assert np.all(np.abs(g_obs - obr) <= 2 * REL * (np.abs(obr) + scale)), np.max(np.abs(g_obs - obr))
    # statistics of the GPU run against the exact discrete moments
    steps = np.arange(0, T + 1, stride)
    ex2, ev2, _, _ = mom.second_moments(p.m, p.k, p.gamma, p.kT, p.dt, T)
    ok = steps > 0
    z = np.abs(g_obs[ok, 0] - ex2[steps][ok]) / (ex2[steps][ok] * math.sqrt(2.0 / (3 * N)))
    assert np.max(z) < 4.5
    after = steps >= t0
    cxx, _ = mom.cross_moments(p.m, p.k, p.gamma, p.kT, p.dt, t0, steps[after] - t0)
    se = np.sqrt((ex2[steps[after]] * ex2[t0] + cxx**2) / (3 * N))
    assert np.max(np.abs(g_obs[after, 4] - cxx) / se) < 4.5


# ---------------------------------------------------------------------------------------------
# config 2 at full size: N = 1e6, h = 0.005; sampled oscillators against the oracle

@pytest.mark.parametrize("kind", ["taus", "ran2"])
def test_config2_full_size_sampled(kind):
    N, T = W.C2["N"], W.C2["steps"]
    p = W.C2["params"].as_f32()
    _say("config2", kind, N, T)
    cfg, st, x, v = _setup(kind, N)
    ens, n_ens = R.make_ensembles([(0, N, _params(p), 0)])
    R.ld_run(cfg, st, ens, n_ens, N, T, x, v)
    torch.cuda.synchronize()
    ids = W.sampled_streams(N, 48)
    xr, vr, _ = orc.ld_run(kind, orc.seed_states(kind, 1234, ids), len(ids), T, p.asdict())
    idx = torch.as_tensor(ids, device="cuda")
    xg = x.view(3, N)[:, idx].cpu().numpy()
    vg = v.view(3, N)[:, idx].cpu().numpy()
    okx, wx = _close(xg, xr, math.sqrt(p.kT / p.k))
    okv, wv = _close(vg, vr, math.sqrt(p.kT / p.m))
    _say(kind, "worst", wx, wv)
    assert okx and okv
    # equipartition over all 3e6 coordinates at the end (stationary after 50 time units)
    x2s, v2s, _ = mom.stationary_closed_form(p.m, p.k, p.gamma, p.kT, p.dt)
    xx = float((x.double() ** 2).mean())
    vv = float((v.double() ** 2).mean())
    assert abs(xx - x2s) < 5 * x2s * math.sqrt(2 / (3 * N)) and abs(vv - v2s) < 5 * v2s * math.sqrt(2 / (3 * N))


def test_config2_lf_full_size_sampled():
    """LF at N = 1e6 with Table I's last row: 4e6 numbers per step in 4 dependent waves."""
    N, T = W.C2["N"], 100
    ll, sl = W.C2["lf_lags"]
    p = W.C2["params"].as_f32()
    _say("config2 lf", N, T)
    cfg, st, x, v = _setup("lf", N, ll=ll, sl=sl)
    ens, n_ens = R.make_ensembles([(0, N, _params(p), 0)])
    R.ld_run(cfg, st, ens, n_ens, N, T, x, v)
    torch.cuda.synchronize()
    ids = W.sampled_streams(N, 48)
    xo, vo, _ = orc.ld_run("lf", orc.lf_seed(1234, ll), N, T, p.asdict(), ll=ll, sl=sl)
    xr, vr = xo[:, ids], vo[:, ids]
    idx = torch.as_tensor(ids, device="cuda")
    okx, wx = _close(x.view(3, N)[:, idx].cpu().numpy(), xr, math.sqrt(p.kT / p.k))
    okv, wv = _close(v.view(3, N)[:, idx].cpu().numpy(), vr, math.sqrt(p.kT / p.m))
    _say("lf worst", wx, wv)
    assert okx and okv


def test_config2_lf_sampled_after_1000_steps():
    """LF at config-2 size (N = 1e6, Table I's last row) for 1000 steps on the persistent path: 48
    sampled oscillators against the oracle, which generates all 4e9 numbers of the one sequence in
    order and integrates only the sampled oscillators, element by element."""
    N, T = W.C2["N"], 1000
    ll, sl = W.C2["lf_lags"]
    p = W.C2["params"].as_f32()
    _say("config2 lf sampled", N, T)
    cfg, st, x, v = _setup("lf", N, ll=ll, sl=sl)
    ens, n_ens = R.make_ensembles([(0, N, _params(p), 0)])
    ws = R.ld_run(cfg, st, ens, n_ens, N, T, x, v)
    assert R.ws_status(ws) == 0 and R.ws_lf_path(ws) == "dataflow"
    ids = W.sampled_streams(N, 48)
    win = orc.lf_seed(1234, ll)
    xr, vr = orc.ld_run_lf_sampled(win, ll, sl, N, T, p.asdict(), ids)
    idx = torch.as_tensor(ids, device="cuda")
    okx, wx = _close(x.view(3, N)[:, idx].cpu().numpy(), xr, math.sqrt(p.kT / p.k))
    okv, wv = _close(v.view(3, N)[:, idx].cpu().numpy(), vr, math.sqrt(p.kT / p.m))
    _say("lf sampled worst", wx, wv)
    assert okx and okv
    pos, _, last = _lf_state(st)
    assert pos == 4 * N * T and np.array_equal(last, win)


def test_config2_lf_full_run_statistics():
    """The whole config-2 LF run (N = 1e6, 1e4 steps, Table I's last row, the persistent path):
    completes without a failed wait, equals the wave path (one launch per wave of sl positions,
    pinned to the oracle elsewhere) bit for bit in x, v and the sequence's last ll values, and
    equipartition holds over all 3e6 coordinates at the end, as for the per-thread generators."""
    N, T = W.C2["N"], W.C2["steps"]
    ll, sl = W.C2["lf_lags"]
    p = W.C2["params"].as_f32()
    _say("config2 lf full run", N, T)
    cfg, st, x, v = _setup("lf", N, ll=ll, sl=sl)
    ens, n_ens = R.make_ensembles([(0, N, _params(p), 0)])
    ws = R.ld_run(cfg, st, ens, n_ens, N, T, x, v)
    assert R.ws_status(ws) == 0 and R.ws_lf_path(ws) == "dataflow"
    assert _lf_state(st)[0] == 4 * N * T
    x2s, v2s, _ = mom.stationary_closed_form(p.m, p.k, p.gamma, p.kT, p.dt)
    xx = float((x.double() ** 2).mean())
    vv = float((v.double() ** 2).mean())
    _say("lf equipartition", xx / x2s, vv / v2s)
    assert abs(xx - x2s) < 5 * x2s * math.sqrt(2 / (3 * N)) and abs(vv - v2s) < 5 * v2s * math.sqrt(2 / (3 * N))
    _say("config2 lf full run, wave path")
    cfg_w, st_w, xw, vw = _setup("lf", N, ll=ll, sl=sl)
    saved = R.ld_get_tuning("lf").astuple()
    R.ld_set_tuning("lf", lf_waves=1)
    try:
        ws_w = R.ld_run(cfg_w, st_w, ens, n_ens, N, T, xw, vw)
        assert R.ws_lf_path(ws_w) == "waves"
    finally:
        R.ld_set_tuning("lf", *saved)
    assert torch.equal(x, xw) and torch.equal(v, vw)
    assert _same_state("lf", st, st_w)


# ---------------------------------------------------------------------------------------------
# protocol equivalences

@pytest.mark.parametrize("kind", ["taus", "ran2", "lf", "lcg"])
def test_resume_is_bit_exact(kind):
    N = 3001
    ll, sl = _lf_lags(N) if kind == "lf" else (0, 0)
    p = _params(W.LDParams(k=1.3, gamma=0.7, kT=0.9, dt=0.01))
    ens, n_ens = R.make_ensembles([(0, N, p, 0)])
    cfg_a, st_a, xa, va = _setup(kind, N, ll=ll, sl=sl)
    cfg_b, st_b, xb, vb = _setup(kind, N, ll=ll, sl=sl)
    R.ld_run(cfg_a, st_a, ens, n_ens, N, 200, xa, va)
    R.ld_run(cfg_b, st_b, ens, n_ens, N, 77, xb, vb)
    R.ld_run(cfg_b, st_b, ens, n_ens, N, 123, xb, vb)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb) and torch.equal(va, vb) and _same_state(kind, st_a, st_b)


@pytest.mark.parametrize("kind", ["taus", "ran2", "lf", "lcg"])
def test_step_protocol_matches_oracle_and_fused_run(kind):
    """ld_step (one launch per step, state through device memory: the paper's protocol)."""
    N, T = 1000, 300
    ll, sl = _lf_lags(N) if kind == "lf" else (0, 0)
    pp = W.LDParams(k=0.8, gamma=1.5, kT=1.2, dt=0.01).as_f32()
    p = _params(pp)
    cfg_s, st_s, xs, vs = _setup(kind, N, ll=ll, sl=sl)
    for _ in range(T):
        R.ld_step(cfg_s, st_s, p, N, xs, vs)
    cfg_r, st_r, xr_, vr_ = _setup(kind, N, ll=ll, sl=sl)
    ens, n_ens = R.make_ensembles([(0, N, p, 0)])
    R.ld_run(cfg_r, st_r, ens, n_ens, N, T, xr_, vr_)
    torch.cuda.synchronize()
    assert _same_state(kind, st_s, st_r)  # identical generator state
    xo, vo, _ = orc.ld_run(kind, _oracle_states(kind, 1234, np.arange(N), ll), N, T, pp.asdict(), ll=ll, sl=sl)
    assert _close(xs.cpu().numpy().reshape(3, N), xo, math.sqrt(pp.kT / pp.k))[0]
    assert _close(vs.cpu().numpy().reshape(3, N), vo, math.sqrt(pp.kT / pp.m))[0]
    d = float((xs - xr_).abs().max())
    _say(kind, "step vs fused max |dx|", d)
    assert d <= 1e-5


@pytest.mark.parametrize("kind", ["taus", "ran2", "lcg"])
def test_batched_equals_plain_bit_exact(kind):
    ens_list = W.batched_ensembles(n_ens=12, n_lo=1, n_hi=3000)
    offs = np.concatenate([[0], np.cumsum([e.n for e in ens_list])])
    n_total = int(offs[-1])
    T, stride, t0 = 150, 10, 50
    specs = [(int(offs[i]), e.n, _params(e.params), e.seed) for i, e in enumerate(ens_list)]
    ens, n_ens = R.make_ensembles(specs)
    cfg = R.make_cfg(kind, n_streams=n_total)
    st = R.new_state(cfg)
    R.rng_init_ensembles(cfg, st, ens, n_ens)
    x = torch.zeros(3 * n_total, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(x)
    P = T // stride + 1
    ob = torch.zeros(n_ens * P * R.NOBS, dtype=torch.float64, device="cuda")
    R.ld_run(cfg, st, ens, n_ens, n_total, T, x, v, R.Obs(stride, t0), ob)
    torch.cuda.synchronize()
    obb = ob.cpu().numpy().reshape(n_ens, P, R.NOBS)
    for i, e in enumerate(ens_list):
        c1, s1, x1, v1 = _setup(kind, e.n, seed=e.seed)
        e1, n1 = R.make_ensembles([(0, e.n, _params(e.params), 0)])
        o1 = torch.zeros(P * R.NOBS, dtype=torch.float64, device="cuda")
        R.ld_run(c1, s1, e1, n1, e.n, T, x1, v1, R.Obs(stride, t0), o1)
        torch.cuda.synchronize()
        sl_ = slice(int(offs[i]), int(offs[i + 1]))
        assert torch.equal(x.view(3, n_total)[:, sl_], x1.view(3, e.n)), i
        assert torch.equal(v.view(3, n_total)[:, sl_], v1.view(3, e.n)), i
        assert np.array_equal(obb[i], o1.cpu().numpy().reshape(P, R.NOBS)), i


def test_config4_ensemble_statistics():
    """Config 4 at full size (512 ensembles, 76.7e6 oscillators, 5000 steps from rest, one batched
    run): each ensemble's <x^2> and <v^2> after the run against the exact discrete second moments
    of its own (k, gamma, kT, h), cov_n = S - A^n S (A^n)^T with S the stationary covariance
    (A S A^T + B B^T = S).  x and v are Gaussian with mean 0, so the estimate over 3 n_e coordinates
    has standard error var sqrt(2 / (3 n_e)); across the ensembles the z-scores must look N(0, 1)."""
    from scipy.linalg import solve_discrete_lyapunov

    c4 = W.C4
    ens_list = W.batched_ensembles(c4["n_ens"], c4["draw_seed"], c4["base_seed"], c4["dt"])
    offs = np.concatenate([[0], np.cumsum([e.n for e in ens_list])])
    n_total, T = int(offs[-1]), c4["steps"]
    specs = [(int(offs[i]), e.n, _params(e.params), e.seed) for i, e in enumerate(ens_list)]
    ens, n_ens = R.make_ensembles(specs)
    cfg = R.make_cfg("taus", n_streams=n_total)
    st = R.new_state(cfg)
    R.rng_init_ensembles(cfg, st, ens, n_ens)
    x = torch.zeros(3 * n_total, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(x)
    ob = torch.zeros(n_ens * 2 * R.NOBS, dtype=torch.float64, device="cuda")
    _say("config 4 statistics", n_ens, n_total, T)
    R.ld_run(cfg, st, ens, n_ens, n_total, T, x, v, R.Obs(T, 0), ob)
    torch.cuda.synchronize()
    del x, v, st
    o = ob.cpu().numpy().reshape(n_ens, 2, R.NOBS)[:, 1]
    z = []
    for i, e in enumerate(ens_list):
        p = e.params
        A, B = mom.scheme_matrices(p.m, p.k, p.gamma, p.kT, p.dt)
        S = solve_discrete_lyapunov(A, B @ B.T)
        An = np.linalg.matrix_power(A, T)
        cov = S - An @ S @ An.T
        for j, var in ((0, cov[0, 0]), (1, cov[1, 1])):
            se = var * math.sqrt(2.0 / (3 * e.n))
            z.append((o[i, j] - var) / se)
    z = np.array(z)
    _say("config 4 z: mean %.3f var %.3f max %.2f" % (z.mean(), z.var(), np.abs(z).max()))
    assert abs(z.mean()) < 0.25 and 0.7 < z.var() < 1.4 and np.abs(z).max() < 5.0


def test_autotune_chooses_installs_caches_and_keeps_results(tmp_path):
    """ld_autotune on a batched workload of uneven ensembles: the chosen tuning is valid and
    installed, it is written to the cache file and read back from it (a second call measures
    nothing and leaves the file alone; an entry edited in the file is what a third call installs),
    a run under it equals the default tuning bit for bit in x, v and the generator state, and it
    matches the oracle on sampled ensembles."""
    ens_list = W.batched_ensembles(n_ens=24, n_lo=300, n_hi=40_000)
    offs = np.concatenate([[0], np.cumsum([e.n for e in ens_list])])
    n_total, T = int(offs[-1]), 3000
    specs = [(int(offs[i]), e.n, _params(e.params), e.seed) for i, e in enumerate(ens_list)]
    ens, n_ens = R.make_ensembles(specs)
    cfg = R.make_cfg("taus", n_streams=n_total)
    cache = tmp_path / "tune.txt"
    default = R.ld_get_tuning("taus").astuple()
    try:
        t = R.ld_autotune(cfg, ens, n_ens, n_total, T, str(cache)).astuple()
        _say("autotune", n_total, T, "->", t)
        assert t[0] in (64, 128, 256, 512) and t[1] in (1, 2) and t[2] in (0, 500, 1000, 2500) and t[3] in (0, 4, 8)
        assert t[4] == 0
        assert R.ld_get_tuning("taus").astuple() == t
        lines = cache.read_text().splitlines()
        assert len(lines) == 1 and lines[0].split()[-4:] == [str(a) for a in t[:4]]
        before = cache.stat().st_mtime_ns, cache.read_text()
        R.ld_set_tuning("taus")
        assert R.ld_autotune(cfg, ens, n_ens, n_total, T, str(cache)).astuple() == t
        assert (cache.stat().st_mtime_ns, cache.read_text()) == before
        edited = (128, 2, 500, 4, 0) if t[:4] != (128, 2, 500, 4) else (256, 1, 0, 0, 0)
        cache.write_text(" ".join(lines[0].split()[:-4] + [str(a) for a in edited[:4]]) + "\n")
        assert R.ld_autotune(cfg, ens, n_ens, n_total, T, str(cache)).astuple() == edited
        assert R.ld_get_tuning("taus").astuple() == edited
        # a run under the chosen tuning against the default tuning and the oracle
        runs = []
        for tune in (t, default):
            R.ld_set_tuning("taus", *tune)
            st = R.new_state(cfg)
            R.rng_init_ensembles(cfg, st, ens, n_ens)
            x = torch.zeros(3 * n_total, dtype=torch.float32, device="cuda")
            v = torch.zeros_like(x)
            R.ld_run(cfg, st, ens, n_ens, n_total, 1000, x, v)
            torch.cuda.synchronize()
            runs.append((x, v, st))
        assert all(torch.equal(a, b) for a, b in zip(runs[0], runs[1]))
        x = runs[0][0].view(3, n_total)
        for i in (0, 7, n_ens - 1):
            e = ens_list[i]
            ids = np.arange(0, e.n, max(1, e.n // 64))
            xr, _, _ = orc.ld_run("taus", orc.seed_states("taus", e.seed, ids), len(ids), 1000, e.params.asdict())
            xg = x[:, int(offs[i]) + torch.as_tensor(ids, device="cuda")].cpu().numpy()
            ok, worst = _close(xg, xr, math.sqrt(e.params.kT / e.params.k))
            _say("autotuned ensemble", i, "worst", worst)
            assert ok
    finally:
        R.ld_set_tuning("taus", *default)


@pytest.mark.parametrize("tuning", [(64, 1, 0, 0), (128, 2, 0, 0), (256, 1, 37, 0), (512, 2, 0, 4), (256, 2, 100, 2)])
def test_tunings_give_identical_trajectories(tuning):
    """Launch shape changes neither the trajectory nor the generator state (observables may differ
    in the last bits because the reduction tree depends on the tile)."""
    N, T = 5000, 120
    p = _params(W.LDParams())
    ens, n_ens = R.make_ensembles([(0, N, p, 0)])
    R.ld_set_tuning("taus")
    c0, s0, x0, v0 = _setup("taus", N)
    R.ld_run(c0, s0, ens, n_ens, N, T, x0, v0)
    R.ld_set_tuning("taus", *tuning)
    try:
        c1, s1, x1, v1 = _setup("taus", N)
        ob = torch.zeros((T // 10 + 1) * R.NOBS, dtype=torch.float64, device="cuda")
        R.ld_run(c1, s1, ens, n_ens, N, T, x1, v1, R.Obs(10, 60), ob)
        torch.cuda.synchronize()
    finally:
        R.ld_set_tuning("taus")
    assert torch.equal(x0, x1) and torch.equal(v0, v1) and torch.equal(s0, s1)


@pytest.mark.parametrize("kind", ["taus", "ran2", "lf", "lcg", "none"])
def test_graph_plan_replays_advance_the_run(kind):
    """A captured plan (hipGraph) replayed three times, with unrelated eager work between the
    replays, equals three eager runs: trajectory and generator state."""
    N, T = 7000, 50
    p = _params(W.LDParams())
    ens, n_ens = R.make_ensembles([(0, N, p, 0)])
    ll, sl = _lf_lags(N) if kind == "lf" else (0, 0)
    ca, sa, xa, va = _setup(kind, N, ll=ll, sl=sl)
    cb, sb, xb, vb = _setup(kind, N, ll=ll, sl=sl)
    plan = R.Plan(cb, sb, ens, n_ens, N, T, xb, vb)
    for rep in range(3):
        R.ld_run(ca, sa, ens, n_ens, N, T, xa, va)
        plan.launch()
        torch.cuda.synchronize()
        _ = (xa * 2).sum().item()  # unrelated eager work between replays
        assert torch.equal(xa, xb) and torch.equal(va, vb) and _same_state(kind, sa, sb), rep
    plan.close()


def _run_chunks(chunks, kind, specs, n_total, T, obs, xi, vi):
    """One run with RNGLD_LD_CHUNKS set to `chunks` ("0": one tile per block for the whole run);
    returns x, v, the generator state, the observables and the status word."""
    import os
    ens, n_ens = R.make_ensembles(specs)
    cfg = R.make_cfg(kind, n_streams=n_total)
    st = R.new_state(cfg)
    R.rng_init_ensembles(cfg, st, ens, n_ens)
    x = torch.as_tensor(xi).cuda()
    v = torch.as_tensor(vi).cuda()
    out = torch.zeros(n_ens * (T // obs.stride + 1) * R.NOBS, dtype=torch.float64, device="cuda")
    old = os.environ.get("RNGLD_LD_CHUNKS")
    os.environ["RNGLD_LD_CHUNKS"] = chunks
    try:
        ws = R.ld_run(cfg, st, ens, n_ens, n_total, T, x, v, obs, out)
    finally:
        if old is None:
            del os.environ["RNGLD_LD_CHUNKS"]
        else:
            os.environ["RNGLD_LD_CHUNKS"] = old
    return x, v, st, out, R.ws_status(ws)


@pytest.mark.skip(reason="the chunked schedule was taken out of the library: its first run at full size (config 2, "
                         "Hybrid Taus, 1e6 oscillators) did not finish within the test time limit and the cause was "
                         "not found; RNGLD_LD_CHUNKS has no effect")
@pytest.mark.parametrize("kind", ["taus", "ran2", "lcg"])
def test_chunked_schedule_equals_whole_run_tiles(kind):
    """The chunked schedule (blocks take (tile, chunk) units in order; a chunk waits for the tile's
    previous one and takes its state from device memory) against one block per tile for the whole
    run, bit for bit in x, v, the generator state and the observables: three uneven ensembles
    (ragged last tiles, tiles of different ensembles next to each other), 250 steps in chunks of
    84, 84 and 82, x(t0) taken inside the second chunk; also 7 chunks and one step per chunk's
    worth of short chunks (50)."""
    sizes = (70_001, 129_999, 33_333)
    n_total, T, obs = sum(sizes), 250, R.Obs(10, 100)
    rng = np.random.default_rng(8)
    xi = rng.standard_normal(3 * n_total).astype(np.float32)
    vi = rng.standard_normal(3 * n_total).astype(np.float32)
    specs, off = [], 0
    for e, n in enumerate(sizes):
        specs.append((off, n, R.make_params(1.0, 0.5 + e, 0.3 + e, 1.0 + 0.25 * e, 0.01), 1234 + e))
        off += n
    _say("chunked schedule", kind, sizes, T)
    ref = _run_chunks("0", kind, specs, n_total, T, obs, xi, vi)
    assert ref[4] == 0
    for chunks in ("3", "7", "50"):
        got = _run_chunks(chunks, kind, specs, n_total, T, obs, xi, vi)
        _say("chunks", chunks, "status", got[4])
        assert got[4] == 0
        for a, b in zip(ref[:4], got[:4]):
            assert torch.equal(a, b)


def _moments(x, v, n_total, lo, n, x0=None, v0=None):
    """The six observables of oscillators [lo, lo + n) from state vectors ([3][n_total] layout), in
    FP64: means over their 3n coordinates of x^2, v^2, x v, x, x x0, v v0."""
    xs = x.double().view(3, n_total)[:, lo:lo + n]
    vs = v.double().view(3, n_total)[:, lo:lo + n]
    m = [float((xs * xs).mean()), float((vs * vs).mean()), float((xs * vs).mean()), float(xs.mean())]
    if x0 is None:
        return m + [0.0, 0.0]
    x0s = x0.double().view(3, n_total)[:, lo:lo + n]
    v0s = v0.double().view(3, n_total)[:, lo:lo + n]
    return m + [float((xs * x0s).mean()), float((vs * v0s).mean())]


@pytest.mark.parametrize("kind", ["taus", "ran2", "lf"])
def test_observables_equal_the_moments_of_the_returned_state(kind):
    """The observables' reduction (per-tile partials, then the fixed-order sum over an ensemble's
    tiles) against the same means taken directly from the state the run returns: N = 300,000
    oscillators (a ragged last tile; more tiles than the final sum has threads, so each thread
    adds several), random initial x and v, observation points 0, 10, 20 with t0 = 10.  Point 0 is
    the initial state, point 20 the returned one, and its x(t0) terms come from a second run of the
    same stream stopped at step 10.  Only the order of the FP64 additions differs, so the two agree
    to about 1e-13."""
    N, T, stride, t0 = 300_000, 20, 10, 10
    rng = np.random.default_rng(5)
    xi = rng.standard_normal(3 * N).astype(np.float32)
    vi = rng.standard_normal(3 * N).astype(np.float32)
    p = W.C1["params"].as_f32()
    lags = dict(zip(("ll", "sl"), _lf_lags(N))) if kind == "lf" else {}
    ens, n_ens = R.make_ensembles([(0, N, _params(p), 0)])
    obs = R.Obs(stride, t0)
    _say("observables vs state moments", kind, N, T)
    cfg, st, x, v = _setup(kind, N, x0=xi, v0=vi, **lags)
    x_init, v_init = x.clone(), v.clone()
    out = torch.zeros(n_ens * (T // stride + 1) * R.NOBS, dtype=torch.float64, device="cuda")
    ws = R.ld_run(cfg, st, ens, n_ens, N, T, x, v, obs, out)
    assert R.ws_status(ws) == 0
    cfg_h, st_h, xh, vh = _setup(kind, N, x0=xi, v0=vi, **lags)
    R.ld_run(cfg_h, st_h, ens, n_ens, N, t0, xh, vh)
    o = out.cpu().numpy().reshape(T // stride + 1, R.NOBS)
    want0 = _moments(x_init, v_init, N, 0, N)
    want2 = _moments(x, v, N, 0, N, xh, vh)
    err = max(abs(o[0, q] - want0[q]) / max(abs(want0[q]), 1e-3) for q in range(R.NOBS))
    err = max(err, max(abs(o[2, q] - want2[q]) / max(abs(want2[q]), 1e-3) for q in range(R.NOBS)))
    _say("largest relative difference", err)
    assert err < 1e-11


def test_batched_observables_equal_the_moments_of_each_ensemble():
    """The same check for a batched run of three uneven Hybrid Taus ensembles (the final sum over
    each ensemble's own tiles, starting at its first tile): point 0 and the last point of each
    ensemble against the means over that ensemble's oscillators."""
    sizes = (70_001, 129_999, 100_000)
    n_total, T, stride = sum(sizes), 20, 20
    rng = np.random.default_rng(6)
    xi = rng.standard_normal(3 * n_total).astype(np.float32)
    vi = rng.standard_normal(3 * n_total).astype(np.float32)
    specs, off = [], 0
    for e, n in enumerate(sizes):
        specs.append((off, n, R.make_params(1.0, 0.5 + e, 0.3 + e, 1.0 + 0.25 * e, 0.01), 1234 + e))
        off += n
    ens, n_ens = R.make_ensembles(specs)
    cfg = R.make_cfg("taus", n_streams=n_total)
    st = R.new_state(cfg)
    R.rng_init_ensembles(cfg, st, ens, n_ens)
    x = torch.as_tensor(xi).cuda()
    v = torch.as_tensor(vi).cuda()
    x_init, v_init = x.clone(), v.clone()
    out = torch.zeros(n_ens * 2 * R.NOBS, dtype=torch.float64, device="cuda")
    _say("batched observables vs state moments", sizes, T)
    R.ld_run(cfg, st, ens, n_ens, n_total, T, x, v, R.Obs(stride, 0), out)
    o = out.cpu().numpy().reshape(n_ens, 2, R.NOBS)
    err = 0.0
    for e, (lo, n, _, _) in enumerate(specs):
        for pt, want in ((0, _moments(x_init, v_init, n_total, lo, n, x_init, v_init)),
                         (1, _moments(x, v, n_total, lo, n, x_init, v_init))):
            err = max(err, max(abs(o[e, pt, q] - want[q]) / max(abs(want[q]), 1e-3) for q in range(R.NOBS)))
    _say("largest relative difference", err)
    assert err < 1e-11


def test_edge_cases():
    p = _params(W.LDParams())
    # one oscillator
    cfg, st, x, v = _setup("taus", 1)
    ens, n_ens = R.make_ensembles([(0, 1, p, 0)])
    R.ld_run(cfg, st, ens, n_ens, 1, 10, x, v)
    xr, _, _ = orc.ld_run("taus", orc.taus_seed(1234, [0]), 1, 10, W.LDParams().as_f32().asdict())
    assert _close(x.cpu().numpy().reshape(3, 1), xr, 1.0)[0]
    # zero steps with observables records the initial state only
    ob = torch.full((R.NOBS,), -1.0, dtype=torch.float64, device="cuda")
    R.ld_run(cfg, st, ens, n_ens, 1, 0, x, v, R.Obs(5, 0), ob)
    xs = x.double()
    assert abs(float(ob[0]) - float((xs ** 2).mean())) < 1e-12
    # an empty ensemble inside a batch
    ens2, n2 = R.make_ensembles([(0, 0, p, 0), (0, 1, p, 0)])
    R.ld_run(cfg, st, ens2, n2, 1, 3, x, v)
    torch.cuda.synchronize()


def test_overdamped_scheme_matches_oracle():
    N, T = 2000, 400
    pp = W.LDParams(m=1.0, k=0.5, gamma=2.0, kT=1.0, dt=0.01).as_f32()
    p = _params(pp, scheme=1)
    rng = np.random.default_rng(0)
    x0 = (10.0 * np.ones((3, N))).astype(np.float32)
    v0 = np.zeros((3, N), np.float32)
    cfg, st, x, v = _setup("taus", N, x0=x0, v0=v0)
    ens, n_ens = R.make_ensembles([(0, N, p, 0)])
    R.ld_run(cfg, st, ens, n_ens, N, T, x, v)
    xr, _, _ = orc.ld_run("taus", orc.taus_seed(1234, np.arange(N)), N, T, pp.asdict(), x0, v0, scheme=1)
    assert _close(x.cpu().numpy().reshape(3, N), xr, math.sqrt(pp.kT / pp.k))[0]
    assert torch.equal(v, torch.zeros_like(v))
    del rng


# ---------------------------------------------------------------------------------------------
# dynamics without random numbers (Fig. 6): the no-noise kind

@pytest.mark.parametrize("scheme", [0, 1])
def test_no_noise_equals_zero_temperature_and_the_oracle(scheme):
    """The no-noise kind runs the deterministic part of the step alone: bit-identical to a Taus run
    with kT = 0 (whose random force is exactly zero), and equal to the FP64 noise-free oracle."""
    N, T, stride, t0 = 5003, 700, 10, 300
    pp = W.LDParams(m=1.3, k=0.8, gamma=0.6, kT=0.0, dt=0.01).as_f32()
    p = _params(pp, scheme)
    rng = np.random.default_rng(3)
    x0 = rng.normal(size=(3, N)).astype(np.float32)
    v0 = rng.normal(size=(3, N)).astype(np.float32)
    ens, n_ens = R.make_ensembles([(0, N, p, 0)])
    P = T // stride + 1
    out = {}
    for kind in ("none", "taus"):
        cfg, st, x, v = _setup(kind, N, x0=x0, v0=v0)
        ob = torch.zeros(P * R.NOBS, dtype=torch.float64, device="cuda")
        R.ld_run(cfg, st, ens, n_ens, N, T, x, v, R.Obs(stride, t0), ob)
        torch.cuda.synchronize()
        out[kind] = (x, v, ob)
    assert torch.equal(out["none"][0], out["taus"][0]) and torch.equal(out["none"][1], out["taus"][1])
    assert torch.equal(out["none"][2], out["taus"][2])
    xr, vr, obr = orc.ld_run("taus", orc.taus_seed(1, np.arange(N)), N, T, pp.asdict(), x0, v0, stride=stride,
                             t0=t0, scheme=scheme)
    assert _close(out["none"][0].cpu().numpy().reshape(3, N), xr, 1.0)[0]
    assert _close(out["none"][1].cpu().numpy().reshape(3, N), vr, 1.0)[0]
    # the one-launch-per-step protocol gives the same trajectory
    cfg, st, xs, vs = _setup("none", N, x0=x0, v0=v0)
    for _ in range(T):
        R.ld_step(cfg, st, p, N, xs, vs)
    torch.cuda.synchronize()
    assert float((xs - out["none"][0]).abs().max()) <= 1e-5 and float((vs - out["none"][1]).abs().max()) <= 1e-5


def test_no_noise_batched_plan_and_null_state():
    N, T = 3000, 64
    p = _params(W.LDParams(kT=0.0))
    ens, n_ens = R.make_ensembles([(0, 1000, p, 0), (1000, 2000, p, 0)])
    cfg = R.make_cfg("none")
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    R.rng_init_ensembles(cfg, st, ens, n_ens)
    x = torch.ones(3 * N, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(x)
    xb, vb = x.clone(), v.clone()
    R.ld_run(cfg, st, ens, n_ens, N, T, x, v)
    plan = R.Plan(cfg, st, ens, n_ens, N, T, xb, vb)
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    assert torch.equal(x, xb) and torch.equal(v, vb)
    # every oscillator starts at x = 1, v = 0 and follows the same deterministic path
    assert float(x.std()) == 0.0 and float(v.std()) == 0.0
    xr, vr, _ = orc.ld_run("taus", orc.taus_seed(1, [0]), 1, T, W.LDParams(kT=0.0).as_f32().asdict(),
                           np.ones((3, 1)), np.zeros((3, 1)))
    assert _close(x.view(3, N)[:, :1].cpu().numpy(), xr, 1.0)[0]
    assert _close(v.view(3, N)[:, :1].cpu().numpy(), vr, 1.0)[0]


# ---------------------------------------------------------------------------------------------
# lagged Fibonacci: persistent dataflow run vs one launch per wave

# lags whose short lag is 1 or 3 mod 4 make consumer groups of four straddle a link's end with one,
# two or three words in it; every b = ll mod sl here is off a multiple of 4, so one producer group per
# link straddles b
@pytest.mark.parametrize("n,lags,T", [(1000, (2281, 1252), 200), (1, (2281, 1252), 2000), (3001, (9689, 5502), 150),
                                      (257, (4423, 3004), 300), (100_000, (132049, 54454), 60),
                                      (2000, (19937, 10095), 100), (5000, (859433, 288477), 200),
                                      # not Table I rows: short lags whose link padding (to 64 words) is
                                      # 3 and 1 words, exactly what the last group of a link spills into
                                      (3000, (2 * 1021 + 517, 1021), 120), (3000, (2 * 1023 + 300, 1023), 120),
                                      # two, three and five tiles per consumer wave (the 2-, 4- and 8-tile
                                      # kernels); the last two runs each hold a step window that starts
                                      # 2 words before a link's end, so its first group straddles it
                                      (300_000, (132049, 54454), 30), (600_000, (132049, 54454), 15),
                                      (1_000_000, (132049, 54454), 5)])
def test_lf_dataflow_equals_waves_and_oracle(n, lags, T):
    ll, sl = lags
    pp = W.LDParams(k=1.1, gamma=0.9, kT=1.0, dt=0.01).as_f32()
    p = _params(pp)
    ens, n_ens = R.make_ensembles([(0, n, p, 0)])
    stride, t0 = 10, T // 2
    P = T // stride + 1
    res = {}
    for waves in (0, 1):
        R.ld_set_tuning("lf", lf_waves=waves)
        try:
            cfg, st, x, v = _setup("lf", n, ll=ll, sl=sl)
            ob = torch.zeros(P * R.NOBS, dtype=torch.float64, device="cuda")
            ws = R.ld_run(cfg, st, ens, n_ens, n, T, x, v, R.Obs(stride, t0), ob)
            assert R.ws_status(ws) == 0
            assert R.ws_lf_path(ws) == ("waves" if waves else "dataflow")
            res[waves] = (x, v, st, ob)
        finally:
            R.ld_set_tuning("lf")
    _say("lf dataflow", n, lags, T)
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])
    sa, sb = _lf_state(res[0][2]), _lf_state(res[1][2])
    assert sa[0] == sb[0] == 4 * n * T and sa[1] == sb[1] and np.array_equal(sa[2], sb[2])
    xo, vo, oo = orc.ld_run("lf", orc.lf_seed(1234, ll), n, T, pp.asdict(), stride=stride, t0=t0, ll=ll, sl=sl)
    assert _close(res[0][0].cpu().numpy().reshape(3, n), xo, math.sqrt(pp.kT / pp.k))[0]
    assert _close(res[0][1].cpu().numpy().reshape(3, n), vo, math.sqrt(pp.kT / pp.m))[0]
    g_obs = res[0][3].cpu().numpy().reshape(P, R.NOBS)
    assert np.all(np.abs(g_obs - oo) <= 2 * REL * (np.abs(oo) + 1.0))


def test_lf_dataflow_resume_and_mixed_calls():
    """Dataflow runs continue the one sequence across calls and interleave with bare draws."""
    n, ll, sl = 2000, 2281, 1252
    p = _params(W.LDParams())
    ens, n_ens = R.make_ensembles([(0, n, p, 0)])
    cfg, st, x, v = _setup("lf", n, ll=ll, sl=sl)
    R.ld_run(cfg, st, ens, n_ens, n, 37, x, v)
    extra = torch.empty(1001, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, 1001, extra)
    R.ld_run(cfg, st, ens, n_ens, n, 23, x, v)
    torch.cuda.synchronize()
    win = orc.lf_seed(1234, ll)
    xo, vo, _ = orc.ld_run("lf", win, n, 37, W.LDParams().as_f32().asdict(), ll=ll, sl=sl)
    assert np.array_equal(extra.cpu().numpy().view(np.uint32), orc.lf_generate(ll, sl, win, 1001))
    xo, vo, _ = orc.ld_run("lf", win, n, 23, W.LDParams().as_f32().asdict(), xo, vo, ll=ll, sl=sl)
    assert _close(x.cpu().numpy().reshape(3, n), xo, 1.0)[0]


def test_lf_ring_size_does_not_change_the_run():
    """The state's ring size (the smallest allowed, ll + sl, the default, a larger one, and one only
    W = 4000 longer than ll) changes neither the persistent run nor the wave path: same trajectory
    and the same last ll values bit for bit, and a second call continues the sequence alike."""
    n, T, ll, sl = 3001, 150, 9689, 5502
    p = _params(W.LDParams(k=1.3, gamma=0.7, dt=0.01))
    ens, n_ens = R.make_ensembles([(0, n, p, 0)])
    ref = None
    cases = [(ring, waves) for ring in (ll + sl, 0, 4 * (ll + sl), ll + 4000) for waves in (0, 1)]
    for ring, waves in cases:
        cfg = R.make_cfg("lf", seed=77, ll=ll, sl=sl, ring=ring, wave=4000 if ring == ll + 4000 else 0)
        st = R.new_state(cfg)
        R.rng_init(cfg, st)
        x = torch.zeros(3 * n, dtype=torch.float32, device="cuda")
        v = torch.zeros_like(x)
        ob = torch.zeros((T // 10 + 1) * R.NOBS, dtype=torch.float64, device="cuda")
        R.ld_set_tuning("lf", lf_waves=waves)
        try:
            ws = R.ld_run(cfg, st, ens, n_ens, n, T, x, v, R.Obs(10, T // 3), ob)
            torch.cuda.synchronize()
            _say("lf ring", ring, R.ws_lf_path(ws))
            assert R.ws_status(ws) == 0 and R.ws_lf_path(ws) == ("waves" if waves else "dataflow")
            R.ld_run(cfg, st, ens, n_ens, n, 7, x, v)
            torch.cuda.synchronize()
        finally:
            R.ld_set_tuning("lf")
        win = _lf_state(st)
        if ref is None:
            ref = (x.clone(), v.clone(), ob.clone(), win)
        else:
            assert torch.equal(x, ref[0]) and torch.equal(v, ref[1]), (ring, waves)
            assert torch.allclose(ob, ref[2], rtol=1e-12, atol=1e-12)
            assert win[0] == ref[3][0] and np.array_equal(win[2], ref[3][2]), (ring, waves)


# ---------------------------------------------------------------------------------------------
# Sec. IV / Fig. 4: overdamped oscillators started away from the minimum

@pytest.mark.parametrize("kind", ["taus", "ran2", "lf", "lcg"])
def test_fig4_overdamped_mean_decay_and_correlation(kind):
    """N = 1e4 oscillators from x0 = 10 in reduced units (tau = xi/k = 100 steps), 2000 overdamped
    steps (Eq. 5).  The ensemble mean <x(t)> follows x0 a^t and the equilibrium correlation
    <x(t0 + s) x(t0)> follows <x^2> a^s (the exact discrete forms of Sec. IV's R0 exp(-t/tau) and
    (kT/k) exp(-t/tau)) within 4.5 standard errors at every observation."""
    N, T, stride, t0 = 10_000, 2000, 10, 1000
    pp = W.LDParams(m=1.0, k=1.0, gamma=1.0, kT=1.0, dt=0.01).as_f32()
    pd = dict(m=float(pp.m), k=float(pp.k), gamma=float(pp.gamma), kT=float(pp.kT), dt=float(pp.dt))
    ll, sl = _lf_lags(N) if kind == "lf" else (0, 0)
    x0 = np.full((3, N), 10.0, np.float32)
    cfg, st, x, v = _setup(kind, N, ll=ll, sl=sl, x0=x0, v0=np.zeros((3, N), np.float32))
    ens, n_ens = R.make_ensembles([(0, N, _params(pp, scheme=1), 0)])
    P = T // stride + 1
    ob = torch.zeros(P * R.NOBS, dtype=torch.float64, device="cuda")
    R.ld_run(cfg, st, ens, n_ens, N, T, x, v, R.Obs(stride, t0), ob)
    obs = ob.cpu().numpy().reshape(P, R.NOBS)
    n = 3 * N
    steps = np.arange(0, T + 1, stride)
    mean, var = mom.overdamped_transient(**pd, n_steps=T, x0=10.0)
    z_mean = np.abs(obs[1:, 3] - mean[steps[1:]]) / np.sqrt(var[steps[1:]] / n)
    after = steps >= t0
    c = mom.overdamped_cross(**pd, t0=t0, taus=steps[after] - t0, x0=10.0)
    s = var[steps[after]] + mean[steps[after]] ** 2
    z_c = np.abs(obs[after, 4] - c) / np.sqrt((s * s[0] + c**2) / n)
    # the paper's continuous forms, for the record (O(h) apart from the discrete ones)
    m_cont, c_cont = mom.overdamped_continuous(pd["k"], pd["m"] * pd["gamma"], pd["kT"], steps * pd["dt"], 10.0)
    _say("fig4", kind, "max z mean %.2f corr %.2f; <x>(tau) %.4f vs continuous %.4f" %
         (z_mean.max(), z_c.max(), obs[10, 3], m_cont[10]))
    assert z_mean.max() < 4.5 and z_c.max() < 4.5


def test_fig4_lcg_correlated_seeding_fails_on_the_gpu():
    """Negative control (Fig. 4b) on the GPU path: LCG streams seeded four values apart along one
    sequence.  The run matches the oracle given the same seeding, fails the Fig. 4 z test that
    independent streams pass, and leaves neighbouring oscillators almost fully correlated."""
    N, T, stride, t0 = 3000, 4000, 20, 800
    pp = W.LDParams(m=1.0, k=1.0, gamma=1.0, kT=1.0, dt=0.01).as_f32()
    pd = dict(m=float(pp.m), k=float(pp.k), gamma=float(pp.gamma), kT=float(pp.kT), dt=float(pp.dt))
    x0 = np.full((3, N), 10.0, np.float32)
    ens, n_ens = R.make_ensembles([(0, N, _params(pp, scheme=1), 0)])
    P = T // stride + 1
    res = {}
    for leap in (0, 4):
        cfg, st, x, v = _setup("lcg", N, x0=x0, v0=np.zeros((3, N), np.float32), leap=leap)
        ob = torch.zeros(P * R.NOBS, dtype=torch.float64, device="cuda")
        R.ld_run(cfg, st, ens, n_ens, N, T, x, v, R.Obs(stride, t0), ob)
        obs = ob.cpu().numpy().reshape(P, R.NOBS)
        xg = x.cpu().numpy().reshape(3, N).astype(np.float64)
        xr, _, _ = orc.ld_run("lcg", orc.seed_states("lcg", 1234, np.arange(N), leap=leap), N, T, pd, x0,
                              np.zeros((3, N)), scheme=1)
        assert _close(xg, xr, math.sqrt(pd["kT"] / pd["k"]))[0], leap
        steps = np.arange(0, T + 1, stride)
        mean, var = mom.overdamped_transient(**pd, n_steps=T, x0=10.0)
        zm = np.max(np.abs(obs[1:, 3] - mean[steps[1:]]) / np.sqrt(var[steps[1:]] / (3 * N)))
        corr = np.mean([np.corrcoef(xg[d, :-1], xg[d, 1:])[0, 1] for d in range(3)])
        res[leap] = (float(zm), float(corr))
    _say("lcg negative control (max z of <x>, neighbour corr):", res)
    assert res[0][0] < 4.5 and abs(res[0][1]) < 0.1
    assert res[4][0] > 10 and res[4][1] > 0.9


def test_fig4_paper_units_fp32_state():
    """Sec. IV / Fig. 4 in the paper's own units (nm, ns, pN): k = 0.01 pN/nm, kT = 4.14 pN nm
    (300 K), D = kT / xi = 0.25 nm^2/ns, h = 1 ps, x0 = 10 nm, so that h / tau = 6.0e-7 per step.
    After 10^7 steps (6 tau) of FP32 state the ensemble mean, <x^2> and the equilibrium correlation
    stay within 4.5 standard errors of the exact discrete forms at every observation: the FP32
    update shows no drift at this soft spring.  The noise-free decay in FP32 is compared with FP64
    (its rounding is deterministic, so it is only bounded loosely and reported)."""
    N, T, stride, t0 = 10_000, 10_000_000, 100_000, 8_000_000
    kT, D, k, h = 4.14, 0.25, 0.01, 1e-3
    pp = W.LDParams(m=1.0, k=k, gamma=kT / D, kT=kT, dt=h).as_f32()
    pd = dict(m=float(pp.m), k=float(pp.k), gamma=float(pp.gamma), kT=float(pp.kT), dt=float(pp.dt))
    x0 = np.full((3, N), 10.0, np.float32)
    ens, n_ens = R.make_ensembles([(0, N, _params(pp, scheme=1), 0)])
    P = T // stride + 1
    cfg, st, x, v = _setup("taus", N, x0=x0, v0=np.zeros((3, N), np.float32))
    ob = torch.zeros(P * R.NOBS, dtype=torch.float64, device="cuda")
    R.ld_run(cfg, st, ens, n_ens, N, T, x, v, R.Obs(stride, t0), ob)
    obs = ob.cpu().numpy().reshape(P, R.NOBS)
    n = 3 * N
    steps = np.arange(0, T + 1, stride)
    xi = pd["m"] * pd["gamma"]
    a = 1.0 - pd["k"] * pd["dt"] / xi
    b2 = 2.0 * pd["kT"] * pd["dt"] / xi
    mean = 10.0 * a ** steps
    var = b2 * (1.0 - a ** (2 * steps)) / (1.0 - a * a)
    z_mean = np.abs(obs[1:, 3] - mean[1:]) / np.sqrt(var[1:] / n)
    m2 = var + mean**2
    z_x2 = np.abs(obs[1:, 0] - m2[1:]) / (np.sqrt(2 * var[1:] ** 2 + 4 * var[1:] * mean[1:] ** 2) / np.sqrt(n))
    after = steps >= t0
    c = a ** (steps[after] - t0) * m2[after][0]
    z_c = np.abs(obs[after, 4] - c) / np.sqrt((m2[after] * m2[after][0] + c**2) / n)
    _say("fig4 paper units: max z mean %.2f, <x^2> %.2f, corr %.2f; <x^2> at the end %.1f nm^2 (kT/k = %.1f)"
         % (z_mean.max(), z_x2.max(), z_c.max(), obs[-1, 0], pd["kT"] / pd["k"]))
    assert z_mean.max() < 4.5 and z_x2.max() < 4.5 and z_c.max() < 4.5
    # the deterministic part alone: FP32 against the FP64 decay x0 a^T
    cfg0, st0, x0d, v0d = _setup("none", N, x0=x0, v0=np.zeros((3, N), np.float32))
    R.ld_run(cfg0, st0, ens, n_ens, N, T, x0d, v0d)
    xt = float(x0d[0])
    rel = abs(xt - 10.0 * a**T) / (10.0 * a**T)
    _say("noise-free FP32 decay after %d steps: %.6g vs FP64 %.6g (relative %.2e)" % (T, xt, 10.0 * a**T, rel))
    assert float(x0d.std()) == 0.0 and rel < 0.05
