"""The allocation-free entry point (ld_run_noalloc) against ld_run with a caller-owned workspace,
through the C ABI: the same runs bit for bit (x, v, observables, generator state, status words),
on calls in a row whose second is smaller than the first, so that what a call leaves in the
library's array cannot leak into the next one."""
import sys

import numpy as np
import pytest
import torch

from paper_1003_1123_amd import workloads as W

pytestmark = pytest.mark.gpu
R = pytest.importorskip("paper_1003_1123_amd._lib")


def _say(*a):
    print("[gpu-noalloc]", *a, flush=True)
    sys.stdout.flush()


def _start(N, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = torch.as_tensor(rng.standard_normal(3 * N).astype(np.float32)).cuda()
    v = torch.as_tensor(rng.standard_normal(3 * N).astype(np.float32)).cuda()
    return x, v


def _pair(kind, specs, n_total, T, obs, ll=0, sl=0, seed=1234):
    """One run through each entry point from identical inputs; asserts they agree bit for bit."""
    _say(kind, "ensembles", [(o, n) for o, n, _ in specs], "steps", T, "obs", obs and (obs.stride, obs.t0))
    cfg = R.make_cfg(kind, seed=seed, n_streams=n_total, ll=ll, sl=sl)
    st_a = R.new_state(cfg)
    R.rng_init(cfg, st_a)
    st_b = st_a.clone()
    xa, va = _start(n_total, seed + 1)
    xb, vb = xa.clone(), va.clone()
    ens, n_ens = R.make_ensembles([(o, n, p, 0) for o, n, p in specs])
    P = (T // obs.stride + 1) if obs and obs.stride else 0
    oa = torch.full((max(n_ens * P * R.NOBS, 1),), -1.0, dtype=torch.float64, device="cuda")
    ob = oa.clone()
    ws = R.ld_run(cfg, st_a, ens, n_ens, n_total, T, xa, va, obs, oa if P else None)
    status = torch.full((2,), 12345, dtype=torch.int32, device="cuda")
    R.ld_run_noalloc(cfg, st_b, ens, n_ens, n_total, T, xb, vb, obs, ob if P else None, status)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb) and torch.equal(va, vb)
    assert torch.equal(oa, ob)
    assert torch.equal(st_a, st_b)
    ref_status = ws[:8].view(torch.int32).cpu().tolist()
    got_status = status.cpu().tolist()
    _say("status words", ref_status, got_status)
    assert got_status == ref_status and got_status[0] == 0
    return got_status


def test_noalloc_equals_ld_run_per_thread_kinds():
    p1 = R.make_params(1.0, 1.3, 0.7, 0.9, 0.01)
    p2 = R.make_params(2.0, 0.5, 2.5, 1.4, 0.01)
    for kind in ("taus", "ran2", "lcg"):
        # a batched run with observables, then a smaller plain run with a later t0
        _pair(kind, [(0, 20000, p1), (20000, 7001, p2)], 27001, 300, R.Obs(10, 100))
        _pair(kind, [(0, 3000, p2)], 3000, 120, R.Obs(7, 50))


def test_noalloc_equals_ld_run_lagged_fibonacci():
    p = R.make_params(1.0, 1.0, 1.0, 1.0, 0.005)
    ll, sl = W.lf_lags_for(4 * 2000)
    assert _pair("lf", [(0, 2000, p)], 2000, 150, R.Obs(10, 40), ll=ll, sl=sl)[1] == 1  # persistent path
    ll, sl = W.lf_lags_for(4 * 300)
    assert _pair("lf", [(0, 300, p)], 300, 90, None, ll=ll, sl=sl)[1] == 1


def test_noalloc_rejects_a_run_beyond_its_array():
    N, T = 10**6, 10**4  # observables every 10 steps: 1001 points x 3907 tiles x 48 bytes
    cfg = R.make_cfg("taus", n_streams=N)
    st = R.new_state(cfg)
    x = torch.zeros(3 * N, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(x)
    out = torch.zeros(((T // 10) + 1) * R.NOBS, dtype=torch.float64, device="cuda")
    ens, n_ens = R.make_ensembles([(0, N, R.make_params(), 0)])
    assert R.ld_workspace_bytes(cfg, ens, n_ens, N, T, R.Obs(10, 0)) > R.NOALLOC_SCRATCH_BYTES
    with pytest.raises(R.RngldError) as e:
        R.ld_run_noalloc(cfg, st, ens, n_ens, N, T, x, v, R.Obs(10, 0), out)
    assert e.value.code == R.ESIZE
