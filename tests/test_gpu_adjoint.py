"""GPU adjoint (checkpointed noise replay) against the FP64 oracle adjoint and exact identities."""
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
A = pytest.importorskip("paper_1003_1123_amd.autograd")


def _say(*a):
    print("[gpu-adj]", *a, flush=True)
    sys.stdout.flush()


def _f32_coef(p):
    """The binary32 coefficients and partials a run iterates, formed as the header states: in
    double precision from the binary32 parameters, then rounded to binary32 once."""
    f = lambda a: float(np.float32(a))
    m, k, g, kT, h = (f(a) for a in (p.m, p.k, p.gamma, p.kT, p.dt))
    s = math.sqrt(2.0 * g * kT * h / m)
    return [f(1.0 - g * h), f(k * h / m), f(s), f(h), f(h / m), f(-h), f(s / (2.0 * g)), f(s / (2.0 * kT))]


def _oracle_per_oscillator(kind, seed, N, T, pd, tb, te):
    """Each oscillator's own loss gradient from the FP64 oracle: [N, 3]."""
    out = np.zeros((N, 3))
    for i in range(N):
        out[i] = orc.ld_adjoint(kind, orc.seed_states(kind, seed, [i]), 1, T, pd, tb, te)[1]
    return out


@pytest.mark.parametrize("kind", ["taus", "ran2"])
def test_adjoint_matches_oracle(kind):
    N, T, tb, te, K = 1000, 400, 201, 400, 64  # K does not divide T: ragged last segment
    pp = W.LDParams(k=1.2, gamma=0.8, kT=1.1, dt=0.01).as_f32()
    run = A.AdjointRun(kind, [(N, pp.m, pp.dt, 1234)], T, tb, te, K, spread=True)
    k = torch.tensor([pp.k], dtype=torch.float64, requires_grad=True)
    g = torch.tensor([pp.gamma], dtype=torch.float64, requires_grad=True)
    kT = torch.tensor([pp.kT], dtype=torch.float64, requires_grad=True)
    L = A.LDAdjoint.apply(k, g, kT, run)
    L.sum().backward()
    grad = np.array([k.grad.item(), g.grad.item(), kT.grad.item()])
    se = run.grad_se[0].cpu().numpy()
    Lo, go = orc.ld_adjoint(kind, orc.seed_states(kind, 1234, np.arange(N)), N, T, pp.asdict(), tb, te)
    _say(kind, "L", L.item(), Lo, "grad", grad, go, "se", se)
    assert abs(L.item() - Lo) <= 1e-4 * abs(Lo)
    # every component on its own scale
    assert np.all(np.abs(grad - go) <= 1e-3 * np.abs(go)), (grad, go)
    # exact pathwise identity from rest
    assert abs(grad[2] - L.item() / pp.kT) <= 1e-4 * abs(L.item() / pp.kT)
    # the standard errors: the spread of the oracle's per-oscillator gradients over sqrt(N)
    per = _oracle_per_oscillator(kind, 1234, N, T, pp.asdict(), tb, te)
    assert np.allclose(per.mean(axis=0), go, rtol=1e-9, atol=1e-12)
    se_o = per.std(axis=0, ddof=1) / math.sqrt(N)
    _say(kind, "se oracle", se_o)
    assert np.all(np.abs(se - se_o) <= 1e-3 * se_o), (se, se_o)


def test_adjoint_batched_equals_plain():
    T, tb, te, K = 300, 151, 300, 100
    shape = [(700, 1.0, 0.01, 11), (300, 1.0, 0.01, 12), (1, 1.0, 0.01, 13)]
    params = [(1.0, 1.0, 1.0), (2.0, 0.5, 1.5), (0.7, 3.0, 0.6)]
    run = A.AdjointRun("taus", shape, T, tb, te, K)
    k = torch.tensor([p[0] for p in params], dtype=torch.float64, requires_grad=True)
    g = torch.tensor([p[1] for p in params], dtype=torch.float64, requires_grad=True)
    kT = torch.tensor([p[2] for p in params], dtype=torch.float64, requires_grad=True)
    L = A.LDAdjoint.apply(k, g, kT, run)
    L.sum().backward()
    for e, (sh, pr) in enumerate(zip(shape, params)):
        r1 = A.AdjointRun("taus", [sh], T, tb, te, K)
        k1 = torch.tensor([pr[0]], dtype=torch.float64, requires_grad=True)
        g1 = torch.tensor([pr[1]], dtype=torch.float64, requires_grad=True)
        t1 = torch.tensor([pr[2]], dtype=torch.float64, requires_grad=True)
        L1 = A.LDAdjoint.apply(k1, g1, t1, r1)
        L1.sum().backward()
        assert L1.item() == L[e].item()
        assert (k1.grad.item(), g1.grad.item(), t1.grad.item()) == (k.grad[e].item(), g.grad[e].item(),
                                                                    kT.grad[e].item())


def _config5_grad(spread=False, kind="taus"):
    c = W.C5
    pp = c["params"].as_f32()
    run = A.AdjointRun(kind, [(c["N"], pp.m, pp.dt, c["seed"])], c["steps"], c["t_begin"], c["t_end"], c["K"],
                       spread=spread)
    k = torch.tensor([pp.k], dtype=torch.float64, requires_grad=True)
    g = torch.tensor([pp.gamma], dtype=torch.float64, requires_grad=True)
    kT = torch.tensor([pp.kT], dtype=torch.float64, requires_grad=True)
    L = A.LDAdjoint.apply(k, g, kT, run)
    L.sum().backward()
    grad = np.array([k.grad.item(), g.grad.item(), kT.grad.item()])
    return run, L.item(), grad


def _config5_loss(q):
    """Loss of the config-5 forward run with parameters q (same seeds, hence the same noise)."""
    c = W.C5
    pp = c["params"].as_f32()
    r = A.AdjointRun("taus", [(c["N"], pp.m, pp.dt, c["seed"])], c["steps"], c["t_begin"], c["t_end"], c["K"])
    return A.LDAdjoint.apply(*(torch.tensor([q[n]], dtype=torch.float64) for n in ("k", "gamma", "kT")), r).item()


def test_config5_gradients():
    """Config 5: N = 1e5, 2000 steps, loss over steps 1001-2000, K = 100 (the register-only,
    segment-parallel backward).  (i) dL/dkT = L/kT exactly; (ii) each gradient within 4 standard
    errors (the per-oscillator spread the backward returns) of d E[L]/d theta from the moment
    recursion; (iii) central differences of the forward kernel under common random numbers with a
    5% step, each component within 1% of its own value plus the truncation error (the change
    from doubling the step) plus the rounding floor of the binary32 coefficients: c = 1 - gamma h
    is held to half an ulp (2^-25), which moves L by up to L / (1 - c) 2^-25 per run (and
    k h / m, sigma by L / kap 2^-31 and 2 L / sigma 2^-27), so a difference over 2 d carries up to
    twice that over 2 d.  At config 5 (gamma h = 0.01) that floor is 6e-5 for d = 0.05, 8% of
    dL/dgamma; the pathwise comparison with the oracle below checks dL/dgamma to 1e-3."""
    c = W.C5
    pp = c["params"].as_f32()
    run, L, grad = _config5_grad(spread=True)
    se = run.grad_se[0].cpu().numpy()
    _say("config5 L", L, "grad", grad, "se", se)
    assert abs(grad[2] - L / pp.kT) <= 1e-4 * abs(L)
    exact = mom.expected_loss_grad(pp.m, pp.k, pp.gamma, pp.kT, pp.dt, c["steps"], c["t_begin"], c["t_end"])
    z = (grad - exact) / se
    _say("config5 d E[L]/d theta", exact, "z", z)
    assert np.all(se > 0) and np.all(np.abs(z) < 4), (grad, exact, se)
    base = dict(k=pp.k, gamma=pp.gamma, kT=pp.kT)
    cq = _f32_coef(pp)
    fd = {}
    for rel in (5e-2, 1e-1):
        out = []
        for name in ("k", "gamma", "kT"):
            d = rel * base[name]
            lp = _config5_loss(dict(base, **{name: base[name] + d}))
            lm = _config5_loss(dict(base, **{name: base[name] - d}))
            out.append((lp - lm) / (2 * d))
        fd[rel] = np.array(out)
    trunc = np.abs(fd[1e-1] - fd[5e-2])
    d = 5e-2 * np.array([base["k"], base["gamma"], base["kT"]])
    per_run = L * (2.0**-25 / (1.0 - cq[0]) + 2.0**-31 / cq[1] + 2.0 * 2.0**-27 / cq[2])
    floor = 2.0 * per_run / (2.0 * d)
    _say("config5 FD", fd[5e-2], fd[1e-1], "floor", floor)
    assert np.all(np.abs(fd[5e-2] - grad) <= 1e-2 * np.abs(grad) + trunc + floor), (fd, grad, floor)


@pytest.mark.parametrize("kind", ["taus", "ran2"])
def test_config5_gradients_match_the_oracle(kind):
    """The config-5 gradients (N = 1e5, 2000 steps, every oscillator) against the FP64 oracle
    adjoint of the same oscillators and noise.  Iterating the binary32 coefficients the run uses,
    each component agrees within 1e-4 of its own value.  Against the oracle with exact
    coefficients the difference is set by their rounding (see the finite-difference test), which
    the difference of the two oracle runs measures.  Config 5 names Hybrid Taus (segment-parallel
    forward); the same workload with Ran2 checks its sequential forward and register-only
    backward at full size."""
    c = W.C5
    pp = c["params"].as_f32()
    _, L, grad = _config5_grad(kind=kind)
    args = (kind, c["seed"], c["N"], c["steps"], pp.asdict(), c["t_begin"], c["t_end"])
    L32, g32 = orc.ld_adjoint_split(*args, coef=_f32_coef(pp))
    L64, g64 = orc.ld_adjoint_split(*args)
    _say(kind, "config5 GPU", L, grad, "oracle (binary32 coefficients)", L32, g32, "relative",
         np.abs(grad - g32) / np.abs(g32))
    _say("oracle (exact coefficients)", L64, g64, "relative", np.abs(grad - g64) / np.abs(g64))
    assert abs(L - L32) <= 1e-5 * abs(L32)
    # measured (Hybrid Taus): 3e-8, 4e-6 and 4e-8 of the three values
    assert np.all(np.abs(grad - g32) <= 1e-4 * np.abs(g32)), (grad, g32)
    assert np.all(np.abs(grad - g64) <= 1e-3 * np.abs(g64) + 2.0 * np.abs(g64 - g32)), (grad, g64, g32)


def _grads(kind, shape, params, T, tb, te, K, replay=False):
    run = A.AdjointRun(kind, shape, T, tb, te, K, replay=replay)
    k = torch.tensor([p[0] for p in params], dtype=torch.float64, requires_grad=True)
    g = torch.tensor([p[1] for p in params], dtype=torch.float64, requires_grad=True)
    kT = torch.tensor([p[2] for p in params], dtype=torch.float64, requires_grad=True)
    L = A.LDAdjoint.apply(k, g, kT, run)
    L.sum().backward()
    torch.cuda.synchronize()
    return run, L.detach().cpu().numpy(), np.stack([k.grad.numpy(), g.grad.numpy(), kT.grad.numpy()], axis=1)


@pytest.mark.parametrize("kind", ["taus", "ran2"])
def test_register_only_backward_equals_replay(kind):
    """The register-only backward (each segment rerun forward from its start checkpoint, the loss
    adjoint carried forward from the one the forward run left there) against the replay backward
    on the same forward run: noise and path are the same bit for bit, so the gradients differ only
    by the rounding of the carried adjoint, each component within 1e-5 of its own value."""
    T, tb, te, K = 500, 101, 500, 64
    shape = [(3000, 1.0, 0.01, 5), (1000, 1.0, 0.01, 6)]
    params = [(1.0, 1.0, 1.0), (2.0, 1.5, 0.7)]
    run_i, Li, gi = _grads(kind, shape, params, T, tb, te, K)
    run_r, Lr, gr = _grads(kind, shape, params, T, tb, te, K, replay=True)
    assert run_i.ws.numel() < run_r.ws.numel()  # no replay scratch on the register-only path
    assert np.array_equal(Li, Lr)
    rel = np.abs(gi - gr) / np.abs(gr)
    _say(kind, "register-only vs replay: relative gradient difference per component", rel)
    # measured: about 1e-8 of each value
    assert np.all(rel <= 1e-5), (gi, gr)


STATE_ROWS = {"taus": 4, "ran2": 35}


@pytest.mark.parametrize("kind", ["taus", "ran2"])
def test_checkpoint_end_record_is_the_final_state(kind):
    N, T, K = 777, 130, 50  # records at steps 0, 50, 100 and the end state (step 130)
    S = STATE_ROWS[kind]
    run, _, _ = _grads(kind, [(N, 1.0, 0.01, 9)], [(1.0, 1.0, 1.0)], T, 1, T, K)
    rec = (6 + S + 6) * N * 4
    last = run.ckpt[3 * rec:4 * rec]
    assert torch.equal(last[:3 * N * 4].view(torch.float32), run.x)
    assert torch.equal(last[3 * N * 4:6 * N * 4].view(torch.float32), run.v)
    assert torch.equal(last[6 * N * 4:(6 + S) * N * 4], run.state[:S * N * 4])
    # no loss term follows the end state: its adjoint rows are zero
    assert not last[(6 + S) * N * 4:].view(torch.float32).any()


@pytest.mark.parametrize("kind", ["taus", "ran2"])
def test_checkpoint_adjoint_rows_are_the_window_gradient_of_the_recorded_state(kind):
    """The adjoint rows of a checkpoint record hold the gradient of the sum of x^2 over the loss
    window's steps after the record with respect to the record's x and v.  Checked against central
    differences of the FP64 oracle's loss, run from the record's own state (its generator rows are
    bit-exact): for fixed noise the loss is quadratic in the starting state, so the difference is
    exact up to rounding.  The window starts and ends inside segments, and the last one is short.
    Hybrid Taus records come from the segment-parallel forward, Ran2 records from the sequential
    one."""
    N, T, tb, te, K = 300, 300, 101, 280, 64  # records at steps 0, 64, 128, 192, 256 and 300
    S = STATE_ROWS[kind]
    pp = W.LDParams(k=1.2, gamma=0.8, kT=1.1, dt=0.01).as_f32()
    pd = pp.asdict()
    run = A.AdjointRun(kind, [(N, pp.m, pp.dt, 77)], T, tb, te, K)
    A.LDAdjoint.apply(*(torch.tensor([a], dtype=torch.float64) for a in (pp.k, pp.gamma, pp.kT)), run)
    torch.cuda.synchronize()
    rows = 6 + S + 6
    ck = run.ckpt.cpu()
    worst = 0.0
    for r in (0, 1, 2, 4):
        step = r * K
        rec = ck[r * rows * N * 4:(r + 1) * rows * N * 4]
        f = rec.view(torch.float32).numpy().reshape(rows, N)
        u = rec.view(torch.int32).numpy().view(np.uint32).reshape(rows, N)
        tb_r, te_r = max(tb - step, 1), te - step
        scale = 3.0 * (te_r - tb_r + 1)  # the oracle's loss is the mean over 3 coordinates and the window
        # the record's generator rows: the seeded streams after 4 draws per step, bit for bit; its
        # x and v: the oracle's run from rest over the same steps
        ids = np.arange(N)
        st_o = orc.seed_states(kind, 77, ids)
        xo, vo, _ = orc.ld_run(kind, st_o, N, step, pd)
        assert np.array_equal(u[6:6 + S].T, st_o.view(np.uint32)), r
        assert np.max(np.abs(f[0:3] - xo)) <= 1e-4 * max(1.0, np.max(np.abs(xo))), r
        assert np.max(np.abs(f[3:6] - vo)) <= 1e-4 * max(1.0, np.max(np.abs(vo))), r
        for i in (0, 7, 255, 299):
            x0 = f[0:3, i:i + 1].astype(np.float64)
            v0 = f[3:6, i:i + 1].astype(np.float64)
            st = np.ascontiguousarray(u[6:6 + S, i][None, :]).view(st_o.dtype)

            def loss(which, d, delta):
                xx, vv = x0.copy(), v0.copy()
                (xx if which == 0 else vv)[d, 0] += delta
                return orc.ld_loss(kind, st.copy(), 1, T - step, pd, tb_r, te_r, xx, vv)

            fd = np.array([[(loss(w, d, 1e-2) - loss(w, d, -1e-2)) / 2e-2 * scale for d in range(3)] for w in (0, 1)])
            got = f[6 + S:12 + S, i].reshape(2, 3).astype(np.float64)
            err = np.max(np.abs(got - fd)) / np.max(np.abs(fd))
            worst = max(worst, err)
            assert err <= 1e-4, (r, i, got, fd)
    _say(kind, "checkpoint adjoint rows vs oracle differences: worst relative error", worst)


@pytest.mark.parametrize("kind", ["taus", "ran2"])
def test_mixed_paths_match_the_oracle(kind):
    """A strongly damped ensemble (gamma dt = 0.06: replay) batched with a weakly damped one
    (register-only); each against the FP64 oracle adjoint."""
    T, tb, te, K = 300, 1, 300, 100
    shape = [(800, 1.0, 0.01, 21), (600, 1.0, 0.01, 22)]
    params = [(1.0, 0.5, 1.0), (1.5, 6.0, 0.8)]
    _, L, grad = _grads(kind, shape, params, T, tb, te, K)
    for e, ((n, m, dt, seed), (k, gm, kT)) in enumerate(zip(shape, params)):
        pd = W.LDParams(m=m, k=k, gamma=gm, kT=kT, dt=dt).as_f32().asdict()
        Lo, go = orc.ld_adjoint(kind, orc.seed_states(kind, seed, np.arange(n)), n, T, pd, tb, te)
        assert abs(L[e] - Lo) <= 1e-4 * abs(Lo)
        scale = np.max(np.abs(go))
        assert np.all(np.abs(grad[e] - go) <= 1e-3 * np.maximum(np.abs(go), 1e-2 * scale)), (e, grad[e], go)
