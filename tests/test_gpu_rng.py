"""GPU parity of seeding, bare uniform streams and Gaussians against the CPU oracle (C ABI path).

Integer streams must match bit for bit; FP32 Gaussians within 1e-5 absolute of the FP64 oracle.
"""
import os
import math
import sys

import numpy as np
import pytest
import torch

import oracle as orc
from paper_1003_1123_amd import workloads as W

pytestmark = pytest.mark.gpu
R = pytest.importorskip("paper_1003_1123_amd._lib")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GAUSS_TOL = 1e-5


def _say(*a):
    print("[gpu-rng]", *a, flush=True)
    sys.stdout.flush()


def _u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def _state_rows(cfg, state):
    S = cfg.n_streams
    rows = R.STATE_ROWS[cfg.kind]
    return state[:rows * S * 4].cpu().numpy().view(np.uint32).reshape(rows, S)


@pytest.mark.parametrize("kind", ["taus", "ran2", "lcg"])
def test_seeding_matches_oracle(kind):
    _say("seeding", kind)
    S = 1000
    cfg = R.make_cfg(kind, seed=1234, n_streams=S)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    torch.cuda.synchronize()
    gpu = _state_rows(cfg, st)
    ref = orc.seed_states(kind, 1234, np.arange(S)).view(np.uint32)  # [S, rows]
    assert np.array_equal(gpu.T, ref)


@pytest.mark.parametrize("kind", ["taus", "ran2", "lcg"])
def test_seeding_with_stream_base(kind):
    base = 2**20 - 7
    cfg = R.make_cfg(kind, seed=99, n_streams=13, stream_base=base)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    gpu = _state_rows(cfg, st)
    ref = orc.seed_states(kind, 99, base + np.arange(13)).view(np.uint32)
    assert np.array_equal(gpu.T, ref)


@pytest.mark.parametrize("leap", [1, 4, 1000])
def test_lcg_leaped_seeding_and_streams(leap):
    """Correlated LCG seeding: stream j starts j * leap steps past the stream-0 seed word."""
    S, per, base = 300, 50, 12345
    cfg = R.make_cfg("lcg", seed=31, n_streams=S, stream_base=base, leap=leap)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    ost = orc.seed_states("lcg", 31, base + np.arange(S), leap=leap)
    assert np.array_equal(_state_rows(cfg, st).T, ost.view(np.uint32))
    out = torch.empty(S * per, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, per, out)
    assert np.array_equal(_u32(out).reshape(per, S), orc.uniform_streams("lcg", ost, per))


def test_taus_seed_lift_streams():
    """Streams whose raw seed words have all-zero significant bits (found by the oracle)."""
    for line in open(os.path.join(GOLDEN, "taus_lift_streams.txt")):
        if line.startswith("#") or not line.strip():
            continue
        seed, comp, stream, raw = (int(v) for v in line.split())
        cfg = R.make_cfg("taus", seed=seed, n_streams=1, stream_base=stream)
        st = R.new_state(cfg)
        R.rng_init(cfg, st)
        gpu = _state_rows(cfg, st)[:, 0]
        assert np.array_equal(gpu, orc.taus_seed(seed, [stream])[0])
        assert gpu[comp] == raw + (1 << (32 - (31, 29, 28)[comp]))


@pytest.mark.parametrize("kind", ["taus", "ran2", "lcg"])
@pytest.mark.parametrize("S,per", [(1, 1), (777, 1000), (256, 3)])
def test_uniform_streams_bit_exact(kind, S, per):
    _say("uniform", kind, S, per)
    cfg = R.make_cfg(kind, seed=4321, n_streams=S)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    out = torch.empty(S * per, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, per, out)
    # a second call continues the streams
    out2 = torch.empty(S * 5, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, 5, out2)
    torch.cuda.synchronize()
    ost = orc.seed_states(kind, 4321, np.arange(S))
    ref = orc.uniform_streams(kind, ost, per)
    ref2 = orc.uniform_streams(kind, ost, 5)
    assert np.array_equal(_u32(out).reshape(per, S), ref)
    assert np.array_equal(_u32(out2).reshape(5, S), ref2)
    assert np.array_equal(_state_rows(cfg, st).T, ost.view(np.uint32))


@pytest.mark.parametrize("kind", ["taus", "ran2", "lcg"])
def test_config3_sampled_streams(kind):
    """2^20 streams x 1024 values in one call; 64 sampled streams checked against the oracle."""
    S, per = W.C3["streams"], W.C3["per_stream"]
    _say("config3", kind, S, per)
    cfg = R.make_cfg(kind, seed=W.C3["seed"], n_streams=S)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    out = torch.empty(S * per, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, per, out)
    torch.cuda.synchronize()
    ids = W.sampled_streams(S, 64)
    gpu = out.view(per, S)[:, torch.as_tensor(ids, device="cuda")].cpu().numpy().view(np.uint32)
    ref = orc.uniform_streams(kind, orc.seed_states(kind, W.C3["seed"], ids), per)
    assert np.array_equal(gpu, ref)
    del out


@pytest.mark.parametrize("kind", ["taus", "ran2", "lcg"])
def test_first_million_values_of_sampled_streams(kind):
    """The first 10^6 values of each of the 64 sampled config-3 streams (0, 1, 2^20 - 1 and 61
    drawn ones), each generated in a run of its own."""
    ids = W.sampled_streams(W.C3["streams"], 64)
    n = 10**6
    _say("first 1e6", kind, len(ids))
    for j in ids:
        cfg = R.make_cfg(kind, seed=W.C3["seed"], n_streams=1, stream_base=int(j))
        st = R.new_state(cfg)
        R.rng_init(cfg, st)
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        R.rng_uniform(cfg, st, n, out)
        ref = orc.uniform_streams(kind, orc.seed_states(kind, W.C3["seed"], [j]), n)[:, 0]
        assert np.array_equal(_u32(out), ref), (kind, j)


@pytest.mark.parametrize("kind", ["taus", "ran2", "lcg"])
def test_gaussian_streams_within_tolerance(kind):
    S, per = 777, 1000
    cfg = R.make_cfg(kind, seed=2024, n_streams=S)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    out = torch.empty(S * per, dtype=torch.float32, device="cuda")
    R.rng_gaussian(cfg, st, per, out)
    ref = orc.gaussian_streams(kind, orc.seed_states(kind, 2024, np.arange(S)), per)
    gpu = out.view(per, S).cpu().numpy().astype(np.float64)
    err = np.max(np.abs(gpu - ref))
    _say("gaussian", kind, "max abs err", err)
    assert err <= GAUSS_TOL


@pytest.mark.parametrize("kind", ["taus", "ran2", "lf"])
def test_config3_gaussian_moments_and_bit_balance(kind):
    """Config 3 at full size: 2^30 Gaussians of one call (2^20 streams x 1024, or one lagged-Fibonacci
    stream of 2^30) have mean 0, variance 1 and fourth moment 3 within 5 standard errors
    (SE = sqrt(Var / n) of the per-value terms: 1, 2 and 96); and 2^30 uint32 words have each bit
    set with frequency 1/2 within 5 standard errors (Ran2's word is iy < 2^31, so its bits 0..30;
    for the lagged Fibonacci stream bits 8..31, see below).  The LCG, whose low bits have short periods, is the paper's counterexample
    and is left out."""
    n = 2**30
    if kind == "lf":
        ll, sl = W.C3["lf_lags"]
        cfg = R.make_cfg("lf", seed=W.C3["seed"], ll=ll, sl=sl)
        per = n
    else:
        cfg = R.make_cfg(kind, seed=W.C3["seed"], n_streams=W.C3["streams"])
        per = W.C3["per_stream"]
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    _say("config3 moments", kind)
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    R.rng_gaussian(cfg, st, per, out)
    s1 = s2 = s4 = 0.0
    for c in out.split(2**26):
        d = c.double()
        s1 += float(d.sum())
        d2 = d * d
        s2 += float(d2.sum())
        s4 += float((d2 * d2).sum())
    m1, m2, m4 = s1 / n, s2 / n, s4 / n
    _say(kind, "mean %.2e var-1 %.2e m4-3 %.2e" % (m1, m2 - 1, m4 - 3))
    assert abs(m1) < 5 * math.sqrt(1 / n) and abs(m2 - 1) < 5 * math.sqrt(2 / n) and abs(m4 - 3) < 5 * math.sqrt(96 / n)
    del out
    u = torch.empty(n, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, per, u)
    ones = torch.zeros(32, dtype=torch.float64, device="cuda")
    for c in u.split(2**26):
        for b in range(32):
            ones[b] += float(((c >> b) & 1).sum())
    f = ones.cpu().numpy() / n
    if kind == "ran2":  # the word is iy in [1, m1 - 1], below 2^31
        assert f[31] == 0.0
        f = f[:31]
    if kind == "lf":
        # the low bits of an additive lagged Fibonacci sequence follow GF(2) recurrences of their own
        # (bit 0: y_n = y_{n-ll} xor y_{n-sl}); from the LCG-filled window they stay unbalanced by
        # up to a few per cent over 2^25-value stretches of the first 2^30 values (the oracle shows
        # the same), so only the 24 bits the uniform mapping uses are held to the 1/2 frequency
        _say("lf bit frequencies - 1/2:", " ".join("%.1e" % d for d in (f - 0.5)))
        f = f[8:]
    _say(kind, "bit frequency worst |f - 1/2| %.2e" % np.max(np.abs(f - 0.5)))
    assert np.all(np.abs(f - 0.5) < 5 * 0.5 / math.sqrt(n))


# ---------------------------------------------------------------------------------------------
# lagged Fibonacci

def _lf_cfg(ll=2281, sl=1252, wave=0, ring=0, seed=1234):
    return R.make_cfg("lf", seed=seed, ll=ll, sl=sl, wave=wave, ring=ring)


@pytest.mark.parametrize("wave", [4, 100, 1252])
def test_lf_uniform_matches_sequential_recurrence_for_any_wave(wave):
    ll, sl = 2281, 1252
    cfg = _lf_cfg(ll, sl, wave=wave)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    counts = [50_000, 33_333, 7, 0, 2281, 1]
    outs = []
    for c in counts:
        o = torch.empty(max(c, 1), dtype=torch.int32, device="cuda")
        R.rng_uniform(cfg, st, c, o)
        outs.append(_u32(o)[:c])
    win = orc.lf_seed(1234, ll)
    for c, o in zip(counts, outs):
        assert np.array_equal(o, orc.lf_generate(ll, sl, win, c)), (wave, c)


def test_lf_gaussian_and_ld_share_the_sequence():
    """rng_gaussian consumes the same sequence; mixing calls keeps one stream."""
    ll, sl = 2281, 1252
    cfg = _lf_cfg(ll, sl, wave=600)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    o1 = torch.empty(1000, dtype=torch.int32, device="cuda")
    g = torch.empty(5000, dtype=torch.float32, device="cuda")
    o2 = torch.empty(999, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, 1000, o1)
    R.rng_gaussian(cfg, st, 5000, g)
    R.rng_uniform(cfg, st, 999, o2)
    win = orc.lf_seed(1234, ll)
    assert np.array_equal(_u32(o1), orc.lf_generate(ll, sl, win, 1000))
    ref_g = orc.lf_gaussian(ll, sl, win, 5000)
    assert np.max(np.abs(g.cpu().numpy().astype(np.float64) - ref_g)) <= GAUSS_TOL
    assert np.array_equal(_u32(o2), orc.lf_generate(ll, sl, win, 999))


def test_lf_config3_one_stream_of_2_30():
    """Config 3: one LF stream of 2^30 values with Table I's largest lags; the output array is the
    lag table.  First and last 10^6 values and a middle window are checked bit for bit."""
    ll, sl = W.C3["lf_lags"]
    n = W.C3["lf_count"]
    _say("lf config3", n)
    cfg = _lf_cfg(ll, sl, seed=W.C3["seed"])
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, n, out)
    torch.cuda.synchronize()
    win = orc.lf_seed(W.C3["seed"], ll)
    ref = orc.lf_generate(ll, sl, win, n)
    m = 10**6
    for lo in (0, n // 2 - m // 2, n - m):
        assert np.array_equal(_u32(out[lo:lo + m]), ref[lo:lo + m]), lo
    # the state continues the sequence
    nxt = torch.empty(1000, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, 1000, nxt)
    assert np.array_equal(_u32(nxt), orc.lf_generate(ll, sl, win, 1000))
    del out


def _low_bit_balance(words: np.ndarray, bits: int = 8):
    """Fraction of values with bit b set, b = 0..bits-1."""
    return [float(((words >> np.uint32(b)) & np.uint32(1)).mean()) for b in range(bits)]


@pytest.mark.parametrize("lags", [(2281, 1252), (44497, 23463), (3021377, 1010202)])
def test_lf_discard_matches_oracle(lags):
    """Seeding with a warm-up discard of 10 ll values (Alg. 3's initial seeds run forward): the
    stream and a fused LD run from the seeded state equal the oracle bit for bit (the LD run to the
    trajectory tolerance), and the state continues the sequence.  Reports the balance of bits 0-7
    over 2^24 values with and without the discard."""
    ll, sl = lags
    D = 10 * ll
    cfg = R.make_cfg("lf", seed=21, ll=ll, sl=sl, discard=D)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    n = 2**24
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, n, out)
    torch.cuda.synchronize()
    win = orc.lf_seed(21, ll, sl, D)
    ref = orc.lf_generate(ll, sl, win, n)
    assert np.array_equal(_u32(out), ref)
    nxt = torch.empty(999, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, 999, nxt)
    assert np.array_equal(_u32(nxt), orc.lf_generate(ll, sl, win, 999))
    cfg0 = R.make_cfg("lf", seed=21, ll=ll, sl=sl)
    st0 = R.new_state(cfg0)
    R.rng_init(cfg0, st0)
    R.rng_uniform(cfg0, st0, n, out)
    _say("lf discard", lags, "bit balance after the discard", _low_bit_balance(ref),
         "without", _low_bit_balance(_u32(out)))
    # a fused LD run from a discarded seeding
    N, T = 500, 50
    cfg = R.make_cfg("lf", seed=21, ll=ll, sl=sl, discard=D)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    p = W.LDParams().as_f32()
    x = torch.zeros(3 * N, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(x)
    ens, n_ens = R.make_ensembles([(0, N, R.make_params(p.m, p.k, p.gamma, p.kT, p.dt), 0)])
    R.ld_run(cfg, st, ens, n_ens, N, T, x, v)
    torch.cuda.synchronize()
    xr, _, _ = orc.ld_run("lf", orc.lf_seed(21, ll, sl, D), N, T, p.asdict(), ll=ll, sl=sl)
    err = np.abs(x.cpu().numpy().reshape(3, N).astype(np.float64) - xr)
    assert np.all(err <= 1e-4 * (np.abs(xr) + 1.0))


@pytest.mark.parametrize("lags,count", [((9689, 5502), 4 * 5502 + 777), ((44497, 23463), 10**6 + 3),
                                        ((132049, 54454), 3 * 10**6 + 17), ((3021377, 1010202), 4 * 1010202)])
def test_lf_persistent_stream_matches_recurrence(lags, count):
    """Bare LF streams long enough for the persistent run (sl >= 4096, at least 4 sl values; the
    first row has ll < 2 sl, so sources also lie in the same link of other producers): every value
    equals the sequential recurrence, nothing is written past the count, the run's status word
    stays zero, and the state continues the sequence through a short (wave-path) call and another
    persistent one."""
    ll, sl = lags
    _say("lf persistent stream", lags, count)
    cfg = _lf_cfg(ll, sl, seed=5)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    out = torch.full((count + 64,), -1, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, count, out)
    torch.cuda.synchronize()
    win = orc.lf_seed(5, ll)
    assert np.array_equal(_u32(out[:count]), orc.lf_generate(ll, sl, win, count))
    assert bool((out[count:] == -1).all())
    hdr = st[:64].cpu().numpy()
    Rr = int(hdr[20:24].view(np.uint32)[0])
    flags = (64 + 4 * Rr + 127) // 128 * 128
    assert int(st[flags:flags + 4].cpu().numpy().view(np.uint32)[0]) == 0
    nxt = torch.empty(1001, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, 1001, nxt)
    again = torch.empty(count, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, count, again)
    torch.cuda.synchronize()
    assert np.array_equal(_u32(nxt), orc.lf_generate(ll, sl, win, 1001))
    assert np.array_equal(_u32(again), orc.lf_generate(ll, sl, win, count))
    del out, again


@pytest.mark.parametrize("lags,count", [((9689, 5502), 4 * 5502 + 10), ((132049, 54454), 3 * 10**6 + 18),
                                        ((3021377, 1010202), 4 * 1010202 + 2), ((19937, 10095), 4 * 10095 + 6)])
def test_lf_persistent_gaussians(lags, count):
    """LF Gaussian streams of a few links: by the persistent uint32 launch (the integers go into the
    output, the lag table; the state's ring takes the last ll of them; every pair is transformed
    after the run), except the third case, whose first 4 n T values come from the producer/consumer
    run and the rest from the waves.  Every Gaussian within 1e-5 of the FP64 oracle, the run's status
    word stays zero, and the state continues the sequence."""
    ll, sl = lags
    cfg = _lf_cfg(ll, sl, seed=8)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    out = torch.empty(count, dtype=torch.float32, device="cuda")
    R.rng_gaussian(cfg, st, count, out)
    assert R.lf_stream_status(st) == 0
    nxt = torch.empty(999, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, 999, nxt)
    torch.cuda.synchronize()
    win = orc.lf_seed(8, ll)
    ref = orc.lf_gaussian(ll, sl, win, count)
    err = float(np.max(np.abs(out.cpu().numpy().astype(np.float64) - ref)))
    _say("lf persistent gaussians", lags, "max abs err", err)
    assert err <= GAUSS_TOL
    assert np.array_equal(_u32(nxt), orc.lf_generate(ll, sl, win, 999))


@pytest.mark.parametrize("lags", [(132049, 54454), (19937, 10095)])
def test_lf_long_gaussian_streams(lags):
    """20 million LF Gaussians by the producer/consumer run (the producers extend the sequence in
    the state's own ring as in the fused LD run, the consumers write the Box-Muller pairs of
    consecutive positions, odd sl included) and the waves for the positions past its 4 n T.  Every
    Gaussian within 1e-5 of the FP64 oracle, the status word stays zero, and the state continues
    the sequence."""
    ll, sl = lags
    count = 2 * 10**7 + 6
    cfg = _lf_cfg(ll, sl, seed=12)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    out = torch.empty(count, dtype=torch.float32, device="cuda")
    R.rng_gaussian(cfg, st, count, out)
    assert R.lf_stream_status(st) == 0
    nxt = torch.empty(999, dtype=torch.int32, device="cuda")
    R.rng_uniform(cfg, st, 999, nxt)
    torch.cuda.synchronize()
    win = orc.lf_seed(12, ll)
    ref = orc.lf_gaussian(ll, sl, win, count)
    err = float(np.max(np.abs(out.cpu().numpy().astype(np.float64) - ref)))
    _say("lf producer/consumer gaussians", lags, "max abs err", err)
    assert err <= GAUSS_TOL
    assert np.array_equal(_u32(nxt), orc.lf_generate(ll, sl, win, 999))
    del out


def test_lf_stream_captured_in_a_graph():
    """rng_uniform on the shared sequence captured in a CUDA graph (the persistent launch is not
    used under capture; the waves are recorded): each replay, with eager work in between, yields
    the next values of the sequence."""
    ll, sl = 9689, 5502
    count = 4 * sl + 100
    cfg = _lf_cfg(ll, sl, seed=3)
    st = R.new_state(cfg)
    R.rng_init(cfg, st)
    out = torch.empty(count, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        R.rng_uniform(cfg, st, count, out)
    torch.cuda.synchronize()
    win = orc.lf_seed(3, ll)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(_u32(out), orc.lf_generate(ll, sl, win, count)), rep
        _ = float((out.float() * 2).sum())  # unrelated eager work between replays


# ---------------------------------------------------------------------------------------------
# the transform over its whole input domain

def test_box_muller_exhaustive_24_bit_domain():
    """Every 24-bit radius input (at angle 0) and every 24-bit angle input (at the largest radius)
    against the FP64 oracle.  A Gaussian r cos(theta) or r sin(theta) is then off by at most
    err_r + r_max err_trig, with err_r the worst radius error over all radius inputs and err_trig
    the worst cosine/sine error over all angle inputs (the final FP32 product's rounding included),
    so that bound covers every pair of words the library can meet."""
    k = np.arange(2**24, dtype=np.uint32) << np.uint32(8)
    zeros = np.zeros_like(k)
    # radius pass: cos 0 = 1 and sin 0 = 0 exactly, so g0 is the radius and g1 is 0
    words = np.stack([k, zeros], 1).ravel()
    d = torch.as_tensor(words.view(np.int32), device="cuda")
    out = torch.empty(words.size, dtype=torch.float32, device="cuda")
    R.rng_box_muller(d, out)
    g = out.cpu().numpy().astype(np.float64)
    ref = orc.box_muller_many(words)
    err_r = float(np.max(np.abs(g[0::2] - ref[0::2])))
    assert np.all(g[1::2] == 0.0)
    r_hat = g[0]  # the largest radius the library produces: u = 2^-24
    r_max = math.sqrt(-2.0 * math.log(2.0**-24))
    assert abs(r_hat - r_max) <= err_r
    # angle pass at the largest radius: the cosine and sine as the library applies them
    words = np.stack([zeros, k], 1).ravel()
    d = torch.as_tensor(words.view(np.int32), device="cuda")
    R.rng_box_muller(d, out)
    g = out.cpu().numpy().astype(np.float64)
    ref = orc.box_muller_many(words)
    err_at_rmax = float(np.max(np.abs(g - ref)))
    theta = 2.0 * math.pi * (k >> np.uint32(8)).astype(np.float64) * 2.0**-24
    err_trig = float(max(np.max(np.abs(g[0::2] / r_hat - np.cos(theta))),
                         np.max(np.abs(g[1::2] / r_hat - np.sin(theta)))))
    bound = err_r + r_max * err_trig
    _say("box-muller exhaustive: radius err", err_r, "trig err", err_trig, "at r_max", err_at_rmax,
         "combined bound", bound)
    assert err_at_rmax <= GAUSS_TOL
    assert bound <= GAUSS_TOL
