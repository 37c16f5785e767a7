"""C-ABI checks that need no GPU: the library loads, exports every entry point the header
declares, and rejects bad arguments on the host (validation happens before any HIP call)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
R = pytest.importorskip("paper_1003_1123_amd._lib")


def _declared():
    src = open(os.path.join(ROOT, "include", "rngld.h")).read()
    return sorted(set(re.findall(r"RNGLD_API\s+(?:int|const char \*)\s*\*?\s*([a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_paper_path_entry_points():
    names = _declared()
    for required in ("rng_init", "rng_uniform", "rng_gaussian", "ld_step", "ld_run", "ld_run_backward"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(R.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared()) == set(R.ENTRY_POINTS)


def test_only_the_c_abi_is_exported():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", R.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert exported == set(_declared())


def test_generator_kinds_match_header():
    src = open(os.path.join(ROOT, "include", "rngld.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define RNGLD_([A-Z0-9_]+)\s+(-?\d+)", src)}
    assert {k: defs[n] for k, n in (("taus", "HYBRID_TAUS"), ("ran2", "RAN2"), ("lf", "LAGFIB"), ("lcg", "LCG"),
                                           ("none", "NO_NOISE"))} \
        == R.KINDS


def test_struct_layouts_match_header():
    assert C.sizeof(R.Cfg) == 64 and R.Cfg.lcg_leap.offset == 48 and R.Cfg.lf_discard.offset == 56
    assert C.sizeof(R.Params) == 24 and C.sizeof(R.Ensemble) == 56
    assert C.sizeof(R.Obs) == 8 and C.sizeof(R.Tuning) == 20 and C.sizeof(R.Loss) == 16
    assert R.Ensemble.seed.offset == 48 and R.Ensemble.p.offset == 16


def _code(fn, *args):
    return fn(*args)


def test_state_bytes():
    out = C.c_size_t()
    assert R.lib.rngld_state_bytes(C.byref(R.make_cfg("taus", n_streams=1000)), C.byref(out)) == 0 and out.value == 16000
    assert R.lib.rngld_state_bytes(C.byref(R.make_cfg("ran2", n_streams=1000)), C.byref(out)) == 0 and out.value == 140000
    assert R.lib.rngld_state_bytes(C.byref(R.make_cfg("lcg", n_streams=1000)), C.byref(out)) == 0 and out.value == 4000
    assert R.lib.rngld_state_bytes(C.byref(R.make_cfg("lcg", n_streams=7, leap=4)), C.byref(out)) == 0 and out.value == 28
    assert R.lib.rngld_state_bytes(C.byref(R.make_cfg("none", n_streams=10**6)), C.byref(out)) == 0 and out.value == 0
    def lf_bytes(ll, sl, R):
        # header and ring; 128-byte aligned, the bare-stream runs' status line and progress words
        # (a line per producer and per consumer); 256-byte aligned, the stream run's padded ring of
        # ceil(2 (ll + sl) / sl) links of sl words rounded up to 64 (when sl >= 256 and it fits)
        up = lambda v, a: (v + a - 1) // a * a
        size = up(64 + 4 * R, 128) + 128 + 2 * 8192 * 32 * 4
        nr, slp = -(-2 * (ll + sl) // sl), up(sl, 64)
        if sl >= 256 and nr * slp < 2**29 and nr * sl < 2**31:
            size = up(size, 256) + 4 * nr * slp
        return size

    assert R.lib.rngld_state_bytes(C.byref(R.make_cfg("lf", ll=2281, sl=1252)), C.byref(out)) == 0
    assert out.value == lf_bytes(2281, 1252, 2 * (2281 + 1252)) == 2156544
    assert R.lib.rngld_state_bytes(C.byref(R.make_cfg("lf", ll=2281, sl=1252, wave=101)), C.byref(out)) == 0
    assert out.value == lf_bytes(2281, 1252, 2 * (2281 + 1252))  # default ring 2 (ll + sl) whatever the wave width
    assert R.lib.rngld_state_bytes(C.byref(R.make_cfg("lf", ll=2281, sl=1252, wave=101, ring=2400)), C.byref(out)) == 0
    assert out.value == lf_bytes(2281, 1252, 2400)
    # lags whose doubled sum reaches 2^30 fall back to a ring of ll + sl (and no stream ring: too long)
    assert R.lib.rngld_state_bytes(C.byref(R.make_cfg("lf", ll=600_000_001, sl=1000)), C.byref(out)) == 0
    assert out.value == lf_bytes(600_000_001, 1000, 600_000_001 + 1000)
    # short lags: no stream ring (sl < 256)
    assert R.lib.rngld_state_bytes(C.byref(R.make_cfg("lf", ll=97, sl=33)), C.byref(out)) == 0
    assert out.value == lf_bytes(97, 33, 2 * (97 + 33)) == 1152 + 128 + 2 * 8192 * 32 * 4
    # ring shorter than ll + W (W = 100 after rounding down to a multiple of 4)
    assert R.lib.rngld_state_bytes(C.byref(R.make_cfg("lf", ll=2281, sl=1252, wave=101, ring=2380)),
                                   C.byref(out)) == R.ELAG


def test_no_noise_kind_generates_no_numbers():
    c = R.make_cfg("none")
    assert R.lib.rng_uniform(C.byref(c), None, 0, 4, None, 0, None) == R.ENOTSUP
    assert R.lib.rng_gaussian(C.byref(c), None, 0, 4, None, 0, None) == R.ENOTSUP


@pytest.mark.parametrize("cfg,code", [
    (dict(kind="lf", ll=100, sl=100), R.ELAG),
    (dict(kind="lf", ll=100, sl=0), R.ELAG),
    (dict(kind="lf", ll=2281, sl=1252, wave=2000), R.ELAG),
    (dict(kind="lf", ll=2281, sl=1252, wave=3), R.ELAG),
    (dict(kind="lf", ll=2281, sl=1252, ring=2281), R.ELAG),
    (dict(kind=7), R.EINVAL),
    (dict(kind="taus", n_streams=2**40), R.EINVAL),
])
def test_bad_configs(cfg, code):
    out = C.c_size_t()
    c = R.make_cfg(cfg.pop("kind"), **cfg)
    assert R.lib.rngld_state_bytes(C.byref(c), C.byref(out)) == code
    assert R.last_error()


def test_null_cfg_and_outputs():
    assert R.lib.rngld_state_bytes(None, None) == R.EINVAL
    c = R.make_cfg("taus", n_streams=10)
    assert R.lib.rngld_state_bytes(C.byref(c), None) == R.EINVAL


def test_entry_points_validate_before_touching_the_device():
    c = R.make_cfg("taus", n_streams=100)
    fake = C.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    assert R.lib.rng_init(C.byref(c), fake, 100, None) == R.ESIZE
    assert R.lib.rng_init(C.byref(c), None, 1600, None) == R.EINVAL
    assert R.lib.rng_uniform(C.byref(c), fake, 1600, 10, fake, 999, None) == R.ESIZE
    assert R.lib.rng_gaussian(C.byref(c), fake, 1600, 3, fake, 10**6, None) == R.EINVAL  # odd count
    p = R.make_params(m=0.0)
    assert R.lib.ld_step(C.byref(c), fake, 1600, C.byref(p), 10, fake, fake, None) == R.EINVAL
    p = R.make_params(dt=float("nan"))
    assert R.lib.ld_step(C.byref(c), fake, 1600, C.byref(p), 10, fake, fake, None) == R.EINVAL
    p = R.make_params(scheme=3)
    assert R.lib.ld_step(C.byref(c), fake, 1600, C.byref(p), 10, fake, fake, None) == R.EINVAL
    p = R.make_params()
    assert R.lib.ld_step(C.byref(c), fake, 1600, C.byref(p), 101, fake, fake, None) == R.ESIZE  # n > S
    assert R.lib.ld_step(C.byref(c), fake, 1600, C.byref(p), 0, None, None, None) == R.OK       # empty


def test_run_validation_and_workspace_sizing():
    c = R.make_cfg("taus", n_streams=1000)
    p = R.make_params()
    ens, n = R.make_ensembles([(0, 600, p, 1), (600, 400, p, 2)])
    ws = C.c_size_t()
    obs = R.Obs(10, 50)
    assert R.lib.ld_workspace_bytes(C.byref(c), ens, n, 1000, 100, C.byref(obs), C.byref(ws)) == R.OK
    tiles = 3 + 2  # 256-oscillator tiles
    assert ws.value >= 256 + tiles * 11 * 6 * 8 + 6 * 1000 * 4
    # overlapping ensembles
    bad, nb = R.make_ensembles([(0, 600, p, 1), (500, 400, p, 2)])
    assert R.lib.ld_workspace_bytes(C.byref(c), bad, nb, 1000, 100, None, C.byref(ws)) == R.EINVAL
    # outside n_total
    bad, nb = R.make_ensembles([(900, 200, p, 1)])
    assert R.lib.ld_workspace_bytes(C.byref(c), bad, nb, 1000, 100, None, C.byref(ws)) == R.EINVAL
    # more oscillators than streams
    assert R.lib.ld_workspace_bytes(C.byref(c), ens, n, 2000, 100, None, C.byref(ws)) == R.ESIZE
    # t0 beyond the run
    obs = R.Obs(10, 500)
    assert R.lib.ld_workspace_bytes(C.byref(c), ens, n, 1000, 100, C.byref(obs), C.byref(ws)) == R.EINVAL
    # lagged Fibonacci runs one ensemble
    lf = R.make_cfg("lf", ll=2281, sl=1252)
    assert R.lib.ld_workspace_bytes(C.byref(lf), ens, n, 1000, 100, None, C.byref(ws)) == R.ENOTSUP
    # a too-small workspace is rejected before any launch
    fake = C.c_void_p(0x1000)
    assert R.lib.ld_run(C.byref(c), fake, 16000, ens, n, 1000, 100, fake, fake, None, None, fake, 8,
                        None) == R.ESIZE


def test_tuning_roundtrip_and_validation():
    t = R.ld_get_tuning("taus")
    assert t.astuple() == (256, 1, 0, 0, 0)
    with pytest.raises(R.RngldError):
        R.ld_set_tuning("taus", block=100)
    with pytest.raises(R.RngldError):
        R.ld_set_tuning("taus", osc_per_thread=3)
    R.ld_set_tuning("ran2", block=128, osc_per_thread=2, steps_per_launch=50, blocks_per_cu=4)
    assert R.ld_get_tuning("ran2").astuple() == (128, 2, 50, 4, 0)
    R.ld_set_tuning("ran2")
    assert R.ld_get_tuning("ran2").astuple() == (256, 1, 0, 0, 0)
    with pytest.raises(R.RngldError):
        R.ld_set_tuning("lf", lf_waves=2)


def test_adjoint_sizing_and_validation():
    c = R.make_cfg("taus", n_streams=1000)
    # 20 checkpoints plus the end state: x, v, the 4 state rows and the 6 adjoint rows
    assert R.ld_ckpt_bytes(c, 1000, 2000, 100) == 21 * 1000 * (6 + 4 + 6) * 4
    assert R.ld_ckpt_bytes(c, 1000, 2001, 100) == 22 * 1000 * (6 + 4 + 6) * 4
    # Ran2: x, v, the 35 state rows and the 6 adjoint rows
    assert R.ld_ckpt_bytes(R.make_cfg("ran2", n_streams=1000), 1000, 2000, 100) == 21 * 1000 * (6 + 35 + 6) * 4
    p = R.make_params()
    ens, n = R.make_ensembles([(0, 1000, p, 1)])
    loss = R.Loss(1001, 2000, 100, 0)
    scratch = 9 * 100 * 1000 * 4  # replay: 9 floats per oscillator-step of one segment
    records = 20 * 1000 * 3 * 8  # register-only backward: 24 bytes per (oscillator, segment)
    fwd_records = 20 * 1000 * 13 * 4  # segment-parallel forward: 52 bytes per (oscillator, segment)
    small = 64 * 1024  # ensemble tables, per-tile partials, jump and coefficient tables
    # weakly damped Hybrid Taus: segment-parallel forward and register-only backward share the space
    ws = R.ld_adjoint_workspace_bytes(c, ens, n, 1000, 2000, loss)
    assert max(records, fwd_records) <= ws < max(records, fwd_records) + small
    assert R.ld_adjoint_workspace_bytes(c, ens, n, 1000, 2000, R.Loss(1001, 2000, 100, R.ADJ_SPREAD)) == ws
    # forced replay and strong damping (gamma dt = 0.05 at K = 100) need the replay scratch
    ws_r = R.ld_adjoint_workspace_bytes(c, ens, n, 1000, 2000, R.Loss(1001, 2000, 100, R.ADJ_REPLAY))
    assert scratch <= ws_r < scratch + small
    ens5, n5 = R.make_ensembles([(0, 500, p, 1), (500, 500, R.make_params(gamma=5.0), 2)])
    assert R.ld_adjoint_workspace_bytes(c, ens5, n5, 1000, 2000, loss) >= scratch + records  # both paths
    # weakly damped Ran2: sequential forward, register-only backward (no replay scratch)
    c2 = R.make_cfg("ran2", n_streams=1000)
    assert records <= R.ld_adjoint_workspace_bytes(c2, ens, n, 1000, 2000, loss) < records + small
    assert scratch <= R.ld_adjoint_workspace_bytes(c2, ens, n, 1000, 2000, R.Loss(1001, 2000, 100, R.ADJ_REPLAY))
    with pytest.raises(R.RngldError) as e:
        R.ld_adjoint_workspace_bytes(c, ens, n, 1000, 2000, R.Loss(0, 2000, 100, 0))
    assert e.value.code == R.EINVAL
    with pytest.raises(R.RngldError) as e:
        R.ld_adjoint_workspace_bytes(c, ens, n, 1000, 2000, R.Loss(1001, 2000, 100, 4))  # unknown flag
    assert e.value.code == R.EINVAL
    with pytest.raises(R.RngldError) as e:
        R.ld_ckpt_bytes(R.make_cfg("lf", ll=2281, sl=1252), 1000, 2000, 100)
    assert e.value.code == R.ENOTSUP
    p0 = R.make_params(kT=0.0)
    ens0, n0 = R.make_ensembles([(0, 1000, p0, 1)])
    with pytest.raises(R.RngldError):
        R.ld_adjoint_workspace_bytes(c, ens0, n0, 1000, 2000, loss)


def test_observable_buffer_length_follows_the_header():
    # double[n_ens][n_steps / stride + 1][6]
    assert R._obs_len(R.Obs(stride=10, t0=500), 1, 1000) == 101 * 6
    assert R._obs_len(R.Obs(stride=100, t0=0), 3, 250) == 3 * 3 * 6
    assert R._obs_len(None, 4, 1000) == 0
    assert R.NOBS == 6


def test_ensemble_table_shorter_than_n_ens_is_rejected_before_the_library():
    p = R.make_params(1.0, 1.0, 1.0, 1.0, 0.01)
    ens, n = R.make_ensembles([(0, 64, p, 1), (64, 64, p, 2)])
    assert n == 2
    R._ens(ens, 2)
    R._ens(ens, 0)
    with pytest.raises(ValueError):
        R._ens(ens, 3)
    with pytest.raises(ValueError):
        R._ens(None, 1)
    with pytest.raises(ValueError):
        R.ld_workspace_bytes(R.make_cfg("taus", n_streams=128), ens, 3, 128, 10)
