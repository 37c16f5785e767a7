"""ctypes binding of librngld (include/rngld.h): same entry-point names, argument marshalling only.

Device buffers are torch CUDA tensors (HIP on ROCm); the library receives their data pointers and
the current stream.  Every compute step runs in librngld's HIP kernels.  If the library has not been
built, importing this module raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librngld.so")

OK, EINVAL, ELAG, ESIZE, EHIP, ENOTSUP = 0, -1, -2, -3, -4, -5
HYBRID_TAUS, RAN2, LAGFIB, LCG, NO_NOISE = 0, 1, 2, 3, 4
KINDS = {"taus": HYBRID_TAUS, "ran2": RAN2, "lf": LAGFIB, "lcg": LCG, "none": NO_NOISE}
NOBS = 6
STATE_ROWS = {HYBRID_TAUS: 4, RAN2: 35, LCG: 1, NO_NOISE: 0}
_ERR_NAMES = {EINVAL: "EINVAL", ELAG: "ELAG", ESIZE: "ESIZE", EHIP: "EHIP", ENOTSUP: "ENOTSUP"}


class RngldError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__("%s failed with %s (%d): %s" % (func, _ERR_NAMES.get(code, "?"), code, msg))
        self.code = code


class Cfg(C.Structure):
    _fields_ = [("kind", C.c_int32), ("lf_ll", C.c_uint32), ("lf_sl", C.c_uint32), ("lf_wave", C.c_uint32),
                ("seed", C.c_uint64), ("n_streams", C.c_uint64), ("stream_base", C.c_uint64),
                ("lf_ring", C.c_uint64), ("lcg_leap", C.c_uint64), ("lf_discard", C.c_uint64)]


class Params(C.Structure):
    _fields_ = [("m", C.c_float), ("k", C.c_float), ("gamma", C.c_float), ("kT", C.c_float), ("dt", C.c_float),
                ("scheme", C.c_int32)]


class Ensemble(C.Structure):
    _fields_ = [("offset", C.c_uint64), ("n", C.c_uint64), ("p", Params), ("pad", C.c_uint32),
                ("seed", C.c_uint64)]


class Obs(C.Structure):
    _fields_ = [("stride", C.c_uint32), ("t0", C.c_uint32)]


class Tuning(C.Structure):
    _fields_ = [("block", C.c_uint32), ("osc_per_thread", C.c_uint32), ("steps_per_launch", C.c_uint32),
                ("blocks_per_cu", C.c_uint32), ("lf_waves", C.c_uint32)]

    def astuple(self):
        return (self.block, self.osc_per_thread, self.steps_per_launch, self.blocks_per_cu, self.lf_waves)


class Loss(C.Structure):
    _fields_ = [("t_begin", C.c_uint32), ("t_end", C.c_uint32), ("K", C.c_uint32), ("flags", C.c_uint32)]


ADJ_REPLAY = 1  # ld_loss.flags: backward by segment replay for every ensemble
ADJ_SPREAD = 2  # ld_loss.flags: ld_run_backward also returns the gradients' standard errors


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("librngld.so is not built (python -m paper_1003_1123_amd.build); there is no fallback")
    L = C.CDLL(LIB_PATH)
    vp, sz, u32, u64, i32 = C.c_void_p, C.c_size_t, C.c_uint32, C.c_uint64, C.c_int32
    P = C.POINTER
    sigs = {
        "rngld_state_bytes": [P(Cfg), P(sz)],
        "rng_init": [P(Cfg), vp, sz, vp],
        "rng_init_ensembles": [P(Cfg), vp, sz, P(Ensemble), u32, vp],
        "rng_uniform": [P(Cfg), vp, sz, u64, vp, u64, vp],
        "rng_gaussian": [P(Cfg), vp, sz, u64, vp, u64, vp],
        "ld_step": [P(Cfg), vp, sz, P(Params), u64, vp, vp, vp],
        "ld_workspace_bytes": [P(Cfg), P(Ensemble), u32, u64, u32, P(Obs), P(sz)],
        "ld_run": [P(Cfg), vp, sz, P(Ensemble), u32, u64, u32, vp, vp, P(Obs), vp, vp, sz, vp],
        "ld_run_noalloc": [P(Cfg), vp, sz, P(Ensemble), u32, u64, u32, vp, vp, P(Obs), vp, vp, vp],
        "ld_get_tuning": [i32, P(Tuning)],
        "ld_set_tuning": [i32, P(Tuning)],
        "ld_autotune": [P(Cfg), P(Ensemble), u32, u64, u32, C.c_char_p, P(Tuning)],
        "ld_plan_create": [P(Cfg), vp, sz, P(Ensemble), u32, u64, u32, vp, vp, P(Obs), vp, vp, sz, vp, P(vp)],
        "ld_plan_launch": [vp, vp],
        "ld_plan_destroy": [vp],
        "ld_ckpt_bytes": [P(Cfg), u64, u32, u32, P(sz)],
        "ld_adjoint_workspace_bytes": [P(Cfg), P(Ensemble), u32, u64, u32, P(Loss), P(sz)],
        "ld_run_ckpt": [P(Cfg), vp, sz, P(Ensemble), u32, u64, u32, vp, vp, P(Loss), vp, sz, vp, vp, sz, vp],
        "ld_run_backward": [P(Cfg), vp, sz, P(Ensemble), u32, u64, u32, P(Loss), vp, vp, sz, vp],
        "rng_box_muller": [vp, u64, vp, vp],
        "rngld_version": [],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.rngld_last_error.argtypes = []
    L.rngld_last_error.restype = C.c_char_p
    return L


lib = _load()

ENTRY_POINTS = ("rngld_state_bytes", "rng_init", "rng_init_ensembles", "rng_uniform", "rng_gaussian", "ld_step",
                "ld_workspace_bytes", "ld_run", "ld_run_noalloc", "ld_get_tuning", "ld_set_tuning", "ld_autotune", "ld_plan_create",
                "ld_plan_launch", "ld_plan_destroy", "ld_ckpt_bytes", "ld_adjoint_workspace_bytes", "ld_run_ckpt",
                "ld_run_backward", "rng_box_muller", "rngld_last_error", "rngld_version")


def _check(rc: int, func: str):
    if rc != OK:
        raise RngldError(rc, func, lib.rngld_last_error().decode())


def last_error() -> str:
    return lib.rngld_last_error().decode()


# ---------------------------------------------------------------------------------------------
# argument helpers

def make_cfg(kind, seed: int = 1234, n_streams: int = 0, stream_base: int = 0, ll: int = 0, sl: int = 0,
             wave: int = 0, ring: int = 0, leap: int = 0, discard: int = 0) -> Cfg:
    k = KINDS[kind] if isinstance(kind, str) else int(kind)
    return Cfg(k, ll, sl, wave, seed & (2**64 - 1), n_streams, stream_base, ring, leap, discard)


def make_params(m=1.0, k=1.0, gamma=1.0, kT=1.0, dt=0.01, scheme: int = 0) -> Params:
    return Params(m, k, gamma, kT, dt, scheme)


def make_ensembles(specs) -> tuple:
    """specs: iterable of (offset, n, Params, seed) -> (ctypes array, count)."""
    specs = list(specs)
    arr = (Ensemble * max(len(specs), 1))()
    for i, (off, n, p, seed) in enumerate(specs):
        arr[i] = Ensemble(off, n, p, 0, seed)
    return arr, len(specs)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ens(ens, n_ens: int):
    """The host ensemble table, checked to hold n_ens entries (the library reads that many)."""
    if n_ens < 0 or (n_ens > 0 and (ens is None or len(ens) < n_ens)):
        have = None if ens is None else len(ens)
        raise ValueError("the ensemble table holds %s entries < n_ens = %d" % (have, n_ens))


def _dev(t: torch.Tensor, dtype, name: str, min_numel: int = 0):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < min_numel:
        raise ValueError("%s holds %d elements < %d" % (name, t.numel(), min_numel))
    return C.c_void_p(t.data_ptr())


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


def _obs_len(obs, n_ens: int, n_steps: int) -> int:
    """Doubles the library writes to d_obs: [n_ens][n_steps / stride + 1][NOBS]."""
    if obs is None or obs.stride == 0:
        return 0
    return n_ens * (n_steps // obs.stride + 1) * NOBS


# ---------------------------------------------------------------------------------------------
# entry points

def rngld_state_bytes(cfg: Cfg) -> int:
    out = C.c_size_t()
    _check(lib.rngld_state_bytes(C.byref(cfg), C.byref(out)), "rngld_state_bytes")
    return out.value


def new_state(cfg: Cfg, device="cuda") -> torch.Tensor:
    """A caller-owned state buffer of the right size (uint8)."""
    return torch.empty(max(rngld_state_bytes(cfg), 1), dtype=torch.uint8, device=device)


def rng_init(cfg: Cfg, state: torch.Tensor):
    _check(lib.rng_init(C.byref(cfg), _dev(state, torch.uint8, "state"), _nbytes(state), _stream()), "rng_init")


def rng_init_ensembles(cfg: Cfg, state: torch.Tensor, ens, n_ens: int):
    _ens(ens, n_ens)
    _check(lib.rng_init_ensembles(C.byref(cfg), _dev(state, torch.uint8, "state"), _nbytes(state), ens, n_ens,
                                  _stream()), "rng_init_ensembles")


def rng_uniform(cfg: Cfg, state: torch.Tensor, per_stream: int, out: torch.Tensor):
    _check(lib.rng_uniform(C.byref(cfg), _dev(state, torch.uint8, "state"), _nbytes(state), per_stream,
                           _dev(out, (torch.uint32, torch.int32), "out"), out.numel(), _stream()), "rng_uniform")


def rng_gaussian(cfg: Cfg, state: torch.Tensor, per_stream: int, out: torch.Tensor):
    _check(lib.rng_gaussian(C.byref(cfg), _dev(state, torch.uint8, "state"), _nbytes(state), per_stream,
                            _dev(out, torch.float32, "out"), out.numel(), _stream()), "rng_gaussian")


def rng_box_muller(words: torch.Tensor, out: torch.Tensor):
    """out[2i], out[2i+1] = Box-Muller pair of words[2i], words[2i+1]."""
    n_pairs = words.numel() // 2
    _check(lib.rng_box_muller(_dev(words, (torch.uint32, torch.int32), "words"), n_pairs,
                              _dev(out, torch.float32, "out", 2 * n_pairs), _stream()), "rng_box_muller")


def ld_step(cfg: Cfg, state: torch.Tensor, params: Params, n: int, x: torch.Tensor, v: torch.Tensor):
    _check(lib.ld_step(C.byref(cfg), _dev(state, torch.uint8, "state"), _nbytes(state), C.byref(params), n,
                       _dev(x, torch.float32, "x", 3 * n), _dev(v, torch.float32, "v", 3 * n), _stream()), "ld_step")


def ld_workspace_bytes(cfg: Cfg, ens, n_ens: int, n_total: int, n_steps: int, obs: Obs | None = None) -> int:
    out = C.c_size_t()
    _ens(ens, n_ens)
    _check(lib.ld_workspace_bytes(C.byref(cfg), ens, n_ens, n_total, n_steps, C.byref(obs) if obs else None,
                                  C.byref(out)), "ld_workspace_bytes")
    return out.value


def ld_run(cfg: Cfg, state: torch.Tensor, ens, n_ens: int, n_total: int, n_steps: int, x: torch.Tensor,
           v: torch.Tensor, obs: Obs | None = None, out_obs: torch.Tensor | None = None,
           ws: torch.Tensor | None = None) -> torch.Tensor:
    """Fused run; returns the workspace used (allocated here when not given)."""
    if ws is None:
        ws = torch.empty(max(ld_workspace_bytes(cfg, ens, n_ens, n_total, n_steps, obs), 256), dtype=torch.uint8,
                         device=x.device)
    d_obs = (_dev(out_obs, torch.float64, "out_obs", _obs_len(obs, n_ens, n_steps)) if out_obs is not None
             else None)
    _ens(ens, n_ens)
    _check(lib.ld_run(C.byref(cfg), _dev(state, torch.uint8, "state"), _nbytes(state), ens, n_ens, n_total, n_steps,
                      _dev(x, torch.float32, "x", 3 * n_total), _dev(v, torch.float32, "v", 3 * n_total),
                      C.byref(obs) if obs else None, d_obs, _dev(ws, torch.uint8, "ws"), _nbytes(ws), _stream()),
           "ld_run")
    return ws


NOALLOC_SCRATCH_BYTES = 48 * 1024 * 1024  # RNGLD_NOALLOC_SCRATCH_BYTES


def ld_run_noalloc(cfg: Cfg, state: torch.Tensor, ens, n_ens: int, n_total: int, n_steps: int, x: torch.Tensor,
                   v: torch.Tensor, obs: Obs | None = None, out_obs: torch.Tensor | None = None,
                   status: torch.Tensor | None = None):
    """ld_run with the library's own per-GPU workspace (nothing is allocated).  `status`: None or a
    device tensor of two 32-bit words that receives the status and lagged-Fibonacci path words."""
    d_obs = (_dev(out_obs, torch.float64, "out_obs", _obs_len(obs, n_ens, n_steps)) if out_obs is not None
             else None)
    d_status = _dev(status, (torch.int32, torch.uint32), "status", 2) if status is not None else None
    _ens(ens, n_ens)
    _check(lib.ld_run_noalloc(C.byref(cfg), _dev(state, torch.uint8, "state"), _nbytes(state), ens, n_ens, n_total,
                              n_steps, _dev(x, torch.float32, "x", 3 * n_total),
                              _dev(v, torch.float32, "v", 3 * n_total), C.byref(obs) if obs else None, d_obs,
                              d_status, _stream()), "ld_run_noalloc")


def ws_status(ws: torch.Tensor) -> int:
    """The workspace status word (synchronises): nonzero after a dataflow run that gave up a wait."""
    torch.cuda.current_stream().synchronize()
    return int(ws[:4].cpu().numpy().view("<u4")[0])


def lf_stream_status(state: torch.Tensor) -> int:
    """Status word of the last persistent rng_uniform / rng_gaussian run on a lagged-Fibonacci
    state (synchronises): nonzero if it gave up a wait, its output then being invalid.  The word
    sits at the first 128-byte boundary after the header and the ring (include/rngld.h)."""
    torch.cuda.current_stream().synchronize()
    R = int(state[20:24].cpu().numpy().view("<u4")[0])
    base = state.data_ptr()
    off = ((base + 64 + 4 * R + 127) & ~127) - base
    return int(state[off:off + 4].cpu().numpy().view("<u4")[0])


LF_PATHS = {1: "dataflow", 2: "waves"}


def ws_lf_path(ws: torch.Tensor) -> str:
    """Which lagged-Fibonacci path the last run on this workspace took (synchronises)."""
    torch.cuda.current_stream().synchronize()
    return LF_PATHS.get(int(ws[4:8].cpu().numpy().view("<u4")[0]), "none")


def ld_get_tuning(kind) -> Tuning:
    t = Tuning()
    _check(lib.ld_get_tuning(KINDS.get(kind, kind) if isinstance(kind, str) else kind, C.byref(t)), "ld_get_tuning")
    return t


def ld_set_tuning(kind, block=256, osc_per_thread=1, steps_per_launch=0, blocks_per_cu=0, lf_waves=0):
    t = Tuning(block, osc_per_thread, steps_per_launch, blocks_per_cu, lf_waves)
    _check(lib.ld_set_tuning(KINDS.get(kind, kind) if isinstance(kind, str) else kind, C.byref(t)), "ld_set_tuning")


def ld_autotune(cfg: Cfg, ens, n_ens: int, n_total: int, n_steps: int, cache_path: str | None = None) -> Tuning:
    t = Tuning()
    _ens(ens, n_ens)
    _check(lib.ld_autotune(C.byref(cfg), ens, n_ens, n_total, n_steps,
                           cache_path.encode() if cache_path else None, C.byref(t)), "ld_autotune")
    return t


class Plan:
    """A captured hipGraph of one ld_run call; launch() replays it on the current stream."""

    def __init__(self, cfg: Cfg, state, ens, n_ens, n_total, n_steps, x, v, obs=None, out_obs=None, ws=None):
        if ws is None:
            ws = torch.empty(max(ld_workspace_bytes(cfg, ens, n_ens, n_total, n_steps, obs), 256),
                             dtype=torch.uint8, device=x.device)
        self._keep = (cfg, state, ens, x, v, obs, out_obs, ws)
        self._h = C.c_void_p()
        d_obs = (_dev(out_obs, torch.float64, "out_obs", _obs_len(obs, n_ens, n_steps)) if out_obs is not None
                 else None)
        _ens(ens, n_ens)
        _check(lib.ld_plan_create(C.byref(cfg), _dev(state, torch.uint8, "state"), _nbytes(state), ens, n_ens,
                                  n_total, n_steps, _dev(x, torch.float32, "x", 3 * n_total),
                                  _dev(v, torch.float32, "v", 3 * n_total), C.byref(obs) if obs else None, d_obs,
                                  _dev(ws, torch.uint8, "ws"), _nbytes(ws), _stream(), C.byref(self._h)),
               "ld_plan_create")

    def launch(self):
        _check(lib.ld_plan_launch(self._h, _stream()), "ld_plan_launch")

    def close(self):
        if self._h:
            lib.ld_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ld_ckpt_bytes(cfg: Cfg, n_total: int, n_steps: int, K: int) -> int:
    out = C.c_size_t()
    _check(lib.ld_ckpt_bytes(C.byref(cfg), n_total, n_steps, K, C.byref(out)), "ld_ckpt_bytes")
    return out.value


def ld_adjoint_workspace_bytes(cfg: Cfg, ens, n_ens: int, n_total: int, n_steps: int, loss: Loss) -> int:
    out = C.c_size_t()
    _ens(ens, n_ens)
    _check(lib.ld_adjoint_workspace_bytes(C.byref(cfg), ens, n_ens, n_total, n_steps, C.byref(loss), C.byref(out)),
           "ld_adjoint_workspace_bytes")
    return out.value


def ld_run_ckpt(cfg: Cfg, state, ens, n_ens, n_total, n_steps, x, v, loss: Loss, ckpt, out_loss, ws):
    _ens(ens, n_ens)
    _check(lib.ld_run_ckpt(C.byref(cfg), _dev(state, torch.uint8, "state"), _nbytes(state), ens, n_ens, n_total,
                           n_steps, _dev(x, torch.float32, "x", 3 * n_total), _dev(v, torch.float32, "v", 3 * n_total),
                           C.byref(loss), _dev(ckpt, torch.uint8, "ckpt"), _nbytes(ckpt),
                           _dev(out_loss, torch.float64, "out_loss", n_ens), _dev(ws, torch.uint8, "ws"),
                           _nbytes(ws), _stream()), "ld_run_ckpt")


def ld_run_backward(cfg: Cfg, ckpt, ens, n_ens, n_total, n_steps, loss: Loss, out_grad, ws):
    """out_grad: [n_ens][3] doubles, or [n_ens][6] (gradients, standard errors) with ADJ_SPREAD."""
    _ens(ens, n_ens)
    width = 6 if loss.flags & ADJ_SPREAD else 3
    _check(lib.ld_run_backward(C.byref(cfg), _dev(ckpt, torch.uint8, "ckpt"), _nbytes(ckpt), ens, n_ens, n_total,
                               n_steps, C.byref(loss), _dev(out_grad, torch.float64, "out_grad", width * n_ens),
                               _dev(ws, torch.uint8, "ws"), _nbytes(ws), _stream()), "ld_run_backward")
