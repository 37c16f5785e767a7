#!/usr/bin/env python3
"""Throughput of the fused RNG + Langevin-dynamics path on one MI355X.

One benchmark step = the config-2 workload for all three generators: seed the generator, then
run N = 1e6 independent 3-D oscillators for 1e4 LD steps (dt = 0.005, m = k = kT = gamma = 1) with
the Gaussian forces generated on the fly and observables recorded every 100 steps -- Hybrid Taus,
Ran2 (32-entry table) and lagged Fibonacci (ll, sl) = (3021377, 1010202).  `value` is the
oscillator-steps per second of that whole step.  The bare generators (config 3, with the per-stream
LCG as a speed reference), the batched run (config 4), the adjoint (config 5) and the Fig. 6 time
breakdown over N are measured once after the timed steps and reported as extra fields; the CPU
oracle is timed on a bounded sample of the config-2 workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "oscillator-steps/s fused LD+RNG; Gaussians/s; plain vs batched/adjoint"
GENERATORS = ("taus", "ran2", "lf")

# Work per oscillator-step.
# Taus and Ran2 are bound by vector-ALU issue: the lane-instructions that the compiled step loop of
# ld_run_kernel (underdamped scheme, gfx950) issues per oscillator-step, LDS accesses not counted,
# as the build counts them in the assembly it compiles (kernel_isa.json, "step_loops").
STEP_LOOP_KERNELS = {"taus": "ld_run_kernel<HybridTaus,256,1>", "ran2": "ld_run_kernel<Ran2,256,1>",
                     "lcg": "ld_run_kernel<Lcg32,256,1>", "adjoint_forward": "ld_fwd_seg_kernel<256>",
                     "adjoint_backward": "ld_adjoint_seg_kernel<HybridTaus,256>"}
# Measured bound of those loops: each instruction class at the issue rate the VALU probe measured
# for it (profiles/valu_issue_rates.md, lane-instructions per second over the chip), times added
# (transcendentals do not overlap other VALU work), except that a 32-bit multiply interleaved with
# other integer work costs what the probe's mixed multiply + xor kernel shows (1.2e-14 s of chip
# time per lane-operation, against 3.0e-14 alone).  Class of each opcode of the compiled loop:
VALU_CLASS_RATES = {"transcendental": 1.905e13, "mul32": 1.0 / 1.2e-14, "cvt": 3.534e13, "three_operand": 3.433e13,
                    "fp32": 5.951e13, "other": 4.917e13}
VALU_CLASSES = {
    "transcendental": ("v_log_f32", "v_exp_f32", "v_sqrt_f32", "v_rsq_f32", "v_rcp_f32", "v_sin_f32", "v_cos_f32"),
    "mul32": ("v_mul_lo_u32", "v_mul_hi_u32", "v_mul_hi_i32", "v_mad_u64_u32", "v_mad_i64_i32"),
    "cvt": ("v_cvt_f32_u32", "v_cvt_f32_i32", "v_cvt_u32_f32", "v_cvt_i32_f32"),
    "three_operand": ("v_and_or_b32", "v_bitop3_b32", "v_alignbit_b32", "v_mad_u32_u24", "v_lshl_add_u32",
                      "v_lshl_or_b32", "v_or3_b32", "v_add3_u32", "v_xad_u32", "v_bfe_u32", "v_bfi_b32",
                      "v_perm_b32", "v_cndmask_b32_e64", "v_add_lshl_u32"),
    "fp32": ("v_mul_f32", "v_add_f32", "v_sub_f32", "v_fma_f32", "v_fmac_f32", "v_mac_f32", "v_fmamk_f32",
             "v_fmaak_f32"),
    "unmeasured": ("v_add_f64", "v_mul_f64", "v_fma_f64", "v_fmac_f64", "v_cvt_f64_f32", "v_cvt_f32_f64"),
}


def valu_classes(by_opcode):
    """Instruction counts of a loop by issue class."""
    out = {}
    for op, n in by_opcode.items():
        cls = "other"
        for c, names in VALU_CLASSES.items():
            if any(op == nm or op.startswith(nm + "_e") for nm in names) or op in names:
                cls = c
                break
        out[cls] = out.get(cls, 0) + n
    return out


def valu_mix_bound(which):
    """Oscillator-steps/s a step loop's instruction mix allows at the measured per-class issue rates
    (None when it holds instructions the probe did not measure, e.g. FP64)."""
    loops = _kernel_isa().get("step_loops", {})
    name = STEP_LOOP_KERNELS[which]
    if name not in loops:
        return None
    cls = valu_classes(loops[name]["by_opcode"])
    if cls.get("unmeasured"):
        return None
    return 1.0 / sum(n / VALU_CLASS_RATES[c] for c, n in cls.items())


# VALU lane-operation peak: 256 CUs x 128 lanes per clock x 2.4 GHz (the published 157.3 TFLOP/s FP32
# vector rate counts an FMA as two flops).
ALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
# Lagged Fibonacci: each of the 4 numbers of an oscillator-step reads two earlier numbers and is
# written once, 4 B each (Alg. 3); the wave path also moves x and v (6 x 4 B each way) per step.
LF_ALGO_BYTES_PER_OSC_STEP = 4 * 12
# One launch per LD step (the paper's protocol), bytes per oscillator-step: x and v (6 floats) read
# and written, and the generator state: Taus 4 words read and written; Ran2 its 3 words read and
# written plus, for each of the 4 draws, the one table entry the draw selects (read and written).
STEP_BYTES_PER_OSC_STEP = {"taus": 2 * 4 * 4 + 48, "ran2": 2 * 3 * 4 + 2 * 4 * 4 + 48, "none": 48}
# What the memory system moves for the Ran2 step at 128-byte lines: a line holds one table slot of 32
# streams and is left alone only if none of them selects that slot in its 4 draws, (7/8)^32 = 1.4%
# of lines, so the whole 128-byte table row of each stream is read and written.
STEP_LINE_BYTES_RAN2 = 2 * 3 * 4 + 2 * 32 * 4 + 48
LF_WAVE_XV_BYTES_PER_OSC_STEP = 48
HBM_PEAK_GBS = 8000.0
# Measured peak for the lagged-Fibonacci run's traffic: device-scope 16-byte loads and stores, two
# loads per store, over a 32 MB region, stores 256-byte aligned and loads 13 words off (as the run's
# long-lag reads), from the wide-access measurement (profiles/wide_access.md, mode 4).
LF_MEASURED_PEAK_GBS = 8130.0
# Bytes past the L2 per launch (to the memory-side cache or HBM: the DRAM-destined request counters
# TCC_EA0_RDREQ_DRAM / TCC_EA0_WRREQ_DRAM count the same requests, and no counter here separates
# the memory-side cache's hits) from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch) at the
# config-2 workload, scaled by what the same counters read for a plain 1 GiB device copy
# (FETCH_SIZE 0.5 GiB: factor 2; WRITE_SIZE 1 GiB: factor 1).  Valid only for the machine code they
# were taken on: the SHA-256 of the gfx950 assembly of the kernel's 8-tile LD instantiation (the one
# this workload runs), which the build records in kernel_isa.json; otherwise the traffic is null.
COUNTER_TRAFFIC = {
    "lf_pc_kernel": {
        "isa_sha256": "25a307333814a2731e5c60e7c4b706f3aef40a24cd6afbd8aa5f9d0e5bb2c2c2",
        # FETCH_SIZE 160394855.0625 KiB x (2^20 / 524308.1875), WRITE_SIZE 158418655.1875 KiB x (2^20 / 1048576)
        "fetch_bytes": 328476015330, "write_bytes": 162220702912,
    },
}


def _kernel_isa():
    path = os.path.join(ROOT, "paper_1003_1123_amd", "kernel_isa.json")
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def built_isa(kernel):
    return _kernel_isa().get(kernel, {}).get("sha256")


def valu_per_osc_step(which):
    """VALU lane-instructions per iteration of a kernel's compiled step loop (one oscillator-step)."""
    loops = _kernel_isa().get("step_loops", {})
    name = STEP_LOOP_KERNELS[which]
    if name not in loops:
        raise RuntimeError("kernel_isa.json has no step-loop count for %s: rebuild the library" % name)
    return loops[name]["valu_per_iteration"]


def windowed_valu(which, n_steps, t_begin, t_end):
    """VALU lane-instructions per oscillator-step of an adjoint kernel (forward or backward),
    averaged over the run: its plain step loop (the smallest) outside the loss window, the loop
    that also handles the window's terms (the largest) inside it."""
    loop = _kernel_isa().get("step_loops", {}).get(STEP_LOOP_KERNELS[which])
    if loop is None:
        raise RuntimeError("kernel_isa.json has no step-loop count for %s: rebuild the library" % which)
    inside = t_end - t_begin + 1
    return ((n_steps - inside) * min(loop["all_loops"]) + inside * loop["valu_per_iteration"]) / n_steps


def valu_entry(kernel, valu_per_unit, units, seconds, mix_bound_units_per_s=None):
    """VALU roofline of `units` oscillator-steps (each `valu_per_unit` lane-instructions) in `seconds`."""
    achieved = valu_per_unit * units / seconds / 1e12
    out = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / ALU_PEAK_TOPS,
           "kernel": kernel, "valu_lane_instr_per_osc_step": valu_per_unit, "osc_steps_per_s": units / seconds}
    if mix_bound_units_per_s:
        pm = valu_per_unit * mix_bound_units_per_s / 1e12
        out.update({"peak_measured": pm, "frac_measured": achieved / pm,
                    "peak_measured_how": "instruction mix of the step loop at the probe's per-class issue rates"})
    return out


def counter_traffic(kernel):
    c = COUNTER_TRAFFIC.get(kernel)
    if c is None or built_isa(kernel) != c["isa_sha256"]:
        return None
    return c["fetch_bytes"] + c["write_bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", default="", help="comma list of generators (profiling runs)")
    ap.add_argument("--extras", default="", help="comma list of extras to run (profiling runs; default: all but step_protocol and wave_rounds)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device (a plain copy of known size, for scaling "
                         "hardware byte counters)")
    return ap.parse_args()


class Config2:
    def __init__(self, R, W, torch, kinds):
        c = W.C2
        self.R, self.torch = R, torch
        self.N, self.T, self.seed = c["N"], c["steps"], c["seed"]
        p = c["params"].as_f32()
        self.params = R.make_params(p.m, p.k, p.gamma, p.kT, p.dt)
        self.ll, self.sl = c["lf_lags"]
        self.kinds = kinds
        self.stride = 100
        self.P = self.T // self.stride + 1
        N = self.N
        self.x = torch.zeros(3 * N, dtype=torch.float32, device="cuda")
        self.v = torch.zeros_like(self.x)
        self.obs = {k: torch.zeros(self.P * R.NOBS, dtype=torch.float64, device="cuda") for k in kinds}
        self.cfg, self.state, self.ws = {}, {}, {}
        self.ens, self.n_ens = R.make_ensembles([(0, N, self.params, 0)])
        for k in kinds:
            cfg = R.make_cfg(k, seed=self.seed, n_streams=N, ll=self.ll if k == "lf" else 0,
                             sl=self.sl if k == "lf" else 0)
            self.cfg[k] = cfg
            self.state[k] = R.new_state(cfg)
            self.ws[k] = torch.empty(max(R.ld_workspace_bytes(cfg, self.ens, 1, N, self.T, R.Obs(self.stride, 0)),
                                         256), dtype=torch.uint8, device="cuda")
        self.events = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                       for k in kinds}

    def step(self):
        R = self.R
        times = {}
        for k in self.kinds:
            e0, e1 = self.events[k]
            R.rng_init(self.cfg[k], self.state[k])
            self.x.zero_()
            self.v.zero_()
            e0.record()
            R.ld_run(self.cfg[k], self.state[k], self.ens, 1, self.N, self.T, self.x, self.v,
                     R.Obs(self.stride, 0), self.obs[k], self.ws[k])
            e1.record()
        return times

    def elapsed(self):
        return {k: self.events[k][0].elapsed_time(self.events[k][1]) for k in self.kinds}

    def check_status(self):
        """Every run of the step finished without a failed wait (a persistent lagged-Fibonacci run
        that gives up stops early and marks its results invalid: its time must not be reported)."""
        for k in self.kinds:
            st = self.R.ws_status(self.ws[k])
            if st != 0:
                raise RuntimeError("the %s run reported status %d: its results are invalid" % (k, st))


def roofline_entry(kind, ms_run, N, T, lf_path=None):
    """Roofline of one ld_run of N oscillators x T steps.  The events bracket the whole ld_run call
    on the stream its kernels run on; the kernel is all but a few microseconds of it."""
    osc_steps = N * T
    if kind == "lf":
        if lf_path == "dataflow":
            kernel, launches, per_os = "lf_pc_kernel", 1, LF_ALGO_BYTES_PER_OSC_STEP
        else:
            kernel, launches = "lf_ld_phase_kernel", 4 * T
            per_os = LF_ALGO_BYTES_PER_OSC_STEP + LF_WAVE_XV_BYTES_PER_OSC_STEP
        per_launch_s = ms_run / 1e3 / launches
        per_launch_bytes = per_os * osc_steps / launches
        achieved = per_launch_bytes / per_launch_s / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(kernel), "kernel": kernel,
                "memory_level": ("memory-side cache: the run's ring (about 32 MB) stays resident in the "
                                 "256 MB infinity cache behind the device-scope accesses, which bypass the "
                                 "XCDs' L2; 'frac' is against the nominal HBM peak only as the contract's "
                                 "reference, 'frac_measured' against what this access mix sustains"),
                "peak_measured": LF_MEASURED_PEAK_GBS, "frac_measured": achieved / LF_MEASURED_PEAK_GBS,
                "peak_measured_how": "device-scope 16-byte loads and stores, 2 loads + 1 store per word, over "
                                     "a 32 MB region (profiles/wide_access.md, mode 4)",
                "lf_path": lf_path, "launches": launches, "avg_launch_us": per_launch_s * 1e6,
                "algorithmic_bytes_per_osc_step": per_os, "algorithmic_bytes_per_launch": per_launch_bytes}
    per_launch_s = ms_run / 1e3
    vpos = valu_per_osc_step(kind)
    e = valu_entry("ld_run_kernel<%s>" % kind, vpos, osc_steps, per_launch_s, valu_mix_bound(kind))
    e.update({"traffic": counter_traffic(e["kernel"]), "launches": 1, "avg_launch_us": per_launch_s * 1e6,
              "algorithmic_ops_per_launch": vpos * osc_steps})
    return e


def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = None
    return {"model": model, "nproc": os.cpu_count(), "available_to_process": avail}


def measured_hbm_copy(torch):
    """An elementwise copy of 2 GiB (read + write), best of three: a measured HBM peak.  (An
    elementwise kernel, so that profiling runs keep the runtime's copy kernel for calibration.)"""
    src = torch.empty(2**29, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    best = None
    for _ in range(3):
        a, b = _ev(torch)
        a.record()
        torch.mul(src, 1.0, out=dst)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2 * 2**31 / (best / 1e3) / 1e9


def cpu_baseline(W):
    """The FP64 oracle on a bounded sample of config 2: N = 3e4 oscillators x 1000 steps per
    generator (about 12 s), single thread, same parameters and lags."""
    import numpy as np
    import oracle as orc

    c = W.C2
    p = c["params"].as_f32().asdict()
    N, T = 30_000, 1000
    ll, sl = c["lf_lags"]
    total_t, total_os = 0.0, 0
    per = {}
    for kind in GENERATORS:
        st = orc.lf_seed(c["seed"], ll) if kind == "lf" else orc.seed_states(kind, c["seed"], np.arange(N))
        t = time.perf_counter()
        orc.ld_run(kind, st, N, T, p, ll=ll, sl=sl, stride=100)
        dt = time.perf_counter() - t
        per[kind] = N * T / dt
        total_t += dt
        total_os += N * T
    return {"value": total_os / total_t, "unit": "oscillator-steps/s", "cores": 1, "kind": "oracle",
            "host": host_cpu(),
            "sample": "config-2 workload at N=3e4 oscillators x 1000 steps per generator (3 x 3e7 "
                      "oscillator-steps, %.1f s), FP64, one thread" % total_t,
            "per_generator": per, "all_cores": cpu_all_cores(W, per["lf"])}


def _oracle_slice(args):
    """One worker of the all-cores leg: the oracle on oscillators [lo, hi) (their own streams)."""
    kind, seed, lo, hi, T, p = args
    import numpy as np
    import oracle as orc

    st = orc.seed_states(kind, seed, np.arange(lo, hi))
    orc.ld_run(kind, st, hi - lo, T, p, stride=100)


def _oracle_warm(_):
    import numpy  # noqa: F401
    import oracle  # noqa: F401


def cpu_all_cores(W, lf_rate):
    """The same oracle on every host core the process may use: Taus and Ran2 oscillators split over
    worker processes (each oscillator has its own stream, so the split changes no value); the lagged
    Fibonacci run stays on one core, its numbers being one sequence."""
    import multiprocessing as mp

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    c = W.C2
    p = c["params"].as_f32().asdict()
    per_core, T = 10_000, 1000
    N = per_core * cores
    per = {"lf": lf_rate}
    with mp.get_context("spawn").Pool(cores) as pool:
        pool.map(_oracle_warm, range(cores), chunksize=1)  # worker start-up is not timed
        for kind in ("taus", "ran2"):
            jobs = [(kind, c["seed"], i * per_core, (i + 1) * per_core, T, p) for i in range(cores)]
            t = time.perf_counter()
            pool.map(_oracle_slice, jobs, chunksize=1)
            per[kind] = N * T / (time.perf_counter() - t)
    value = len(GENERATORS) / sum(1.0 / per[k] for k in GENERATORS)
    return {"value": value, "unit": "oscillator-steps/s", "cores": cores, "per_generator": per,
            "sample": "Taus and Ran2: %d processes x 1e4 oscillators x 1000 steps each; lagged Fibonacci: "
                      "the one-thread figure (one sequence)" % cores}


def _c3_slice(args):
    """One worker of the config-3 all-cores leg: uniform streams [lo, hi) of the oracle."""
    kind, seed, lo, hi, per = args
    import numpy as np
    import oracle as orc

    orc.uniform_streams(kind, orc.seed_states(kind, seed, np.arange(lo, hi)), per)


def cpu_extras(W):
    """The oracle on bounded samples of configs 3-5, every figure labelled with what was measured
    and how it scales: config 3 (bare streams, one core and all cores; the lagged Fibonacci stream
    on one core, being one sequence), config 4 (8 sampled ensembles, extrapolated to the whole
    batch), config 5 (adjoint and the common-random-number differences at N = 10^4, extrapolated)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    import numpy as np
    import oracle as orc

    out = {}
    c3 = W.C3
    S_s, per = 2**12, 1024  # 4.2e6 values per generator
    c3o = {}
    for kind in ("taus", "ran2", "lcg"):
        st = orc.seed_states(kind, c3["seed"], np.arange(S_s))
        t = time.perf_counter()
        orc.uniform_streams(kind, st, per)
        c3o[kind] = {"uint32_per_s_1core": S_s * per / (time.perf_counter() - t)}
        st = orc.seed_states(kind, c3["seed"], np.arange(S_s // 4))
        t = time.perf_counter()
        orc.gaussian_streams(kind, st, per)
        c3o[kind]["gaussians_per_s_1core"] = S_s // 4 * per / (time.perf_counter() - t)
    ll, sl = c3["lf_lags"]
    win = orc.lf_seed(c3["seed"], ll)
    t = time.perf_counter()
    orc.lf_generate(ll, sl, win, 2**23, keep=False)
    c3o["lf"] = {"uint32_per_s_1core": 2**23 / (time.perf_counter() - t)}
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(_c3_slice, [("taus", 1, 0, 8, 8)] * cores))  # worker start-up is not timed
        for kind in ("taus", "ran2", "lcg"):
            per_core = 2**14
            jobs = [(kind, c3["seed"], i * per_core, (i + 1) * per_core, per) for i in range(cores)]
            t = time.perf_counter()
            list(ex.map(_c3_slice, jobs))
            c3o[kind]["uint32_per_s_all_cores"] = cores * per_core * per / (time.perf_counter() - t)
    out["config3"] = {"per_generator": c3o, "cores": cores,
                      "sample": "uint32: 4096 streams x 1024 values per generator on one core, 16384 streams x 1024 "
                                "per core on all cores; Gaussians: 1024 streams x 1024; lagged Fibonacci: 2^23 values "
                                "of the one sequence on one core"}
    c4 = W.C4
    ens_list = W.batched_ensembles(c4["n_ens"], c4["draw_seed"], c4["base_seed"], c4["dt"])
    total = sum(e.n for e in ens_list) * c4["steps"]
    n_os, t_os = 0, 0.0
    for i in range(0, c4["n_ens"], c4["n_ens"] // 8):
        e = ens_list[i]
        n = min(e.n, 400)
        st = orc.seed_states("taus", e.seed, np.arange(n))
        t = time.perf_counter()
        orc.ld_run("taus", st, n, c4["steps"], e.params.asdict())
        t_os += time.perf_counter() - t
        n_os += n * c4["steps"]
    out["config4"] = {"osc_steps_per_s_1core": n_os / t_os, "extrapolated_s_whole_batch_1core": total * t_os / n_os,
                      "sample": "8 ensembles (every 64th), the first min(n, 400) oscillators of each x 5000 steps "
                                "(%d oscillator-steps), extrapolated to all %d" % (n_os, total)}
    c5 = W.C5
    pp = c5["params"].as_f32().asdict()
    N5 = 10**4
    t = time.perf_counter()
    orc.ld_adjoint("taus", orc.seed_states("taus", c5["seed"], np.arange(N5)), N5, c5["steps"], pp, c5["t_begin"],
                   c5["t_end"])
    t_adj = time.perf_counter() - t
    t = time.perf_counter()
    for name in ("k", "gamma", "kT"):
        for sgn in (1, -1):
            q = dict(pp)
            q[name] *= 1 + sgn * 5e-2
            orc.ld_loss("taus", orc.seed_states("taus", c5["seed"], np.arange(N5)), N5, c5["steps"], q,
                        c5["t_begin"], c5["t_end"])
    t_fd = time.perf_counter() - t
    out["config5"] = {"N": N5, "adjoint_s_1core": t_adj, "crn_fd_6_forwards_s_1core": t_fd,
                      "extrapolated_to_N_1e5": {"adjoint_s_1core": t_adj * 1e5 / N5,
                                                "crn_fd_6_forwards_s_1core": t_fd * 1e5 / N5},
                      "sample": "N = 1e4 oscillators, 2000 steps, extrapolated linearly to config 5's N = 1e5"}
    return out


def _ev(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def extra_config3(R, W, torch):
    """Bare generators: 2^30 uint32 and 2^30 Gaussians per generator (per-thread kinds: 2^20 streams
    x 1024 values; lagged Fibonacci: one stream).  Each call is timed with events on the stream it
    runs on, after an untimed warm-up call.  Bytes per value: the 4 written, plus for the lagged
    Fibonacci stream the long-lag source read back from the output (its short-lag source stays in
    registers); the per-thread generators' state (16 or 140 bytes per stream, in and out) adds
    0.03 and 0.27 bytes per value."""
    ev = lambda: _ev(torch)
    c3 = W.C3
    S, per = c3["streams"], c3["per_stream"]
    n_vals = S * per
    buf_u = torch.empty(n_vals, dtype=torch.int32, device="cuda")
    buf_g = torch.empty(n_vals, dtype=torch.float32, device="cuda")
    bare = {}
    state_bytes = {"taus": 16, "ran2": 140, "lcg": 4}
    for kind in GENERATORS + ("lcg",):
        if kind == "lf":
            cfg = R.make_cfg("lf", seed=c3["seed"], ll=c3["lf_lags"][0], sl=c3["lf_lags"][1])
            count = c3["lf_count"]
        else:
            cfg = R.make_cfg(kind, seed=c3["seed"], n_streams=S)
            count = per
        st = R.new_state(cfg)
        R.rng_init(cfg, st)
        R.rng_uniform(cfg, st, count, buf_u)  # warm-up
        a, b = ev()
        a.record()
        R.rng_uniform(cfg, st, count, buf_u)
        b.record()
        if kind == "lf" and R.lf_stream_status(st) != 0:
            raise RuntimeError("the persistent lagged-Fibonacci stream gave up a wait: invalid output")
        c, d = ev()
        c.record()
        R.rng_gaussian(cfg, st, count, buf_g)
        d.record()
        torch.cuda.synchronize()
        if kind == "lf" and R.lf_stream_status(st) != 0:
            raise RuntimeError("the persistent lagged-Fibonacci stream gave up a wait: invalid output")
        tu, tg = a.elapsed_time(b) / 1e3, c.elapsed_time(d) / 1e3
        if kind == "lf":
            # uniforms: each value written once and read once as a long-lag source (the output is
            # the lag table); Gaussians (the producer/consumer run): each integer written into the
            # run's ring, read there as a long-lag source and by a consumer, and its float written
            # once to the output: 12 B in the ring (memory-side cache) + 4 B to HBM
            bpv_u, bpv_g = 8.0, 16.0
        else:
            bpv_u = bpv_g = 4.0 + 2.0 * state_bytes[kind] * S / n_vals
        ru, rg = bpv_u * n_vals / tu / 1e9, bpv_g * n_vals / tg / 1e9
        bare[kind] = {"uint32_per_s": n_vals / tu, "gaussians_per_s": n_vals / tg,
                      "uint32_GBps_written": 4 * n_vals / tu / 1e9,
                      "roofline_uint32": {"bound": "hbm", "achieved": ru, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                          "frac": ru / HBM_PEAK_GBS, "bytes_per_value": bpv_u},
                      "roofline_gaussian": {"bound": "hbm", "achieved": rg, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                            "frac": rg / HBM_PEAK_GBS, "bytes_per_value": bpv_g}}
        del st
    del buf_u, buf_g
    return bare


def extra_config4(R, W, torch):
    """512 uneven ensembles in one hipGraph-captured plan vs 512 plain ld_run launches."""
    ev = lambda: _ev(torch)
    c4 = W.C4
    ens_list = W.batched_ensembles(c4["n_ens"], c4["draw_seed"], c4["base_seed"], c4["dt"])
    offs = [0]
    for e in ens_list:
        offs.append(offs[-1] + e.n)
    n_total = offs[-1]
    specs = [(offs[i], e.n, R.make_params(e.params.m, e.params.k, e.params.gamma, e.params.kT, e.params.dt), e.seed)
             for i, e in enumerate(ens_list)]
    ens, n_ens = R.make_ensembles(specs)
    cfg = R.make_cfg("taus", n_streams=n_total)
    # RNGLD_AUTOTUNE_CACHE names a file that keeps the chosen launch shape between runs (none by default)
    t_tune = time.perf_counter()
    tune = R.ld_autotune(cfg, ens, n_ens, n_total, c4["steps"], os.environ.get("RNGLD_AUTOTUNE_CACHE") or None)
    t_tune = time.perf_counter() - t_tune
    st = R.new_state(cfg)
    x = torch.zeros(3 * n_total, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(x)
    R.rng_init_ensembles(cfg, st, ens, n_ens)
    plan = R.Plan(cfg, st, ens, n_ens, n_total, c4["steps"], x, v)
    a, b = ev()
    a.record()
    plan.launch()
    b.record()
    torch.cuda.synchronize()
    t_batched = a.elapsed_time(b) / 1e3
    plan.close()
    R.rng_init_ensembles(cfg, st, ens, n_ens)
    x.zero_()
    v.zero_()
    ws = torch.empty(max(R.ld_workspace_bytes(cfg, ens, n_ens, n_total, c4["steps"]), 256), dtype=torch.uint8,
                     device="cuda")
    a, b = ev()
    a.record()
    for i in range(n_ens):
        e1, _ = R.make_ensembles([specs[i]])
        R.ld_run(cfg, st, e1, 1, n_total, c4["steps"], x, v, ws=ws)
    b.record()
    torch.cuda.synchronize()
    t_plain = a.elapsed_time(b) / 1e3
    R.ld_set_tuning("taus")
    osc_steps = n_total * c4["steps"]
    res = {"ensembles": n_ens, "oscillators": n_total, "steps": c4["steps"],
           "osc_steps": osc_steps, "tuning": list(tune.astuple()), "autotune_s": t_tune,
           "batched_graph_osc_steps_per_s": osc_steps / t_batched,
           "plain_512_launches_osc_steps_per_s": osc_steps / t_plain,
           "speedup_batched_vs_plain": t_plain / t_batched,
           "roofline": valu_entry("ld_run_kernel<HybridTaus> (batched)", valu_per_osc_step("taus"), osc_steps,
                                  t_batched, valu_mix_bound("taus"))}
    del x, v, st, ws
    return res


def extra_config5(R, W, torch):
    """Adjoint at config 5 (N = 1e5, 2000 steps from rest, loss over steps 1001-2000, K = 100):
    forward with checkpoints (segment-parallel) and backward, for the register-only
    (segment-parallel) backward and the replay backward, each timed with events on the stream
    around the library call, and end to end through torch's autograd; every pass starts a fresh run
    from rest (one untimed pass first loads the kernels).  Also the 6 forward runs of
    common-random-number central differences that the gradient replaces, and both backward paths
    for Ran2 after its sequential forward."""
    from paper_1003_1123_amd import autograd as A
    c5 = W.C5
    p5 = c5["params"].as_f32()
    N, T = c5["N"], c5["steps"]
    out = {"N": N, "steps": T, "K": c5["K"]}
    osc = N * T

    def one(replay, kind="taus"):
        run = A.AdjointRun(kind, [(N, p5.m, p5.dt, c5["seed"])], T, c5["t_begin"], c5["t_end"], c5["K"],
                           replay=replay, spread=True)
        run.timed = True
        k = torch.tensor([p5.k], dtype=torch.float64, requires_grad=True)
        g = torch.tensor([p5.gamma], dtype=torch.float64, requires_grad=True)
        kT = torch.tensor([p5.kT], dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        e0, e1 = _ev(torch)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record()
        L = A.LDAdjoint.apply(k, g, kT, run)
        e1.record()
        L.sum().backward()
        e2.record()
        torch.cuda.synchronize()
        lib = [p[0].elapsed_time(p[1]) for p in (run.fwd_events, run.bwd_events)]
        return run, L.item(), [k.grad.item(), g.grad.item(), kT.grad.item()], lib, [e0.elapsed_time(e1),
                                                                                    e1.elapsed_time(e2)]

    for replay in (False, True):
        one(replay)  # loads the kernels
        run, L, grad, (fwd_ms, bwd_ms), (fwd_ag, bwd_ag) = one(replay)
        res = {"backward_path": "replay" if replay else "register-only, segment-parallel",
               "loss": L, "grad_k_gamma_kT": grad, "grad_standard_errors": run.grad_se[0].tolist(),
               "forward_ms": fwd_ms, "backward_ms": bwd_ms, "fwd_plus_bwd_over_fwd": (fwd_ms + bwd_ms) / fwd_ms,
               "timed": "forward_ms and backward_ms: events on the stream around ld_run_ckpt and ld_run_backward; "
                        "the *_autograd_ms include torch's autograd engine (LDAdjoint.apply, L.sum().backward())",
               "forward_autograd_ms": fwd_ag, "backward_autograd_ms": bwd_ag,
               "forward_osc_steps_per_s": osc / (fwd_ms / 1e3),
               "roofline_forward": valu_entry("ld_fwd_seg_kernel (+ tables and join)",
                                              windowed_valu("adjoint_forward", T, c5["t_begin"], c5["t_end"]), osc,
                                              fwd_ms / 1e3)}
        if not replay:
            res["roofline_backward"] = valu_entry("ld_adjoint_seg_kernel + sum",
                                                  windowed_valu("adjoint_backward", T, c5["t_begin"], c5["t_end"]),
                                                  osc, bwd_ms / 1e3)
            # the common-random-number central differences the gradient replaces: 6 forward runs
            e0, e1 = _ev(torch)
            runs = []
            for name in ("k", "gamma", "kT"):
                for sgn in (1, -1):
                    q = {"k": p5.k, "gamma": p5.gamma, "kT": p5.kT}
                    q[name] *= 1 + sgn * 5e-2
                    runs.append((A.AdjointRun("taus", [(N, p5.m, p5.dt, c5["seed"])], T, c5["t_begin"], c5["t_end"],
                                              c5["K"]), q))
            torch.cuda.synchronize()
            e0.record()
            for r, q in runs:
                A.LDAdjoint.apply(*(torch.tensor([q[n]], dtype=torch.float64) for n in ("k", "gamma", "kT")), r)
            e1.record()
            torch.cuda.synchronize()
            res["crn_fd_6_forwards_ms"] = e0.elapsed_time(e1)
            out.update(res)
        else:
            out["replay"] = res
    # the same workload with Ran2: a sequential forward (its shuffle table has no jump-ahead), then
    # the register-only or the replay backward
    r2 = {}
    for replay in (False, True):
        one(replay, "ran2")
        _, L, grad, (fwd_ms, bwd_ms), _ = one(replay, "ran2")
        r2["replay" if replay else "register_only"] = {"loss": L, "grad_k_gamma_kT": grad, "forward_ms": fwd_ms,
                                                       "backward_ms": bwd_ms}
    out["ran2"] = r2
    return out


def extra_fig6_breakdown(R, W, torch, cpu=True):
    """Fig. 6 on this GPU: time per 10^3 LD steps against N for the fused full step of each generator,
    the dynamics alone (the no-noise kind: same kernel, zero random force), the generator alone (bare
    uniform streams, 4 words per oscillator-step written to HBM, in chunks), and the paper's
    one-launch-per-step protocol (ld_step) for Hybrid Taus with and without noise (called from Python,
    and replayed from a captured graph); plus the speedup
    of the fused step over the FP64 oracle (one thread), whose per-oscillator-step time is measured
    on about 2e5 oscillator-steps at each N.  Underdamped, h = 0.005, m = k = kT = gamma = 1, from
    rest, no observables; LF uses the smallest Table I pair with sl > 4N."""
    import numpy as np
    Ns = (10**2, 10**3, 10**4, 10**5, 10**6)
    T = 1000
    kinds = ("taus", "ran2", "lf", "lcg")
    pp = W.C2["params"].as_f32()
    p = R.make_params(pp.m, pp.k, pp.gamma, pp.kT, pp.dt)
    seed = W.C2["seed"]

    def timed(fn):
        a, b = _ev(torch)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    rows = []
    chunk_words = 2**28  # bare-stream output buffer: 1 GiB
    buf = torch.empty(chunk_words, dtype=torch.int32, device="cuda")
    for N in Ns:
        row = {"N": N, "full_ms": {}, "rng_only_ms": {}, "cpu_ms_extrapolated": {}, "cpu_measured_osc_steps": {},
               "speedup_vs_cpu": {}}
        ens, n_ens = R.make_ensembles([(0, N, p, 0)])
        x = torch.zeros(3 * N, dtype=torch.float32, device="cuda")
        v = torch.zeros_like(x)
        ll, sl = W.lf_lags_for(4 * N)
        for kind in kinds + ("none",):
            cfg = R.make_cfg(kind, seed=seed, n_streams=N, ll=ll if kind == "lf" else 0,
                             sl=sl if kind == "lf" else 0)
            st = R.new_state(cfg)
            ws = torch.empty(max(R.ld_workspace_bytes(cfg, ens, n_ens, N, T), 256), dtype=torch.uint8,
                             device="cuda")
            R.rng_init(cfg, st)
            R.ld_run(cfg, st, ens, n_ens, N, 8, x, v, ws=ws)  # first launch of this kernel shape
            x.zero_()
            v.zero_()
            ms = timed(lambda: R.ld_run(cfg, st, ens, n_ens, N, T, x, v, ws=ws))
            if kind == "none":
                row["dynamics_wo_rng_ms"] = ms
            else:
                row["full_ms"][kind] = ms
            if kind == "lf":
                row["lf_lags"] = [ll, sl]
                row["lf_path"] = R.ws_lf_path(ws)
                if R.ws_status(ws) != 0:
                    raise RuntimeError("the lagged-Fibonacci run at N=%d gave up a wait: invalid results" % N)
            if kind != "none":
                R.rng_init(cfg, st)
                total = 4 * N * T
                if kind == "lf":
                    per_call = min(total, chunk_words)
                    calls = [(per_call if i + per_call <= total else total - i) for i in range(0, total, per_call)]
                    run = lambda: [R.rng_uniform(cfg, st, c, buf) for c in calls]
                else:
                    per_stream = max(1, min(4 * T, chunk_words // N))
                    calls = [min(per_stream, 4 * T - i) for i in range(0, 4 * T, per_stream)]
                    run = lambda: [R.rng_uniform(cfg, st, c, buf) for c in calls]
                row["rng_only_ms"][kind] = timed(run)
            del st, ws
        for kind in ("taus", "ran2", "none"):
            cfg = R.make_cfg(kind, seed=seed, n_streams=N)
            st = R.new_state(cfg)
            R.rng_init(cfg, st)
            R.ld_step(cfg, st, p, N, x, v)
            ms = timed(lambda: [R.ld_step(cfg, st, p, N, x, v) for _ in range(T)])
            row["step_protocol_ms_" + kind] = ms
            # the same 10^3 launches captured in a graph: the device-side cost without the host's
            # per-call overhead
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                for _ in range(T):
                    R.ld_step(cfg, st, p, N, x, v)
            g.replay()
            row["step_protocol_graph_ms_" + kind] = timed(g.replay)
            # bytes each launch moves per oscillator-step: the generator state and x, v in and out
            row["step_protocol_graph_GBps_" + kind] = (STEP_BYTES_PER_OSC_STEP[kind] * N * T /
                                                       (row["step_protocol_graph_ms_" + kind] / 1e3) / 1e9)
            if kind == "ran2":
                row["step_protocol_graph_GBps_ran2_whole_lines"] = (
                    STEP_LINE_BYTES_RAN2 * N * T / (row["step_protocol_graph_ms_ran2"] / 1e3) / 1e9)
            del g, st
        if cpu:
            import oracle as orc
            pd = pp.asdict()
            n_cpu = max(1, 200_000 // N)
            for kind in kinds:
                stc = orc.lf_seed(seed, ll) if kind == "lf" else orc.seed_states(kind, seed, np.arange(N))
                t = time.perf_counter()
                orc.ld_run(kind, stc, N, n_cpu, pd, ll=ll, sl=sl)
                per_os = (time.perf_counter() - t) / (N * n_cpu)
                row["cpu_measured_osc_steps"][kind] = N * n_cpu
                row["cpu_ms_extrapolated"][kind] = per_os * N * T * 1e3
                row["speedup_vs_cpu"][kind] = row["cpu_ms_extrapolated"][kind] / row["full_ms"][kind]
        rows.append(row)
        log("fig6 N=%d: %s" % (N, json.dumps(row)))
        del x, v
    del buf
    return {"steps": T, "ms_per_1000_steps": rows,
            "cpu": "FP64 oracle, one thread: timed on N x max(1, 2e5 // N) oscillator-steps per point "
                   "(cpu_measured_osc_steps) and extrapolated linearly to N x 1000 (cpu_ms_extrapolated)"}


def extra_step_protocol(R, W, torch):
    """The one-launch-per-step protocol alone at N = 10^6: 50 eager ld_step launches per kind, for
    counter runs that need the step kernels without graph replays around them."""
    N, T = 10**6, 50
    pp = W.C2["params"].as_f32()
    p = R.make_params(pp.m, pp.k, pp.gamma, pp.kT, pp.dt)
    x = torch.zeros(3 * N, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(x)
    out = {"N": N, "launches": T, "us_per_launch": {}}
    for kind in ("taus", "ran2", "none"):
        cfg = R.make_cfg(kind, seed=W.C2["seed"], n_streams=N)
        st = R.new_state(cfg)
        R.rng_init(cfg, st)
        R.ld_step(cfg, st, p, N, x, v)
        a, b = _ev(torch)
        a.record()
        for _ in range(T):
            R.ld_step(cfg, st, p, N, x, v)
        b.record()
        torch.cuda.synchronize()
        out["us_per_launch"][kind] = a.elapsed_time(b) * 1e3 / T
        out.setdefault("GBps_algorithmic", {})[kind] = (STEP_BYTES_PER_OSC_STEP[kind] * N /
                                                        (out["us_per_launch"][kind] * 1e-6) / 1e9)
        del st
    out["GBps_ran2_whole_lines"] = STEP_LINE_BYTES_RAN2 * N / (out["us_per_launch"]["ran2"] * 1e-6) / 1e9
    return out


def extra_wave_rounds(R, W, torch):
    """The fused Hybrid Taus and Ran2 runs of config 2 (10^4 steps, observables every 100) at
    N = 10^6 and at the nearest N below it whose waves spread evenly over the SIMDs (15 per SIMD on
    256 CUs).  At N = 10^6 the 15,625 waves leave 265 SIMDs a 16th wave, which runs after the others
    have finished; the even N shows the step loop's rate without that tail."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    simds = 4 * cus
    N_even = (10**6 // (64 * simds)) * 64 * simds
    c = W.C2
    pp = c["params"].as_f32()
    p = R.make_params(pp.m, pp.k, pp.gamma, pp.kT, pp.dt)
    T, stride = c["steps"], 100
    out = {"simds": simds, "steps": T, "runs": []}
    for kind in ("taus", "ran2"):
        bound = valu_mix_bound(kind)
        for N in (N_even, 10**6):
            cfg = R.make_cfg(kind, seed=c["seed"], n_streams=N)
            st = R.new_state(cfg)
            ens, n_ens = R.make_ensembles([(0, N, p, 0)])
            x = torch.zeros(3 * N, dtype=torch.float32, device="cuda")
            v = torch.zeros_like(x)
            obs = torch.zeros((T // stride + 1) * R.NOBS, dtype=torch.float64, device="cuda")
            ws = torch.empty(max(R.ld_workspace_bytes(cfg, ens, n_ens, N, T, R.Obs(stride, 0)), 256),
                             dtype=torch.uint8, device="cuda")
            ms = []
            for rep in range(3):  # the first run is a warm-up
                R.rng_init(cfg, st)
                x.zero_()
                v.zero_()
                a, b = _ev(torch)
                a.record()
                R.ld_run(cfg, st, ens, n_ens, N, T, x, v, R.Obs(stride, 0), obs, ws)
                b.record()
                torch.cuda.synchronize()
                if rep:
                    ms.append(a.elapsed_time(b))
            rate = N * T / (min(ms) * 1e-3)
            out["runs"].append({"kind": kind, "N": N, "waves_per_simd": N / 64 / simds, "ms": min(ms),
                                "osc_steps_per_s": rate,
                                "frac_of_mix_bound": rate / bound if bound else None})
            del st, x, v, obs, ws
    return out


def extras(R, W, torch, only=()):
    out = {}
    named_only = {"step_protocol": extra_step_protocol,  # run only when asked for by name
                  "wave_rounds": extra_wave_rounds}
    for name, fn in (("config3_bare_generators", extra_config3), ("config4_batched", extra_config4),
                     ("config5_adjoint", extra_config5), ("fig6_breakdown", extra_fig6_breakdown),
                     *named_only.items()):
        if (only and name not in only) or (not only and name in named_only):
            continue
        try:
            out[name] = fn(R, W, torch)
            log("%s: %s" % (name, json.dumps(out[name])))
        except Exception as e:  # reported in the JSON line, never hidden
            out[name] = {"error": "%s: %s" % (type(e).__name__, e)}
            log("%s failed: %s" % (name, e))
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (each GPU would run "
              "its own range of oscillators, with one all-reduce of the observables). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1003_1123_amd import _lib as R
    from paper_1003_1123_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration * 2**18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d MiB copied" % args.copy_calibration)
        del src, dst
    hbm_copy = None if args.copy_calibration else measured_hbm_copy(torch)
    if hbm_copy:
        log("measured HBM copy: %.0f GB/s (read + write)" % hbm_copy)
    kinds = tuple(k for k in (args.only.split(",") if args.only else GENERATORS) if k)
    c2 = Config2(R, W, torch, kinds)
    log("config 2: N=%d, %d steps, generators %s" % (c2.N, c2.T, ",".join(kinds)))
    for i in range(args.warmup):
        c2.step()
        torch.cuda.synchronize()
        c2.check_status()
        log("warmup step %d done" % i)
    acc = {k: 0.0 for k in kinds}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        c2.step()
        torch.cuda.synchronize()
        for k, ms in c2.elapsed().items():
            acc[k] += ms
        c2.check_status()
        log("step %d done" % i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    osc_steps_per_step = len(kinds) * c2.N * c2.T
    value = osc_steps_per_step * args.steps / wall
    per_gen = {}
    rooflines = {}
    for k in kinds:
        ms = acc[k] / args.steps
        per_gen[k] = {"ms_per_run": ms, "osc_steps_per_s": c2.N * c2.T / (ms / 1e3),
                      "gaussians_per_s": 3 * c2.N * c2.T / (ms / 1e3)}
        lf_path = R.ws_lf_path(c2.ws[k]) if k == "lf" else None
        if k == "lf":
            per_gen[k]["lf_path"] = lf_path
        rooflines[k] = roofline_entry(k, ms, c2.N, c2.T, lf_path)
    dominant = max(kinds, key=lambda k: acc[k])
    res = {
        "metric": METRIC, "value": value, "unit": "oscillator-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "config 2: N=1e6 independent 3-D harmonic oscillators, 1e4 underdamped LD steps "
                               "(dt=0.005, m=k=kT=gamma=1) per generator, observables every 100 steps",
                   "generators": list(kinds), "N": c2.N, "ld_steps_per_run": c2.T, "lf_lags": [c2.ll, c2.sl]},
        "roofline": rooflines[dominant],
        "measured_peaks": {"hbm_copy_GBps": hbm_copy,
                           "lf_device_scope_mix_GBps": LF_MEASURED_PEAK_GBS},
        "per_generator": per_gen,
        "rooflines_all": rooflines,
    }
    log("config 2 value %.4g osc-steps/s; per generator ms: %s" %
        (value, {k: round(v["ms_per_run"], 2) for k, v in per_gen.items()}))
    if not args.no_extras:
        res["extras"] = extras(R, W, torch, tuple(e for e in args.extras.split(",") if e))
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(W)
        res["cpu_baseline"]["gpu_over_cpu"] = value / res["cpu_baseline"]["value"]
        if not args.no_extras:
            try:
                res["cpu_baseline"]["configs_3_to_5"] = cpu_extras(W)
            except Exception as e:  # reported, never hidden
                res["cpu_baseline"]["configs_3_to_5"] = {"error": "%s: %s" % (type(e).__name__, e)}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
