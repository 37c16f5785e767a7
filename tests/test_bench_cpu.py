"""Host logic of bench.py, without a GPU: the one-GPU guard, the roofline arithmetic, the counter
traffic that is reported only for the machine code it was taken on, and the per-oscillator-step
byte and instruction counts the roofline uses."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_lf_roofline_is_algorithmic_bytes_over_the_launch_time():
    N, T, ms = 1_000_000, 10_000, 72.0
    e = bench.roofline_entry("lf", ms, N, T, "dataflow")
    # 4 numbers per oscillator-step, each written once and read twice (Eq. 3), 4 bytes each
    assert e["algorithmic_bytes_per_osc_step"] == 48
    assert e["algorithmic_bytes_per_launch"] == 48 * N * T
    assert e["achieved"] == pytest.approx(48 * N * T / (ms / 1e3) / 1e9)
    assert e["frac"] == pytest.approx(e["achieved"] / 8000.0)
    assert e["frac_measured"] == pytest.approx(e["achieved"] / bench.LF_MEASURED_PEAK_GBS)
    assert e["launches"] == 1 and e["avg_launch_us"] == pytest.approx(ms * 1e3)
    assert e["bound"] == "hbm" and e["unit"] == "GB/s"
    # the wave path: one launch per wave, x and v through memory as well
    w = bench.roofline_entry("lf", ms, N, T, "waves")
    assert w["kernel"] == "lf_ld_phase_kernel" and w["launches"] == 4 * T
    assert w["algorithmic_bytes_per_osc_step"] == 48 + 48


# the opcode histogram of the Hybrid Taus step loop as compiled when the probe's class table was
# made (117 VALU per oscillator-step)
TAUS_LOOP = {"v_add_u32_e32": 6, "v_and_b32_e32": 3, "v_and_or_b32": 9, "v_bitop3_b32": 7, "v_cos_f32_e32": 2,
             "v_cvt_f32_u32_e32": 4, "v_fma_f32": 5, "v_fmac_f32_e32": 4, "v_log_f32_e32": 2,
             "v_lshlrev_b32_e32": 24, "v_lshrrev_b32_e32": 16, "v_mul_f32_e32": 12, "v_mul_lo_u32": 4,
             "v_or_b32_e32": 3, "v_sin_f32_e32": 1, "v_sqrt_f32_e32": 2, "v_xor_b32_e32": 13}


def test_valu_classes_and_mix_bound():
    cls = bench.valu_classes(TAUS_LOOP)
    assert cls == {"transcendental": 7, "mul32": 4, "cvt": 4, "three_operand": 16, "fp32": 21, "other": 65}
    t = sum(n / bench.VALU_CLASS_RATES[c] for c, n in cls.items())
    assert 1.0 / t == pytest.approx(3.75e11, rel=2e-3)
    assert bench.valu_classes({"v_fmac_f64_e32": 3, "v_xor_b32_e32": 1}) == {"unmeasured": 3, "other": 1}


@pytest.mark.parametrize("kind", ["taus", "ran2"])
def test_valu_roofline_uses_the_loop_counts_and_the_mix_bound(kind):
    if "step_loops" not in bench._kernel_isa():
        pytest.skip("the library has not been built (no kernel_isa.json)")
    N, T, ms = 1_000_000, 10_000, 30.0
    e = bench.roofline_entry(kind, ms, N, T)
    vpos = bench.valu_per_osc_step(kind)
    assert 40 < vpos < 200
    assert e["achieved"] == pytest.approx(vpos * N * T / (ms / 1e3) / 1e12)
    assert e["peak"] == pytest.approx(256 * 128 * 2.4e9 / 1e12)
    # the measured peak is the mix bound in oscillator-steps/s times the loop's instructions
    bound = bench.valu_mix_bound(kind)
    assert e["peak_measured"] == pytest.approx(vpos * bound / 1e12)
    assert e["frac_measured"] == pytest.approx((N * T / (ms / 1e3)) / bound)
    assert e["traffic"] is None  # no counters are recorded for these kernels


def test_adjoint_loops_mix_bounds():
    if "step_loops" not in bench._kernel_isa():
        pytest.skip("the library has not been built (no kernel_isa.json)")
    # the backward reruns each segment's generator, Box-Muller and update steps and adds the
    # carried adjoint and its FP32 sums: more instructions and a lower bound than the forward
    assert bench.valu_per_osc_step("adjoint_backward") > bench.valu_per_osc_step("adjoint_forward")
    assert bench.valu_per_osc_step("adjoint_forward") >= bench.valu_per_osc_step("taus")
    bwd, fwd = bench.valu_mix_bound("adjoint_backward"), bench.valu_mix_bound("adjoint_forward")
    assert bwd is not None and fwd is not None
    assert bwd < fwd <= bench.valu_mix_bound("taus")
    # an FP64 instruction in a loop leaves it without a bound (the probe measured no FP64 rates)
    assert bench.valu_classes({"v_fma_f64": 2, "v_xor_b32_e32": 3}) == {"unmeasured": 2, "other": 3}


def test_counter_traffic_only_for_the_recorded_machine_code(monkeypatch):
    c = bench.COUNTER_TRAFFIC["lf_pc_kernel"]
    monkeypatch.setattr(bench, "built_isa", lambda k: c["isa_sha256"])
    assert bench.counter_traffic("lf_pc_kernel") == c["fetch_bytes"] + c["write_bytes"]
    monkeypatch.setattr(bench, "built_isa", lambda k: "0" * 64)
    assert bench.counter_traffic("lf_pc_kernel") is None
    monkeypatch.setattr(bench, "built_isa", lambda k: None)
    assert bench.counter_traffic("lf_pc_kernel") is None
    # the counted bytes stay close to the algorithmic 480 GB of the config-2 run
    assert 0.98 < (c["fetch_bytes"] + c["write_bytes"]) / 480e9 < 1.1


def test_step_protocol_bytes():
    # x and v (6 floats) in and out, plus the state each launch reads and writes
    assert bench.STEP_BYTES_PER_OSC_STEP["none"] == 48
    assert bench.STEP_BYTES_PER_OSC_STEP["taus"] == 48 + 2 * 16
    assert bench.STEP_BYTES_PER_OSC_STEP["ran2"] == 48 + 2 * 12 + 2 * 4 * 4


def test_ran2_step_line_bytes():
    # the three state words and the whole 32-entry table row in and out, plus x and v
    assert bench.STEP_LINE_BYTES_RAN2 == 2 * 12 + 2 * 128 + 48 == 328


def test_profiling_extras_run_only_when_named(monkeypatch):
    ran = []
    for name in ("extra_config3", "extra_config4", "extra_config5", "extra_fig6_breakdown", "extra_step_protocol",
                 "extra_wave_rounds"):
        monkeypatch.setattr(bench, name, lambda R, W, torch, _n=name: ran.append(_n) or {})
    bench.extras(None, None, None)
    assert ran == ["extra_config3", "extra_config4", "extra_config5", "extra_fig6_breakdown"]
    ran.clear()
    bench.extras(None, None, None, ("step_protocol",))
    assert ran == ["extra_step_protocol"]
    ran.clear()
    bench.extras(None, None, None, ("wave_rounds",))
    assert ran == ["extra_wave_rounds"]


def test_windowed_valu_weights_the_window_loop():
    if "step_loops" not in bench._kernel_isa():
        pytest.skip("the library has not been built (no kernel_isa.json)")
    for which in ("adjoint_forward", "adjoint_backward"):
        loop = bench._kernel_isa()["step_loops"][bench.STEP_LOOP_KERNELS[which]]
        lo, hi = min(loop["all_loops"]), loop["valu_per_iteration"]
        assert bench.windowed_valu(which, 2000, 1, 2000) == hi  # the whole run is the window
        assert bench.windowed_valu(which, 2000, 2000, 2000) == pytest.approx((1999 * lo + hi) / 2000)
        assert bench.windowed_valu(which, 2000, 1001, 2000) == pytest.approx((lo + hi) / 2)
