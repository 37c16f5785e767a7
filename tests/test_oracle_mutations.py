"""The oracle's pins catch plausible mistakes: each case plants one mistake in a temporary copy of
oracle/rngld_oracle.c (a wrong shift, mask, constant, update order, lag, branch, sign, index, scale
or term) and runs the pins that must then fail, in a subprocess against that copy.  The unmodified
copy passes the same pins.  CPU only; the oracle in the repository is never modified."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
G = "tests/test_oracle_generators.py::"
L = "tests/test_oracle_ld.py::"

# (name, original text, planted text, pins that must fail)
MUTATIONS = [
    ("Tausworthe shift", "uint32_t feedback = ((z << q) ^ z) >> (k - s);",
     "uint32_t feedback = ((z << q) ^ z) >> (k - s + 1);", [G + "test_taus_component_matches_bitwise_definition"]),
    ("Tausworthe mask", "uint32_t keep_mask = (uint32_t)(0xFFFFFFFFu << (32 - k));", "uint32_t keep_mask = 0xFFFFFFFFu;",
     [G + "test_taus_component_matches_bitwise_definition"]),
    ("LCG increment", "#define LCG_C 1013904223u", "#define LCG_C 1013904221u", [G + "test_lcg_constants_match_paper"]),
    ("Hybrid Taus output before the LCG step", "    z[3] = orc_lcg_next(z[3]);\n    return z[0] ^ z[1] ^ z[2] ^ z[3];",
     "    uint32_t o = z[0] ^ z[1] ^ z[2] ^ z[3];\n    z[3] = orc_lcg_next(z[3]);\n    return o;",
     [G + "test_hybrid_taus_is_xor_of_independent_components"]),
    ("Ran2 wrap at 0", "if (iy < 1) iy += (int32_t)R2_IMM1;", "if (iy < 0) iy += (int32_t)R2_IMM1;",
     [G + "test_ran2_output_range_boundary"]),
    ("Ran2 table filled backwards", "if (j < R2_NTAB) iv[j] = idum;", "if (j < R2_NTAB) iv[R2_NTAB - 1 - j] = idum;",
     [G + "test_ran2_seeding_follows_alg2_initialisation"]),
    ("LF short lag read as ll - sl", "uint32_t y_sl = buf[(head + (ll - sl)) % ll];",
     "uint32_t y_sl = buf[(head + sl) % ll];", [G + "test_lf_output_satisfies_recurrence"]),
    ("Box-Muller sin/cos swapped", "*g0 = r * cos(theta);\n    *g1 = r * sin(theta);",
     "*g0 = r * sin(theta);\n    *g1 = r * cos(theta);", [G + "test_box_muller_identity_and_special_angles"]),
    ("uniform offset dropped", "return (double)((w >> 8) + 1u) * (1.0 / 16777216.0); }",
     "return (double)((w >> 8) + 0u) * (1.0 / 16777216.0) + 1e-300; }", [G + "test_uniform_mapping_edges"]),
    ("position update scaled", "x[d] = x[d] + q->h * v[d];", "x[d] = x[d] + q->h * v[d] * 1.0000001;",
     [L + "test_ld_noise_free_is_matrix_power"]),
    ("noise amplitude 5% high", "q.sig = sqrt(2.0 * gamma * kT * dt / m);",
     "q.sig = sqrt(2.0 * gamma * kT * dt / m) * 1.05;", [L + "test_config1_ensemble_statistics"]),
    ("z force from the sine branch", "orc_box_muller(w[2], w[3], &g[2], &unused);",
     "orc_box_muller(w[2], w[3], &unused, &g[2]);", [L + "test_forces_use_four_words_per_oscillator_step"]),
    ("adjoint noise term scaled", "gT += mu * (dsig_dkT * g);", "gT += mu * (dsig_dkT * g) * 1.001;",
     [L + "test_adjoint_dkT_equals_L_over_kT"]),
    ("adjoint velocity factor dropped", "lv[d] = q.c * mu;", "lv[d] = mu;",
     [L + "test_adjoint_matches_crn_central_differences"]),
    ("adjoint loss term one step off", "lx[d] += 2.0 * scale * path[6 * ((size_t)s + 1) + d];",
     "lx[d] += 2.0 * scale * path[6 * ((size_t)s) + d];", [L + "test_adjoint_matches_crn_central_differences"]),
    ("observable <xv> computed as <xx>", "s[2] += x[i] * v[i];", "s[2] += x[i] * x[i];",
     [L + "test_observables_are_means_over_coordinates"]),
    ("Tausworthe seed lift dropped", "if (z[c] < floor_val) z[c] += floor_val;", "",
     [G + "test_taus_lift_values"]),
    ("polynomial reduction shifted", "poly_xor_shl(a, nw, high, nw, sl);", "poly_xor_shl(a, nw, high, nw, sl + 1);",
     [G + "test_trinomial_checker_matches_brute_force_lfsr_period"]),
    ("LCG stream leap off by one", "uint64_t n = (stream * leap) & 0xFFFFFFFFULL;",
     "uint64_t n = (stream * leap + 1) & 0xFFFFFFFFULL;", [G + "test_lcg_stream_seeding_independent_and_leaped"]),
    ("overdamped displacement multiplied by xi", "q.ods = sqrt(2.0 * kT * dt / xi);",
     "q.ods = sqrt(2.0 * kT * dt * xi);", [L + "test_fig4_overdamped_statistics_oracle"]),
    ("overdamped drift 1% high", "q.odc = k * dt / xi;", "q.odc = k * dt / xi * 1.01;",
     [L + "test_overdamped_noise_free_decay_and_closed_forms"]),
    ("LF discard one value short", "return orc_lf_generate(ll, sl, win, discard, NULL);",
     "return orc_lf_generate(ll, sl, win, discard ? discard - 1 : 0, NULL);",
     [G + "test_lf_discard_shifts_the_sequence"]),
    ("sampled LF run with the short lag read as ll - sl", "uint32_t head = 0, tail = ll - sl;",
     "uint32_t head = 0, tail = sl;", [L + "test_lf_sampled_run_equals_the_full_run"]),
]


def _run_pins(src_text, pins, workdir):
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(workdir, "oracle"),
                    ignore=shutil.ignore_patterns("*.so", "*.so.*", "__pycache__"))
    shutil.copytree(os.path.join(ROOT, "tests"), os.path.join(workdir, "tests"),
                    ignore=shutil.ignore_patterns("__pycache__", "native"))
    with open(os.path.join(workdir, "oracle", "rngld_oracle.c"), "w") as f:
        f.write(src_text)
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1")
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + pins,
                          cwd=workdir, capture_output=True, text=True, timeout=600, env=env)


def _case(args):
    name, old, new, pins = args
    src = open(os.path.join(ROOT, "oracle", "rngld_oracle.c")).read()
    assert src.count(old) == 1, "anchor of '%s' not found once" % name
    with tempfile.TemporaryDirectory() as d:
        r = _run_pins(src.replace(old, new), pins, d)
    return name, r.returncode, r.stdout[-400:]


@pytest.mark.timeout(900)
def test_every_planted_mistake_fails_a_pin():
    src = open(os.path.join(ROOT, "oracle", "rngld_oracle.c")).read()
    all_pins = sorted({p for m in MUTATIONS for p in m[3]})
    with tempfile.TemporaryDirectory() as d:
        control = _run_pins(src, all_pins, d)
    assert control.returncode == 0, control.stdout[-2000:]
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(_case, MUTATIONS))
    # caught = a pin failed (not a build or collection error)
    survived = [(name, out) for name, rc, out in results if rc == 0 or " failed" not in out or " error" in out]
    assert not survived, survived
