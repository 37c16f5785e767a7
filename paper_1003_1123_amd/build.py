"""Build librngld.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1003_1123_amd.build          # compiles every csrc/*.hip, links librngld.so

Object files go to <repo>/_build/; the shared library is written next to this file, with
kernel_isa.json: the SHA-256 of the gfx950 assembly of the kernels whose hardware counters are
recorded (so a measurement can tell whether the machine code it was taken on is still the one
built).
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import json
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "librngld.so")
ISA_JSON = os.path.join(HERE, "kernel_isa.json")
# kernels whose machine code is fingerprinted: name -> (source file, substring of the mangled
# symbols covered).  The lagged-Fibonacci entry covers the 8-tile instantiation, the one that runs
# 10^6 oscillators on 256 CUs.
FINGERPRINTED = {"lf_pc_kernel": ("k_lf.hip", "lf_pc_kernelILi8E"), "ld_run_kernel": ("k_ld.hip", "ld_run_kernel")}
# kernels whose step loop's vector-ALU instructions are counted (the loop that holds the Box-Muller
# logarithm: one oscillator-step per iteration): name -> (source file, exact mangled symbol)
STEP_LOOPS = {
    "ld_run_kernel<HybridTaus,256,1>": ("k_ld.hip", "_ZN5rngld12_GLOBAL__N_113ld_run_kernelINS_10HybridTausELi256ELi1EEEvNS_6LdArgsE"),
    "ld_run_kernel<Ran2,256,1>": ("k_ld.hip", "_ZN5rngld12_GLOBAL__N_113ld_run_kernelINS_4Ran2ELi256ELi1EEEvNS_6LdArgsE"),
    "ld_run_kernel<Lcg32,256,1>": ("k_ld.hip", "_ZN5rngld12_GLOBAL__N_113ld_run_kernelINS_5Lcg32ELi256ELi1EEEvNS_6LdArgsE"),
    "ld_fwd_seg_kernel<256>": ("k_adj.hip", "_ZN5rngld12_GLOBAL__N_117ld_fwd_seg_kernelILi256EEEvNS_7AdjArgsE"),
    "ld_adjoint_seg_kernel<HybridTaus,256>": ("k_adj.hip",
                                              "_ZN5rngld12_GLOBAL__N_121ld_adjoint_seg_kernelINS_10HybridTausELi256EEEvNS_7AdjArgsE"),
}
ARCH = os.environ.get("RNGLD_OFFLOAD_ARCH", "gfx950")

# Packed-FP32 instructions are disabled for all device code (the compiler would otherwise form
# v_pk_* ops from scalar float code).
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wall", "-fvisibility=hidden", "-Wno-unused-command-line-argument", "-I" + os.path.join(ROOT, "include")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [hipcc()] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def _function_bodies(asm: str, name: str):
    """Bodies of the device functions whose mangled symbol contains `name`, with comments and
    compiler-numbered labels normalised (they change when unrelated functions are added)."""
    out = {}
    cur, lines = None, []
    for line in asm.splitlines():
        m = re.match(r"^([_A-Za-z0-9.$]+):", line)
        if cur is None and m and name in m.group(1) and not m.group(1).startswith("."):
            cur, lines = m.group(1), []
            continue
        if cur is not None:
            if re.match(r"^\.Lfunc_end\d+:", line):
                out[cur] = "\n".join(lines)
                cur = None
                continue
            t = line.split(";")[0].rstrip()
            t = re.sub(r"\.LBB\d+_", ".LBB_", t)
            t = re.sub(r"\.Ltmp\d+", ".Ltmp", t)
            if t:
                lines.append(t)
    return out


def step_loop_valu(asm: str, symbol: str) -> dict:
    """Vector-ALU instructions of the step loop of `symbol`, by opcode: among the loops that contain
    a v_log_f32 (one oscillator-step per iteration) and no other loop, the largest one (the
    underdamped scheme where a kernel holds both).  Every instruction of the loop body counts once, including
    any branch that runs on some iterations only."""
    lines = asm.splitlines()
    start = next(i for i, l in enumerate(lines) if l.startswith(symbol + ":"))
    end = next(i for i in range(start, len(lines)) if lines[i].startswith(".Lfunc_end"))
    body = [l.split(";")[0].rstrip() for l in lines[start:end]]
    labels = {m.group(1): i for i, l in enumerate(body) for m in [re.match(r"^(\.LBB\d+_\d+):", l)] if m}
    spans = []
    for i, l in enumerate(body):
        m = re.search(r"s_(?:cbranch_\w+|branch)\s+(\.LBB\d+_\d+)", l)
        if m and m.group(1) in labels and labels[m.group(1)] < i:
            spans.append((labels[m.group(1)], i))
    ops_of = {(a, b): [x.split()[0] for x in body[a:b + 1] if x.strip().startswith("v_")] for a, b in spans}
    stepping = [sp for sp in spans if "v_log_f32_e32" in ops_of[sp]]
    # loops with no loop inside them (a loop around a step loop, or around the code between events
    # with its reduction loops, is not one)
    innermost = [sp for sp in stepping
                 if not any(sp[0] <= c and d <= sp[1] and (c, d) != sp for c, d in spans)]
    if not innermost:
        raise RuntimeError("no step loop found in %s" % symbol)
    best = max((ops_of[sp] for sp in innermost), key=len)
    counts = {}
    for op in best:
        counts[op] = counts.get(op, 0) + 1
    # every step loop's size, for kernels whose steps take different loops (e.g. inside and outside
    # a loss window)
    return {"valu_per_iteration": len(best), "by_opcode": dict(sorted(counts.items())),
            "all_loops": sorted(len(ops_of[sp]) for sp in innermost)}


def _assembly(src: str) -> str:
    """The gfx950 assembly listing of one source (written to _build/)."""
    asm_path = os.path.join(BUILD, src[:-4] + ".gfx950.s")
    cmd = [hipcc()] + [f for f in FLAGS if f != "-fPIC"] + ["--cuda-device-only", "-S",
                                                          os.path.join(CSRC, src), "-o", asm_path]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("assembly listing failed: %s\n%s" % (" ".join(cmd), r.stderr))
    return open(asm_path).read()


def fingerprint_kernels() -> dict:
    """SHA-256 over the sorted assembly bodies of each fingerprinted kernel family, and the VALU
    instruction counts of the step loops."""
    srcs = sorted({src for src, _ in FINGERPRINTED.values()} | {src for src, _ in STEP_LOOPS.values()})
    with cf.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        asm = dict(zip(srcs, ex.map(_assembly, srcs)))
    res = {}
    for name, (src, pattern) in FINGERPRINTED.items():
        bodies = _function_bodies(asm[src], pattern)
        if not bodies:
            raise RuntimeError("no %s in the assembly of %s" % (name, src))
        h = hashlib.sha256()
        for sym in sorted(bodies):
            h.update(sym.encode() + b"\n" + bodies[sym].encode() + b"\n")
        res[name] = {"sha256": h.hexdigest(), "functions": len(bodies)}
    loops = {}
    for name, (src, symbol) in STEP_LOOPS.items():
        loops[name] = step_loop_valu(asm[src], symbol)
    res["step_loops"] = loops
    return res


def build(verbose: bool = False) -> str:
    """Compile every kernel/ABI source and link librngld.so; always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    with open(ISA_JSON + ".tmp", "w") as f:
        json.dump(fingerprint_kernels(), f, indent=1, sort_keys=True)
    os.replace(ISA_JSON + ".tmp", ISA_JSON)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
