"""Benchmark: direct line-by-line emission spectrum + gradient on one MI355X.

One step = one HMC-style evaluation of the whole path on the full
configuration-2 workload (two absorbers x 1e5 lines, 20,000-point
log-uniform grid at R0 ~ 2.2e6, 100 power-law layers, CIA, rotation + RV +
instrumental response): line-parameter precompute, FP32 compensated Voigt sum
with temperature tangents, transfer, response, and the adjoint back to
(T0, alpha, log10 X_1, log10 X_2, RV, vsini), i.e. exo_flux_vjp returning the
spectrum and its gradient.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  The metric value is Voigt evaluations per second
(lines x grid points x layers per step / time per step).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Voigt evals/s (lines×grid×layers) + spectra/s & p99 latency, FP32 vs FP64 @1e-4"
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak (packed FMA)
C_KMS = 2.99792458e5          # km/s
# Algorithmic FP32 operations per (line, grid point, layer) pair of the Voigt
# sum in tangent mode (FMA = 2).  Near tier (full wing polynomial; core pairs
# are counted at this rate too): offset 1, D 2, 1/D 1, value polynomial
# 12 + 1, tangent polynomial 14 + 1, two accumulations 2.  Far tier
# (polynomial truncated below FP32 rounding): offset 1, D 2, 1/D 1, value
# polynomial 4, tangent polynomial 6 (4 in layers where it stops at r^3),
# two accumulations 4.  Beyond the outer reach both polynomials stop at r^2:
# value 2, tangent 2.
FLOPS_PER_EVAL_NEAR = 34.0
FLOPS_PER_EVAL_FAR = 18.0
FLOPS_PER_EVAL_FAR_CUT = 16.0   # far pair whose tangent polynomial stops at r^3
FLOPS_PER_EVAL_OUTER = 12.0     # far pair beyond the outer reach


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", default="full", choices=["small", "medium", "full"])
    ap.add_argument("--fp64-reps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modit", action="store_true", help="skip the MODIT-vs-direct cross-section runs")
    ap.add_argument("--modit-only", action="store_true", help="only the MODIT-vs-direct runs (for profiling)")
    ap.add_argument("--modit-emission-only", action="store_true",
                    help="only the config-3 emission with MODIT opacities (for profiling)")
    ap.add_argument("--cpu-points", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the Poisson serving run (0: skip)")
    ap.add_argument("--serve-streams", type=int, default=4, help="serving slots (1..16)")
    ap.add_argument("--serve-policy", nargs="+", default=["fifo", "shortest"], choices=["fifo", "shortest"],
                    help="admission orders to measure, each at every load")
    ap.add_argument("--serve-capacity-requests", type=int, default=200,
                    help="requests of the closed-loop capacity run that sets the arrival rate")
    ap.add_argument("--no-config3", action="store_true", help="skip the full config-3 direct-sum spectrum")
    ap.add_argument("--serve-load", type=float, nargs="+", default=[0.9],
                    help="arrival rates of the serving runs as fractions of the measured capacity")
    ap.add_argument("--serving-only", action="store_true", help="only the serving runs")
    ap.add_argument("--config3-direct", action="store_true",
                    help="only one direct-sum FP32 spectrum of the whole config-3 workload (~1e14 evaluations)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic summary from two --pmc runs of --counters and exit")
    ap.add_argument("--summarize-valu", metavar="VALU_CSV",
                    help="write the VALU-issue summary from a --pmc run of --counters and exit")
    ap.add_argument("--summarize-response", metavar="STATS_CSV",
                    help="write the response-kernel summary from the rocprofv3 --stats run of the bench")
    ap.add_argument("--summarize-flops", metavar="FLOPS_CSV",
                    help="write the hardware FLOP summary from a --pmc run (FLOP_COUNTERS) of --counters and exit")
    ap.add_argument("--summarize-stats", metavar="STATS_CSV",
                    help="write the kernel-time summary from a rocprofv3 --stats run and exit")
    ap.add_argument("--summarize-modit-stats", metavar="STATS_CSV",
                    help="write the MODIT kernel-time summary from a rocprofv3 --stats run of --modit-only")
    ap.add_argument("--summarize-modit-emission-stats", metavar="STATS_CSV",
                    help="write the kernel-time summary from a rocprofv3 --stats run of --modit-emission-only")
    ap.add_argument("--counters", action="store_true",
                    help="one step plus a 512 MiB device copy (calibration), for rocprofv3 --pmc runs")
    return ap.parse_args()


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(wl, theta, n_points):
    """The FP64 oracle on a bounded sample: F0 at n_points grid points, all
    lines and layers, on every CPU this process may use (at most 16, a
    one-GPU host's share)."""
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    threads = max(1, min(16, usable))
    os.environ["ORACLE_THREADS"] = str(threads)
    from oracle import oracle as O
    O.N_THREADS = threads
    rng = np.random.default_rng(99)
    idx = np.sort(rng.choice(wl.nu.size, n_points, replace=False))
    t0 = time.perf_counter()
    O.emission_F0(wl, theta, nu_idx=idx)
    dt = time.perf_counter() - t0
    evals = sum(l.n for l in wl.lines) * wl.atmos.P_bar.size * n_points
    return {"value": evals / dt, "unit": "Voigt evals/s", "cores": threads, "kind": "oracle",
            "nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": _cpu_model(),
            "evals_per_s_per_core": evals / dt / threads,
            "sample": f"F0 at {n_points} random grid points x all {sum(l.n for l in wl.lines)} lines "
                      f"x {wl.atmos.P_bar.size} layers (FP64 scipy wofz + exact E3), {dt:.1f} s"}


VOIGT_SOURCES = ["paper_2105_14782_amd/csrc/k_voigt.hip", "paper_2105_14782_amd/csrc/exo_device.h",
                 "paper_2105_14782_amd/csrc/exo_launch.h", "paper_2105_14782_amd/csrc/exo_lines.h"]
TRAFFIC_PROFILE = "profiles/voigt_tangent_config2_traffic.md"


def voigt_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in VOIGT_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def _profile_values(rel_path):
    """The "- key: value" lines of a committed counter summary, or None when
    the kernel sources changed since its counters were taken."""
    path = os.path.join(ROOT, rel_path)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            kv[k.strip()] = v.strip().strip("`")
    if kv.get("kernel_source_sha256") != voigt_source_hash():
        return None
    return kv


def recorded_traffic():
    """HBM bytes per tangent Voigt launch from the committed counter summary
    (None if stale)."""
    kv = _profile_values(TRAFFIC_PROFILE)
    return None if kv is None else float(kv["traffic_bytes_per_launch"])


def recorded_counter_flops():
    """FP32 and FP64 operations per tangent Voigt launch counted by the
    hardware (64 lanes x (ADD + MUL + TRANS + 2 FMA) wave instructions), from
    the committed counter summary (None if stale)."""
    kv = _profile_values(FLOPS_PROFILE)
    if kv is None:
        return None
    return float(kv["fp32_flop_per_launch"]), float(kv["fp64_flop_per_launch"])


def summarize_counters(fetch_csv, write_csv, out_path):
    """Write the traffic summary from two rocprofv3 --pmc runs of `bench.py --counters`:
    FETCH_SIZE / WRITE_SIZE of the tangent Voigt launches, calibrated by the same
    counters on the 512 MiB device copy that run ends with."""
    import csv

    def read(path, counter):
        voigt, copy = [], None
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            if "k_voigt_f32<true" in r["Kernel_Name"]:
                voigt.append(v)
            elif "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) >= 65536:
                copy = v
        return voigt, copy

    fv, fc = read(fetch_csv, "FETCH_SIZE")
    wv, wc = read(write_csv, "WRITE_SIZE")
    nbytes = 512 * 2 ** 20
    f_fac, w_fac = nbytes / (fc * 1024.0), nbytes / (wc * 1024.0)
    fetch = float(np.mean(fv)) * 1024.0 * f_fac
    write = float(np.mean(wv)) * 1024.0 * w_fac
    lines = [
        "# HBM traffic of the tangent-mode Voigt sum (config-2 emission, one species per launch)", "",
        "Commands (repository root, one MI355X):", "", "```",
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_FETCH_SIZE -o run -- python3 bench.py --counters --warmup 1",
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_WRITE_SIZE -o run -- python3 bench.py --counters --warmup 1",
        "python3 bench.py --summarize-counters gpurun_out/pmc_FETCH_SIZE/run_counter_collection.csv "
        "gpurun_out/pmc_WRITE_SIZE/run_counter_collection.csv", "```", "",
        "Calibration: the run ends with a 512 MiB device-to-device copy; the counters read "
        f"{fc:.0f} KiB fetched and {wc:.0f} KiB written for it, so FETCH_SIZE is scaled by "
        f"{f_fac:.3f} and WRITE_SIZE by {w_fac:.3f}.", "",
        f"Tangent Voigt launches measured: {len(fv)} (1e5 lines x 20,000 points x 100 layers each).", "",
        "Algorithmic bytes per launch: line records 1e7 x (64 + 64) B + centres 0.8 MB read, "
        "outputs 2 x 100 x 20,000 x 8 B (split partial sums) written: 1.33e9 B.  The kernel runs at",
        "5 waves per SIMD with 96 registers per lane and spills nothing around its out-of-line",
        "core-branch call; the split partial sums (5 splits x 100 layers x 20,000 points x 2 x 8 B",
        "= 1.6e8 B) are most of the written bytes.", "",
        f"- fetch_kib_per_launch: {np.mean(fv):.1f}",
        f"- write_kib_per_launch: {np.mean(wv):.1f}",
        f"- traffic_bytes_per_launch: {fetch + write:.4e}",
        f"- kernel_source_sha256: `{voigt_source_hash()}`", "",
        "The fetched bytes exceed the algorithmic record stream because every wave loads the",
        "records of its (layer, split) chunk by chunk into its own LDS slice, and the per-XCD L2",
        "does not hold the streams of all resident workgroups.  At the kernel's duration this is",
        "well below HBM bandwidth (the kernel is VALU-issue bound).",
    ]
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


VALU_PROFILE = "profiles/voigt_tangent_config2_valu.md"
FLOPS_PROFILE = "profiles/voigt_tangent_config2_flops.md"
FLOP_COUNTERS = ("SQ_INSTS_VALU_ADD_F32 SQ_INSTS_VALU_MUL_F32 SQ_INSTS_VALU_FMA_F32 SQ_INSTS_VALU_TRANS_F32 "
                 "SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64")
STATS_PROFILE = "profiles/voigt_config2_kernel_stats.md"
MODIT_EMISSION_PROFILE = "profiles/modit_emission_config3_kernel_stats.md"
MODIT_PROFILE = "profiles/modit_config3_kernel_stats.md"
VALU_COUNTERS = "SQ_INSTS_VALU SQ_INSTS_VALU_TRANS_F32 SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES GRBM_GUI_ACTIVE"


def summarize_valu(csv_path, out_path):
    """VALU issue of the tangent Voigt launches from one rocprofv3 --pmc run of
    `bench.py --counters`: wave instructions per 64 pairs and the fraction of
    the SIMDs' issue cycles they occupy (a non-packed FP32 or FP64 VALU
    instruction of a 64-wide wave holds a 16-lane SIMD for 4 cycles)."""
    import csv
    acc = {}
    for r in csv.DictReader(open(csv_path)):
        if "k_voigt_f32<true" in r["Kernel_Name"]:
            acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    m = {k: float(np.mean(v)) for k, v in acc.items()}
    n = len(acc["SQ_INSTS_VALU"])
    pairs = 1e5 * 2e4 * 100
    groups = pairs / 64.0
    xcd = 8
    cycles = m["GRBM_GUI_ACTIVE"] / xcd          # summed over the 8 XCDs
    simds = 256 * 4
    issue = m["SQ_INSTS_VALU"] * 4.0 / (simds * cycles)
    lines = [
        "# VALU issue of the tangent-mode Voigt sum (config-2 emission, one species per launch)", "",
        "Command (repository root, one MI355X):", "", "```",
        f"rocprofv3 --pmc {VALU_COUNTERS} --output-format csv -d gpurun_out/pmc_valu -o run -- "
        "python3 bench.py --counters --warmup 1",
        "python3 bench.py --summarize-valu gpurun_out/pmc_valu/run_counter_collection.csv", "```", "",
        f"Launches measured: {n} (1e5 lines x 20,000 points x 100 layers = 2e11 pairs each).", "",
        f"- SQ_INSTS_VALU per launch: {m['SQ_INSTS_VALU']:.4e} wave instructions "
        f"= {m['SQ_INSTS_VALU'] / groups:.2f} per 64 pairs",
        f"- SQ_INSTS_VALU_TRANS_F32 per launch: {m['SQ_INSTS_VALU_TRANS_F32']:.4e} "
        f"= {m['SQ_INSTS_VALU_TRANS_F32'] / groups:.3f} per 64 pairs (the reciprocal 1/D, plus core-branch transcendentals)",
        f"- GRBM_GUI_ACTIVE per launch: {m['GRBM_GUI_ACTIVE']:.4e} (8 XCDs) = {cycles:.4e} cycles per XCD",
        f"- SQ_BUSY_CYCLES per launch: {m['SQ_BUSY_CYCLES']:.4e}",
        f"- SQ_ACTIVE_INST_VALU per launch: {m['SQ_ACTIVE_INST_VALU']:.4e}",
        f"- VALU issue occupancy (instructions x 4 cycles / (1024 SIMDs x cycles)): {issue:.3f}",
        "",
        "A throughput probe (independent FMA chains, packed FP32 disabled) runs a 64-wide",
        "v_fma_f32 every 4 cycles per SIMD (76.9 TFLOP/s, 98 % of 78.6) and a v_rcp_f32 with",
        "its dependent add every 12.  An occupancy near or above 1 therefore means the SIMDs",
        "issue VALU work on (nearly) every cycle; above 1, some counted instructions (moves,",
        "masks, lane operations) hold the SIMD for fewer than 4 cycles.  The kernel is bound",
        "by VALU issue, not by memory: the lever is the instruction count per pair.",
    ]
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_flops(csv_path, out_path):
    """Hardware FP32/FP64 operation counts of the tangent Voigt launches from
    one rocprofv3 --pmc run of `bench.py --counters` (FLOP_COUNTERS): each
    counter counts wave instructions, so operations = 64 lanes x (ADD + MUL +
    TRANS + 2 FMA), whatever the execution mask (masked-off lanes count)."""
    import csv
    acc = {}
    for r in csv.DictReader(open(csv_path)):
        if "k_voigt_f32<true" in r["Kernel_Name"]:
            acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    m = {k: float(np.mean(v)) for k, v in acc.items()}
    n = len(next(iter(acc.values())))
    f32 = 64.0 * (m["SQ_INSTS_VALU_ADD_F32"] + m["SQ_INSTS_VALU_MUL_F32"] + m["SQ_INSTS_VALU_TRANS_F32"]
                  + 2.0 * m["SQ_INSTS_VALU_FMA_F32"])
    f64 = 64.0 * (m["SQ_INSTS_VALU_ADD_F64"] + m["SQ_INSTS_VALU_MUL_F64"] + m["SQ_INSTS_VALU_TRANS_F64"]
                  + 2.0 * m["SQ_INSTS_VALU_FMA_F64"])
    pairs = 1e5 * 2e4 * 100
    groups = pairs / 64.0
    lines = [
        "# Hardware FP32/FP64 operations of the tangent-mode Voigt sum (config-2 emission, one species per launch)", "",
        "Command (repository root, one MI355X):", "", "```",
        f"rocprofv3 --pmc {FLOP_COUNTERS} --output-format csv -d gpurun_out/pmc_flops -o run -- "
        "python3 bench.py --counters --warmup 1",
        "python3 bench.py --summarize-flops gpurun_out/pmc_flops/run_counter_collection.csv", "```", "",
        f"Launches measured: {n} (1e5 lines x 20,000 points x 100 layers = 2e11 pairs each).", "",
        "Wave instructions per 64 pairs (per launch / 3.125e9):", "",
    ]
    for k in FLOP_COUNTERS.split():
        lines.append(f"- {k}: {m[k]:.4e} per launch = {m[k] / groups:.3f} per 64 pairs")
    lines += [
        "",
        "Operations = 64 x (ADD + MUL + TRANS + 2 FMA) wave instructions (FMA = 2, masked lanes included):", "",
        f"- fp32_flop_per_launch: {f32:.4e}",
        f"- fp64_flop_per_launch: {f64:.4e}",
        f"- fp32_flop_per_pair: {f32 / pairs:.3f}",
        f"- fp64_flop_per_pair: {f64 / pairs:.3f}",
        f"- kernel_source_sha256: `{voigt_source_hash()}`", "",
        "bench.py divides these per-launch counts by the launch time it measures with HIP events",
        "(`roofline.counter_tflops`), beside the algorithmic count (`roofline.achieved`, tier-aware",
        "model FLOPs per pair).  The hardware count is the larger: it includes the reciprocal",
        "sharing (one reciprocal and three multiplications per two far points), the FP64 offset",
        "and core-branch work, compares and selects counted as FP32 operations, and lanes",
        "masked off in the core branch.",
    ]
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_stats(csv_path, out_path, modit=False):
    """Markdown table of a rocprofv3 --kernel-trace --stats run of the bench."""
    import csv
    rows = list(csv.DictReader(open(csv_path)))
    if modit == "emission":
        head = [
            "# Kernel trace summary: config-3 emission with MODIT opacities (rocprofv3 --kernel-trace --stats)", "",
            "Command (repository root, one MI355X):", "", "```",
            "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_modit_em -o modit_em -- \\",
            "    python3 bench.py --modit-emission-only",
            "python3 bench.py --summarize-modit-emission-stats gpurun_out/prof_modit_em/modit_em_kernel_stats.csv",
            "```", "",
            "Workload: the config-3 line list (1e7 lines) on its 100,000-point grid at R0 = 1e6, 100 layers",
            "(1e-8 .. 100 bar, T0 = 1300 K, alpha = 0.1), one species, no response: 6 spectra in FP32 and 6 in",
            "FP64 (1 warm-up + 5 timed each).  The layers go 14 (FP32) or 10 (FP64) to a launch; each launch",
            "has 9 radix-4 Stockham passes over 32 width rows per layer forward and 9 over one row inverse.", "",
        ]
    elif modit:
        head = [
            "# Kernel trace summary: MODIT vs direct cross-section, config-3 grid (rocprofv3 --kernel-trace --stats)", "",
            "Command (repository root, one MI355X):", "", "```",
            "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_modit -o modit -- \\",
            "    python3 bench.py --modit-only",
            "python3 bench.py --summarize-modit-stats gpurun_out/prof_modit/modit_kernel_stats.csv", "```", "",
            "Workload: one layer (700 K, 1 bar) of the config-3 line list, 100,000-point grid at R0 = 1e6,",
            "at 1e5, 1e6 and 1e7 lines: each size runs 6 MODIT cross-sections in FP32 and 6 in FP64",
            "(transform length 262,144: 9 radix-4 Stockham passes forward over the width rows, 9 inverse),",
            "and 4, 4 and 2 direct FP32 cross-sections (`k_voigt_f32<false, 4>`).", "",
        ]
    else:
        head = [
            "# Kernel trace summary: config-2 emission bench (rocprofv3 --kernel-trace --stats)", "",
            "Command (repository root, one MI355X):", "", "```",
            "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_bench -o bench -- \\",
            "    python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline --fp64-reps 1 --serve-requests 0 --no-modit "
            "--no-config3",
            "python3 bench.py --summarize-stats gpurun_out/prof_bench/bench_kernel_stats.csv", "```", "",
            "Workload: 2 species x 1e5 lines, 20,000-point log-uniform grid, 100 layers.",
            "The run does 1 warm-up + 3 timed flux_vjp steps (two tangent-mode Voigt sums each),",
            "then 4 FP32 forward spectra, 2 plain-FP64 and 4 tiled-FP64 forward spectra (two Voigt sums each),",
            "then 4 loss_grad (leapfrog step) and 4 flux_jvp calls (tangent-mode Voigt sums as well),",
            "then the config-1 cross-section timing (1000 lines x 4000 points, one layer: 51 FP32 and",
            "51 plain-FP64 calls, hence the many short `k_voigt_f32<false, 4>` and `k_voigt_f64` launches).", "",
        ]
    lines = head + ["| kernel | calls | avg ms | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        name = r["Name"] if len(r["Name"]) <= 70 else r["Name"][:67] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


RESPONSE_PROFILE = "profiles/response_config2_kernel_stats.md"


def response_shapes(nu, resp):
    """Tap counts and lengths of the response stages on a log-uniform grid, as
    the library plans them (rotation taps d = i - j from dlo, IP taps -K..K)."""
    dv = C_KMS * math.log(nu[-1] / nu[0]) / (nu.size - 1)
    dmin = math.ceil((-resp.vsini_kms - resp.rv_kms) / dv) - 1
    dmax = math.floor((resp.vsini_kms - resp.rv_kms) / dv) + 1
    beta_ip = C_KMS / (2.0 * math.sqrt(2.0 * math.log(2.0)) * resp.R_inst)
    K = math.floor(6.0 * beta_ip / dv)
    return {"ng": nu.size, "nrot": dmax - dmin + 1, "K": K, "ol": resp.out_len, "nmid": resp.out_len + 2 * K}


def summarize_response(csv_path, out_path):
    """Response-stage kernels of the config-2 bench trace (the same rocprofv3
    --kernel-trace --stats run as STATS_PROFILE): average duration, the
    algorithmic bytes each launch must move (inputs, taps, outputs once) and
    FLOPs (2 per tap and output), and the rates they imply."""
    import csv
    import synth
    wl = synth.make_config(2, "full")
    sh = response_shapes(wl.nu, wl.response)
    ng, nrot, K, ol, nmid = sh["ng"], sh["nrot"], sh["K"], sh["ol"], sh["nmid"]
    nip = 2 * K + 1
    model = {   # kernel name prefix: (bytes, flops)
        "exo::k_conv_rot(": ((nmid + nrot - 1) * 8 + nrot * 8 + nmid * 8, 2 * nrot * nmid),
        "void exo::k_conv_ip<float>": (nmid * 8 + nip * 8 + ol * 4, 2 * nip * ol),
        "void exo::k_conv_ip<double>": (nmid * 8 + nip * 8 + ol * 8, 2 * nip * ol),
        "void exo::k_convT_ip<float>": (ol * 4 + nip * 8 + nmid * 8, 2 * nip * nmid),
        "void exo::k_convT_ip<double>": (ol * 8 + nip * 8 + nmid * 8, 2 * nip * nmid),
        "exo::k_convT_rot(": (nmid * 8 + nrot * 8 + ng * 8, 2 * nrot * ng),
        "exo::k_rot_param_grad(": ((nmid + nrot - 1) * 8 + 2 * nrot * 8 + nmid * 8, 4 * nrot * nmid),
        "exo::k_conv_rot_jvp(": (2 * (nmid + nrot - 1) * 8 + 3 * nrot * 8 + nmid * 8, 4 * nrot * nmid),
    }
    lines = [
        "# Response-stage kernels (config-2 bench, rocprofv3 --kernel-trace --stats)", "",
        "From the same run as `profiles/voigt_config2_kernel_stats.md`:", "", "```",
        "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_bench -o bench -- \\",
        "    python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline --fp64-reps 1 --serve-requests 0 --no-modit "
        "--no-config3",
        "python3 bench.py --summarize-response gpurun_out/prof_bench/bench_kernel_stats.csv", "```", "",
        f"Shapes (config 2): model grid {ng} points, output {ol}, rotation output {nmid}, {nrot} rotation taps, "
        f"{nip} IP taps.  Each kernel stages its taps and the input window of a 256-output block in LDS.",
        "Algorithmic bytes: inputs, taps and outputs moved once; FLOPs: one FMA (2) per tap and output.", "",
        "| kernel | calls | avg us | algorithmic bytes | GB/s | FP64 GFLOP/s |", "|---|---:|---:|---:|---:|---:|",
    ]
    for r in csv.DictReader(open(csv_path)):
        for pre, (nb, nf) in model.items():
            if r["Name"].startswith(pre):
                us = float(r["AverageNs"]) / 1e3
                lines.append(f"| `{r['Name'][:60]}` | {r['Calls']} | {us:.1f} | {nb:.3e} | "
                             f"{nb / (us * 1e-6) / 1e9:.1f} | {nf / (us * 1e-6) / 1e9:.1f} |")
    lines += ["", "At these sizes (tens of thousands of outputs, 75 workgroups) the launches are bound by",
              "latency, far below HBM bandwidth (8 TB/s) and FP64 peak; they are a few tens of microseconds",
              "of a ~114 ms step."]
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def modit_bench(wl=None, reps=5):
    """MODIT (Sec. 2.1.2) against the direct sum on the throughput workload
    (config 3: lines U(4340, 4796.44) cm^-1, 100,000-point grid at R0 = 1e6),
    one layer at T = 700 K, P = 1 bar, as the paper benchmarks opacity time
    against the number of lines: 1e5, 1e6 and 1e7 lines (every 100th, every
    10th, all).  700 K: the synthetic strengths (S0 <= 1e-18 at 296 K,
    E_low ~ Exp(3000)) reach 1e36 cm/molecule there, so every cross-section
    fits the FP32 range; at 1300 K they reach 1e54 and no FP32 output can
    hold the result."""
    import torch
    import synth
    from dataclasses import replace
    from paper_2105_14782_amd import api
    wl = wl if wl is not None else synth.make_config(3, "full")
    full = wl.lines[0]
    ctx = api.Context(0)
    ctx.set_grid(wl.nu)
    T, P = 700.0, 1.0
    atm = api.Atmos.from_workload(wl.atmos, [0])
    T_scan = np.arange(500.0, 1701.0, 100.0)
    out = {"workload": "config-3 single layer (T = 700 K, P = 1 bar), 100,000-point grid at R0 = 1e6; "
                       "line selection on the config-3 100-layer pressure grid",
           "runs": []}

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / n

    for stride in (100, 10, 1):
        sub = full if stride == 1 else replace(
            full, nu_c=full.nu_c[::stride], S0=full.S0[::stride], E_low=full.E_low[::stride],
            alpha_ref=full.alpha_ref[::stride], n_texp=full.n_texp[::stride])
        ctx.set_lines(0, sub)
        run = {"lines": int(sub.n)}
        for prec in ("fp32", "fp64"):
            run[f"modit_{prec}_ms"] = 1e3 * timed(lambda: ctx.cross_section_modit(0, T, P, prec), reps)
        run["direct_fp32_ms"] = 1e3 * timed(lambda: ctx.cross_section(0, T, P, "fp32"), 1 if stride == 1 else 3)
        run["direct_over_modit_fp32"] = run["direct_fp32_ms"] / run["modit_fp32_ms"]
        run["direct_fp32_evals_per_s"] = sub.n * wl.nu.size / (1e-3 * run["direct_fp32_ms"])
        # weak-line pre-selection (App. G) of the same list on the config-3 atmosphere:
        # isothermal 1700 K, strengths scanned over 500-1700 K, margin 2 layers
        run["select_ms"] = 1e3 * timed(lambda: ctx.select_lines(0, math.log10(0.0023), atm, 1700.0, T_scan, 2),
                                       reps)
        run["select_kept"] = ctx.select_lines(0, math.log10(0.0023), atm, 1700.0, T_scan, 2)[1]
        out["runs"].append(run)
    ctx.close()
    out["emission"] = modit_emission_bench(wl, reps)
    out["emission"]["direct_single_layer_fp32_ms"] = out["runs"][-1]["direct_fp32_ms"]
    return out


def config1_bench(reps=50):
    """Configuration 1: one layer (1000 K, 1 bar) of 1000 lines on a
    4000-point linear grid, FP32 and the plain FP64 form; median time per
    call after a warm-up (a latency-bound call)."""
    import torch
    import synth
    from paper_2105_14782_amd import api
    wl = synth.make_config(1, "full")
    ctx = api.Context(0)
    ctx.set_lines(0, wl.lines[0])
    ctx.set_grid(wl.nu)
    out = {"workload": "config-1 cross-section: 1000 lines, 4000-point linear grid, 1000 K, 1 bar"}
    for prec in ("fp32", "fp64"):
        ctx.cross_section(0, wl.T, wl.P_bar, prec)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            ctx.cross_section(0, wl.T, wl.P_bar, prec)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        us = 1e6 * float(np.median(ts))
        out[f"{prec}_us"] = us
        out[f"{prec}_evals_per_s"] = wl.lines[0].n * wl.nu.size / (1e-6 * us)
    ctx.close()
    return out


def config3_direct_bench(wl=None, fp64_layer=True):
    """The throughput workload by the direct sum: one FP32 forward spectrum
    (F0, no response) of all of config 3 (1e7 lines x 100,000 points x 100
    layers = 1e14 pair evaluations), with the Voigt kernel's share and its
    per-tier pair fractions; then one layer (700 K, 1 bar) of the same list
    in FP32 and in the plain FP64 form (1e12 evaluations each)."""
    import torch
    import synth
    from paper_2105_14782_amd import api
    wl = wl if wl is not None else synth.make_config(3, "full")
    ctx = api.Context(0)
    ctx.set_lines(0, wl.lines[0])
    ctx.set_grid(wl.nu)
    atm = api.Atmos.from_workload(wl.atmos, [0])
    ctx.profile(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.emission_flux(atm, None, "fp32")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    nl, kms, evals = ctx.profile_read()
    near = ctx.profile_read_near()
    cut = ctx.profile_read_far_cut()
    outer = ctx.profile_read_far_outer()
    ctx.profile(False)
    total = wl.lines[0].n * wl.nu.size * wl.atmos.P_bar.size
    out = {"workload": "config-3 direct-sum FP32 spectrum: 1e7 lines, 100,000 points, 100 layers",
           "s": dt, "evals": total, "evals_per_s": total / dt, "voigt_kernel_ms": kms,
           "voigt_launches": nl, "voigt_share": 1e-3 * kms / dt,
           "near_fraction": near / max(evals, 1.0), "far_cut_fraction": cut / max(evals, 1.0),
           "outer_fraction": outer / max(evals, 1.0),
           "far_fraction": (evals - near - cut - outer) / max(evals, 1.0)}
    if fp64_layer:
        # one layer at 700 K, where the FP32 cross-section fits its range (see modit_bench)
        T, P = 700.0, 1.0
        ts = {}
        for prec in ("fp32", "fp64"):
            ctx.cross_section(0, T, P, prec)
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.cross_section(0, T, P, prec)
            torch.cuda.synchronize()
            ts[prec] = time.perf_counter() - t
        out["one_layer"] = {"T_K": T, "P_bar": P, "evals": wl.lines[0].n * wl.nu.size,
                            "fp32_ms": 1e3 * ts["fp32"], "fp64_plain_ms": 1e3 * ts["fp64"],
                            "fp32_over_fp64_plain": ts["fp64"] / ts["fp32"]}
    ctx.close()
    return out


def modit_emission_bench(wl=None, reps=5):
    """The whole config-3 emission spectrum (all 1e7 lines, 100 layers, no
    response) with MODIT opacities, FP32 and FP64; the direct sum would take
    100 single-layer sums of all lines."""
    import torch
    import synth
    from dataclasses import replace
    from paper_2105_14782_amd import api
    wl = wl if wl is not None else synth.make_config(3, "full")
    ctx = api.Context(0)
    ctx.set_lines(0, wl.lines[0])
    ctx.set_grid(wl.nu)
    atm = replace(api.Atmos.from_workload(wl.atmos, [0]), opacity="modit")
    em = {"workload": "config-3 emission, 1e7 lines, 100 layers, 100,000-point grid, MODIT opacities"}
    for prec in ("fp32", "fp64"):
        ctx.emission_flux(atm, None, prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            ctx.emission_flux(atm, None, prec)
        torch.cuda.synchronize()
        em[f"modit_{prec}_ms"] = 1e3 * (time.perf_counter() - t) / reps
    # the FP32 form against the FP64 one: per-layer cross-sections spanning more
    # decades than an FP32 transform resolves lose their weak end
    f32 = ctx.emission_flux(atm, None, "fp32").double()
    f64 = ctx.emission_flux(atm, None, "fp64")
    rel = ((f32 - f64).abs() / f64.abs()).cpu().numpy()
    em["fp32_vs_fp64_rel"] = {"median": float(np.median(rel)), "p99": float(np.percentile(rel, 99)),
                              "max": float(rel.max())}
    ctx.close()
    return em


SERVE_MARGIN = 260   # output margin (points) at R0 = 1e6: rotation + RV + 6-sigma IP reach < 200


def serving_bench(n_req, loads=(0.9,), n_streams=4, budget=48 << 30, n_cap=200, policies=("fifo",)):
    """Continuous batching on a stream shaped like the serving configuration:
    16 resident lists (1e3-1e6 lines, 3900-5100 cm^-1), windows of 2e3-1e5
    points on an R0 = 1e6 grid, 50-200 layers, HMC-like parameter walk.
    Capacity is measured closed-loop first (n_cap requests submitted at
    once); then n_req Poisson arrivals at each load x capacity give the
    latency distribution, from each request's scheduled arrival to its
    spectrum on the device, for each admission policy ("fifo": arrival
    order; "shortest": fewest evaluations first, a request passed over at
    most 16 times; the same arrival sequence for both).  The top-level
    latency fields are those of the first policy at the first load."""
    import torch
    import synth
    from paper_2105_14782_amd import api, serve
    lists, nu = synth.serving_pool()
    ctx = api.Context(0)
    for s, ll in enumerate(lists):
        ctx.set_lines(s, ll)
    ctx.set_grid(nu)
    u1, u2 = 0.5366563145999494, 0.35777087639996635

    def args(reqs):
        out = []
        for q in reqs:
            P, T0, al, logx, rv, vs = synth.serving_atmosphere(q)
            atm = api.Atmos(P, T0, al, list(q.species), list(logx), cia_alpha0=5e-46, cia_Tpow=1.0,
                            cia_slope=0.1, cia_nu_c=4500.0, vmr_h2=0.75 * 2.33 / 2.016,
                            grid_begin=q.grid_begin, grid_len=q.grid_len)
            out.append((atm, api.Response(rv, vs, u1, u2, 1e5, SERVE_MARGIN, q.grid_len - 2 * SERVE_MARGIN)))
        return out

    warm = args(synth.serving_requests(n_streams, 0.0, nu_master=nu, seed=7))
    srv = serve.Server(ctx, n_streams=n_streams, mem_budget_bytes=budget)
    serve.run_stream(srv, warm)
    closed = args(synth.serving_requests(n_cap, 0.0, nu_master=nu, seed=11))
    cap = serve.run_stream(srv, closed)
    print(f"serving: capacity {cap['spectra_per_s']:.2f} spectra/s over {n_cap} requests", file=sys.stderr,
          flush=True)
    evals = lambda reqs: sum((lists[a.species[0]].n + lists[a.species[1]].n) * a.grid_len * len(a.P_bar)
                             for a, _ in reqs)
    runs = []
    for policy in policies:
        srv.set_policy(policy, 16)
        for rho in loads:
            rate = rho * cap["spectra_per_s"]
            reqs = synth.serving_requests(n_req, rate, nu_master=nu)
            arr = np.array([q.arrival_s for q in reqs])
            st0 = srv.stats()
            res = serve.run_stream(srv, args(reqs), arr, progress=max(250, n_req // 20))
            st1 = srv.stats()
            lat = res["latency_s"]
            runs.append({"policy": policy, "load": rho, "arrival_rate_hz": rate,
                         "spectra_per_s": res["spectra_per_s"], "p50_ms": res["p50_ms"], "p99_ms": res["p99_ms"],
                         "p90_ms": float(np.percentile(lat, 90) * 1e3), "max_ms": float(lat.max() * 1e3),
                         "bypasses": st1["bypasses"] - st0["bypasses"]})
            print(f"serving: {policy}, load {rho}: p50 {res['p50_ms']:.0f} ms, p99 {res['p99_ms']:.0f} ms",
                  file=sys.stderr, flush=True)
    st = srv.stats()
    srv.close()
    ctx.close()
    first = runs[0]
    return {"requests": n_req, "capacity_requests": n_cap, "streams": n_streams,
            "capacity_spectra_per_s": cap["spectra_per_s"],
            "capacity_evals_per_s": evals(closed) / cap["wall_s"],
            "arrival_rate_hz": first["arrival_rate_hz"], "spectra_per_s": first["spectra_per_s"],
            "p50_ms": first["p50_ms"], "p99_ms": first["p99_ms"], "latency_from": "scheduled arrival",
            "loads": runs, "peak_in_flight": st["peak_in_flight"],
            "mem_peak_gb": st["mem_peak_bytes"] / 2 ** 30, "mem_budget_gb": st["mem_budget_bytes"] / 2 ** 30}


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, os.path.join(ROOT, TRAFFIC_PROFILE))
        return
    if args.summarize_valu:
        summarize_valu(args.summarize_valu, os.path.join(ROOT, VALU_PROFILE))
        return
    if args.summarize_response:
        summarize_response(args.summarize_response, os.path.join(ROOT, RESPONSE_PROFILE))
        return
    if args.summarize_flops:
        summarize_flops(args.summarize_flops, os.path.join(ROOT, FLOPS_PROFILE))
        return
    if args.summarize_stats:
        summarize_stats(args.summarize_stats, os.path.join(ROOT, STATS_PROFILE))
        return
    if args.summarize_modit_stats:
        summarize_stats(args.summarize_modit_stats, os.path.join(ROOT, MODIT_PROFILE), modit=True)
        return
    if args.summarize_modit_emission_stats:
        summarize_stats(args.summarize_modit_emission_stats, os.path.join(ROOT, MODIT_EMISSION_PROFILE),
                        modit="emission")
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.modit_only:
        print(json.dumps({"modit": modit_bench()}), flush=True)
        return
    if args.modit_emission_only:
        print(json.dumps({"modit_emission": modit_emission_bench()}), flush=True)
        return
    if args.config3_direct:
        print(json.dumps({"config3_direct": config3_direct_bench()}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_bench(args.serve_requests, args.serve_load, n_streams=args.serve_streams,
                                                   n_cap=args.serve_capacity_requests,
                                                   policies=args.serve_policy)}), flush=True)
        return
    import torch
    import synth
    from paper_2105_14782_amd import api

    wl = synth.make_config(2, args.size)
    theta = wl.theta_star
    ctx = api.Context(0)
    for s, ll in enumerate(wl.lines):
        ctx.set_lines(s, ll)
    ctx.set_grid(wl.nu)
    torch.cuda.synchronize()
    # the one-time upload (the paper's "with transfer" case): both line lists
    # and the grid again, validated, sorted on the host and copied to HBM
    tu = time.perf_counter()
    for s, ll in enumerate(wl.lines):
        ctx.set_lines(s, ll)
    ctx.set_grid(wl.nu)
    torch.cuda.synchronize()
    upload_ms = 1e3 * (time.perf_counter() - tu)
    atm = api.Atmos.from_workload(wl.atmos, [0, 1], theta)
    resp = api.Response.from_workload(wl.response, theta)
    n_out = resp.out_len
    rng = np.random.default_rng(5)
    # cotangent of an independent-Gaussian loss: seeded residuals / sigma
    cot = torch.tensor(rng.normal(size=n_out) * 1e-2, dtype=torch.float32, device="cuda")
    evals = wl.evals_per_spectrum
    stream = torch.cuda.current_stream()

    def step():
        return ctx.flux_vjp(atm, resp, cot, want_flux=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.counters:
        # one step, then a plain copy of known size whose FETCH_SIZE/WRITE_SIZE
        # calibrate the counters (512 MiB read + 512 MiB written)
        step()
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "counters", "copy_bytes": src.numel() * 4,
                          "voigt_launches_per_step": len(wl.lines)}), flush=True)
        ctx.close()
        return
    ctx.profile(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        step()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    nl, kms, kevals = ctx.profile_read()
    knear = ctx.profile_read_near()
    kcut = ctx.profile_read_far_cut()
    kout = ctx.profile_read_far_outer()
    ctx.profile(False)
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    ms = 1e3 * T / args.steps

    # forward-only spectra/s, FP32 and the plain FP64 form
    def time_fwd(prec, reps):
        ctx.emission_flux(atm, resp, prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            ctx.emission_flux(atm, resp, prec)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    t32 = time_fwd("fp32", max(3, args.steps))
    t64 = time_fwd("fp64", args.fp64_reps)
    t64t = time_fwd("fp64_tiled", max(3, args.fp64_reps))

    # agreement of the forms on this workload (outside the timed regions):
    # the FP32 spectrum against both FP64 spectra, and the FP32 gradient of
    # the bench's cotangent against the FP64 one
    F32 = ctx.emission_flux(atm, resp, "fp32").double()
    F64 = ctx.emission_flux(atm, resp, "fp64")
    F64t = ctx.emission_flux(atm, resp, "fp64_tiled")
    g32, _, _ = ctx.flux_vjp(atm, resp, cot)
    g64, _, _ = ctx.flux_vjp(atm, resp, cot.double(), precision="fp64_tiled")
    agreement = {
        "fp32_vs_fp64_plain_max_rel": float(((F32 - F64).abs() / F64.abs()).max()),
        "fp32_vs_fp64_tiled_max_rel": float(((F32 - F64t).abs() / F64t.abs()).max()),
        "fp64_tiled_vs_plain_max_rel": float(((F64t - F64).abs() / F64.abs()).max()),
        "gradient_fp32_vs_fp64_max_rel": float(np.max(np.abs(g32 - g64) / np.maximum(np.abs(g64), 1e-6 * np.abs(g64).max()))),
    }

    # one leapfrog step of the sampler: Gaussian likelihood and its gradient in one pass
    Fd = ctx.emission_flux(atm, resp, "fp32")
    dat = (Fd * (1.0 + 0.01 * torch.randn(Fd.numel(), device="cuda", generator=None))).contiguous()
    sig = (0.01 * Fd).contiguous()
    ctx.loss_grad(atm, resp, dat, sig)
    torch.cuda.synchronize()
    tl0 = time.perf_counter()
    for _ in range(max(3, args.steps // 2)):
        ctx.loss_grad(atm, resp, dat, sig)
    torch.cuda.synchronize()
    tloss = (time.perf_counter() - tl0) / max(3, args.steps // 2)

    # forward-mode derivative along a parameter tangent plus a per-layer
    # temperature tangent (spectrum and J dtheta in one call)
    dth = np.array([5.0, 1e-3, 1e-2, -1e-2, 0.1, 0.1])
    dT = np.random.default_rng(6).normal(size=atm.P_bar.size)
    ctx.flux_jvp(atm, resp, dth, dT)
    torch.cuda.synchronize()
    tj0 = time.perf_counter()
    for _ in range(max(3, args.steps // 2)):
        ctx.flux_jvp(atm, resp, dth, dT)
    torch.cuda.synchronize()
    tjvp = (time.perf_counter() - tj0) / max(3, args.steps // 2)

    avg_launch_ms = kms / max(nl, 1)
    flops_per_launch = (FLOPS_PER_EVAL_NEAR * knear + FLOPS_PER_EVAL_FAR * (kevals - knear - kcut - kout)
                        + FLOPS_PER_EVAL_FAR_CUT * kcut + FLOPS_PER_EVAL_OUTER * kout) / max(nl, 1)
    achieved = flops_per_launch / (avg_launch_ms * 1e-3) / 1e12
    hw = recorded_counter_flops()
    counter_tflops = None if hw is None else hw[0] / (avg_launch_ms * 1e-3) / 1e12
    counter_tflops64 = None if hw is None else hw[1] / (avg_launch_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": evals / (ms * 1e-3),
        "unit": "Voigt evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"config-2 emission forward+gradient ({args.size}): 2 species x "
                               f"{wl.lines[0].n} lines, {wl.nu.size}-point log-uniform grid, "
                               f"{wl.atmos.P_bar.size} layers, rotation+RV+IP response, flux_vjp",
                   "evals_per_step": evals, "precision": "FP32 Voigt + compensated sum, FP64 line params/offsets"},
        "spectra_per_s": 1e3 / ms,
        "upload_ms": upload_ms,
        "step_with_upload_ms": upload_ms + ms,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "forward_fp32": {"spectra_per_s": 1.0 / t32, "evals_per_s": evals / t32},
        "forward_fp64_plain": {"spectra_per_s": 1.0 / t64, "evals_per_s": evals / t64},
        "forward_fp64_tiled": {"spectra_per_s": 1.0 / t64t, "evals_per_s": evals / t64t,
                               "form": "the FP32 form's tiling, staging, near/far split and core branch in "
                                       "FP64, full asymptotic polynomial on every wing pair"},
        "fp32_over_fp64_spectra": t64 / t32,
        "fp32_over_fp64_plain_spectra": t64 / t32,
        "fp32_over_fp64_tiled_spectra": t64t / t32,
        "agreement": agreement,
        "flux_jvp": {"ms_per_call": tjvp * 1e3, "evals_per_s": evals / tjvp},
        "leapfrog_loss_grad": {"ms_per_call": tloss * 1e3, "evals_per_s": evals / tloss},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": recorded_traffic(),
                     "model_tflops": achieved,
                     "counter_tflops": counter_tflops, "counter_fp64_tflops": counter_tflops64,
                     "counter_frac": None if counter_tflops is None else counter_tflops / PEAK_FP32_TFLOPS,
                     "non_packed_peak": PEAK_FP32_TFLOPS / 2,
                     "evals_counted": "every (line, grid point, layer) pair is evaluated, but by tier: the "
                                      "full wing polynomial (near tier, core pairs by the rational w), the "
                                      "polynomial cut after r^3 (far) or after r^2 (outer), each cut below "
                                      "FP32 rounding of that pair; see the *_fraction fields",
                     "kernel": "k_voigt_f32<tangent>", "avg_launch_ms": avg_launch_ms,
                     "launches": nl, "evals_per_launch": kevals / max(nl, 1),
                     "near_fraction": knear / max(kevals, 1.0),
                     "far_cut_fraction": kcut / max(kevals, 1.0),
                     "outer_fraction": kout / max(kevals, 1.0),
                     "flops_per_eval": {"near": FLOPS_PER_EVAL_NEAR, "far": FLOPS_PER_EVAL_FAR,
                                        "far_cut": FLOPS_PER_EVAL_FAR_CUT, "outer": FLOPS_PER_EVAL_OUTER},
                     "evals_per_s": kevals / (kms * 1e-3)},
    }
    ctx.close()
    if args.serve_requests > 0:
        out["serving"] = serving_bench(args.serve_requests, args.serve_load, n_streams=args.serve_streams,
                                       n_cap=args.serve_capacity_requests, policies=args.serve_policy)
    wl3 = None
    if not args.no_config3 or not args.no_modit:
        wl3 = synth.make_config(3, "full")
    if not args.no_config3:
        out["config3"] = config3_direct_bench(wl3)
        print(f"config3: direct FP32 spectrum {out['config3']['s']:.2f} s", file=sys.stderr, flush=True)
    if not args.no_modit:
        out["modit"] = modit_bench(wl3)
    out["config1"] = config1_bench()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, theta, args.cpu_points)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
