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
# Algorithmic FP32 operations per (line, grid point, layer) pair of the Voigt
# sum in tangent mode (wing branch, FMA = 2): offset 1, D 2, 1/D 1, value
# polynomial 12 + 1, tangent polynomial 14 + 1, two accumulations 2.
FLOPS_PER_EVAL_TANGENT = 34.0
FLOPS_PER_EVAL_FORWARD = 18.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", default="full", choices=["small", "medium", "full"])
    ap.add_argument("--fp64-reps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-points", type=int, default=16)
    return ap.parse_args()


def cpu_baseline(wl, theta, n_points):
    """The FP64 oracle on a bounded sample: F0 at n_points grid points, all lines and layers."""
    threads = min(16, os.cpu_count() or 1)
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
            "sample": f"F0 at {n_points} random grid points x all {sum(l.n for l in wl.lines)} lines "
                      f"x {wl.atmos.P_bar.size} layers (FP64 scipy wofz + exact E3), {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import synth
    from paper_2105_14782_amd import api

    wl = synth.make_config(2, args.size)
    theta = wl.theta_star
    ctx = api.Context(0)
    for s, ll in enumerate(wl.lines):
        ctx.set_lines(s, ll)
    ctx.set_grid(wl.nu)
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

    avg_launch_ms = kms / max(nl, 1)
    flops_per_launch = FLOPS_PER_EVAL_TANGENT * kevals / max(nl, 1)
    achieved = flops_per_launch / (avg_launch_ms * 1e-3) / 1e12
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
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "forward_fp32": {"spectra_per_s": 1.0 / t32, "evals_per_s": evals / t32},
        "forward_fp64_plain": {"spectra_per_s": 1.0 / t64, "evals_per_s": evals / t64},
        "fp32_over_fp64_spectra": t64 / t32,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "k_voigt_f32<tangent>", "avg_launch_ms": avg_launch_ms,
                     "launches": nl, "flops_per_eval": FLOPS_PER_EVAL_TANGENT},
    }
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, theta, args.cpu_points)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
