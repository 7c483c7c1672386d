#!/usr/bin/env python3
"""Throughput of the lattice scalar-field hot path on one MI355X.

Workload (default): two-field preheating, V = phi^4/4 + q phi^2 chi^2/2 with
q = 100, 256^3 lattice, k_IR = 0.5, 4th-order velocity Verlet, dt = 0.05 dx,
FP32 fields with FP64 lattice sums and scale factor, self-consistent
expansion, seeded vacuum fluctuations.  One bench step = one full time step
(three fused drift-kick-reduce passes over the lattice).  The same run is
repeated with FP64 fields; the FP32 form's deviation from it on the volume
averages is reported next to both rates (the comparison at fixed error).

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "site-updates/s + %HBM peak: FP64 vs FP32 vs surrogate at fixed error"
HBM_PEAK_GBS = 8000.0


def bytes_per_site(precision: str, nf: int) -> int:
    """Algorithmic HBM bytes of one fused drift-kick pass per lattice site:
    read f and pi, write f and pi, per field."""
    return 4 * nf * (4 if precision == "fp32" else 8)


def kpass_bytes_per_site(precision: str, nf: int) -> int:
    """Opening kick: read f and pi, write pi."""
    return 3 * nf * (4 if precision == "fp32" else 8)


def make(w, precision, stream):
    from paper_2607_24978_amd import _lib
    lat = _lib.Lattice(w.N, w.dx, w.n_fields, precision)
    lat.set_stream(stream.cuda_stream)
    lat.set_background(w.alpha, w.expansion, w.mp, w.a0)
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    lat.seed(w.seed, w.fbar[:w.n_fields], w.pbar[:w.n_fields], w.cutoff_modes, w.amp)
    return lat


def timed_run(w, precision, steps, warmup, chunk):
    """Seed, run `warmup` untimed steps, then `steps` timed steps in calls of
    `chunk` steps.  Returns (records of all steps, seconds, event ms, passes)."""
    import torch
    stream = torch.cuda.Stream()
    lat = make(w, precision, stream)
    recs = []
    for _ in range(warmup // chunk):
        recs.append(lat.step(w.integrator, w.dt, chunk))
    if warmup % chunk:
        recs.append(lat.step(w.integrator, w.dt, warmup % chunk))
    ncalls = steps // chunk
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(ncalls):
        recs.append(lat.step(w.integrator, w.dt, chunk))
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat.close()
    per = 3 if w.integrator == "vv4" else 1
    dk_passes = ncalls * chunk * per
    return np.concatenate(recs), t1 - t0, e0.elapsed_time(e1), dk_passes, ncalls


def linear_regime_deviation(r32, r64, nf):
    """Max relative deviation of the FP32 run's volume averages from the FP64
    run's, over the steps where every field's variance is still within
    1e4 of its initial value (the linear regime)."""
    v0 = r64["var"][0, :nf]
    lin = np.all(r64["var"][:, :nf] <= 1e4 * v0, axis=1)
    end = int(np.argmin(lin)) if not np.all(lin) else len(lin)
    out = {"linear_regime_steps": end}
    worst = 0.0
    for k in ("a", "EV"):
        d = np.max(np.abs(r32[k][:end] - r64[k][:end]) / np.abs(r64[k][:end]))
        out[k] = float(d)
        worst = max(worst, d)
    for k in ("EK", "EG", "var"):
        for j in range(nf):
            d = np.max(np.abs(r32[k][:end, j] - r64[k][:end, j]) / np.abs(r64[k][:end, j]))
            out[f"{k}{j}"] = float(d)
            worst = max(worst, d)
    out["max"] = float(worst)
    return out


def cpu_baseline(w, steps=1):
    """The FP64 oracle as it stands, on the same 256^3 workload, for a bounded
    number of full steps on the host (numpy, single thread)."""
    from oracle import lattice as L
    from oracle import seed as S
    P = L.Params(N=w.N, dx=w.dx, n_fields=w.n_fields, alpha=w.alpha, mp=w.mp, expansion=w.expansion,
                 m2=w.m2, lam=w.lam, g2=w.g2, V0=w.V0)
    s = S.seed_state(P, w.k_ir, w.fbar[:w.n_fields], w.pbar[:w.n_fields], w.seed, cutoff=w.cutoff_modes)
    t0 = time.perf_counter()
    for _ in range(steps):
        s = L.step(s, w.dt, P, w.integrator)
    dt = time.perf_counter() - t0
    return {"value": w.sites * steps / dt, "unit": "site-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} full {w.integrator} step(s) of the {w.N}^3 {w.n_fields}-field workload "
                      f"in FP64 numpy on one host core ({platform.processor() or platform.machine()}, "
                      f"{os.cpu_count()} logical CPUs visible), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--chunk", type=int, default=500)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)

    w = W.C1
    chunk = max(1, min(args.chunk, args.steps))
    if args.steps % chunk:
        chunk = math.gcd(args.steps, chunk)
    r32, sec32, ms32, dk32, calls32 = timed_run(w, "fp32", args.steps, args.warmup, chunk)
    value = w.sites * args.steps / sec32
    ms_per_step = 1e3 * sec32 / args.steps
    # dominant kernel: the fused drift-kick-reduce pass (plus one opening kick per call)
    alg = dk32 * bytes_per_site("fp32", w.n_fields) * w.sites + calls32 * kpass_bytes_per_site("fp32", 2) * w.sites
    launches = dk32 + calls32
    avg_ms = ms32 / launches
    achieved = alg / launches / (avg_ms * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": value, "unit": "site-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32", "data": "synthetic (seeded vacuum fluctuations)",
        "config": {"workload": w.name, "N": w.N, "n_fields": w.n_fields, "k_ir": w.k_ir, "q": w.g2,
                   "integrator": w.integrator, "dt": w.dt, "sums_and_scale_factor": "fp64",
                   "steps_per_call": chunk, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "lattice_pass<float,2>", "avg_launch_us": avg_ms * 1e3,
                     "alg_bytes_per_launch": alg / launches},
    }
    forms = {"fp32": {"site_updates_per_s": value, "hbm_frac": achieved / HBM_PEAK_GBS}}
    if not args.no_fp64:
        r64, sec64, ms64, dk64, calls64 = timed_run(w, "fp64", args.steps, args.warmup, chunk)
        alg64 = dk64 * bytes_per_site("fp64", 2) * w.sites + calls64 * kpass_bytes_per_site("fp64", 2) * w.sites
        ach64 = alg64 / (ms64 * 1e-3) / 1e9
        forms["fp64"] = {"site_updates_per_s": w.sites * args.steps / sec64, "hbm_frac": ach64 / HBM_PEAK_GBS}
        forms["fp32_vs_fp64_rel_dev"] = linear_regime_deviation(r32, r64, w.n_fields)
        forms["fp32_speedup_vs_fp64"] = value / forms["fp64"]["site_updates_per_s"]
    line["forms"] = forms
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, steps=1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
