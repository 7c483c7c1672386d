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


def progress(msg: str):
    """One progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)
HBM_PEAK_GBS = 8000.0


def bytes_per_site(precision: str, nf: int) -> int:
    """Algorithmic HBM bytes of one fused drift-kick pass per lattice site:
    read f and pi, write f and pi, per field."""
    return 4 * nf * (4 if precision == "fp32" else 8)


def kpass_bytes_per_site(precision: str, nf: int) -> int:
    """Opening kick: read f and pi, write pi."""
    return 3 * nf * (4 if precision == "fp32" else 8)


def measured_traffic(workload: str, tile: dict):
    """HBM bytes per launch from the committed rocprofv3 counter record, or None
    when the kernel source changed since the counters were taken or the tile
    differs (the prefetch depth, which does not change the bytes a pass
    touches, is not compared)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["kernel_source"]), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != rec["sha256_prefix"]:
        return None
    key = [tile["tz"], tile["ty"], tile["cx"], tile["ry"]]
    for e in rec["entries"]:
        if e["workload"] == workload and e["tile"][:4] == key:
            return e["traffic_bytes_per_launch"]
    return None


def make(w, precision, stream, tune=True, tile=None):
    from paper_2607_24978_amd import _lib
    lat = _lib.Lattice(w.N, w.dx, w.n_fields, precision)
    lat.set_stream(stream.cuda_stream)
    lat.set_background(w.alpha, w.expansion, w.mp, w.a0)
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    progress(f"seeding {w.N}^3 {precision}")
    lat.seed(w.seed, w.fbar[:w.n_fields], w.pbar[:w.n_fields], w.cutoff_modes, w.amp)
    if tile is not None:
        lat.set_tile(*tile)
    elif tune:
        progress("autotuning the pass tile")
        lat.autotune(reps=3)  # the library's own tile search (state is left unchanged)
    progress(f"tile {lat.get_tile()}")
    return lat


def timed_run(w, precision, steps, warmup, chunk, tune=True, tile=None):
    """Seed, autotune, run `warmup` untimed steps, then `steps` timed steps in
    calls of `chunk` steps.  Returns (records of all steps, seconds, event ms,
    fused passes, calls, tile)."""
    import torch
    stream = torch.cuda.Stream()
    lat = make(w, precision, stream, tune, tile)
    tile = lat.get_tile()
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
    for i in range(ncalls):
        recs.append(lat.step(w.integrator, w.dt, chunk))
        if time.perf_counter() - t0 > 30 and i % 10 == 0:
            progress(f"timed call {i + 1}/{ncalls}")
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat.close()
    per = 3 if w.integrator == "vv4" else 1
    dk_passes = ncalls * chunk * per
    return np.concatenate(recs), t1 - t0, e0.elapsed_time(e1), dk_passes, ncalls, tile


def linear_regime_deviation(r32, r64, nf):
    """Max relative deviation of the FP32 run's volume averages from the FP64
    run's, over the steps where every field's variance is still within 1e4 of
    its initial value (the linear regime).  a, H, EG and var are compared to
    themselves; EK and EV, which pass through zero as the homogeneous field
    oscillates, relative to the total energy density of the same step."""
    v0 = r64["var"][0, :nf]
    lin = np.all(r64["var"][:, :nf] <= 1e4 * v0, axis=1)
    end = int(np.argmin(lin)) if not np.all(lin) else len(lin)
    out = {"linear_regime_steps": end}
    rho = (r64["EK"][:end, :nf].sum(1) + r64["EG"][:end, :nf].sum(1) + r64["EV"][:end])
    worst = 0.0
    for k in ("a", "H", "EV"):
        scale = rho if k == "EV" else np.abs(r64[k][:end])
        d = np.max(np.abs(r32[k][:end] - r64[k][:end]) / scale)
        out[k] = float(d)
        worst = max(worst, d)
    for k in ("EK", "EG", "var"):
        for j in range(nf):
            scale = rho if k == "EK" else np.abs(r64[k][:end, j])
            d = np.max(np.abs(r32[k][:end, j] - r64[k][:end, j]) / scale)
            out[f"{k}{j}"] = float(d)
            worst = max(worst, d)
    out["max"] = float(worst)
    return out


def batched_run(steps, warmup, solo_steps=100):
    """The 96-member uneven ensemble (48 x 32^3, 32 x 64^3, 16 x 128^3, FP32,
    one field, leapfrog): all members advanced together, one persistent
    launch per pass, passes captured in a HIP graph.  Also times every member
    run on its own for `solo_steps` steps, for the batching gain."""
    import torch
    from paper_2607_24978_amd import _lib
    ws = W.ensemble_members()
    lats = []
    for w in ws:
        lat = _lib.Lattice(w.N, w.dx, 1, "fp32")
        lat.set_potential(w.m2, w.lam, w.g2, w.V0)
        lat.seed(w.seed, w.fbar[:1], w.pbar[:1], w.cutoff_modes, w.amp)
        lats.append(lat)
    progress(f"ensemble: {len(lats)} members seeded")
    sites = sum(w.sites for w in ws)
    # solo: each member on its own stream-less handle, back to back
    torch.cuda.synchronize()
    for lat, w in zip(lats, ws):
        lat.step("leapfrog", w.dt, 2)
    t0 = time.perf_counter()
    for lat, w in zip(lats, ws):
        lat.step("leapfrog", w.dt, solo_steps)
    solo_s = time.perf_counter() - t0
    progress(f"ensemble: members run one by one ({solo_s:.2f} s)")
    ens = _lib.Ensemble(lats)
    for i, w in enumerate(ws):
        ens.set_dt(i, w.dt)
    progress("ensemble: created, searching the work layout")
    tune = ens.autotune(reps=3)  # the library's decomposition search (states unchanged)
    progress(f"ensemble layout {tune['best']}")
    chunk = min(steps, 500)
    ens.step("leapfrog", chunk)  # warm-up call captures the graph
    for _ in range(max(0, warmup - chunk) // chunk):
        ens.step("leapfrog", chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // chunk):
        r = ens.step("leapfrog", chunk)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    nsteps = (steps // chunk) * chunk
    ok = not bool(np.any(r["nonfinite"]))
    ens.close()
    for lat in lats:
        lat.close()
    launches = nsteps + steps // chunk
    achieved = sites * 16 * launches / sec / 1e9
    return {"members": len(ws), "sites": sites, "steps": nsteps, "site_updates_per_s": sites * nsteps / sec,
            "ms_per_step": 1e3 * sec / nsteps, "hbm_frac": achieved / HBM_PEAK_GBS,
            "solo_site_updates_per_s": sites * solo_steps / solo_s,
            "batched_speedup_vs_solo": (sites * nsteps / sec) / (sites * solo_steps / solo_s), "finite": ok,
            "layout": tune["best"]}


def _scalar_errors(rec, ref, nf):
    """Max relative deviation of per-jump volume averages from the reference
    (a, H, EG, var relative to themselves; EK and EV relative to the total
    energy density, as they pass through zero)."""
    rho = ref["EK"][:, :nf].sum(1) + ref["EG"][:, :nf].sum(1) + ref["EV"]
    out = {}
    for k in ("a", "H", "EV"):
        scale = rho if k == "EV" else np.abs(ref[k])
        out[k] = float(np.max(np.abs(rec[k] - ref[k]) / scale))
    for k in ("EK", "EG", "var"):
        for j in range(nf):
            scale = rho if k == "EK" else np.abs(ref[k][:, j])
            out[f"{k}{j}"] = float(np.max(np.abs(rec[k][:, j] - ref[k][:, j]) / scale))
    out["max"] = max(out.values())
    return out


def _field_error(lat, ref_lat):
    """Norm-wise relative field error max_j ||f_j - f_ref_j||_inf / ||f_ref_j - <f_ref_j>||_inf
    (fluctuations, since the homogeneous value would hide them)."""
    f, p = lat.get_fields()
    fr, pr = ref_lat.get_fields()
    err = 0.0
    for x, xr in ((f, fr), (p, pr)):
        for j in range(x.shape[0]):
            d = xr[j] - xr[j].mean()
            err = max(err, float(np.max(np.abs(x[j].astype(np.float64) - xr[j])) / np.max(np.abs(d))))
    return err


def surrogate_flops_per_site(extra_inputs: int, nf: int = 2, hidden: int = 32, layers: int = 5) -> int:
    """Useful multiply-add flops of one network evaluation per lattice site
    (2 x 27 x c_in x c_out summed over the layers, real channel counts)."""
    ch = [2 * nf + extra_inputs] + [hidden] * (layers - 1) + [2 * nf]
    return sum(2 * 27 * a * b for a, b in zip(ch[:-1], ch[1:]))


MFMA_BF16_PEAK = 2.5e15


def surrogate_forward_profile(N=256, reps=5):
    """Forward passes of the 8-input surrogate network (random weights,
    seeded random inputs of shape [8, N, N, N]) for a kernel-level profile of
    the BF16 MFMA convolutions: the host copies of each call are outside the
    kernels, whose durations a trace reports; useful flops per call are
    surrogate_flops_per_site * N^3."""
    from paper_2607_24978_amd import _lib
    s = _lib.Surrogate(n_fields=2, extra_inputs=4, init_seed=7)
    x = np.random.default_rng(5).standard_normal((8, N, N, N)).astype(np.float32)
    s.forward(x)
    t0 = time.perf_counter()
    for _ in range(reps):
        y = s.forward(x)
    sec = time.perf_counter() - t0
    s.close()
    return {"N": N, "calls": reps, "flops_per_call": surrogate_flops_per_site(4) * N ** 3,
            "wall_s_per_call_incl_host_copies": sec / reps, "finite": bool(np.all(np.isfinite(y)))}


def surrogate_train_profile(N=128, pairs=4, epochs=5):
    """Training steps of the 8-input surrogate at N^3 (pairs recorded from a
    seeded two-field VV4 run) for a kernel-level profile of one training
    step: forward with pre-activations, MSE gradient, weight gradients and
    their reduction, input gradients through the hidden layers, GELU
    derivative, Adam and the BF16 weight refresh."""
    from paper_2607_24978_amd import _lib
    K = 16
    w = W.C1.with_(N=N, precision="fp64")
    s = _lib.Surrogate(n_fields=2, extra_inputs=4, layers=5, jump_steps=K, init_seed=0)
    s.dataset_reserve(N, pairs)
    lat = _lib.Lattice(w.N, w.dx, 2, "fp64")
    lat.set_background(w.alpha, w.expansion, w.mp, w.a0)
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    lat.seed(w.seed, w.fbar[:2], w.pbar[:2], w.cutoff_modes, w.amp)
    for _ in range(pairs):
        s.record_input(lat)
        lat.step("vv4", w.dt, K, record=False)
        s.record_target(lat)
    lat.close()
    rep = s.train(epochs=epochs, lr=5e-4, lr_final=5e-6, shuffle_seed=0, holdout=0)
    s.close()
    return {"N": N, "steps": rep["steps"], "steps_per_s": rep["steps"] / rep["seconds"],
            "flops_per_step": 3 * surrogate_flops_per_site(4) * N ** 3}


def linear_jump_profile(N=256, jumps=10, k_ir=0.25):
    """Linear jumps (CL_JUMP_LINEAR, 16 VV4 steps each, default gates) on the
    seeded two-field FP32 workload at N^3 (k_IR = 0.25: the training grid
    spacing of the surrogate study at 256^3) for a kernel-level profile of
    one jump: packing fused with the forward z pass, the FP32 y and x
    passes, the transfer table, the modes, the inverse x and y passes, the
    inverse z pass fused with the unpacking, and the gates' reduction."""
    from paper_2607_24978_amd import _lib
    K = 16
    w = W.C1.with_(N=N, k_ir=k_ir, seed=3000)
    lat = _lib.Lattice(w.N, w.dx, 2, "fp32")
    lat.set_background(w.alpha, w.expansion, w.mp, w.a0)
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    lat.seed(w.seed, w.fbar[:2], w.pbar[:2], w.cutoff_modes, w.amp)
    sg = _lib.Surrogate(n_fields=2, extra_inputs=2, layers=2, jump_steps=K, init_seed=1)
    sg.set_jump("linear")
    sg.advance(lat, "vv4", w.dt, 1)
    _, rep = sg.advance(lat, "vv4", w.dt, jumps)
    lat.close()
    sg.close()
    sites = float(N) ** 3
    return {"N": N, "jumps": jumps, "fallbacks": rep["fallbacks"], "seconds": rep["seconds"],
            "device_ms_per_jump": 1e3 * rep["net_seconds"] / jumps,
            "effective_site_updates_per_s": jumps * K * sites / rep["seconds"]}


def surrogate_run(epochs=12, pairs_per_seed=64, train_seeds=range(2000, 2008), eval_seed=3000, jumps=312,
                  extra_inputs=4, eval_256=True, ablation=False):
    """The learned surrogate on the two-field q = 100 workload: training pairs
    (state, state 16 VV4 steps later) from seeded 128^3 runs (k_IR = 0.5,
    dt = 0.05 dx), start steps spread over 5000 steps; training with the
    library's kernels; evaluation on an unseen seed against the FP64 VV4
    integrator over `jumps` jumps, next to the FP32 integrator forms, with the
    Hubble-residual fallback at 1e-3."""
    import torch
    from paper_2607_24978_amd import _lib
    K = 16
    wt = W.C1.with_(N=128, precision="fp64")
    out = {"train_N": wt.N, "k_ir": wt.k_ir, "dt": wt.dt, "jump_steps": K, "extra_inputs": extra_inputs}
    s = _lib.Surrogate(n_fields=2, extra_inputs=extra_inputs, layers=5, jump_steps=K, init_seed=0)
    seeds = list(train_seeds)
    s.dataset_reserve(wt.N, len(seeds) * pairs_per_seed)
    t0 = time.perf_counter()
    tiles = {}

    def tuned(lat, N, prec):
        """The library's tile search once per lattice size and precision."""
        if (N, prec) not in tiles:
            lat.autotune(reps=3)
            tiles[(N, prec)] = lat.get_tile()
        else:
            t = tiles[(N, prec)]
            lat.set_tile(t["tz"], t["ty"], t["cx"], t["ry"], t["pd"])
        return lat

    gap = (5000 - K) // pairs_per_seed   # start steps 0, gap, 2 gap, ... within the 5000-step run
    for seed in seeds:
        w = wt.with_(seed=seed)
        lat = _lib.Lattice(w.N, w.dx, 2, "fp64")
        lat.set_background(w.alpha, w.expansion, w.mp, w.a0)
        lat.set_potential(w.m2, w.lam, w.g2, w.V0)
        lat.seed(w.seed, w.fbar[:2], w.pbar[:2], w.cutoff_modes, w.amp)
        # the library's default tile, not a timed choice: the order of the
        # lattice sums (and so the training pairs, bit for bit) is the same
        # in every run
        for i in range(pairs_per_seed):
            if i and gap > K:
                lat.step("vv4", w.dt, gap - K, record=False)
            s.record_input(lat)
            lat.step("vv4", w.dt, K, record=False)
            s.record_target(lat)
        lat.close()
        progress(f"surrogate: training pairs of seed {seed} recorded")
    torch.cuda.synchronize()
    out["pairs"] = s.dataset_size()
    out["datagen_s"] = time.perf_counter() - t0
    progress(f"surrogate: training ({epochs} epochs)")
    rep = s.train(epochs=epochs, lr=5e-4, lr_final=5e-6, shuffle_seed=0, holdout=pairs_per_seed // 2)
    out["train"] = rep
    out["train_steps_per_s"] = rep["steps"] / rep["seconds"]
    progress(f"surrogate: trained, held-out loss {rep['holdout_loss']:.4g}")

    def evaluate(N, k_ir, njumps):
        w = W.C1.with_(N=N, k_ir=k_ir, seed=eval_seed)

        def lattice(prec):
            lat = _lib.Lattice(w.N, w.dx, 2, prec)
            lat.set_background(w.alpha, w.expansion, w.mp, w.a0)
            lat.set_potential(w.m2, w.lam, w.g2, w.V0)
            lat.seed(w.seed, w.fbar[:2], w.pbar[:2], w.cutoff_modes, w.amp)
            return tuned(lat, N, prec)

        res = {"N": N, "k_ir": k_ir, "dx": w.dx, "jumps": njumps, "steps": njumps * K}
        progress(f"surrogate: evaluation at {N}^3, k_IR = {k_ir}")
        # every form makes one untimed jump first (graph capture, buffers), then njumps timed ones
        ref = lattice("fp64")
        rr = np.concatenate([ref.step("vv4", w.dt, K)[-1:] for _ in range(njumps + 1)])[1:]
        forms = {}
        for name, prec, integ, mult in (("fp32_vv4", "fp32", "vv4", 1), ("fp64_vv4", "fp64", "vv4", 1),
                                        ("fp32_leapfrog", "fp32", "leapfrog", 1),
                                        ("fp32_leapfrog_dt4", "fp32", "leapfrog", 4),
                                        ("fp32_leapfrog_dt8", "fp32", "leapfrog", 8)):
            lat = lattice(prec)
            n = K // mult
            lat.step(integ, w.dt * mult, n, record=False)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            recs = np.concatenate([lat.step(integ, w.dt * mult, n)[-1:] for _ in range(njumps)])
            torch.cuda.synchronize()
            sec = time.perf_counter() - t1
            e = {"effective_site_updates_per_s": w.sites * njumps * K / sec, "seconds": sec}
            if name != "fp64_vv4":
                e["error_vs_fp64_vv4"] = _scalar_errors(recs, rr, 2)["max"]
                e["field_error"] = _field_error(lat, ref)
            forms[name] = e
            lat.close()
        lat = lattice("fp32")
        s.advance(lat, "vv4", w.dt, 1, threshold=1e-3)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        recs, srep = s.advance(lat, "vv4", w.dt, njumps, threshold=1e-3)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t1
        errs = _scalar_errors(recs, rr, 2)
        flops = surrogate_flops_per_site(extra_inputs) * w.sites * njumps
        progress("surrogate: surrogate form done")
        forms["surrogate"] = {"effective_site_updates_per_s": w.sites * njumps * K / sec, "seconds": sec,
                              "fallbacks": srep["fallbacks"], "fallback_rate": srep["fallbacks"] / max(1, njumps),
                              "accepted_fraction": 1.0 - srep["fallbacks"] / max(1, njumps),
                              "fluct_gate_rejects": srep["fluct_rejects"],
                              "max_residual": srep["max_residual"], "error_vs_fp64_vv4": errs["max"],
                              "errors": errs, "field_error": _field_error(lat, ref),
                              "network_ms_per_jump": 1e3 * srep["net_seconds"] / max(1, njumps),
                              "network_tflops": flops / srep["net_seconds"] / 1e12,
                              "mfma_frac": flops / srep["net_seconds"] / MFMA_BF16_PEAK}
        lat.close()
        # the linear propagation of the fluctuations instead of the network,
        # with the same gates and fallback
        lat = lattice("fp32")
        s.set_jump("linear")
        s.advance(lat, "vv4", w.dt, 1, threshold=1e-3)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        recs, srep = s.advance(lat, "vv4", w.dt, njumps, threshold=1e-3)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t1
        errs = _scalar_errors(recs, rr, 2)
        progress("surrogate: linear jump form done")
        forms["linear_jump"] = {"effective_site_updates_per_s": w.sites * njumps * K / sec, "seconds": sec,
                                "accepted_fraction": 1.0 - srep["fallbacks"] / max(1, njumps),
                                "fluct_gate_rejects": srep["fluct_rejects"], "max_residual": srep["max_residual"],
                                "error_vs_fp64_vv4": errs["max"], "errors": errs,
                                "field_error": _field_error(lat, ref),
                                "propagation_ms_per_jump": 1e3 * srep["net_seconds"] / max(1, njumps)}
        lat.close()
        # ... with the Hubble-residual gate alone (a resonance may grow a
        # variance by more than the second gate's 25 % within one jump)
        lat = lattice("fp32")
        s.set_gate(0.0)
        s.advance(lat, "vv4", w.dt, 1, threshold=1e-3)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        recs, srep = s.advance(lat, "vv4", w.dt, njumps, threshold=1e-3)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t1
        s.set_gate(0.25)
        s.set_jump("network")
        errs = _scalar_errors(recs, rr, 2)
        progress("surrogate: linear jump hubble gate only form done")
        forms["linear_jump_hubble_gate_only"] = {"effective_site_updates_per_s": w.sites * njumps * K / sec,
                                                 "accepted_fraction": 1.0 - srep["fallbacks"] / max(1, njumps),
                                                 "max_residual": srep["max_residual"],
                                                 "error_vs_fp64_vv4": errs["max"], "errors": errs,
                                                 "field_error": _field_error(lat, ref)}
        lat.close()
        # the Hubble-residual gate alone (second gate off)
        lat = lattice("fp32")
        s.set_gate(0.0)
        s.advance(lat, "vv4", w.dt, 1, threshold=1e-3)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        recs, srep = s.advance(lat, "vv4", w.dt, njumps, threshold=1e-3)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t1
        s.set_gate(0.25)
        errs = _scalar_errors(recs, rr, 2)
        progress("surrogate: surrogate hubble gate only form done")
        forms["surrogate_hubble_gate_only"] = {"effective_site_updates_per_s": w.sites * njumps * K / sec,
                                               "accepted_fraction": 1.0 - srep["fallbacks"] / max(1, njumps),
                                               "max_residual": srep["max_residual"],
                                               "error_vs_fp64_vv4": errs["max"], "errors": errs}
        # the network alone: no residual gate (non-finite jumps still fall back), until the
        # evolution breaks down
        lat.close()
        lat = lattice("fp32")
        s.advance(lat, "vv4", w.dt, 1, threshold=float("inf"))
        done, chunks, sec, fb, maxr = 0, [], 0.0, 0, 0.0
        while done < njumps:
            n = min(10, njumps - done)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            try:
                recs, srep = s.advance(lat, "vv4", w.dt, n, threshold=float("inf"))
            except _lib.CLError:
                break
            torch.cuda.synchronize()
            sec += time.perf_counter() - t1
            chunks.append(recs)
            fb += srep["fallbacks"]
            maxr = max(maxr, srep["max_residual"])
            done += n
        e = {"jumps_completed": done, "fallbacks_nonfinite": fb, "max_residual": maxr}
        if done:
            e["effective_site_updates_per_s"] = w.sites * done * K / sec
            e["errors"] = _scalar_errors(np.concatenate(chunks), rr[:done], 2)
            e["error_vs_fp64_vv4"] = e["errors"]["max"]
        forms["surrogate_no_gate"] = e
        lat.close()
        ref.close()
        res["forms"] = forms
        return res

    out["eval"] = [evaluate(128, 0.5, jumps)]
    if ablation:
        # the literal 6-channel layout (fluctuations + a, H): trained and
        # evaluated the same way at 128^3
        s.close()
        s = _lib.Surrogate(n_fields=2, extra_inputs=2, layers=5, jump_steps=K, init_seed=0)
        s.dataset_reserve(wt.N, len(seeds) * pairs_per_seed)
        for seed in seeds:
            w = wt.with_(seed=seed)
            lat = _lib.Lattice(w.N, w.dx, 2, "fp64")
            lat.set_background(w.alpha, w.expansion, w.mp, w.a0)
            lat.set_potential(w.m2, w.lam, w.g2, w.V0)
            lat.seed(w.seed, w.fbar[:2], w.pbar[:2], w.cutoff_modes, w.amp)
            # default tile, as for the main training set
            for i in range(pairs_per_seed):
                if i and gap > K:
                    lat.step("vv4", w.dt, gap - K, record=False)
                s.record_input(lat)
                lat.step("vv4", w.dt, K, record=False)
                s.record_target(lat)
            lat.close()
        rep6 = s.train(epochs=epochs, lr=5e-4, lr_final=5e-6, shuffle_seed=0, holdout=pairs_per_seed // 2)
        extra_inputs, saved = 2, extra_inputs
        e6 = evaluate(128, 0.5, jumps)
        extra_inputs = saved
        out["ablation_6_channels"] = {"train": rep6, "eval": e6["forms"]["surrogate"],
                                      "eval_no_gate": e6["forms"]["surrogate_no_gate"]}
        s.close()
        s = None
    if eval_256 and s is not None:
        out["eval"].append(evaluate(256, 0.25, jumps))        # training dx, larger box
        out["eval"].append(evaluate(256, 0.5, min(jumps, 40)))  # half the training dx: out of distribution
    if s is not None:
        s.close()
    out["summary"] = surrogate_summary(out["eval"])
    return out


def surrogate_summary(evals):
    """The comparison the metric names, per evaluated 256^3 workload: rate
    (site-updates/s) and error (worst relative error of the volume averages
    against FP64 VV4) of FP64 VV4, FP32 VV4, FP32 leapfrog at dt, the linear
    jump and the network jump (both gates), and the linear jump's rate over
    FP64 VV4's and over the fastest integrator form whose error is no larger
    than its own."""
    out = []
    for e in evals:
        if e["N"] != 256:
            continue
        f = e["forms"]

        def form(k):
            v = f[k]
            r = {"site_updates_per_s": v["effective_site_updates_per_s"], "error": v.get("error_vs_fp64_vv4", 0.0)}
            if "accepted_fraction" in v:
                r["accepted_fraction"] = v["accepted_fraction"]
            return r

        rows = {k: form(k) for k in ("fp64_vv4", "fp32_vv4", "fp32_leapfrog", "fp32_leapfrog_dt4",
                                     "linear_jump", "surrogate")}
        lj = rows["linear_jump"]
        peers = [v["site_updates_per_s"] for k, v in rows.items()
                 if k not in ("linear_jump", "surrogate") and v["error"] <= lj["error"]]
        out.append({"workload": f"256^3 two-field FP32, k_IR = {e['k_ir']}, {e['jumps']} jumps of 16 VV4 steps",
                    "forms": rows,
                    "linear_jump_over_fp64_vv4": lj["site_updates_per_s"] / rows["fp64_vv4"]["site_updates_per_s"],
                    "linear_jump_over_fastest_integrator_at_no_larger_error":
                        lj["site_updates_per_s"] / max(peers) if peers else None})
    return out


def rk_bytes_per_step(stages: int, precision: str, nf: int, classic: bool = False) -> int:
    """Algorithmic bytes per site of one Runge-Kutta step.  Low storage: the
    first stage reads f, pi and writes f, pi and their registers; every
    later stage also reads the registers.  Standard RK4: stage 1 reads the
    state and writes the next stage input and the stage sum; stages 2 and 3
    also read the step's start and the sum; stage 4 writes no sum."""
    e = 4 if precision == "fp32" else 8
    if classic:
        return nf * e * 2 * (3 + 5 + 5 + 4)
    return nf * e * (6 + 8 * (stages - 1))


def rk_run(w, steps, r64, tile, scheme="rk4"):
    """A fourth-order Runge-Kutta scheme (RK4-5, 5 stages, or the standard
    RK4) in FP32 on the same workload and tile, from the same seed: rate,
    HBM fraction and deviation from the FP64 VV4 run over the same steps."""
    import torch
    stream = torch.cuda.Stream()
    lat = make(w, "fp32", stream, tune=False,
               tile=(tile["tz"], tile["ty"], tile["cx"], tile["ry"], tile["pd"]))
    chunk = min(steps, 100)
    recs = [lat.step(scheme, w.dt, chunk)]   # untimed first call (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // chunk - 1):
        recs.append(lat.step(scheme, w.dt, chunk))
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    lat.close()
    timed = (steps // chunk - 1) * chunk
    r = np.concatenate(recs)
    classic = scheme == "rk4_classic"
    per_site = rk_bytes_per_step(5, "fp32", w.n_fields, classic)
    alg = per_site * w.sites * timed / sec / 1e9
    return {"scheme": "standard RK4 (4 stages, 3 auxiliary arrays)" if classic else "rk4 (Carpenter-Kennedy 5-stage)",
            "steps": timed, "site_updates_per_s": w.sites * timed / sec, "ms_per_step": 1e3 * sec / timed,
            "hbm_frac": alg / HBM_PEAK_GBS, "bytes_per_site_step": per_site,
            "vs_fp64_vv4_rel_dev": linear_regime_deviation(r, r64[:len(r)], w.n_fields)}


def lowdim_run(w, steps, warmup, chunk=500):
    """The reduced (2+1)-dimensional form: the 4096^2 two-field FP32 VV4
    lattice (seeded noise state), steps in calls of `chunk`: rate and the
    fraction of the HBM peak at 32 B per site and pass (three passes per
    step plus one opening kick per call)."""
    import torch
    from paper_2607_24978_amd import _lib
    lat = _lib.Lattice(w.N, w.dx, w.n_fields, "fp32", dim=2)
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    f, p = W.random_state(w.N, w.n_fields, w.seed, fbar=w.fbar[:w.n_fields], famp=1e-3, pamp=1e-3, dim=2)
    lat.set_fields(f, p)
    del f, p
    chunk = min(chunk, steps)
    lat.step(w.integrator, w.dt, chunk)
    for _ in range(max(0, warmup - chunk) // chunk):
        lat.step(w.integrator, w.dt, chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    calls = steps // chunk
    for _ in range(calls):
        r = lat.step(w.integrator, w.dt, chunk)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    lat.close()
    sites = w.N ** 2
    n = calls * chunk
    alg = (3 * n * 32 + calls * 24) * sites
    return {"workload": w.name, "steps": n, "site_updates_per_s": sites * n / sec, "ms_per_step": 1e3 * sec / n,
            "hbm_frac": alg / sec / 1e9 / HBM_PEAK_GBS, "finite": not bool(np.any(r["nonfinite"]))}


def spectrum_run(w, reps=5):
    """Cost of one power spectrum of f_0 on the workload's lattice: device
    FFT in FP64 (extraction fused with the z pass, the y pass, the x pass
    fused with the binning) plus the copy of the bins; algorithmic bytes per
    site: 4 (or 8) read + 16 P / N written by the first pass, 32 P / N by the
    y pass, 16 P / N read by the last, where P is the number of z of the
    half transform that the y and x passes hold (z <= N / 2 rounded up to
    whole batches of L = 2048 / N lines: 136 at N = 256)."""
    import torch
    stream = torch.cuda.Stream()
    lat = make(w, w.precision, stream, tune=False)
    lat.power_spectrum(0, "f", 1.0)  # first call allocates
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k, c, s, d = lat.power_spectrum(0, "f", 1.0)
        times.append(time.perf_counter() - t0)
    lat.close()
    sec = float(np.median(times))
    e = 4 if w.precision == "fp32" else 8
    L = w.N if w.N <= 32 else 2048 // w.N
    P = min(w.N, -(-(w.N // 2 + 1) // L) * L)
    alg = int((e + 64 * P / w.N) * w.sites)
    return {"field": "f_0", "binning": "canonical (width 1)", "bins": int(len(k)), "ms": 1e3 * sec,
            "hbm_frac": alg / sec / 1e9 / HBM_PEAK_GBS, "alg_bytes": alg}


def gw_run(w, steps=200, warmup=20, tune=True):
    """The 256^3 two-field FP32 VV4 workload with the gravitational-wave
    tensor carried in the fused pass (five traceless components and their
    momenta: 16 (n_fields + 5) bytes per site and pass), timed on the stream
    the passes run on; then the cost of one binned wave spectrum."""
    import torch
    from paper_2607_24978_amd import _lib
    stream = torch.cuda.Stream()
    lat = _lib.Lattice(w.N, w.dx, w.n_fields, "fp32")
    lat.set_stream(stream.cuda_stream)
    lat.set_background(w.alpha, w.expansion, w.mp, w.a0)
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    lat.gw_enable(True)
    lat.seed(w.seed, w.fbar[:w.n_fields], w.pbar[:w.n_fields], w.cutoff_modes, w.amp)
    if tune:
        lat.autotune(reps=3)
    tile = lat.get_tile()
    lat.step(w.integrator, w.dt, warmup)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    r = lat.step(w.integrator, w.dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    per = 3 if w.integrator == "vv4" else 1
    launches = steps * per + 1
    bps = 16 * (w.n_fields + 5)
    alg = (steps * per * bps + 12 * (w.n_fields + 5)) * w.sites
    achieved = alg / launches / (ms / launches * 1e-3) / 1e9
    lat.gw_spectrum()  # first call allocates
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        counts, rho, omega, tot = lat.gw_spectrum()
    spec_ms = 1e3 * (time.perf_counter() - t0) / reps
    lat.close()
    return {"workload": w.name + "+gw", "steps": steps, "tile": tile, "bytes_per_site_pass": bps,
            "site_updates_per_s": w.sites * steps / sec, "ms_per_step": 1e3 * sec / steps,
            "hbm_frac": achieved / HBM_PEAK_GBS, "achieved_GBps": achieved, "finite": not bool(np.any(r["nonfinite"])),
            "spectrum_ms": spec_ms, "rho_gw": tot, "omega_gw_max": float(np.max(omega)),
            "rho_gw_over_rho": tot / float(r["EK"][-1].sum() + r["EG"][-1].sum() + r["EV"][-1])}


def cpu_model() -> str:
    """CPU model name of the host (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def c3_run(warmup=50, steps=200, tune=True):
    """The 1024^3 two-field FP32 leapfrog workload (1.07e9 sites, 17.2 GB of
    state): library seed, autotuned tile, `warmup` untimed steps, then `steps`
    timed steps in one call, with the roofline of its fused pass."""
    w = W.C3
    r, sec, ms, dk, calls, tile = timed_run(w, "fp32", steps, warmup, steps, tune)
    alg = dk * bytes_per_site("fp32", w.n_fields) * w.sites + calls * kpass_bytes_per_site("fp32", 2) * w.sites
    launches = dk + calls
    avg_ms = ms / launches
    achieved = alg / launches / (avg_ms * 1e-3) / 1e9
    return {"workload": w.name, "N": w.N, "k_ir": w.k_ir, "integrator": w.integrator, "dt": w.dt,
            "warmup": warmup, "steps": steps, "tile": tile, "site_updates_per_s": w.sites * steps / sec,
            "ms_per_step": 1e3 * sec / steps, "finite": not bool(np.any(r["nonfinite"])),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(w.name, tile),
                         "kernel": "lattice_pass<float,2>", "avg_launch_us": avg_ms * 1e3,
                         "alg_bytes_per_launch": alg / launches}}


def oracle_worker(seed: int, start_at: float):
    """One process of the all-cores oracle baseline: seed the 256^3
    workload, wait for the common start time, time one full step, print it."""
    from oracle import lattice as L
    from oracle import seed as S
    w = W.C1
    P = L.Params(N=w.N, dx=w.dx, n_fields=w.n_fields, alpha=w.alpha, mp=w.mp, expansion=w.expansion,
                 m2=w.m2, lam=w.lam, g2=w.g2, V0=w.V0)
    s = S.seed_state(P, w.k_ir, w.fbar[:w.n_fields], w.pbar[:w.n_fields], seed, cutoff=w.cutoff_modes)
    while time.time() < start_at:
        time.sleep(0.01)
    t0 = time.perf_counter()
    L.step(s, w.dt, P, w.integrator)
    print(json.dumps({"seconds": time.perf_counter() - t0}), flush=True)


def cpu_all_cores(procs):
    """The same oracle step (256^3 workload) in `procs` concurrent worker
    processes (one thread each, started as child programs), all timed from a
    common start: the aggregate rate of the untuned oracle over the host's
    cores."""
    import subprocess
    w = W.C1
    start_at = time.time() + 25.0  # every worker has seeded by then
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    ps = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker", str(w.seed + i),
                            "--start-at", repr(start_at)], stdout=subprocess.PIPE, env=env, text=True)
          for i in range(procs)]
    secs = []
    for p in ps:
        out, _ = p.communicate(timeout=300)
        if p.returncode == 0 and out.strip():
            secs.append(json.loads(out.strip().splitlines()[-1])["seconds"])
    if len(secs) != procs:
        return None
    return {"value": sum(w.sites / t for t in secs), "unit": "site-updates/s", "cores": procs, "kind": "oracle",
            "sample": f"one full {w.integrator} step of the {w.N}^3 workload in each of {procs} concurrent "
                      f"single-thread processes, slowest {max(secs):.1f} s"}


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
                      f"in FP64 numpy on one host core ({cpu_model()}, "
                      f"{os.cpu_count()} logical CPUs visible), {dt:.1f} s", "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (5000 for c1, 200 for c3)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (500 for c1, 50 for c3)")
    ap.add_argument("--chunk", type=int, default=500)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--tile", default=None, help="force the FP32 tile tz,ty,cx,ry,pd instead of autotuning")
    ap.add_argument("--no-surrogate", action="store_true", help="skip training and evaluating the learned surrogate")
    ap.add_argument("--sg-epochs", type=int, default=12)
    ap.add_argument("--sg-pairs", type=int, default=64, help="training pairs per seed (8 seeds)")
    ap.add_argument("--sg-jumps", type=int, default=312)
    ap.add_argument("--sg-extra", type=int, default=4, help="broadcast inputs: 4 = (a, H, <phi>, <pi_phi>), 2 = (a, H)")
    ap.add_argument("--sg-ablation", action="store_true", help="also train and evaluate the 6-channel input layout")
    ap.add_argument("--oracle-worker", type=int, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--start-at", type=float, default=0.0, help=argparse.SUPPRESS)
    ap.add_argument("--sg-forward-profile", action="store_true",
                    help="only run surrogate forward passes at 256^3 (for a kernel profile) and print their figures")
    ap.add_argument("--sg-linear-profile", action="store_true",
                    help="only run linear jumps at 256^3 (for a kernel profile) and print their figures")
    ap.add_argument("--sg-train-profile", action="store_true",
                    help="only run a few surrogate training steps at 128^3 (for a kernel profile) and print their figures")
    ap.add_argument("--cpu-procs", type=int, default=16, help="processes of the all-cores oracle baseline (0: skip)")
    ap.add_argument("--no-c3", action="store_true", help="skip the 1024^3 leapfrog leg of the default run")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the power-spectrum, gravitational-wave and 2+1 legs of the default run")
    ap.add_argument("--profile-leg", choices=["gw", "batched", "surrogate", "spectrum", "lowdim"], default=None,
                    help="only run that leg (for a kernel profile; --steps / --warmup set the length of gw and "
                         "batched) and print it")
    ap.add_argument("--workload", choices=["c1", "c3"], default="c1",
                    help="c1: 256^3 two-field VV4 (default); c3: 1024^3 two-field leapfrog")
    args = ap.parse_args()
    if args.oracle_worker is not None:
        oracle_worker(args.oracle_worker, args.start_at)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.sg_forward_profile:
        print(json.dumps(surrogate_forward_profile()), flush=True)
        return
    if args.sg_train_profile:
        print(json.dumps(surrogate_train_profile()), flush=True)
        return
    if args.sg_linear_profile:
        print(json.dumps(linear_jump_profile()), flush=True)
        return
    if args.profile_leg == "gw":
        print(json.dumps(gw_run(W.C1, steps=args.steps or 200, warmup=args.warmup or 20, tune=not args.no_tune)),
              flush=True)
        return
    if args.profile_leg == "surrogate":
        print(json.dumps(surrogate_run(epochs=args.sg_epochs, pairs_per_seed=args.sg_pairs, jumps=args.sg_jumps,
                                       extra_inputs=args.sg_extra, ablation=args.sg_ablation)), flush=True)
        return
    if args.profile_leg == "lowdim":
        print(json.dumps(lowdim_run(W.C4, args.steps or 2000, args.warmup or 200)), flush=True)
        return
    if args.profile_leg == "spectrum":
        print(json.dumps(spectrum_run(W.C1, reps=args.steps or 20)), flush=True)
        return
    if args.profile_leg == "batched":
        # one solo step per member only: the solo comparison is not what is profiled
        print(json.dumps(batched_run(args.steps or 1000, args.warmup or 500, solo_steps=1)), flush=True)
        return

    from paper_2607_24978_amd import _lib
    w = W.C1 if args.workload == "c1" else W.C3
    if args.workload == "c3":
        args.no_fp64 = True  # the all-FP64 form of the 1024^3 run is not part of this workload
    if args.steps is None:
        args.steps = 5000 if args.workload == "c1" else 200
    if args.warmup is None:
        args.warmup = 500 if args.workload == "c1" else 50
    chunk = max(1, min(args.chunk, args.steps))
    if args.steps % chunk:
        chunk = math.gcd(args.steps, chunk)
    copy_gbs = _lib.copy_bandwidth(1 << 30, 10)
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    r32, sec32, ms32, dk32, calls32, tile32 = timed_run(w, "fp32", args.steps, args.warmup, chunk,
                                                       not args.no_tune, tile)
    value = w.sites * args.steps / sec32
    progress(f"fp32 form: {value:.4g} site-updates/s")
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
                   "steps_per_call": chunk, "tile": tile32, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(w.name, tile32),
                     "kernel": "lattice_pass<float,2>", "avg_launch_us": avg_ms * 1e3,
                     "alg_bytes_per_launch": alg / launches,
                     "copy_ceiling_GBps": copy_gbs, "frac_of_copy_ceiling": achieved / copy_gbs},
    }
    forms = {"fp32": {"site_updates_per_s": value, "hbm_frac": achieved / HBM_PEAK_GBS}}
    if not args.no_fp64:
        progress("fp64 form")
        r64, sec64, ms64, dk64, calls64, _ = timed_run(w, "fp64", args.steps, args.warmup, chunk,
                                                        not args.no_tune)
        alg64 = dk64 * bytes_per_site("fp64", 2) * w.sites + calls64 * kpass_bytes_per_site("fp64", 2) * w.sites
        ach64 = alg64 / (ms64 * 1e-3) / 1e9
        forms["fp64"] = {"site_updates_per_s": w.sites * args.steps / sec64, "hbm_frac": ach64 / HBM_PEAK_GBS}
        forms["fp32_vs_fp64_rel_dev"] = linear_regime_deviation(r32, r64, w.n_fields)
        forms["fp32_speedup_vs_fp64"] = value / forms["fp64"]["site_updates_per_s"]
        if args.workload == "c1":
            progress("rk4 form")
            forms["rk4_fp32"] = rk_run(w, 1000, r64, tile32)
            progress("standard rk4 form")
            forms["rk4_classic_fp32"] = rk_run(w, 1000, r64, tile32, scheme="rk4_classic")
    if args.workload == "c1" and not args.no_c3:
        progress("1024^3 two-field leapfrog form (50 warm-up + 200 timed steps)")
        forms["c3_1024"] = c3_run()
    if args.workload == "c1" and not args.no_forms:
        progress("power spectrum form")
        forms["spectrum"] = spectrum_run(w)
    if args.workload == "c1" and not args.no_forms:
        progress("gravitational-wave form")
        forms["gw"] = gw_run(w)
    if args.workload == "c1" and not args.no_forms:
        progress("reduced 2+1 form")
        forms["lowdim_2d"] = lowdim_run(W.C4, 2000, 200)
    if not args.no_batched and args.workload == "c1":
        progress("batched ensemble form")
        forms["batched"] = batched_run(1000, 500)
    if not args.no_surrogate and args.workload == "c1":
        progress("surrogate form (training pairs, training, evaluation)")
        forms["surrogate"] = surrogate_run(epochs=args.sg_epochs, pairs_per_seed=args.sg_pairs,
                                           jumps=args.sg_jumps, extra_inputs=args.sg_extra,
                                           ablation=args.sg_ablation)
    line["forms"] = forms
    if not args.no_cpu:
        # the oracle on the 256^3 workload (the 1024^3 one does not fit a numpy run of ~30 s)
        progress("oracle on the host (cpu_baseline)")
        line["cpu_baseline"] = cpu_baseline(W.C1, steps=1)
        procs = min(args.cpu_procs, os.cpu_count() or 1)
        if procs > 1:
            progress(f"oracle on {procs} host cores")
            line["cpu_baseline"]["all_cores"] = cpu_all_cores(procs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
