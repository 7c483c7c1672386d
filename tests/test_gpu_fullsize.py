"""Parity at the full benchmark sizes, in the launch configuration the
benchmark times (library seed, autotuned tile, graph-launched calls), through
the C ABI.

* 256^3 two-field preheating (q = 100) in FP32: the library's seed against
  the oracle's, then VV4 and RK4-5 steps against the FP64 oracle on the whole
  lattice.
* 1024^3 (too large for the oracle): a property that holds at any size.  A
  state made of 4 x 4 x 4 periodic images of a 256^3 oracle seed is an exact
  solution of the 1024^3 lattice equations (same dx, translation-invariant
  stencil, volume averages equal), so every image must stay bitwise equal to
  the first, and the first must follow the oracle's 256^3 run.

FP32 bars.  Volume averages within 1e-4 (as on small lattices).  Fields:
worst-case bounds from FP32 storage, derived in `fp32_bounds`.
"""
import math
import time

import numpy as np
import pytest

from oracle import lattice as L
import workloads as W
from test_gpu_parity import compare_records, make_lattice, oracle_seed, params

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24  # unit roundoff of FP32


def say(msg):
    print(f"[fullsize] {msg}", flush=True)


def abs_kick_weight(scheme: str) -> float:
    """Sum over one step of the absolute weights with which force
    evaluations enter pi (in units of dt).  Leapfrog 1; VV4 2|w1| + |w0|
    (Yoshida's middle weight is negative); a low-storage RK scheme
    sum_s sum_{t >= s} |B_t| prod_{s < r <= t} |A_r|."""
    if scheme == "leapfrog":
        return 1.0
    if scheme == "vv4":
        w1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
        return 2.0 * w1 + abs(1.0 - 2.0 * w1)
    A, B = L.RK_SCHEMES[scheme]
    total = 0.0
    for s in range(len(A)):
        c = 1.0
        for t in range(s, len(A)):
            if t > s:
                c *= abs(A[t])
            total += abs(B[t]) * c
    return total


def fp32_bounds(w, s, steps: int, scheme: str, a_max: float):
    """Worst-case max-norm deviations of FP32-stored fields from the FP64
    oracle after `steps` steps.  Every stored f carries a rounding of at most
    u|f|, one more per drift (D drifts in the run, D + 1 with the initial
    storage); the 7-point Laplacian weighs the seven stored values with
    absolute coefficients 12, and its FP32 neighbour sum
    ((x- + x+) + (y- + y+)) + (z- + z+) rounds at partial sums of about
    2, 2, 4, 2, 6 |f|: force error E <= (16 + 12 (D + 1)) u f_max a^(1+alpha)
    / dx^2.  pi collects it with the scheme's absolute kick weights, plus its
    own storage rounding; f collects its drifts' roundings and dt times the
    pi error."""
    f_max = float(np.max(np.abs(s.f)))
    p_max = float(np.max(np.abs(s.p)))
    drifts = {"leapfrog": 1, "vv4": 3}.get(scheme, len(L.RK_SCHEMES.get(scheme, ([],))[0]))
    D = steps * drifts
    kw = abs_kick_weight(scheme)
    E = (16 + 12 * (D + 1)) * U32 * f_max * a_max ** (1.0 + w.alpha) / w.dx ** 2
    bar_p = steps * kw * w.dt * E + (D + 2) * U32 * p_max
    bar_f = (D + 2) * U32 * f_max + steps * kw * w.dt * bar_p
    return bar_f, bar_p


def check_fields(f, p, s, w, steps, scheme, recs):
    bar_f, bar_p = fp32_bounds(w, s, steps, scheme, float(np.max(recs["a"])))
    ef = float(np.max(np.abs(f - s.f)))
    ep = float(np.max(np.abs(p - s.p)))
    say(f"{scheme}: max |df| {ef:.3g} (bound {bar_f:.3g}), max |dpi| {ep:.3g} (bound {bar_p:.3g})")
    assert ef <= bar_f and ep <= bar_p


@pytest.fixture(scope="module")
def c1_oracle_seed():
    t = time.time()
    s = oracle_seed(W.C1)
    say(f"oracle seed 256^3: {time.time() - t:.1f} s")
    return s


def c1_lattice(s0):
    """The benchmark's lattice: library seed, then its tile search.  Checks
    the seed against the oracle's to FP32 rounding."""
    w = W.C1
    lat = make_lattice(w)
    lat.seed(w.seed, w.fbar[:2], w.pbar[:2], w.cutoff_modes, w.amp)
    f, p = lat.get_fields()
    for j in range(2):
        # library FP64 seed within 1e-12 of the oracle's, then one rounding
        df = 1e-12 * np.max(np.abs(s0.f[j] - w.fbar[j]))
        dp = 1e-12 * np.max(np.abs(s0.p[j]))
        assert np.all(np.abs(f[j] - s0.f[j]) <= U32 * (np.abs(s0.f[j]) + df) + df)
        assert np.all(np.abs(p[j] - s0.p[j]) <= U32 * (np.abs(s0.p[j]) + dp) + dp)
    del f, p
    t = time.time()
    lat.autotune(reps=3)
    say(f"autotune 256^3: {time.time() - t:.1f} s, tile {lat.get_tile()}")
    return lat


def test_config1_fullsize_vv4(c1_oracle_seed):
    """256^3 FP32 VV4: one graph-launched call of two steps in the tuned
    tile against two FP64 oracle steps from the oracle's seed."""
    w, s0, n = W.C1, c1_oracle_seed, 2
    lat = c1_lattice(s0)
    recs = lat.step("vv4", w.dt, n)
    f, p = lat.get_fields()
    lat.close()
    t = time.time()
    s, orecs = L.run(s0, w.dt, n, params(w), "vv4")
    say(f"oracle {n} vv4 steps 256^3: {time.time() - t:.1f} s")
    assert not np.any(recs["nonfinite"])
    compare_records(recs, orecs, 2, 1e-4, energy_scale=True)
    check_fields(f, p, s, w, n, "vv4", recs)


def test_config1_fullsize_rk4(c1_oracle_seed):
    """256^3 FP32 RK4-5 in the tile the VV4 search picks (as the benchmark's
    RK form runs it): one graph-launched call of two steps against the
    oracle."""
    w, s0, n = W.C1, c1_oracle_seed, 2
    lat = c1_lattice(s0)
    recs = lat.step("rk4", w.dt, n)
    f, p = lat.get_fields()
    lat.close()
    t = time.time()
    s, orecs = L.run(s0, w.dt, n, params(w), "rk4")
    say(f"oracle {n} rk4 steps 256^3: {time.time() - t:.1f} s")
    assert not np.any(recs["nonfinite"])
    compare_records(recs, orecs, 2, 1e-4, energy_scale=True)
    check_fields(f, p, s, w, n, "rk4", recs)


def test_config3_fullsize_periodic_images():
    """1024^3 FP32 leapfrog in the tuned tile, one graph-launched call of
    three steps, from 64 periodic images of a 256^3 oracle seed (same dx, so
    k_IR four times larger for the block): all images bitwise equal after the
    call, image 0 against three oracle steps on the 256^3 block, volume
    averages of the 1024^3 run against the block's."""
    import torch
    big_w = W.C3
    n, N, nf = 256, big_w.N, big_w.n_fields
    R = N // n
    w = big_w.with_(N=n, k_ir=big_w.k_ir * R)
    assert math.isclose(w.dx, big_w.dx, rel_tol=1e-15) and math.isclose(w.dt, big_w.dt, rel_tol=1e-15)
    s0 = oracle_seed(w)
    A = [torch.empty(2 * nf * n ** 3, dtype=torch.float32, device="cuda") for _ in range(2)]
    small = make_lattice(w)
    small.attach_device_buffers(A[0].data_ptr(), A[1].data_ptr())
    small.set_fields(s0.f, s0.p)
    b0 = small.get_state()["b"]
    assert small.state_buffer() == A[0].data_ptr()
    small.close()
    big = make_lattice(big_w)
    B = [torch.empty(2 * nf * N ** 3, dtype=torch.float32, device="cuda") for _ in range(2)]
    big.attach_device_buffers(B[0].data_ptr(), B[1].data_ptr())
    assert big.state_buffer() == B[0].data_ptr()
    # array a of row (x, y) at ((x N + y) 2nf + a) N + z, with x = i n + x' etc.
    B[0].view(R, n, R, n, 2 * nf, R, n).copy_(A[0].view(1, n, 1, n, 2 * nf, 1, n).expand(R, n, R, n, 2 * nf, R, n))
    torch.cuda.synchronize()
    del A
    big.set_state(big_w.a0, b0, 0.0)
    big.read_observables()  # re-centres the variance sums on the new means
    t = time.time()
    big.autotune(reps=3)
    say(f"autotune 1024^3: {time.time() - t:.1f} s, tile {big.get_tile()}")
    steps = 3
    recs = big.step("leapfrog", big_w.dt, steps)
    cur = big.state_buffer()
    V = next(x for x in B if x.data_ptr() == cur).view(R, n, R, n, 2 * nf, R, n)
    ref = V[0, :, 0, :, :, 0, :].clone()
    unequal = [(i, j, k) for i in range(R) for j in range(R) for k in range(R)
               if not torch.equal(V[i, :, j, :, :, k, :], ref)]
    host = ref.cpu().numpy().astype(np.float64)
    big.close()
    del V, B, ref
    torch.cuda.empty_cache()
    assert not unequal, f"{len(unequal)} of {R ** 3} images differ, first {unequal[0]}"
    t = time.time()
    s, orecs = L.run(s0, w.dt, steps, params(w), "leapfrog")
    say(f"oracle {steps} leapfrog steps 256^3: {time.time() - t:.1f} s")
    assert not np.any(recs["nonfinite"])
    compare_records(recs, orecs, nf, 1e-4, energy_scale=True)
    f = np.stack([host[:, :, j, :] for j in range(nf)])
    p = np.stack([host[:, :, nf + j, :] for j in range(nf)])
    check_fields(f, p, s, w, steps, "leapfrog", recs)


def linear_regime_max_dev(r32, r64, nf):
    """Largest relative deviation of the FP32 run's volume averages from the
    FP64 run's over the linear regime -- the steps while every field's
    variance stays within 1e4 of its initial value.  a, H, EG and var are
    taken relative to themselves; EK and EV, which pass through zero as the
    homogeneous field oscillates, relative to rho of the same step; the mean
    of the field whose homogeneous value is zero relative to its spread."""
    v0 = r64["var"][0, :nf]
    lin = np.all(r64["var"][:, :nf] <= 1e4 * v0, axis=1)
    end = int(np.argmin(lin)) if not np.all(lin) else len(lin)
    rho = r64["EK"][:end, :nf].sum(1) + r64["EG"][:end, :nf].sum(1) + r64["EV"][:end]
    dev = {}
    for k in ("a", "H", "EV"):
        scale = rho if k == "EV" else np.abs(r64[k][:end])
        dev[k] = float(np.max(np.abs(r32[k][:end] - r64[k][:end]) / scale))
    for j in range(nf):
        for k in ("EK", "EG", "var"):
            scale = rho if k == "EK" else np.abs(r64[k][:end, j])
            dev[f"{k}{j}"] = float(np.max(np.abs(r32[k][:end, j] - r64[k][:end, j]) / scale))
        spread = np.sqrt(np.max(r64["var"][:end, j]))
        scale = max(float(np.max(np.abs(r64["mean"][:end, j]))), spread)
        dev[f"mean{j}"] = float(np.max(np.abs(r32["mean"][:end, j] - r64["mean"][:end, j])) / scale)
    return end, dev


def test_config1_full_length_fp32_vs_fp64():
    """The 256^3 two-field workload at its stated length: 5000 VV4 steps
    with FP32 fields and again in all-FP64, both from the library seed, in
    calls of 500 steps; the FP32 volume averages stay within 1e-4 of the
    FP64 run's through the linear regime.  (The FP64 form itself is tied to
    the oracle at 1e-11 on shorter runs.)"""
    w = W.C1
    recs = {}
    for prec in ("fp32", "fp64"):
        lat = make_lattice(w, precision=prec)
        lat.seed(w.seed, w.fbar[:2], w.pbar[:2], w.cutoff_modes, w.amp)
        t = time.time()
        recs[prec] = np.concatenate([lat.step("vv4", w.dt, 500) for _ in range(w.steps // 500)])
        say(f"{prec}: {w.steps} vv4 steps 256^3 in {time.time() - t:.1f} s, a = {recs[prec]['a'][-1]:.4f}")
        lat.close()
        assert len(recs[prec]) == w.steps
        assert not np.any(recs[prec]["nonfinite"])
    end, dev = linear_regime_max_dev(recs["fp32"], recs["fp64"], 2)
    say(f"linear regime: {end} of {w.steps} steps; deviations {dev}")
    assert end >= 1000
    assert max(dev.values()) <= 1e-4, dev
