"""GPU parity of the HIP lattice path against the CPU FP64 oracle.

All calls go through the C ABI (ctypes binding).  Tolerances: FP64 fields
and scalars within 1e-11 relative of the oracle (per step for a, H, EK,
EG, EV, var; norm-wise for the final fields); FP32 fields with FP64 sums
within 1e-4 relative on volume averages.
"""
import math

import numpy as np
import pytest

from oracle import lattice as L
from oracle import seed as S
import workloads as W

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2607_24978_amd import _lib
    return _lib


def make_lattice(w, precision=None, expansion="self"):
    lat = _lib().Lattice(w.N, w.dx, w.n_fields, precision or w.precision)
    lat.set_background(w.alpha, expansion, w.mp, w.a0)
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    return lat


def params(w, expansion="self"):
    return L.Params(N=w.N, dx=w.dx, n_fields=w.n_fields, alpha=w.alpha, mp=w.mp, expansion=expansion,
                    m2=w.m2, lam=w.lam, g2=w.g2, V0=w.V0)


def oracle_seed(w, expansion="self", amp=None):
    return S.seed_state(params(w, expansion), w.k_ir, w.fbar[:w.n_fields], w.pbar[:w.n_fields], w.seed,
                        a0=w.a0, cutoff=w.cutoff_modes, amp=w.amp if amp is None else amp)


def rel_err(got, want):
    got, want = np.asarray(got, float), np.asarray(want, float)
    return np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-300))


def compare_records(recs_gpu, recs_orc, nf, tol, expansion="self", skip_var=False):
    keys = ["a", "H", "EV"] if expansion == "self" else ["EV"]
    for k in keys:
        g = recs_gpu[k]
        o = np.array([r[k] for r in recs_orc])
        assert rel_err(g, o) <= tol, (k, rel_err(g, o))
    g = recs_gpu["eta"]
    o = np.array([r["eta"] for r in recs_orc])
    assert np.max(np.abs(g - o)) <= 1e-12 * np.max(np.abs(o))
    for j in range(nf):
        for k in (["EK", "EG"] + ([] if skip_var else ["var"])):
            g = recs_gpu[k][:, j]
            o = np.array([r[k][j] for r in recs_orc])
            assert rel_err(g, o) <= tol, (k, j, rel_err(g, o))
        g = recs_gpu["mean"][:, j]
        o = np.array([r["mean"][j] for r in recs_orc])
        scale = max(np.max(np.abs(o)), 1e-300)
        assert np.max(np.abs(g - o)) <= tol * scale, ("mean", j)


# ------------------------------------------------------------------ seed (P16)
@pytest.mark.parametrize("w", [W.C0, W.C1.with_(N=32, k_ir=2.0)], ids=["1field32", "2field32"])
def test_seed_matches_oracle(w):
    """Library host seed and oracle seed are two implementations of one
    written spec (RNG stream, left/right movers, DFT convention)."""
    s = oracle_seed(w)
    lat = make_lattice(w, precision="fp64")
    lat.seed(w.seed, w.fbar[:w.n_fields], w.pbar[:w.n_fields], w.cutoff_modes, w.amp)
    f, p = lat.get_fields()
    for j in range(w.n_fields):
        df = s.f[j] - w.fbar[j]
        assert np.max(np.abs(f[j] - s.f[j])) <= 1e-12 * np.max(np.abs(df))
        assert np.max(np.abs(p[j] - s.p[j])) <= 1e-12 * np.max(np.abs(s.p[j]))
    st = lat.get_state()
    assert abs(st["b"] - s.b) <= 1e-13 * abs(s.b)
    assert st["a"] == 1.0 and st["eta"] == 0.0 and st["step"] == 0
    lat.close()


# ------------------------------------------------------------------ FP64 parity
def run_both(w, n, integrator, expansion="self", precision="fp64", amp=None):
    s0 = oracle_seed(w, expansion, amp)
    P = params(w, expansion)
    lat = make_lattice(w, precision=precision, expansion=expansion)
    lat.set_fields(s0.f, s0.p)
    st = lat.get_state()
    if expansion == "self":
        assert abs(st["b"] - s0.b) <= 1e-12 * s0.b
    recs = lat.step(integrator, w.dt, n)
    f, p = lat.get_fields()
    s, orecs = L.run(s0, w.dt, n, P, integrator)
    lat.close()
    return recs, orecs, (f, p), s


def test_fp64_parity_config0_200_steps():
    """32^3 single field, lambda phi^4, self-consistent expansion, leapfrog,
    200 steps: per-step scalars and final fields within 1e-11 relative."""
    w = W.C0
    recs, orecs, (f, p), s = run_both(w, w.steps, "leapfrog")
    assert not np.any(recs["nonfinite"])
    compare_records(recs, orecs, 1, 1e-11)
    assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))
    assert np.max(np.abs(p - s.p)) <= 1e-11 * np.max(np.abs(s.p))
    assert recs["a"][-1] > 10.0  # the run really expands


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
@pytest.mark.parametrize("N", [8, 16])
def test_fp64_parity_two_field(integrator, N):
    """Two-field lphi4 preheating potential (q = 100), small lattices that
    exercise the halo and wrap-around paths: 30 steps within 1e-11."""
    w = W.C1.with_(N=N, k_ir=2.0 * 16 / N, precision="fp64")
    recs, orecs, (f, p), s = run_both(w, 30, integrator, amp=20.0)
    compare_records(recs, orecs, 2, 1e-11)
    assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))
    assert np.max(np.abs(p - s.p)) <= 1e-11 * np.max(np.abs(s.p))


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_fp64_parity_static(integrator):
    """Static space (a == 1): energies per step within 1e-11."""
    w = W.C0.with_(N=16, k_ir=0.4)
    recs, orecs, (f, p), s = run_both(w, 40, integrator, expansion="static", amp=30.0)
    compare_records(recs, orecs, 1, 1e-11, expansion="static")
    assert np.all(recs["a"] == 1.0) and np.all(recs["H"] == 0.0)
    assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))


def test_fp64_parity_vv4_config0_size():
    w = W.C0
    recs, orecs, (f, p), s = run_both(w, 40, "vv4")
    compare_records(recs, orecs, 1, 1e-11)
    assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))


# ------------------------------------------------------------------ FP32 form
def test_fp32_parity_config0():
    """FP32 fields with FP64 sums and scale factor against the FP64 oracle:
    volume averages within 1e-4 relative over the 200-step run."""
    w = W.C0
    recs, orecs, (f, p), s = run_both(w, w.steps, "leapfrog", precision="fp32")
    compare_records(recs, orecs, 1, 1e-4)
    # fields: FP32 storage rounding bounds the norm-wise error
    assert np.max(np.abs(f - s.f)) <= 1e-5 * np.max(np.abs(s.f))


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_fp32_parity_two_field(integrator):
    w = W.C1.with_(N=32, k_ir=2.0, precision="fp32")
    recs, orecs, (f, p), s = run_both(w, 30, integrator, amp=1.0)
    compare_records(recs, orecs, 2, 1e-4)


# ------------------------------------------------------------------ runtime properties
def test_observables_of_current_state():
    w = W.C0.with_(N=16)
    s0 = oracle_seed(w, amp=10.0)
    lat = make_lattice(w)
    lat.set_fields(s0.f, s0.p)
    o = lat.read_observables()
    ref = L.observe(s0, params(w))
    for k in ("a", "EV"):
        assert abs(o[k] - ref[k]) <= 1e-12 * abs(ref[k])
    assert abs(o["EK"][0] - ref["EK"][0]) <= 1e-12 * abs(ref["EK"][0]) + 1e-300
    assert abs(o["EG"][0] - ref["EG"][0]) <= 1e-12 * abs(ref["EG"][0])
    assert abs(o["var"][0] - ref["var"][0]) <= 1e-11 * abs(ref["var"][0])
    assert o["r"] <= 1e-14
    lat.close()


def test_deterministic_and_checkpoint_resume():
    """Two identical runs are bitwise equal, and a run resumed from a
    checkpoint (fields + background state) equals the uninterrupted run."""
    w = W.C1.with_(N=16, k_ir=2.0, precision="fp64")
    s0 = oracle_seed(w, amp=20.0)
    outs = []
    for _ in range(2):
        lat = make_lattice(w)
        lat.set_fields(s0.f, s0.p)
        r1 = lat.step("leapfrog", w.dt, 10)
        r2 = lat.step("leapfrog", w.dt, 10)
        outs.append((r1, r2, lat.get_fields()))
        lat.close()
    assert outs[0][1].tobytes() == outs[1][1].tobytes()
    assert np.array_equal(outs[0][2][0], outs[1][2][0])
    # checkpoint after 10 steps
    lat = make_lattice(w)
    lat.set_fields(s0.f, s0.p)
    lat.step("leapfrog", w.dt, 10)
    fck, pck = lat.get_fields()
    st = lat.get_state()
    lat.close()
    lat = make_lattice(w)
    lat.set_fields(fck, pck)
    lat.set_state(st["a"], st["b"], st["eta"], st["step"])
    r2b = lat.step("leapfrog", w.dt, 10)
    f2b, _ = lat.get_fields()
    assert lat.get_state()["step"] == 20
    lat.close()
    assert np.array_equal(f2b, outs[0][2][0])
    for k in ("a", "H", "EK", "EG", "EV"):
        assert np.array_equal(r2b[k], outs[0][1][k]), k


def test_graph_and_direct_launch_agree():
    """Repeated calls with the same shape replay a cached HIP graph; the
    first call and n = 1 calls launch directly.  All give the same numbers."""
    w = W.C0.with_(N=16)
    s0 = oracle_seed(w, amp=10.0)
    lat = make_lattice(w)
    lat.set_fields(s0.f, s0.p)
    ra = np.concatenate([lat.step("leapfrog", w.dt, 1) for _ in range(6)])
    fa, _ = lat.get_fields()
    lat.set_fields(s0.f, s0.p)
    rb = np.concatenate([lat.step("leapfrog", w.dt, 3) for _ in range(2)])
    fb, _ = lat.get_fields()
    lat.close()
    assert np.array_equal(fa, fb)
    assert np.array_equal(ra["a"], rb["a"]) and np.array_equal(ra["EG"], rb["EG"])


def test_errors_and_instability():
    lib = _lib()
    with pytest.raises(lib.CLError) as e:
        lib.Lattice(24, 1.0, 1, "fp64")
    assert e.value.status == lib.CL_EINVAL
    w = W.C0.with_(N=16)
    lat = make_lattice(w)
    s0 = oracle_seed(w)
    lat.set_fields(s0.f, s0.p)
    with pytest.raises(lib.CLError) as e:
        lat.step("leapfrog", 0.6 * w.dx, 2)  # dt sqrt(12)/dx > 2
    assert e.value.status == lib.CL_EUNSTABLE
    f = s0.f.copy()
    f[0, 3, 4, 5] = np.nan
    with pytest.raises(lib.CLError) as e:
        lat.set_fields(f, s0.p)  # non-finite input is reported at once
    assert e.value.status == lib.CL_EUNSTABLE
    # a field amplitude far beyond the stability range of dt blows up within
    # a few steps; the non-finite sums are reported as CL_EUNSTABLE
    lat.set_fields(s0.f * 1e4, s0.p)
    with pytest.raises(lib.CLError) as e:
        lat.step("leapfrog", w.dt, 50)
    assert e.value.status == lib.CL_EUNSTABLE
    lat.set_fields(s0.f, s0.p)
    assert lat.step("leapfrog", w.dt, 0).size == 0
    lat.close()
