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


def compare_records(recs_gpu, recs_orc, nf, tol, expansion="self", skip_var=False, energy_scale=True):
    """Per-step relative comparison.  With energy_scale, the kinetic and
    potential energies -- which pass through zero as the homogeneous field
    oscillates -- are compared relative to the total energy density rho of
    the same step instead of to themselves."""
    keys = ["a", "H"] if expansion == "self" else []
    for k in keys:
        g = recs_gpu[k]
        o = np.array([r[k] for r in recs_orc])
        assert rel_err(g, o) <= tol, (k, rel_err(g, o))
    rho = np.array([sum(r["EK"]) + sum(r["EG"]) + r["EV"] for r in recs_orc])
    o = np.array([r["EV"] for r in recs_orc])
    scale = rho if energy_scale else np.abs(o)
    assert np.max(np.abs(recs_gpu["EV"] - o) / scale) <= tol, ("EV", np.max(np.abs(recs_gpu["EV"] - o) / scale))
    g = recs_gpu["eta"]
    o = np.array([r["eta"] for r in recs_orc])
    assert np.max(np.abs(g - o)) <= 1e-12 * np.max(np.abs(o))
    for j in range(nf):
        for k in (["EK", "EG"] + ([] if skip_var else ["var"])):
            g = recs_gpu[k][:, j]
            o = np.array([r[k][j] for r in recs_orc])
            sc = rho if (energy_scale and k == "EK") else np.abs(o)
            err = np.max(np.abs(g - o) / np.maximum(sc, 1e-300))
            assert err <= tol, (k, j, err)
        # the volume average of a field with zero homogeneous value is a sum of
        # fluctuations: it is known to the precision of their spread
        g = recs_gpu["mean"][:, j]
        o = np.array([r["mean"][j] for r in recs_orc])
        spread = np.sqrt(np.max(np.array([r["var"][j] for r in recs_orc])))
        scale = max(np.max(np.abs(o)), spread, 1e-300)
        assert np.max(np.abs(g - o)) <= tol * scale, ("mean", j, np.max(np.abs(g - o)) / scale)


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
        # FP32 storage rounds f, p at ~6e-8 relative, which moves rho and b0
        assert abs(st["b"] - s0.b) <= (1e-12 if precision == "fp64" else 1e-6) * s0.b
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
    compare_records(recs, orecs, 1, 1e-4, energy_scale=True)
    # fields: FP32 storage rounding bounds the norm-wise error
    assert np.max(np.abs(f - s.f)) <= 1e-5 * np.max(np.abs(s.f))


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_fp32_parity_two_field(integrator):
    w = W.C1.with_(N=32, k_ir=2.0, precision="fp32")
    recs, orecs, (f, p), s = run_both(w, 30, integrator, amp=1.0)
    compare_records(recs, orecs, 2, 1e-4, energy_scale=True)


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_fp32_reductions_with_order_one_fluctuations(integrator):
    """FP32 form with fluctuations as large as the fields (values of both
    signs, neighbours that differ by O(f), so differences of neighbours are not
    exact): the energies and moments the FP32 pass reduces, against the FP64
    oracle on the same FP32-rounded values.  Each site term is a few correctly
    rounded FP32 operations (relative error a few 2^-24) and a thread adds at
    most 16 of them per plane in FP32 before the FP64 sums, so the sums of
    these positive terms are within 16 * 2^-24 ~ 1e-6 relative; the test
    allows 3e-6.  Then one step, compared the same way."""
    w = W.C1.with_(N=32, k_ir=2.0, precision="fp32")
    rng = np.random.default_rng(4242)
    shape = (2, w.N, w.N, w.N)
    f = rng.uniform(-1.0, 1.0, shape) + np.array([0.3, 0.0])[:, None, None, None]
    p = rng.uniform(-1.0, 1.0, shape)
    lat = make_lattice(w, precision="fp32")
    lat.set_fields(f, p)
    f32, p32 = lat.get_fields()
    assert np.array_equal(f32, f.astype(np.float32)) and np.array_equal(p32, p.astype(np.float32))
    P = params(w)
    st = lat.get_state()
    s0 = L.State(f32, p32, st["a"], st["b"], st["eta"])

    def check(o, ref, tol):
        assert abs(o["EV"] - ref["EV"]) <= tol * ref["EV"], ("EV", o["EV"], ref["EV"])
        for j in range(2):
            for k in ("EK", "EG", "var"):
                assert abs(o[k][j] - ref[k][j]) <= tol * ref[k][j], (k, j, o[k][j], ref[k][j])
            spread = math.sqrt(ref["var"][j])
            assert abs(o["mean"][j] - ref["mean"][j]) <= tol * spread, ("mean", j)

    check(lat.read_observables(), L.observe(s0, P), 3e-6)
    # one full step from the same state: the stepped fields differ from the
    # oracle's by FP32 rounding of the update, so the bar is the FP32 form's
    recs = lat.step(integrator, w.dt, 1)
    s1, orecs = L.run(s0, w.dt, 1, P, integrator)
    compare_records(recs, orecs, 2, 1e-5, energy_scale=False)
    lat.close()


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


def test_graph_and_direct_launch_agree(monkeypatch):
    """Repeated calls of one shape replay a cached HIP graph (one per
    starting buffer); CL_NO_GRAPH=1 launches every pass directly.  Both give
    bitwise equal results.  Calls of different lengths agree to rounding
    only (adjacent half kicks are merged inside a call)."""
    w = W.C0.with_(N=16)
    s0 = oracle_seed(w, amp=10.0)
    outs = []
    for env in ("0", "1"):
        monkeypatch.setenv("CL_NO_GRAPH", env)
        lat = make_lattice(w)
        lat.set_fields(s0.f, s0.p)
        r = np.concatenate([lat.step("leapfrog", w.dt, 3) for _ in range(3)]
                           + [lat.step("vv4", w.dt, 2) for _ in range(3)])
        outs.append((r, lat.get_fields()[0]))
        lat.close()
    assert outs[0][0].tobytes() == outs[1][0].tobytes()
    assert np.array_equal(outs[0][1], outs[1][1])
    lat = make_lattice(w)
    lat.set_fields(s0.f, s0.p)
    r1 = np.concatenate([lat.step("leapfrog", w.dt, 1) for _ in range(9)])
    lat.close()
    assert rel_err(r1["EG"][:, 0], outs[0][0]["EG"][:9, 0]) <= 1e-12
    assert rel_err(r1["a"], outs[0][0]["a"][:9]) <= 1e-14


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("expansion", ["static", "self"])
def test_tiles_agree(precision, expansion):
    """Every candidate tile computes the same site updates.  In static space
    the fields do not depend on the lattice sums, so they are bitwise equal
    across tiles; with expansion the scale factor carries the summation
    order of the sums (tile dependent) into the coefficients, so fields and
    sums agree to rounding."""
    w = W.C1.with_(N=32, k_ir=2.0, precision=precision)
    s0 = oracle_seed(w, expansion=expansion, amp=5.0)
    lat = make_lattice(w, expansion=expansion)
    lat.set_fields(s0.f, s0.p)
    rep = lat.autotune(reps=1)
    lat.close()
    tiles = rep["candidates"]
    assert len(tiles) >= 4
    ref = None
    tol = 1e-12 if precision == "fp64" else 1e-5
    for t in tiles[:: max(1, len(tiles) // 12)] + [rep["best"]]:
        lat = make_lattice(w, expansion=expansion)
        lat.set_tile(t["tz"], t["ty"], t["cx"], t["ry"], t["pd"])
        lat.set_fields(s0.f, s0.p)
        r = lat.step("vv4", w.dt, 4)
        f, p = lat.get_fields()
        lat.close()
        if ref is None:
            ref = (r, f, p)
            continue
        if expansion == "static":
            assert np.array_equal(f, ref[1]) and np.array_equal(p, ref[2]), t
        else:
            assert np.max(np.abs(f - ref[1])) <= tol * np.max(np.abs(ref[1])), t
            assert rel_err(r["a"], ref[0]["a"]) <= (1e-13 if precision == "fp64" else 1e-9), t
        for k in ("EV",):
            assert rel_err(r[k], ref[0][k]) <= tol, (t, k)
        assert rel_err(r["EG"][:, 1], ref[0]["EG"][:, 1]) <= tol, t


def test_autotune_keeps_state():
    w = W.C0.with_(N=16)
    s0 = oracle_seed(w, amp=10.0)
    lat = make_lattice(w)
    lat.set_fields(s0.f, s0.p)
    st0 = lat.get_state()
    rep = lat.autotune(reps=2)
    assert lat.get_tile() == {k: rep["best"][k] for k in ("tz", "ty", "cx", "ry", "pd")}
    assert lat.get_state() == st0
    f, p = lat.get_fields()
    assert np.array_equal(f, s0.f) and np.array_equal(p, s0.p)
    lib = _lib()
    with pytest.raises(lib.CLError):
        lat.set_tile(12, 4, 4, 1)
    lat.close()


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


def test_scheme_stability_bounds():
    """Each scheme's own limit on w_max dt, with w_max^2 = 12/dx^2 + a^2 V''
    at the field means (a = 1, V'' = 3 lambda phi0^2 here): at w_max dt = 1.8
    leapfrog (limit 2) and RK4-5 (3.34) run, while VV4 (1.5735), RK3-3
    (sqrt 3) and RK2 (0.532, its growth cap) are refused before any pass."""
    lib = _lib()
    w = W.C0.with_(N=16)
    s0 = oracle_seed(w)
    wmax = math.sqrt(12.0 / w.dx ** 2 + 3.0)
    dt = 1.8 / wmax
    for scheme, ok in (("leapfrog", True), ("rk4", True), ("vv4", False), ("rk3", False), ("rk2", False)):
        lat = make_lattice(w)
        lat.set_fields(s0.f, s0.p)
        if ok:
            r = lat.step(scheme, dt, 2)
            assert not np.any(r["nonfinite"])
        else:
            with pytest.raises(lib.CLError) as e:
                lat.step(scheme, dt, 2)
            assert e.value.status == lib.CL_EUNSTABLE, scheme
            assert lat.get_state()["step"] == 0
            # just inside the limit the same scheme runs
            lat.step(scheme, {"vv4": 1.55, "rk3": 1.7, "rk2": 0.5}[scheme] / wmax, 2)
        lat.close()


def test_attached_torch_buffers_layout_and_results():
    """Borrowed device memory (two torch tensors) gives bitwise the same run
    as library-owned buffers, and holds the documented row-interleaved
    layout: array a of row (x, y) at ((x*N + y)*2*nf + a)*N."""
    import torch
    w = W.C1.with_(N=16, k_ir=2.0, precision="fp64")
    s0 = oracle_seed(w, amp=20.0)
    own = make_lattice(w)
    own.set_fields(s0.f, s0.p)
    r_own = own.step("leapfrog", w.dt, 5)
    f_own, p_own = own.get_fields()
    own.close()
    N, nf = w.N, 2
    bufs = [torch.empty(2 * nf * N ** 3, dtype=torch.float64, device="cuda") for _ in range(2)]
    lat = make_lattice(w)
    lat.attach_device_buffers(bufs[0].data_ptr(), bufs[1].data_ptr())
    lat.set_fields(s0.f, s0.p)
    torch.cuda.synchronize()
    view = bufs[0].view(N, N, 2 * nf, N).cpu().numpy()
    assert np.array_equal(view[3, 5, 0], s0.f[0, 3, 5])
    assert np.array_equal(view[3, 5, 1], s0.f[1, 3, 5])
    assert np.array_equal(view[7, 2, 2], s0.p[0, 7, 2])
    assert np.array_equal(view[7, 2, 3], s0.p[1, 7, 2])
    r = lat.step("leapfrog", w.dt, 5)
    f, p = lat.get_fields()
    lat.close()
    assert r.tobytes() == r_own.tobytes()
    assert np.array_equal(f, f_own) and np.array_equal(p, p_own)
