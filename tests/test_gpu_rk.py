"""GPU parity of the low-storage Runge-Kutta schemes (RK2 midpoint, RK3-3,
RK4-5) against the CPU FP64 oracle, through the C ABI.  Same bars as the
symplectic schemes: FP64 within 1e-11 relative per step and norm-wise on the
final fields; FP32 fields with FP64 sums within 1e-4 on volume averages."""
import numpy as np
import pytest

from oracle import lattice as L
import workloads as W
from test_gpu_parity import compare_records, make_lattice, oracle_seed, params, run_both

pytestmark = pytest.mark.gpu

SCHEMES = ["rk2", "rk3", "rk34", "rk4", "rk4_classic"]


@pytest.mark.parametrize("scheme", SCHEMES)
def test_rk_fp64_config0(scheme):
    """32^3 single field, lambda phi^4, self-consistent expansion.  Seed
    amplitude 10: at the literal amplitude (fluctuations ~3e-4 of the mean)
    the variance is ill-conditioned -- an ulp of the field is 3e-13 of the
    fluctuation -- and the midpoint rule, which amplifies oscillating modes
    slightly, carries that to ~1e-11 of the variance within 40 steps."""
    w = W.C0
    recs, orecs, (f, p), s = run_both(w, 40, scheme, amp=10.0)
    assert not np.any(recs["nonfinite"])
    compare_records(recs, orecs, 1, 1e-11)
    assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))
    assert np.max(np.abs(p - s.p)) <= 1e-11 * np.max(np.abs(s.p))


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("N", [8, 16])
def test_rk_fp64_two_field(scheme, N):
    """Two-field preheating potential on small lattices (halo and
    wrap-around paths, workgroups of fewer than 64 threads at N = 8)."""
    w = W.C1.with_(N=N, k_ir=2.0 * 16 / N, precision="fp64")
    recs, orecs, (f, p), s = run_both(w, 20, scheme, amp=20.0)
    compare_records(recs, orecs, 2, 1e-11)
    assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))
    assert np.max(np.abs(p - s.p)) <= 1e-11 * np.max(np.abs(s.p))


@pytest.mark.parametrize("scheme", SCHEMES)
def test_rk_fp64_static(scheme):
    w = W.C0.with_(N=16, k_ir=0.4)
    recs, orecs, (f, p), s = run_both(w, 30, scheme, expansion="static", amp=30.0)
    compare_records(recs, orecs, 1, 1e-11, expansion="static")
    assert np.all(recs["a"] == 1.0) and np.all(recs["H"] == 0.0)
    assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))


def test_rk4_fp32_two_field():
    w = W.C1.with_(N=32, k_ir=2.0, precision="fp32")
    recs, orecs, (f, p), s = run_both(w, 20, "rk4", amp=1.0)
    compare_records(recs, orecs, 2, 1e-4, energy_scale=True)


def test_schemes_interleaved_with_symplectic_calls():
    """Calls of different schemes on one lattice hand the scale factor, its
    derivative and the pass coefficients over correctly: the sequence
    rk4, vv4, rk2, leapfrog, rk3 agrees with the oracle doing the same."""
    w = W.C1.with_(N=16, k_ir=2.0, precision="fp64")
    s = oracle_seed(w, amp=20.0)
    P = params(w)
    lat = make_lattice(w, precision="fp64")
    lat.set_fields(s.f, s.p)
    got, want = [], []
    for scheme, n in (("rk4", 3), ("vv4", 2), ("rk2", 4), ("leapfrog", 3), ("rk3", 2)):
        got.append(lat.step(scheme, w.dt, n))
        s, r = L.run(s, w.dt, n, P, scheme)
        want += r
    f, p = lat.get_fields()
    lat.close()
    compare_records(np.concatenate(got), want, 2, 1e-11)
    assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))


def test_rk_graph_and_direct_launch_agree(monkeypatch):
    w = W.C0.with_(N=16)
    s0 = oracle_seed(w, amp=10.0)
    outs = []
    for env in ("0", "1"):
        monkeypatch.setenv("CL_NO_GRAPH", env)
        lat = make_lattice(w)
        lat.set_fields(s0.f, s0.p)
        r = np.concatenate([lat.step("rk4", w.dt, 3) for _ in range(3)])
        outs.append((r, lat.get_fields()[0]))
        lat.close()
    assert outs[0][0].tobytes() == outs[1][0].tobytes()
    assert np.array_equal(outs[0][1], outs[1][1])


def test_rk_tiles_agree_static_bitwise():
    """In static space every candidate tile gives bitwise the same stage
    updates (the site arithmetic is the same in every instantiation)."""
    w = W.C0.with_(N=32, k_ir=0.4)
    s0 = oracle_seed(w, expansion="static", amp=30.0)
    lat = make_lattice(w, precision="fp64", expansion="static")
    lat.set_fields(s0.f, s0.p)
    tiles = lat.autotune(reps=1)["candidates"][:12]
    lat.close()
    ref = None
    for t in tiles:
        lat = make_lattice(w, precision="fp64", expansion="static")
        lat.set_fields(s0.f, s0.p)
        lat.set_tile(t["tz"], t["ty"], t["cx"], t["ry"], t["pd"])
        lat.step("rk3", w.dt, 4)
        f, p = lat.get_fields()
        lat.close()
        if ref is None:
            ref = (f, p)
        else:
            assert np.array_equal(f, ref[0]) and np.array_equal(p, ref[1]), t


def test_rk_rejected_by_ensembles():
    lib = __import__("paper_2607_24978_amd._lib", fromlist=["_lib"])
    ws = [W.C0.with_(N=32, seed=5 + i, precision="fp32") for i in range(2)]
    lats = []
    for w in ws:
        lat = lib.Lattice(w.N, w.dx, 1, "fp32")
        lat.seed(w.seed, w.fbar[:1], w.pbar[:1], w.cutoff_modes, w.amp)
        lats.append(lat)
    ens = lib.Ensemble(lats)
    for i, w in enumerate(ws):
        ens.set_dt(i, w.dt)
    with pytest.raises(lib.CLError):
        ens.step("rk4", 2)
    ens.close()
    for lat in lats:
        lat.close()
