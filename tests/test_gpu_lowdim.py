"""Reduced (1+1)- and (2+1)-dimensional lattices on the GPU against the CPU
FP64 oracle, through the C ABI.  Same bars as in three dimensions: FP64
within 1e-11 relative per step and norm-wise on the final fields, FP32
fields with FP64 sums within 1e-4 on volume averages."""
import numpy as np
import pytest

from oracle import lattice as L
import workloads as W
from test_gpu_parity import compare_records

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2607_24978_amd import _lib
    return _lib


def run_both(d, N, integrator, n, precision="fp64", seed=61, expansion="self", famp=0.3, pamp=0.2):
    w = W.C1.with_(N=N, k_ir=2.0 * 16 / N)
    P = L.Params(N=N, dx=w.dx, n_fields=2, m2=w.m2, lam=w.lam, g2=w.g2, expansion=expansion, dim=d)
    f, p = W.random_state(N, 2, seed, fbar=(1.0, 0.05), famp=famp, pamp=pamp, dim=d)
    lat = _lib().Lattice(N, w.dx, 2, precision, dim=d)
    lat.set_background(1.0, expansion, 1.0, 1.0)
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    lat.set_fields(f, p)
    st = lat.get_state()
    E = L.energies(f, p, 1.0, P)
    b0 = L.hubble_from_rho(1.0, L.rho_pressure(*E)[0], P)
    if expansion == "self":
        assert abs(st["b"] - b0) <= (1e-12 if precision == "fp64" else 1e-6) * b0
    recs = lat.step(integrator, w.dt, n)
    fg, pg = lat.get_fields()
    lat.close()
    s, orecs = L.run(L.State(f, p, 1.0, b0), w.dt, n, P, integrator)
    return recs, orecs, (fg, pg), s


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
@pytest.mark.parametrize("d,N", [(1, 64), (1, 1000), (2, 16), (2, 36), (2, 128), (2, 256)])
def test_lowdim_fp64_parity(d, N, integrator):
    """Two-field preheating potential, self-consistent expansion, 30 steps:
    per-step scalars and final fields within 1e-11 (ragged sizes: 1000 and
    36 are not powers of two)."""
    recs, orecs, (f, p), s = run_both(d, N, integrator, 30)
    assert not np.any(recs["nonfinite"])
    compare_records(recs, orecs, 2, 1e-11)
    assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))
    assert np.max(np.abs(p - s.p)) <= 1e-11 * np.max(np.abs(s.p))


@pytest.mark.parametrize("N,steps", [(1024, 3), (2048, 2)])
def test_lowdim_fp64_parity_long_marches(N, steps):
    """2-D lattices large enough that a work item marches several rows (4 at
    1024^2: one unrolled group of three and a remainder; 16 at 2048^2), in
    FP64 against the oracle: per-step scalars and final fields within
    1e-11."""
    recs, orecs, (f, p), s = run_both(2, N, "vv4", steps)
    assert not np.any(recs["nonfinite"])
    compare_records(recs, orecs, 2, 1e-11)
    assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))
    assert np.max(np.abs(p - s.p)) <= 1e-11 * np.max(np.abs(s.p))


@pytest.mark.parametrize("d,N", [(1, 4096), (2, 64)])
def test_lowdim_fp32_parity(d, N):
    recs, orecs, _, _ = run_both(d, N, "vv4", 30, precision="fp32", famp=0.05, pamp=0.05)
    compare_records(recs, orecs, 2, 1e-4, energy_scale=True)


def test_lowdim_static():
    recs, orecs, (f, p), s = run_both(2, 32, "leapfrog", 40, expansion="static")
    compare_records(recs, orecs, 2, 1e-11, expansion="static")
    assert np.all(recs["a"] == 1.0)
    assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))


def test_lowdim_graph_and_direct_launch_agree(monkeypatch):
    w = W.C1.with_(N=64, k_ir=0.5)
    f, p = W.random_state(64, 2, 3, fbar=(1.0, 0.05), famp=0.2, pamp=0.1, dim=2)
    outs = []
    for env in ("0", "1"):
        monkeypatch.setenv("CL_NO_GRAPH", env)
        lat = _lib().Lattice(64, w.dx, 2, "fp32", dim=2)
        lat.set_potential(w.m2, w.lam, w.g2, w.V0)
        lat.set_fields(f, p)
        r = np.concatenate([lat.step("vv4", w.dt, 4) for _ in range(3)])
        outs.append((r, lat.get_fields()))
        lat.close()
    assert outs[0][0].tobytes() == outs[1][0].tobytes()
    assert np.array_equal(outs[0][1][0], outs[1][1][0]) and np.array_equal(outs[0][1][1], outs[1][1][1])


def test_lowdim_unsupported_calls():
    lib = _lib()
    lat = lib.Lattice(32, 0.5, 1, "fp32", dim=2)
    f, p = W.random_state(32, 1, 2, dim=2)
    lat.set_fields(f, p)
    for call in (lambda: lat.seed(1, (1.0,), (0.0,)), lambda: lat.step("rk4", 0.01, 2),
                 lambda: lat.power_spectrum(0, "f"), lambda: lat.autotune(1),
                 lambda: lat.set_tile(32, 8, 4, 1, 1), lambda: lib.Ensemble([lat])):
        with pytest.raises(lib.CLError) as e:
            call()
        assert e.value.status == lib.CL_EUNSUPPORTED
    for bad in ((4, 32), (2, 10), (0, 32)):
        with pytest.raises(lib.CLError):
            lib.Lattice(bad[1], 0.5, 1, "fp32", dim=bad[0])
    lat.close()


def test_lowdim_4096sq_as_benchmarked():
    """The 4096^2 two-field FP32 VV4 workload the benchmark times, one
    graph-launched call of two steps against two FP64 oracle steps on the
    whole lattice: volume averages within 1e-4."""
    w = W.C4
    P = L.Params(N=w.N, dx=w.dx, n_fields=2, m2=w.m2, lam=w.lam, g2=w.g2, dim=2)
    f, p = W.random_state(w.N, 2, w.seed, fbar=(1.0, 0.0), famp=1e-3, pamp=1e-3, dim=2)
    lat = _lib().Lattice(w.N, w.dx, 2, "fp32", dim=2)
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    lat.set_fields(f, p)
    recs = lat.step("vv4", w.dt, 2)
    lat.close()
    E = L.energies(f, p, 1.0, P)
    b0 = L.hubble_from_rho(1.0, L.rho_pressure(*E)[0], P)
    _, orecs = L.run(L.State(f, p, 1.0, b0), w.dt, 2, P, "vv4")
    assert not np.any(recs["nonfinite"])
    compare_records(recs, orecs, 2, 1e-4, energy_scale=True)
