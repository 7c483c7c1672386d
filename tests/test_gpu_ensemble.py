"""Batched ensembles: members of uneven sizes advanced in one persistent
launch per pass (HIP-graph captured) equal their solo runs bitwise when the
solo run uses the member's ensemble tile, and match the FP64 oracle."""
import numpy as np
import pytest

from oracle import lattice as L
from oracle import seed as S
import workloads as W

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2607_24978_amd import _lib
    return _lib


def member_lattice(w, tile=None):
    lat = _lib().Lattice(w.N, w.dx, w.n_fields, w.precision)
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    lat.seed(w.seed, w.fbar[:w.n_fields], w.pbar[:w.n_fields], w.cutoff_modes, w.amp)
    if tile is not None:
        lat.set_tile(**tile)
    return lat


def small_members(precision="fp32"):
    out = []
    for r, N in enumerate((32, 64, 32, 128, 64)):
        out.append(W.C0.with_(N=N, seed=1000 + r, precision=precision, amp=30.0))
    return out


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_ensemble_equals_solo_bitwise(integrator):
    ws = small_members()
    lats = [member_lattice(w) for w in ws]
    ens = _lib().Ensemble(lats)
    for i, w in enumerate(ws):
        ens.set_dt(i, w.dt)
    r = np.concatenate([ens.step(integrator, 6), ens.step(integrator, 6)])  # second call replays the graph
    fields = [lat.get_fields() for lat in lats]
    states = [lat.get_state() for lat in lats]
    tiles = [ens.get_tile(i) for i in range(len(ws))]
    ens.close()
    for lat in lats:
        lat.close()
    assert r.shape == (12, len(ws))
    for i, w in enumerate(ws):
        solo = member_lattice(w, tiles[i])
        rs = np.concatenate([solo.step(integrator, w.dt, 6), solo.step(integrator, w.dt, 6)])
        f, p = solo.get_fields()
        assert solo.get_state() == states[i]
        solo.close()
        assert rs.tobytes() == np.ascontiguousarray(r[:, i]).tobytes(), i
        assert np.array_equal(f, fields[i][0]) and np.array_equal(p, fields[i][1]), i


def test_ensemble_autotune_keeps_state_and_solo_equality():
    """The ensemble autotuner times distinct decompositions on the members'
    states without changing them (fields and background bitwise), and with
    the decomposition it keeps every member still equals its solo run bitwise:
    the solo lattice takes the same calls, three leapfrog steps in the
    default ensemble tile and five VV4 steps in the tuned one."""
    ws = small_members()
    lats = [member_lattice(w) for w in ws]
    ens = _lib().Ensemble(lats)
    for i, w in enumerate(ws):
        ens.set_dt(i, w.dt)
    tiles0 = [ens.get_tile(i) for i in range(len(ws))]
    r0 = ens.step("leapfrog", 3)
    before = [(lat.get_fields(), lat.get_state()) for lat in lats]
    rep = ens.autotune(reps=2)
    after = [(lat.get_fields(), lat.get_state()) for lat in lats]
    assert len(rep["candidates"]) >= 2 and rep["best"]["us"] > 0
    assert {c["item_sites"] for c in rep["candidates"]} <= {8192, 16384, 32768, 65536, 131072}
    for (fb, sb), (fa, sa) in zip(before, after):
        assert np.array_equal(fb[0], fa[0]) and np.array_equal(fb[1], fa[1])
        assert sb == sa
    r = ens.step("vv4", 5)
    fields = [lat.get_fields() for lat in lats]
    tiles = [ens.get_tile(i) for i in range(len(ws))]
    ens.close()
    for lat in lats:
        lat.close()
    for i, w in enumerate(ws):
        solo = member_lattice(w, tiles0[i])
        rs0 = solo.step("leapfrog", w.dt, 3)
        solo.set_tile(**tiles[i])
        rs = solo.step("vv4", w.dt, 5)
        f, p = solo.get_fields()
        solo.close()
        assert rs0.tobytes() == np.ascontiguousarray(r0[:, i]).tobytes(), i
        assert np.array_equal(f, fields[i][0]) and np.array_equal(p, fields[i][1]), (i, tiles[i])
        assert rs.tobytes() == np.ascontiguousarray(r[:, i]).tobytes(), i


def test_ensemble_fp64_matches_oracle():
    ws = [W.C0.with_(N=32, seed=1000 + r, amp=30.0) for r in range(2)] + [W.C0.with_(N=64, seed=7, amp=30.0)]
    lats = [member_lattice(w) for w in ws]
    ens = _lib().Ensemble(lats)
    for i, w in enumerate(ws):
        ens.set_dt(i, w.dt)
    n = 25
    r = ens.step("leapfrog", n)
    for i, w in enumerate(ws):
        P = L.Params(N=w.N, dx=w.dx, n_fields=1, lam=w.lam)
        s0 = S.seed_state(P, w.k_ir, w.fbar[:1], w.pbar[:1], w.seed, amp=w.amp)
        s, orecs = L.run(s0, w.dt, n, P, "leapfrog")
        for k in ("a", "H", "EV"):
            o = np.array([x[k] for x in orecs])
            assert np.max(np.abs(r[k][:, i] - o) / np.abs(o)) <= 1e-11, (i, k)
        o = np.array([x["EG"][0] for x in orecs])
        assert np.max(np.abs(r["EG"][:, i, 0] - o) / o) <= 1e-11
        f, _ = lats[i].get_fields()
        assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))
    ens.close()


def test_ensemble_errors():
    lib = _lib()
    a = member_lattice(W.C0.with_(N=32, precision="fp32"))
    b = member_lattice(W.C0.with_(N=32, precision="fp64"))
    with pytest.raises(lib.CLError) as e:
        lib.Ensemble([a, b])
    assert e.value.status == lib.CL_EINVAL
    c = member_lattice(W.C0.with_(N=16, precision="fp32"))
    with pytest.raises(lib.CLError) as e:
        lib.Ensemble([a, c])
    assert e.value.status == lib.CL_EUNSUPPORTED
    ens = lib.Ensemble([a])
    with pytest.raises(lib.CLError) as e:
        ens.step("leapfrog", 2)  # dt not set
    assert e.value.status == lib.CL_ESTATE
    with pytest.raises(lib.CLError) as e:
        ens.set_dt(0, 10 * a.dx)
    assert e.value.status == lib.CL_EUNSTABLE
    ens.close()
    for x in (a, b, c):
        x.close()


def test_config2_ensemble_sampled_members():
    """The 96-member uneven ensemble (48 x 32^3, 32 x 64^3, 16 x 128^3, FP32)
    at its stated length of 1000 leapfrog steps, in the decomposition its
    autotuner picks, as benchmarked: every record finite, a(eta) grows, and
    sampled members equal their solo runs bitwise."""
    ws = W.ensemble_members()
    assert len(ws) == 96
    lats = [member_lattice(w) for w in ws]
    ens = _lib().Ensemble(lats)
    for i, w in enumerate(ws):
        ens.set_dt(i, w.dt)
    ens.autotune(reps=3)
    n = 1000
    r = np.concatenate([ens.step("leapfrog", 250) for _ in range(n // 250)])
    assert not np.any(r["nonfinite"])
    assert np.all(r["a"][-1] > r["a"][0])
    picks = [0, 47, 48, 79, 80, 95]
    tiles = {i: ens.get_tile(i) for i in picks}
    fields = {i: lats[i].get_fields()[0] for i in picks}
    ens.close()
    for lat in lats:
        lat.close()
    for i in picks:
        solo = member_lattice(ws[i], tiles[i])
        rs = np.concatenate([solo.step("leapfrog", ws[i].dt, 250) for _ in range(n // 250)])
        f, _ = solo.get_fields()
        solo.close()
        assert rs.tobytes() == np.ascontiguousarray(r[:, i]).tobytes(), i
        assert np.array_equal(f, fields[i]), i
