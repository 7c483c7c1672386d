"""GPU tests of the linear-propagation jump of cl_surrogate_advance
(CL_JUMP_LINEAR) against the oracle (oracle/propagator.py) and the
integrator."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2607_24978_amd import _lib
    return _lib


def _free_static(N=32, precision="fp64"):
    """Two free fields of different masses on a static background."""
    from oracle import lattice as L
    P = L.Params(N=N, dx=0.4, n_fields=2, expansion="static", m2=(0.6, 2.3), lam=(0.0, 0.0), g2=0.0)
    rng = np.random.default_rng(3)
    f = np.stack([0.9 + 0.3 * rng.standard_normal((N, N, N)), 0.05 + 0.3 * rng.standard_normal((N, N, N))])
    p = np.stack([0.02 + 0.3 * rng.standard_normal((N, N, N)), -0.01 + 0.3 * rng.standard_normal((N, N, N))])
    lat = _lib().Lattice(N, P.dx, 2, precision)
    lat.set_background(1.0, "static", 1.0, 1.0)
    lat.set_potential(P.m2, P.lam, P.g2, 0.0)
    lat.set_fields(f, p)
    return P, L.State(f, p, 1.0, 0.0), lat


@pytest.mark.parametrize("integrator", ["vv4", "leapfrog"])
def test_free_fields_static_equal_the_integrator(integrator):
    """Free fields, static background: two linear jumps of 16 steps equal 32
    steps of the library's integrator and of the lattice oracle (the
    equations are linear, the propagation exact up to rounding)."""
    from oracle import lattice as L
    lib = _lib()
    P, s0, lat = _free_static()
    ref = lib.Lattice(32, P.dx, 2, "fp64")
    ref.set_background(1.0, "static", 1.0, 1.0)
    ref.set_potential(P.m2, P.lam, P.g2, 0.0)
    ref.set_fields(s0.f, s0.p)
    dt = 0.05
    sg = lib.Surrogate(n_fields=2, extra_inputs=2, layers=2, jump_steps=16, init_seed=1)
    sg.set_jump("linear")
    sg.set_gate(0.0)
    recs, rep = sg.advance(lat, integrator, dt, 2, threshold=float("inf"))
    assert rep["fallbacks"] == 0
    ref.step(integrator, dt, 32, record=False)
    f, p = lat.get_fields()
    fr, pr = ref.get_fields()
    so, _ = L.run(s0.copy(), dt, 32, P, integrator)
    for got, want, scale in ((f, fr, np.max(np.abs(fr))), (p, pr, np.max(np.abs(pr))),
                             (f, so.f, np.max(np.abs(so.f))), (p, so.p, np.max(np.abs(so.p)))):
        err = np.max(np.abs(got - want))
        print(f"max deviation {err:.3g} of scale {scale:.3g}", flush=True)
        assert err <= 1e-11 * scale
    st = lat.get_state()
    assert st["step"] == 32 and st["eta"] == pytest.approx(32 * dt, rel=1e-14)
    for h in (lat, ref, sg):
        h.close()


@pytest.mark.parametrize("nf", [1, 2])
def test_linear_jump_against_oracle(nf):
    """Two accepted linear jumps (threshold = inf, second gate off) on an
    expanding, interacting lattice seeded by the oracle (one field: lambda
    phi^4 at 16^3; two fields: the q = 100 preheating model at 32^3), against
    the oracle's linear jump: fields and momenta within 1e-11 of their scale,
    a, a' and the Hubble residual within 1e-12."""
    from oracle import lattice as L
    from oracle import propagator as PR
    from oracle import seed as S
    lib = _lib()
    N = 32 if nf == 2 else 16
    w = W.C1.with_(N=N, k_ir=1.0, precision="fp64")
    m2 = w.m2 if nf == 2 else (0.0, 0.0)
    g2 = w.g2 if nf == 2 else 0.0
    P = L.Params(N=N, dx=w.dx, n_fields=nf, m2=m2, lam=w.lam, g2=g2, V0=w.V0)
    s0 = S.seed_state(P, w.k_ir, w.fbar[:nf], w.pbar[:nf], w.seed, amp=20.0)
    lat = lib.Lattice(N, w.dx, nf, "fp64")
    lat.set_potential(m2, w.lam, g2, w.V0)
    lat.set_fields(s0.f, s0.p)
    sg = lib.Surrogate(n_fields=nf, extra_inputs=2, layers=2, jump_steps=16, init_seed=1)
    sg.set_jump("linear")
    sg.set_gate(0.0)
    recs, rep = sg.advance(lat, "vv4", w.dt, 2, threshold=float("inf"))
    assert rep["fallbacks"] == 0
    f, p = lat.get_fields()
    st = lat.get_state()
    s, rs = s0, []
    for _ in range(2):
        s, r = PR.linear_jump(s, w.dt, 16, "vv4", P)
        rs.append(r)
    print(f"a {st['a']:.15g} vs {s.a:.15g}; r {recs['r']} vs {rs}", flush=True)
    assert abs(st["a"] - s.a) <= 1e-12 * s.a and abs(st["b"] - s.b) <= 1e-12 * abs(s.b)
    assert np.max(np.abs(recs["r"] - np.array(rs))) <= 1e-12
    ef = np.max(np.abs(f - s.f)) / np.max(np.abs(s.f - s.f.mean(axis=tuple(range(1, 4)), keepdims=True)))
    ep = np.max(np.abs(p - s.p)) / np.max(np.abs(s.p - s.p.mean(axis=tuple(range(1, 4)), keepdims=True)))
    print(f"fluctuation-relative deviation: fields {ef:.3g}, momenta {ep:.3g}", flush=True)
    assert ef <= 1e-11 and ep <= 1e-11
    lat.close()
    sg.close()


def test_linear_jump_fp32_state_and_gates():
    """The same jump on an FP32 lattice stays within FP32 rounding of the FP64
    one, and with the default gates the early jumps of the preheating lattice
    (physical seed amplitude, linear regime) are all accepted.  Against the
    FP64 integrator the fluctuations deviate by the neglected mode coupling,
    which is first order in the amplitude relative to the signal: 2.5 % after
    four jumps here (the oracle's own jump gives the same), bounded at 5 %."""
    lib = _lib()
    from oracle import lattice as L
    from oracle import seed as S
    w = W.C1.with_(N=32, k_ir=1.0, precision="fp64")
    P = L.Params(N=32, dx=w.dx, n_fields=2, m2=w.m2, lam=w.lam, g2=w.g2, V0=w.V0)
    s0 = S.seed_state(P, w.k_ir, w.fbar[:2], w.pbar[:2], w.seed, amp=1.0)
    out = {}
    for prec in ("fp64", "fp32"):
        lat = lib.Lattice(32, w.dx, 2, prec)
        lat.set_potential(w.m2, w.lam, w.g2, w.V0)
        lat.set_fields(s0.f, s0.p)
        sg = lib.Surrogate(n_fields=2, extra_inputs=2, layers=2, jump_steps=16, init_seed=1)
        sg.set_jump("linear")
        recs, rep = sg.advance(lat, "vv4", w.dt, 4)
        out[prec] = (lat.get_fields(), rep)
        lat.close()
        sg.close()
    (f64, p64), rep64 = out["fp64"]
    (f32, p32), rep32 = out["fp32"]
    assert rep64["fallbacks"] == 0 and rep32["fallbacks"] == 0
    assert np.max(np.abs(f32 - f64)) <= 2e-6 * np.max(np.abs(f64))
    ref = lib.Lattice(32, w.dx, 2, "fp64")
    ref.set_potential(w.m2, w.lam, w.g2, w.V0)
    ref.set_fields(s0.f, s0.p)
    ref.step("vv4", w.dt, 64, record=False)
    fr, _ = ref.get_fields()
    fl = fr - fr.mean(axis=(1, 2, 3), keepdims=True)
    dev = np.max(np.abs((f64 - f64.mean(axis=(1, 2, 3), keepdims=True)) - fl)) / np.max(np.abs(fl))
    print(f"linear jumps vs FP64 VV4 after 64 steps: fluctuation-relative deviation {dev:.3g}", flush=True)
    assert dev < 5e-2
    ref.close()


def test_one_handle_two_spacings():
    """One surrogate handle advancing two lattices of the same N but
    different spacing: the mode table follows each lattice's dx (both equal
    their integrator for free fields on a static background)."""
    lib = _lib()
    sg = lib.Surrogate(n_fields=2, extra_inputs=2, layers=2, jump_steps=16, init_seed=1)
    sg.set_jump("linear")
    sg.set_gate(0.0)
    for dx in (0.4, 0.9):
        P, s0, lat = _free_static()
        lat.close()
        lat = lib.Lattice(32, dx, 2, "fp64")
        ref = lib.Lattice(32, dx, 2, "fp64")
        for h in (lat, ref):
            h.set_background(1.0, "static", 1.0, 1.0)
            h.set_potential(P.m2, P.lam, P.g2, 0.0)
            h.set_fields(s0.f, s0.p)
        recs, rep = sg.advance(lat, "vv4", 0.05, 1, threshold=float("inf"))
        assert rep["fallbacks"] == 0
        ref.step("vv4", 0.05, 16, record=False)
        f, p = lat.get_fields()
        fr, pr = ref.get_fields()
        err = max(np.max(np.abs(f - fr)) / np.max(np.abs(fr)), np.max(np.abs(p - pr)) / np.max(np.abs(pr)))
        print(f"dx {dx}: relative deviation from the integrator {err:.3g}", flush=True)
        assert err <= 1e-11
        lat.close()
        ref.close()
    sg.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_rejected_linear_jumps_are_the_integrator(precision):
    """Every jump rejected (threshold 0): the jump's result went to the other
    state buffer and is dropped, so the lattice ends bitwise where the
    integrator alone takes it, with the same background."""
    lib = _lib()
    w = W.C1.with_(N=32, k_ir=1.0, precision=precision)
    from oracle import lattice as L
    from oracle import seed as S
    P = L.Params(N=32, dx=w.dx, n_fields=2, m2=w.m2, lam=w.lam, g2=w.g2, V0=w.V0)
    s0 = S.seed_state(P, w.k_ir, w.fbar[:2], w.pbar[:2], w.seed, amp=1.0)
    hs = []
    for _ in range(2):
        h = lib.Lattice(32, w.dx, 2, precision)
        h.set_potential(w.m2, w.lam, w.g2, w.V0)
        h.set_fields(s0.f, s0.p)
        hs.append(h)
    lat, ref = hs
    sg = lib.Surrogate(n_fields=2, extra_inputs=2, layers=2, jump_steps=16, init_seed=1)
    sg.set_jump("linear")
    recs, rep = sg.advance(lat, "vv4", w.dt, 3, threshold=0.0)
    assert rep["fallbacks"] == 3
    for _ in range(3):
        ref.step("vv4", w.dt, 16, record=False)
    f, p = lat.get_fields()
    fr, pr = ref.get_fields()
    assert np.array_equal(f, fr) and np.array_equal(p, pr)
    assert lat.get_state() == ref.get_state()
    for h in (lat, ref, sg):
        h.close()


@pytest.mark.parametrize("nf", [1, 2])
def test_linear_jump_fp32_against_oracle(nf):
    """FP32 lattice (the fluctuations then go through the FP32 line FFT) on
    the interacting model (one field: lambda phi^4 at 16^3; two fields: the
    q = 100 model at 32^3), one accepted jump (threshold = inf, second gate
    off), against the oracle's FP64 jump from the same FP32-rounded state.  Error budget per element: the rounding of the result
    to FP32 (half an ulp of the field value, allowed 4 eps32 |f|) plus the
    FP32 transforms, packing and unpacking of the fluctuations (a few eps32
    per radix-2 stage, 2 log2(N^3) stages; allowed 64 eps32 max|fluct|)."""
    from oracle import lattice as L
    from oracle import propagator as PR
    from oracle import seed as S
    lib = _lib()
    N = 32 if nf == 2 else 16
    w = W.C1.with_(N=N, k_ir=1.0, precision="fp32")
    m2 = w.m2 if nf == 2 else (0.0, 0.0)
    g2 = w.g2 if nf == 2 else 0.0
    P = L.Params(N=N, dx=w.dx, n_fields=nf, m2=m2, lam=w.lam, g2=g2, V0=w.V0)
    s0 = S.seed_state(P, w.k_ir, w.fbar[:nf], w.pbar[:nf], w.seed, amp=20.0)
    f32 = s0.f.astype(np.float32).astype(np.float64)
    p32 = s0.p.astype(np.float32).astype(np.float64)
    rho, _ = L.rho_pressure(*L.energies(f32, p32, s0.a, P))
    sr = L.State(f32, p32, s0.a, L.hubble_from_rho(s0.a, rho, P))
    lat = lib.Lattice(N, w.dx, nf, "fp32")
    lat.set_potential(m2, w.lam, g2, w.V0)
    lat.set_fields(f32, p32)
    sg = lib.Surrogate(n_fields=nf, extra_inputs=2, layers=2, jump_steps=16, init_seed=1)
    sg.set_jump("linear")
    sg.set_gate(0.0)
    recs, rep = sg.advance(lat, "vv4", w.dt, 1, threshold=float("inf"))
    assert rep["fallbacks"] == 0
    f, p = lat.get_fields()
    s, r = PR.linear_jump(sr, w.dt, 16, "vv4", P)
    st = lat.get_state()
    eps = float(np.finfo(np.float32).eps)
    for got, want in ((f, s.f), (p, s.p)):
        fl = want - want.mean(axis=(1, 2, 3), keepdims=True)
        tol = 4 * eps * np.max(np.abs(want)) + 64 * eps * np.max(np.abs(fl))
        err = np.max(np.abs(got - want))
        print(f"max deviation {err:.3g}, allowed {tol:.3g} (fluctuation scale {np.max(np.abs(fl)):.3g})", flush=True)
        assert err <= tol
    print(f"a {st['a']:.10g} vs {s.a:.10g}; r {recs['r'][0]:.6g} vs {r:.6g}", flush=True)
    assert abs(st["a"] - s.a) <= 1e-6 * s.a
    assert abs(recs["r"][0] - r) <= 1e-5
    lat.close()
    sg.close()


@pytest.mark.parametrize("N,precision", [(64, "fp32"), (128, "fp32"), (256, "fp32"), (256, "fp64"), (512, "fp32")])
def test_free_fields_at_size_equal_the_integrator(N, precision):
    """The launch shapes the benchmark times (256^3: 2048-value fused z
    batches, 16-line FP32 axis batches with radix-16 passes, 129^3 folded
    index triples) and the sizes between: free fields of two masses on a
    static background, where one linear jump of 16 VV4 steps equals the
    integrator up to rounding, against the library's FP64 integrator.
    Allowed: 1e-11 of the field scale in FP64; in FP32 the rounding of the
    state (4 eps32 of the scale) plus the FP32 transforms (64 eps32 of the
    fluctuations), plus the FP32 state's own rounding at the start."""
    lib = _lib()
    rng = np.random.default_rng(11)
    m2 = (0.6, 2.3)
    dx = 0.4
    f = np.stack([0.9 + 0.3 * rng.standard_normal((N, N, N)), 0.05 + 0.3 * rng.standard_normal((N, N, N))])
    p = np.stack([0.02 + 0.3 * rng.standard_normal((N, N, N)), -0.01 + 0.3 * rng.standard_normal((N, N, N))])
    if precision == "fp32":
        f = f.astype(np.float32).astype(np.float64)
        p = p.astype(np.float32).astype(np.float64)
    hs = []
    for prec in (precision, "fp64"):
        h = lib.Lattice(N, dx, 2, prec)
        h.set_background(1.0, "static", 1.0, 1.0)
        h.set_potential(m2, (0.0, 0.0), 0.0, 0.0)
        h.set_fields(f, p)
        hs.append(h)
    lat, ref = hs
    del f, p
    sg = lib.Surrogate(n_fields=2, extra_inputs=2, layers=2, jump_steps=16, init_seed=1)
    sg.set_jump("linear")
    sg.set_gate(0.0)
    _, rep = sg.advance(lat, "vv4", 0.05, 1, threshold=float("inf"))
    assert rep["fallbacks"] == 0
    ref.step("vv4", 0.05, 16, record=False)
    got = lat.get_fields()
    want = ref.get_fields()
    eps = float(np.finfo(np.float32).eps)
    for g, w in zip(got, want):
        scale = float(np.max(np.abs(w)))
        fl = float(np.max(np.abs(w - w.mean(axis=(1, 2, 3), keepdims=True))))
        tol = 1e-11 * scale if precision == "fp64" else 4 * eps * scale + 64 * eps * fl
        err = float(np.max(np.abs(g - w)))
        print(f"N={N} {precision}: max deviation {err:.3g}, allowed {tol:.3g}", flush=True)
        assert err <= tol
    for h in (lat, ref, sg):
        h.close()
