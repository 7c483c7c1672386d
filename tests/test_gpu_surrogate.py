"""GPU tests of the learned surrogate: BF16 MFMA forward and gradients
against the FP64 oracle, training on integrator-generated pairs, and the
Hubble-constraint fallback gate."""
import numpy as np
import pytest

from oracle import surrogate as SG
import workloads as W

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2607_24978_amd import _lib
    return _lib


def unflatten(theta, channels):
    """Flat parameter vector -> [(W[o][i][3][3][3], b[o])] (layout of cl_surrogate.h)."""
    params, off = [], 0
    for cin, cout in zip(channels[:-1], channels[1:]):
        n = cout * cin * 27
        Wt = theta[off:off + n].astype(np.float64).reshape(cout, cin, 3, 3, 3)
        off += n
        b = theta[off:off + cout].astype(np.float64)
        off += cout
        params.append((Wt, b))
    assert off == theta.size
    return params


def emulated_forward(params, x):
    """FP64 forward with the GPU's BF16 roundings: weights and the inputs of
    every layer rounded to BF16.  Also returns, per output element, the
    convolution of absolute values (the scale of the rounding error)."""
    h = SG.bf16_round(x).astype(np.float64)
    absacc = None
    for l, (Wt, b) in enumerate(params):
        Wb = SG.bf16_round(Wt).astype(np.float64)
        z = SG.conv3d(h, Wb, b)
        absacc = SG.conv3d(np.abs(h), np.abs(Wb), np.abs(b))
        if l + 1 < len(params):
            h = SG.bf16_round(SG.gelu(z)).astype(np.float64)
        else:
            h = z
    return h, absacc


@pytest.mark.parametrize("layers,extra,tolf,N", [(2, 2, 2 ** -7, 16), (5, 4, 2 ** -5, 16), (3, 4, 2 ** -6, 64)])
def test_forward_matches_oracle(layers, extra, tolf, N):
    """Every output of the network against the FP64 forward on the same
    BF16-rounded operands.  At 16^3 every tile of the convolutions touches a
    periodic image; at 64^3 most tiles lie inside the lattice (the kernels'
    path without wrap-around)."""
    lib = _lib()
    s = lib.Surrogate(n_fields=2, extra_inputs=extra, layers=layers, init_seed=3)
    chans = [s.cin] + [32] * (layers - 1) + [s.cout]
    rng = np.random.default_rng(5)
    theta = s.get_params()
    # non-zero biases exercise the bias path
    params = unflatten(theta, chans)
    for l, (Wt, b) in enumerate(params):
        params[l] = (Wt, rng.uniform(-0.1, 0.1, b.shape))
    flat = np.concatenate([np.concatenate([Wt.ravel(), b]) for Wt, b in params]).astype(np.float32)
    s.set_params(flat)
    params = unflatten(flat, chans)
    x = rng.standard_normal((s.cin, N, N, N)).astype(np.float32)
    y = s.forward(x)
    ref, absacc = emulated_forward(params, x)
    err = np.abs(y - ref)
    bound = tolf * absacc + 1e-6
    assert np.all(err <= bound), (float(np.max(err / bound)), float(np.max(err)))
    # and the error is far below the signal: the bound is not vacuous
    assert np.max(err) < 0.05 * np.max(np.abs(ref))
    s.close()


def emulated_backward(params, x, t):
    """FP64 forward and backward with the GPU's BF16 roundings (the layer
    inputs and weights, the output gradient 2 (y - t) / n, the
    pre-activations GELU' is evaluated at and the GELU-scaled layer
    gradients rounded to BF16), together with the same
    computation on absolute values -- the scale of the rounding error of
    every gradient element (the forward's accumulated scale enters at the
    output and at every layer input)."""
    L_ = len(params)
    Wb = [SG.bf16_round(Wt).astype(np.float64) for Wt, _ in params]
    hs, zs, fabs = [SG.bf16_round(x).astype(np.float64)], [], [np.zeros_like(x, dtype=np.float64)]
    for l, (_, b) in enumerate(params):
        z = SG.conv3d(hs[-1], Wb[l], b)
        fa = SG.conv3d(np.abs(hs[-1]), np.abs(Wb[l]), np.abs(b))
        zs.append(z)
        if l + 1 < L_:
            hs.append(SG.bf16_round(SG.gelu(z)).astype(np.float64))
            fabs.append(fa)
        else:
            y, yabs = z, fa
    n = y.size
    loss = float(np.mean((y - t) ** 2))
    dz = SG.bf16_round(2.0 * (y - t) / n).astype(np.float64)
    dz_abs = np.abs(dz) + 2.0 * yabs / n
    grads, gabs = [None] * L_, [None] * L_
    for l in range(L_ - 1, -1, -1):
        dW, db = SG.conv3d_grad_weight(dz, hs[l])
        aW, ab = SG.conv3d_grad_weight(dz_abs, np.abs(hs[l]) + fabs[l])
        grads[l], gabs[l] = (dW, db), (aW, ab)
        dA = SG.conv3d_grad_input(dz, Wb[l])
        dA_abs = SG.conv3d_grad_input(dz_abs, np.abs(Wb[l]))
        if l == 0:
            return loss, grads, gabs, dA, dA_abs
        g = SG.gelu_grad(SG.bf16_round(zs[l - 1]).astype(np.float64))  # pre-activations kept in BF16
        dz = SG.bf16_round(dA * g).astype(np.float64)
        dz_abs = dA_abs * np.abs(g) + np.abs(dz)


@pytest.mark.parametrize("N", [32, 64])
def test_gradients_match_oracle_elementwise(N):
    """Every weight, bias and input gradient element of a 3-layer network at
    N^3 (at 64^3 most convolution tiles lie inside the lattice, at 32^3 none
    does) against the FP64 oracle's backward pass on the same BF16-rounded
    operands: |g_gpu - g_oracle| <= 2^-6 g_abs, where g_abs is the same
    backward pass on absolute values (the convolution-of-absolute-values
    bound of the forward check, carried through the backward pass).  A
    wrong element, a transposed weight or a dropped bias gradient breaks
    the bound; it is not vacuous (the typical error is far below it)."""
    lib = _lib()
    layers = 3
    s = lib.Surrogate(n_fields=2, extra_inputs=4, layers=layers, init_seed=11)
    chans = [s.cin] + [32] * (layers - 1) + [s.cout]
    rng = np.random.default_rng(9)
    params = unflatten(s.get_params(), chans)
    params = [(Wt, rng.uniform(-0.05, 0.05, b.shape)) for Wt, b in params]
    flat = np.concatenate([np.concatenate([Wt.ravel(), b]) for Wt, b in params]).astype(np.float32)
    s.set_params(flat)
    x = rng.standard_normal((s.cin, N, N, N)).astype(np.float32)
    t = rng.standard_normal((s.cout, N, N, N)).astype(np.float32)
    loss, g, gx = s.loss_grad(x, t, input_grad=True)
    pb = [(Wt, b) for Wt, b in unflatten(flat, chans)]
    lo, go, ga, dx, dx_abs = emulated_backward(pb, x.astype(np.float64), t.astype(np.float64))
    assert abs(loss - lo) <= 2e-2 * lo
    gamma = 2.0 ** -6
    off = 0
    for l, ((dW, db), (aW, ab)) in enumerate(zip(go, ga)):
        for ref, scale in ((dW, aW), (db, ab)):
            got = g[off:off + ref.size].astype(np.float64).reshape(ref.shape)
            off += ref.size
            err = np.abs(got - ref)
            ratio = float(np.max(err / (gamma * scale + 1e-30)))
            print(f"layer {l} {ref.shape}: max err {err.max():.3g}, max err/bound {ratio:.3g}, "
                  f"median rel {np.median(err / (np.abs(ref) + 1e-30)):.3g}", flush=True)
            assert ratio <= 1.0, (l, ref.shape, ratio)
            assert err.max() <= 2e-2 * np.abs(ref).max()
    assert off == g.size
    err = np.abs(gx.astype(np.float64) - dx)
    ratio = float(np.max(err / (gamma * dx_abs + 1e-30)))
    print(f"input gradient: max err {err.max():.3g}, max err/bound {ratio:.3g}", flush=True)
    assert ratio <= 1.0 and err.max() <= 2e-2 * np.abs(dx).max()
    s.close()


def test_adam_matches_oracle():
    """Three Adam steps of the device kernel (FP32) on caller-supplied
    gradients against the FP64 oracle step (Kingma and Ba, bias-corrected).
    The hyper-parameters are those the device holds, FP32 values of
    beta = (0.9, 0.999), eps = 1e-8 and lr (1 - float32(0.999) is 1.3e-5 off
    1e-3, far more than the arithmetic's rounding).  Bound per parameter,
    from the FP32 arithmetic: the moments carry rounding of at most a few
    units of 2^-24 of their terms (cancellations in m included as absolute
    errors), the update inherits them and its own rounding, and every stored
    weight rounds once per step."""
    lib = _lib()
    s = lib.Surrogate(n_fields=2, extra_inputs=2, layers=2, init_seed=4)
    theta0 = s.get_params().astype(np.float64)
    rng = np.random.default_rng(17)
    lr = 1e-3
    base = rng.standard_normal(theta0.size)
    grads = [(base * (1.0 + 0.5 * rng.standard_normal(theta0.size)) * 10.0 ** rng.uniform(-4, 1, theta0.size))
             .astype(np.float32) for _ in range(3)]
    for gr in grads:
        s.apply_grad(gr, lr)
    got = s.get_params().astype(np.float64)
    u = 2.0 ** -24
    th, m, v = theta0.copy(), np.zeros_like(theta0), np.zeros_like(theta0)
    dm = np.zeros_like(theta0)
    dv = np.zeros_like(theta0)
    bound = np.zeros_like(theta0)
    b1, b2, eps = (float(np.float32(x)) for x in (0.9, 0.999, 1e-8))
    lr32 = float(np.float32(lr))
    for t, gr in enumerate(grads, start=1):
        g64 = gr.astype(np.float64)
        dm = b1 * dm + 8 * u * (b1 * np.abs(m) + (1 - b1) * np.abs(g64))
        dv = b2 * dv + 8 * u * (b2 * v + (1 - b2) * g64 ** 2)
        th_new, m, v = SG.adam_step(th, g64, m, v, t, lr32, beta1=b1, beta2=b2, eps=eps)
        c1, c2 = 1 - b1 ** t, 1 - b2 ** t
        den = np.sqrt(v / c2) + eps
        step = np.abs(th_new - th)
        bound += lr32 / c1 * dm / den + step * (0.5 * dv / np.maximum(v, 1e-300) + 16 * u) \
            + np.spacing(np.abs(th_new).astype(np.float32)).astype(np.float64)
        th = th_new
    err = np.abs(got - th)
    print(f"adam: max err {err.max():.3g}, max err/bound {np.max(err / bound):.3g}", flush=True)
    assert np.all(err <= bound)
    # the three steps moved the weights by much more than the bound
    assert np.median(np.abs(th - theta0) / bound) > 10
    s.close()


def test_training_sizes_rejected():
    lib = _lib()
    s = lib.Surrogate(n_fields=2, extra_inputs=4, layers=2)
    with pytest.raises(lib.CLError):
        s.dataset_reserve(16, 2)
    x = np.zeros((s.cin, 16, 16, 16), np.float32)
    with pytest.raises(lib.CLError):
        s.loss_grad(x, np.zeros((s.cout, 16, 16, 16), np.float32))
    with pytest.raises(lib.CLError):
        s.train(epochs=1)
    with pytest.raises(lib.CLError):
        lib.Surrogate(n_fields=2, extra_inputs=6)   # 10 input channels
    with pytest.raises(lib.CLError):
        lib.Surrogate(hidden=64)
    s.close()


def seeded(w):
    lat = _lib().Lattice(w.N, w.dx, w.n_fields, w.precision)
    lat.set_background(w.alpha, w.expansion, w.mp, w.a0)
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    lat.seed(w.seed, w.fbar[:w.n_fields], w.pbar[:w.n_fields], w.cutoff_modes, w.amp)
    return lat


def make_pairs(s, seeds, N, k_ir, warm, jumps, precision="fp32"):
    """Record (state, state jump_steps later) pairs from seeded two-field
    preheating runs (the q = 100 workload at a smaller size) integrated with
    the library's VV4."""
    w0 = W.C1.with_(N=N, k_ir=k_ir, precision=precision)
    for seed in seeds:
        w = w0.with_(seed=seed)
        lat = seeded(w)
        lat.step("vv4", w.dt, warm)
        for _ in range(jumps):
            s.record_input(lat)
            lat.step("vv4", w.dt, s.jump_steps)
            s.record_target(lat)
            lat.step("vv4", w.dt, 3)
        lat.close()
    return w0


def test_training_reduces_loss_and_beats_zero_predictor():
    lib = _lib()
    s = lib.Surrogate(n_fields=2, extra_inputs=4, layers=5, jump_steps=16, init_seed=1)
    N = 32
    s.dataset_reserve(N, 40)
    make_pairs(s, [2000, 2001, 2002, 2003], N, 1.0, 10, 10)
    assert s.dataset_size() == 40
    rep = s.train(epochs=12, lr=2e-3, lr_final=1e-4, shuffle_seed=0, holdout=8)
    assert rep["steps"] == 12 * 32
    assert rep["last_epoch_loss"] < 0.5 * rep["first_loss"], rep
    assert rep["holdout_loss"] < 0.5 * rep["holdout_zero"], rep
    s.close()


def test_fallback_gate_forced_and_save_load(tmp_path):
    """Threshold 0 makes every jump fall back: the result is then bitwise the
    integrator's.  Saved and reloaded parameters are identical."""
    lib = _lib()
    s = lib.Surrogate(n_fields=2, extra_inputs=4, layers=5, jump_steps=16, init_seed=2)
    N = 32
    s.dataset_reserve(N, 4)
    w = make_pairs(s, [2100], N, 2.0, 4, 4)
    s.train(epochs=1, lr=1e-3, holdout=0)
    path = str(tmp_path / "net.bin")
    s.save(path)
    s2 = lib.Surrogate(n_fields=2, extra_inputs=4, layers=5, jump_steps=16, init_seed=99)
    s2.load(path)
    assert np.array_equal(s.get_params(), s2.get_params())
    a = seeded(w.with_(seed=7))
    b = seeded(w.with_(seed=7))
    recs, rep = s2.advance(a, "vv4", w.dt, 3, threshold=0.0)
    assert rep["fallbacks"] == 3
    ref = np.concatenate([b.step("vv4", w.dt, 16) for _ in range(3)])
    fa, pa = a.get_fields()
    fb, pb = b.get_fields()
    assert np.array_equal(fa, fb) and np.array_equal(pa, pb)
    assert recs[-1]["a"] == ref[-1]["a"]
    assert a.get_state() == b.get_state()
    # corrupted weights: huge outputs trip the gate as well
    theta = s2.get_params()
    s2.set_params(theta * 1e3)
    _, rep = s2.advance(a, "vv4", w.dt, 2, threshold=1e-3)
    assert rep["fallbacks"] == 2
    for _ in range(2):
        b.step("vv4", w.dt, 16)
    # overflowing outputs: non-finite jumps fall back even with no residual threshold
    s2.set_params(theta * 1e30)
    _, rep = s2.advance(a, "vv4", w.dt, 2, threshold=float("inf"))
    assert rep["fallbacks"] == 2
    for _ in range(2):
        b.step("vv4", w.dt, 16)
    fa, pa = a.get_fields()
    fb, pb = b.get_fields()
    assert np.all(np.isfinite(fa)) and np.array_equal(fa, fb) and np.array_equal(pa, pb)
    assert a.get_state() == b.get_state()
    for x in (a, b, s, s2):
        x.close()


def _jump_lattice(amp=20.0):
    """32^3 two-field preheating lattice in FP64 from the oracle's seed."""
    from oracle import lattice as L
    from oracle import seed as S
    w = W.C1.with_(N=32, k_ir=1.0, precision="fp64")
    P = L.Params(N=w.N, dx=w.dx, n_fields=2, m2=w.m2, lam=w.lam, g2=w.g2, V0=w.V0)
    s0 = S.seed_state(P, w.k_ir, w.fbar[:2], w.pbar[:2], w.seed, amp=amp)
    lat = _lib().Lattice(w.N, w.dx, 2, "fp64")
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    lat.set_fields(s0.f, s0.p)
    return w, P, s0, lat


def test_accepted_jump_exact_against_oracle():
    """Two accepted jumps (threshold = inf) with a network whose output is
    exactly its last-layer bias (all weights zero), so that everything
    after the network is plain arithmetic: predictor, state update,
    corrector and Hubble residual against the jump oracle -- fields within
    1e-11 (norm-wise) and a, a', residual within 1e-12 of FP64."""
    from oracle import surrogate_jump as J
    lib = _lib()
    w, P, s0, lat = _jump_lattice()
    sg = lib.Surrogate(n_fields=2, extra_inputs=4, layers=2, jump_steps=16, init_seed=5)
    theta = np.zeros(sg.num_params(), dtype=np.float32)
    bias = np.array([0.3, -0.2, 0.5, 0.1], dtype=np.float32)
    theta[-4:] = bias
    sg.set_params(theta)
    out_scale = [2e-4, 1e-4, 3e-3, 1e-3]
    sg.set_normalisation([1e-2] * 4, out_scale)
    sg.set_gate(0.0)  # arithmetic parity: no gating
    recs, rep = sg.advance(lat, "vv4", w.dt, 2, threshold=float("inf"))
    assert rep["fallbacks"] == 0
    f, p = lat.get_fields()
    st = lat.get_state()
    s, rs = s0, []
    y = np.broadcast_to(bias.astype(np.float64)[:, None, None, None], (4, 32, 32, 32))
    for _ in range(2):
        s, r = J.jump(s, y, out_scale, w.dt, 16, "vv4", P)
        rs.append(r)
    print(f"a {st['a']:.15g} vs {s.a:.15g}; r {recs['r']} vs {rs}", flush=True)
    assert abs(st["a"] - s.a) <= 1e-12 * s.a and abs(st["b"] - s.b) <= 1e-12 * abs(s.b)
    assert abs(st["eta"] - s.eta) <= 1e-14 * s.eta and st["step"] == 32
    assert np.max(np.abs(recs["r"] - np.array(rs))) <= 1e-12
    assert np.max(np.abs(f - s.f)) <= 1e-11 * np.max(np.abs(s.f))
    assert np.max(np.abs(p - s.p)) <= 1e-11 * np.max(np.abs(s.p))
    # the increment is visible: a jump with a zero output ends far from this one
    z = s0
    for _ in range(2):
        z, _ = J.jump(z, np.zeros_like(y), out_scale, w.dt, 16, "vv4", P)
    assert np.max(np.abs(f - z.f)) > 1e4 * 1e-11 * np.max(np.abs(s.f))
    lat.close()
    sg.close()


def test_accepted_jump_network_against_oracle():
    """One accepted jump with a random 5-layer network: the oracle packs the
    network input from the state (normalised fluctuations and broadcast
    features, rounded as the device rounds them), evaluates the network on
    BF16-rounded operands in FP64 and runs the jump; every field and
    momentum element within out_scale times the forward's BF16 bound
    (2^-5 of the convolution of absolute values).  The increments are small
    (out_scale 1e-3 of the fluctuations), so the network's rounding moves
    the endpoint sums -- hence a and a' -- by less than 1e-8 relative."""
    from oracle import lattice as L
    from oracle import surrogate_jump as J
    lib = _lib()
    w, P, s0, lat = _jump_lattice()
    sg = lib.Surrogate(n_fields=2, extra_inputs=4, layers=5, jump_steps=16, init_seed=6)
    chans = [8, 32, 32, 32, 32, 4]
    rng = np.random.default_rng(21)
    params = [(Wt, rng.uniform(-0.1, 0.1, b.shape)) for Wt, b in unflatten(sg.get_params(), chans)]
    flat = np.concatenate([np.concatenate([Wt.ravel(), b]) for Wt, b in params]).astype(np.float32)
    sg.set_params(flat)
    fl = [s0.f[0], s0.f[1], s0.p[0], s0.p[1]]
    rms = [float(np.std(c)) for c in fl]
    in_scale = rms
    out_scale = [1e-3 * r for r in rms]
    ex_mean, ex_std = [1.0, 0.3, 1.0, 0.0], [0.5, 0.2, 0.5, 0.1]
    sg.set_normalisation(in_scale, out_scale, ex_mean, ex_std)
    sg.set_gate(0.0)  # arithmetic parity: no gating
    recs, rep = sg.advance(lat, "vv4", w.dt, 1, threshold=float("inf"))
    assert rep["fallbacks"] == 0
    f, p = lat.get_fields()
    st = lat.get_state()
    # network input as the device packs it
    x = np.zeros((8, 32, 32, 32), dtype=np.float32)
    for c in range(4):
        v = fl[c] - np.mean(fl[c])
        x[c] = SG.bf16_round(np.float32(v * (1.0 / in_scale[c])))
    e = [s0.a, s0.b / s0.a, np.mean(s0.f[0]), np.mean(s0.p[0])]
    for k in range(4):
        x[4 + k] = SG.bf16_round(np.float32((e[k] - ex_mean[k]) / ex_std[k]))
    y, absacc = emulated_forward(unflatten(flat, chans), x)
    s, r = J.jump(s0, y, out_scale, w.dt, 16, "vv4", P)
    for j, (got, want) in enumerate([(f[0], s.f[0]), (f[1], s.f[1]), (p[0], s.p[0]), (p[1], s.p[1])]):
        bound = out_scale[j] * (2.0 ** -5 * absacc[j] + 1e-6) + 1e-12 * np.max(np.abs(want))
        err = np.abs(got - want)
        print(f"channel {j}: max err/bound {np.max(err / bound):.3g}", flush=True)
        assert np.all(err <= bound), j
        # the comparison resolves the network's share of the new state
        assert np.max(err) < 1e-2 * np.max(np.abs(out_scale[j] * y[j]))
    assert abs(st["a"] - s.a) <= 1e-8 * s.a and abs(st["b"] - s.b) <= 1e-8 * abs(s.b)
    assert abs(recs["r"][0] - r) <= 1e-8
    lat.close()
    sg.close()


def test_fluctuation_gate():
    """The second gate sees what the Hubble residual does not: with the
    residual gate off (threshold = inf), a network whose increments are
    twice the fluctuations (variance changed far beyond 25 %) is refused and
    the integrator runs instead -- bitwise the integrator's result -- while
    increments of 1e-3 of the fluctuations pass."""
    lib = _lib()
    chans = [8, 32, 4]
    for scale, expect_fallback in ((2.0, True), (1e-3, False)):
        w, P, s0, lat = _jump_lattice()
        sg = lib.Surrogate(n_fields=2, extra_inputs=4, layers=2, jump_steps=16, init_seed=8)
        rng = np.random.default_rng(4)
        params = [(Wt, rng.uniform(-0.1, 0.1, b.shape)) for Wt, b in unflatten(sg.get_params(), chans)]
        sg.set_params(np.concatenate([np.concatenate([Wt.ravel(), b]) for Wt, b in params]).astype(np.float32))
        rms = [float(np.std(c)) for c in (s0.f[0], s0.f[1], s0.p[0], s0.p[1])]
        y_rms = float(np.std(sg.forward(np.zeros((8, 16, 16, 16), np.float32) + 0.3)))
        sg.set_normalisation(rms, [scale * r / max(y_rms, 1e-6) for r in rms])
        sg.set_gate(0.25)
        recs, rep = sg.advance(lat, "vv4", w.dt, 1, threshold=float("inf"))
        assert rep["fallbacks"] == (1 if expect_fallback else 0), (scale, rep)
        assert rep["fluct_rejects"] == (1 if expect_fallback else 0), (scale, rep)
        if expect_fallback:
            ref = _lib().Lattice(w.N, w.dx, 2, "fp64")
            ref.set_potential(w.m2, w.lam, w.g2, w.V0)
            ref.set_fields(s0.f, s0.p)
            ref.step("vv4", w.dt, 16)
            assert np.array_equal(lat.get_fields()[0], ref.get_fields()[0])
            ref.close()
        lat.close()
        sg.close()
