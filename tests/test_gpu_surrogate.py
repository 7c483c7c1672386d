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


@pytest.mark.parametrize("layers,extra,tolf", [(2, 2, 2 ** -7), (5, 4, 2 ** -5)])
def test_forward_matches_oracle(layers, extra, tolf):
    lib = _lib()
    N = 16
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


def test_gradients_match_oracle():
    lib = _lib()
    N = 32
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
    loss, g = s.loss_grad(x, t)
    # oracle: FP64 forward/backward on the BF16-rounded weights and input
    pb = [(SG.bf16_round(Wt).astype(np.float64), b) for Wt, b in unflatten(flat, chans)]
    yo, cache = SG.forward(pb, SG.bf16_round(x).astype(np.float64))
    lo, dy = SG.mse(yo, t.astype(np.float64))
    go = SG.backward(pb, cache, dy)
    assert abs(loss - lo) <= 2e-2 * lo
    gref = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in go])
    off = 0
    for (dW, db) in go:
        n = dW.size + db.size
        a, b = g[off:off + n].astype(np.float64), gref[off:off + n]
        off += n
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        assert rel < 3e-2 and cos > 0.999, (rel, cos)
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
