"""Pins of the surrogate oracle (FP64): brute-force convolution on tiny
lattices, the circular-convolution identity of the DFT, central finite
differences for every gradient, closed forms of GELU and Adam, and bfloat16
rounding cases.  CPU only."""
import math

import numpy as np
import pytest

from oracle import surrogate as SG


def brute_conv(x, W, b):
    """Direct six-fold loop over sites, channels and offsets."""
    cin, X, Y, Z = x.shape
    cout = W.shape[0]
    y = np.zeros((cout, X, Y, Z))
    for o in range(cout):
        for i in range(X):
            for j in range(Y):
                for k in range(Z):
                    s = b[o]
                    for c in range(cin):
                        for dx in (-1, 0, 1):
                            for dy in (-1, 0, 1):
                                for dz in (-1, 0, 1):
                                    s += W[o, c, dx + 1, dy + 1, dz + 1] * x[c, (i + dx) % X, (j + dy) % Y, (k + dz) % Z]
                    y[o, i, j, k] = s
    return y


def test_conv_matches_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 5, 6))
    W = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    assert np.max(np.abs(SG.conv3d(x, W, b) - brute_conv(x, W, b))) <= 1e-12


def test_conv_circular_convolution_identity():
    """Periodic cross-correlation with a kernel embedded on the lattice:
    FFT(y)_o = sum_i FFT(x_i) * conj(FFT(w_oi)) for y[n] = sum_d w[d] x[n + d]."""
    rng = np.random.default_rng(1)
    N = 8
    x = rng.standard_normal((2, N, N, N))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    y = SG.conv3d(x, W, np.zeros(3))
    X = np.fft.fftn(x, axes=(1, 2, 3))
    for o in range(3):
        acc = np.zeros((N, N, N), dtype=complex)
        for i in range(2):
            k = np.zeros((N, N, N))
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        k[dx % N, dy % N, dz % N] = W[o, i, dx + 1, dy + 1, dz + 1]
            acc += X[i] * np.conj(np.fft.fftn(k))
        assert np.max(np.abs(np.fft.ifftn(acc).real - y[o])) <= 1e-12


def test_gelu_closed_forms():
    assert SG.gelu(np.array(0.0)) == 0.0
    assert abs(SG.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15  # Phi(1)
    z = np.linspace(-5, 5, 101)
    assert np.max(np.abs(SG.gelu(z) - SG.gelu(-z) - z)) < 1e-14  # Phi(z) + Phi(-z) = 1
    h = 1e-6
    fd = (SG.gelu(z + h) - SG.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - SG.gelu_grad(z))) < 1e-8


def test_adam_first_step_closed_form():
    """With bias correction the first Adam step moves by lr * g/(|g| + eps)."""
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = SG.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(t1, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # second step with the same gradient: m and v are the bias-corrected g, g^2 again
    t2, _, _ = SG.adam_step(t1, g, m, v, 2, lr=0.01)
    assert np.allclose(t2, t1 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_bf16_rounding_cases():
    one = 1.0
    cases = {
        one: one,
        1.0 + 2 ** -8: 1.0,                    # halfway, ties to even (down)
        1.0 + 3 * 2 ** -8: 1.0 + 2 ** -6,      # halfway, ties to even (up)
        1.0 + 2 ** -8 + 2 ** -20: 1.0 + 2 ** -7,  # above halfway
        -3.14159265: -3.140625,
        65504.0: 65536.0,
    }
    for x, want in cases.items():
        assert float(SG.bf16_round(np.array([x]))[0]) == want, x


@pytest.mark.parametrize("channels", [(3, 4, 2), (2, 3, 3, 1)])
def test_gradients_finite_differences(channels):
    rng = np.random.default_rng(7)
    N = 4
    params = SG.init_params(channels, 3)
    params = [(W, rng.standard_normal(W.shape[0]) * 0.1) for W, _ in params]
    x = rng.standard_normal((channels[0], N, N, N))
    t = rng.standard_normal((channels[-1], N, N, N))

    def loss(ps, xx):
        y, _ = SG.forward(ps, xx)
        return SG.mse(y, t)[0]

    y, cache = SG.forward(params, x)
    _, dy = SG.mse(y, t)
    grads = SG.backward(params, cache, dy)
    h = 1e-6
    for l, (W, b) in enumerate(params):
        for idx in [(0, 0, 1, 1, 1), (W.shape[0] - 1, W.shape[1] - 1, 0, 2, 1), (0, W.shape[1] - 1, 2, 0, 0)]:
            Wp = W.copy(); Wp[idx] += h
            Wm = W.copy(); Wm[idx] -= h
            pp = list(params); pp[l] = (Wp, b)
            pm = list(params); pm[l] = (Wm, b)
            fd = (loss(pp, x) - loss(pm, x)) / (2 * h)
            assert abs(fd - grads[l][0][idx]) <= 1e-7 * max(1.0, abs(fd)), (l, idx)
        bp = b.copy(); bp[0] += h
        bm = b.copy(); bm[0] -= h
        pp = list(params); pp[l] = (W, bp)
        pm = list(params); pm[l] = (W, bm)
        fd = (loss(pp, x) - loss(pm, x)) / (2 * h)
        assert abs(fd - grads[l][1][0]) <= 1e-7 * max(1.0, abs(fd))
    # input gradient through the whole net (the chain backward() follows)
    g = dy
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        hh, z = cache[l]
        dz = g if l + 1 == len(params) else g * SG.gelu_grad(z)
        g = SG.conv3d_grad_input(dz, W)
    for idx in [(0, 1, 2, 3), (channels[0] - 1, 0, 0, 0)]:
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = (loss(params, xp) - loss(params, xm)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(fd))
