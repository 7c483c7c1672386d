"""GPU power spectrum (own FP64 FFT + shell binning) against the oracle's
numpy DFT, through the C ABI.  Counts are integers and must match exactly;
bin sums within 1e-9 relative (FP64 FFT rounding, atomically accumulated
bins), with an absolute floor of 1e-13 of the total power for bins that
hold almost nothing."""
import numpy as np
import pytest

from oracle import spectrum as SP
import workloads as W

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2607_24978_amd import _lib
    return _lib


def check(lat, f_host, field, what, width, dx):
    N = f_host.shape[0]
    nb = int(np.ceil(np.sqrt(3.0) * (N // 2) / width)) + 1
    k, c, s, d = lat.power_spectrum(field, what, width, nb)
    ko, co, so, do = SP.power_spectrum(f_host, dx, width, nb)
    assert np.array_equal(c, co)
    floor = 1e-13 * so.sum()
    assert np.all(np.abs(s - so) <= 1e-9 * so + floor), np.max(np.abs(s - so) / np.maximum(so, floor))
    assert np.allclose(k, ko, rtol=1e-15, atol=0)
    assert np.all(np.abs(d - do) <= 1e-9 * np.abs(do) + 1e-13 * np.abs(do).sum())


@pytest.mark.parametrize("N,precision", [(16, "fp64"), (32, "fp64"), (64, "fp32"), (128, "fp64")])
@pytest.mark.parametrize("width", [1.0, 0.5, 2.0])
def test_spectrum_matches_oracle(N, precision, width):
    """Seeded two-field state (after a few steps, so f and pi carry
    structure): f_0, pi_0 and f_1 against the numpy DFT of the same values."""
    w = W.C1.with_(N=N, k_ir=2.0 * 32 / N, precision=precision)
    lat = _lib().Lattice(N, w.dx, 2, precision)
    lat.set_background(w.alpha, w.expansion, w.mp, w.a0)
    lat.set_potential(w.m2, w.lam, w.g2, w.V0)
    lat.seed(w.seed, w.fbar[:2], w.pbar[:2], w.cutoff_modes, 20.0)
    lat.step("leapfrog", w.dt, 5)
    f, p = lat.get_fields()
    check(lat, f[0], 0, "f", width, w.dx)
    check(lat, p[0], 0, "pi", width, w.dx)
    check(lat, f[1], 1, "f", width, w.dx)
    lat.close()


def test_spectrum_matches_oracle_256_fp32():
    """The benchmark's shape: 256^3 two-field FP32 lattice, where the y and x
    passes run over the half z <= N / 2 of the transform (136 of 256 stored z,
    the last batch partly padding) and count the mirrored modes twice."""
    N = 256
    rng = np.random.default_rng(77)
    f = np.stack([1.0 + 0.1 * rng.standard_normal((N, N, N)), 0.05 * rng.standard_normal((N, N, N))])
    p = 0.01 * rng.standard_normal((2, N, N, N))
    lat = _lib().Lattice(N, 0.1, 2, "fp32")
    lat.set_background(1.0, "static", 1.0, 1.0)
    lat.set_fields(f, p)
    del f, p
    f32, _ = lat.get_fields()
    check(lat, f32[1], 1, "f", 1.0, 0.1)
    lat.close()


def test_spectrum_plane_wave_256():
    """A single plane wave on 256^3 (the y and x passes with four- and
    sixteen-line batches): all power in one bin, A^2 N^6 / 2."""
    N, A = 256, 0.25
    n = np.arange(N)
    X, Y, Z = np.meshgrid(n, n, n, indexing="ij", sparse=True)
    f = np.broadcast_to(1.0 + A * np.cos(2 * np.pi * (3 * X + 4 * Y + 12 * Z) / N), (N, N, N))
    f = np.ascontiguousarray(f[None], dtype=np.float64)
    p = np.zeros_like(f)
    lat = _lib().Lattice(N, 0.1, 1, "fp64")
    lat.set_background(1.0, "static", 1.0, 1.0)
    lat.set_fields(f, p)
    _, c, s, _ = lat.power_spectrum(0, "f", 1.0, 300)
    lat.close()
    want = A ** 2 * float(N) ** 6 / 2
    assert abs(s[13] - want) <= 1e-12 * want          # |(3, 4, 12)| = 13
    assert abs(s[0] - float(N) ** 6) <= 1e-12 * float(N) ** 6  # the mean, 1.0
    rest = np.delete(s, [0, 13])
    assert np.max(rest) <= 1e-20 * want
    assert c.sum() == N ** 3


def test_spectrum_argument_errors():
    lib = _lib()
    lat = lib.Lattice(16, 0.5, 1, "fp64")
    lat.seed(1, (1.0,), (0.0,))
    for kw in (dict(field=1), dict(width=0.0), dict(nbins=0), dict(nbins=5000)):
        args = dict(field=0, what="f", width=1.0, nbins=10)
        args.update(kw)
        with pytest.raises(lib.CLError):
            lat.power_spectrum(**args)
    lat.close()
