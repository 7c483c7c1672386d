"""Pins of the power-spectrum oracle against closed forms and brute force
(CPU only)."""
import math

import numpy as np
import pytest

from oracle import spectrum as SP


def test_parseval_all_modes_binned():
    """Every mode lands in exactly one bin: the bin sums add up to
    N^3 sum_n f(n)^2 (Parseval for the unnormalised forward DFT)."""
    N = 12
    f = np.random.default_rng(0).standard_normal((N, N, N))
    _, counts, sums, _ = SP.power_spectrum(f, dx=0.3, width=1.0, nbins=100)
    assert counts.sum() == N ** 3
    assert abs(sums.sum() - N ** 3 * np.sum(f * f)) <= 1e-12 * N ** 3 * np.sum(f * f)


@pytest.mark.parametrize("a,expect_bin", [((3, 4, 0), 5), ((1, 2, 2), 3), ((0, 0, 5), 5), ((2, 3, 6), 7)])
def test_single_plane_wave(a, expect_bin):
    """f = A cos(2 pi a.n / N): the only power sits at n~ = +-a with
    |f(n~)| = A N^3 / 2 each, so one bin holds A^2 N^6 / 2."""
    N, A = 16, 0.7
    n = np.arange(N)
    X, Y, Z = np.meshgrid(n, n, n, indexing="ij")
    f = A * np.cos(2 * np.pi * (a[0] * X + a[1] * Y + a[2] * Z) / N)
    _, counts, sums, _ = SP.power_spectrum(f, dx=1.0, width=1.0, nbins=N)
    want = A ** 2 * N ** 6 / 2
    assert abs(sums[expect_bin] - want) <= 1e-10 * want
    others = np.delete(sums, expect_bin)
    assert np.max(np.abs(others)) <= 1e-12 * want


def test_nyquist_mode_counted_once():
    """n~ = N/2 is one DFT index (no -N/2 partner): cos(pi n_x) puts A N^3
    there, all in bin N/2."""
    N, A = 8, 1.3
    n = np.arange(N)
    X, _, _ = np.meshgrid(n, n, n, indexing="ij")
    f = A * np.cos(np.pi * X)
    _, _, sums, _ = SP.power_spectrum(f, dx=1.0, width=1.0, nbins=N)
    want = (A * N ** 3) ** 2
    assert abs(sums[N // 2] - want) <= 1e-10 * want
    assert abs(sums.sum() - want) <= 1e-10 * want


@pytest.mark.parametrize("N,width", [(8, 1.0), (10, 1.0), (8, 0.5), (12, 2.0)])
def test_bin_counts_brute_force(N, width):
    """Shell multiplicities against a direct count over the integer modes
    n~_i in {-N/2+1, ..., N/2}."""
    nbins = int(math.ceil(math.sqrt(3) * (N // 2) / width)) + 2
    want = np.zeros(nbins, dtype=np.int64)
    rng = range(-N // 2 + 1, N // 2 + 1)
    for i in rng:
        for j in rng:
            for k in rng:
                r = math.sqrt(i * i + j * j + k * k)
                lb = int(math.floor(r / width + 0.5))
                if lb < nbins:
                    want[lb] += 1
    _, counts, _, _ = SP.power_spectrum(np.zeros((N, N, N)), dx=1.0, width=width, nbins=nbins)
    assert np.array_equal(counts, want)


def test_delta_forms_agree():
    """The two forms of Eq. discretePST2 agree: (k/2pi)(dx/N^5) # <|f|^2>
    and k^3/(2 pi^2) Upsilon (dx/N)^3 <|f|^2> with Upsilon = #/(4 pi |n~|^2)."""
    N, dx = 16, 0.37
    f = np.random.default_rng(3).standard_normal((N, N, N))
    k, counts, sums, delta = SP.power_spectrum(f, dx=dx, width=1.0, nbins=N)
    for l in range(1, N):
        if counts[l] == 0:
            continue
        mean = sums[l] / counts[l]
        ups = counts[l] / (4 * np.pi * l ** 2)
        alt = k[l] ** 3 / (2 * np.pi ** 2) * ups * (dx / N) ** 3 * mean
        assert abs(delta[l] - alt) <= 1e-12 * abs(alt)
    assert delta[0] == 0.0
