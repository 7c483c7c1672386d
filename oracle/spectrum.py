"""Lattice power spectrum -- TEST INFRASTRUCTURE ONLY (see the package header).

Sect. 4.3 (arbitrary binning): with the forward DFT
    f(n~) = sum_n exp(-2 pi i n~.n / N) f(n)
(the inverse of the DFT convention of Eq. discretePSaux), the volume average
is <f^2>_V = N^-6 sum_n~ |f(n~)|^2, and a radial binning groups the modes by
|n~| with n~_i in {-N/2+1, ..., N/2}.  Reading of the bins: bin l collects
the modes with l*w - w/2 <= |n~| < l*w + w/2 (centred shells, as the
canonical binning w = 1 is described), l = 0, 1, ...; the bin's momentum is
k_l = k_IR * l * w.  The spectrum of a bin in the exact-multiplicity form of
Eq. discretePST2 (Type I: Upsilon = #/(4 pi |n~|^2)) is
    Delta_f(k_l) = (k_l / 2 pi) (dx / N^5) sum_{n~ in bin} |f(n~)|^2,
which equals k^3/(2 pi^2) Upsilon (dx/N)^3 <|f|^2>_bin.
"""
import numpy as np


def mode_radii(N: int) -> np.ndarray:
    """|n~| for every DFT index (m -> m for m <= N/2, m - N above)."""
    m = np.arange(N)
    n = np.where(m <= N // 2, m, m - N).astype(np.float64)
    X, Y, Z = np.meshgrid(n, n, n, indexing="ij")
    return np.sqrt(X * X + Y * Y + Z * Z)


def bin_index(r: np.ndarray, width: float) -> np.ndarray:
    """Centred shells: l = floor(r / w + 1/2)."""
    return np.floor(r / width + 0.5).astype(np.int64)


def power_spectrum(f: np.ndarray, dx: float, width: float = 1.0, nbins: int | None = None):
    """Counts, sums of |f(n~)|^2 and Delta_f per bin for one real N^3 field.
    Returns (k, counts, sums, delta) for bins l = 0 .. nbins-1 (modes beyond
    the last bin are dropped)."""
    N = f.shape[0]
    F = np.fft.fftn(f)  # numpy's forward transform has the exp(-2 pi i ...) sign and no scale
    p = (F.real ** 2 + F.imag ** 2).ravel()
    lb = bin_index(mode_radii(N), width).ravel()
    if nbins is None:
        nbins = int(lb.max()) + 1
    keep = lb < nbins
    counts = np.bincount(lb[keep], minlength=nbins)[:nbins]
    sums = np.bincount(lb[keep], weights=p[keep], minlength=nbins)[:nbins]
    k_ir = 2.0 * np.pi / (N * dx)
    k = k_ir * width * np.arange(nbins)
    delta = k / (2.0 * np.pi) * dx / float(N) ** 5 * sums
    return k, counts, sums, delta
