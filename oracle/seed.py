"""Oracle (test infrastructure only): vacuum-fluctuation initial conditions.

Follows Sect. 2.3 (Eqs. QuantumFlucts, fpr_influct, fpr_influct2), the DFT
convention and mode range of Sect. 4.3, and the normalisation of Eq.
varFandDFgeneral with Upsilon = 1 (Type-II).  The paper names no random
generator; both this oracle and the library implement the same
counter-based generator from its published definition:

  SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom
  number generators", OOPSLA 2014): state s_k = seed + k * gamma with
  gamma = 0x9E3779B97F4A7C15, output mix(s_k) with the finaliser
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
  z *= 0x94D049BB133111EB; z ^= z >> 31.

Draw k is the k-th output (k >= 1) after starting at `seed`.  Uniforms are
u = ((z >> 11) + 1) * 2^-53 in (0, 1]; Gaussians come from the Box-Muller
cosine branch g = sqrt(-2 ln u1) cos(2 pi u2).

Counter layout (shared written reading): for field j, representative mode
index m = (ix N + iy) N + iz (ix = n_x mod N, ...), draw d in 0..3
(Re f_l, Im f_l, Re f_r, Im f_r) and Box-Muller component c in {0, 1},
k = 2 * (((j * N^3 + m) * 4) + d) + c + 1.
"""
from __future__ import annotations

import math

import numpy as np

from . import lattice as L

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, k):
    """k-th SplitMix64 output started from state `seed` (k is an array of
    uint64 counters >= 1)."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + k * GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, k):
    """53-bit uniform in (0, 1] from draw k."""
    z = splitmix64(seed, k)
    return ((z >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53


def gaussian(seed: int, k0):
    """Standard normal from the uniforms at counters k0 and k0 + 1."""
    k0 = np.asarray(k0, dtype=np.uint64)
    u1 = uniform(seed, k0)
    u2 = uniform(seed, k0 + np.uint64(1))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def mode_numbers(N: int):
    """Integer mode number along one axis for array index i: n = i for
    i <= N/2, else i - N (range -N/2+1 .. N/2, Sect. 4.3)."""
    i = np.arange(N)
    return np.where(i <= N // 2, i, i - N)


def representative_mask(N: int):
    """True where mode n is the representative of its pair {n, -n}: its first
    nonzero component (in x, y, z order) is positive."""
    n = mode_numbers(N)
    nx, ny, nz = np.meshgrid(n, n, n, indexing="ij")
    return (nx > 0) | ((nx == 0) & (ny > 0)) | ((nx == 0) & (ny == 0) & (nz > 0))


def fourier_fluctuations(N, dx, k_ir, j, seed, omega2, a0, alpha, H_hom, cutoff, amp):
    """Fourier amplitudes (df(n), dp(n)) of one field on the full mode lattice.

    Eq. QuantumFlucts: P(k) = 1 / (2 a^2 w_k), w_k^2 = k^2 + a^2 m^2.
    Reading of the normalisation: <|df(n)|^2> = S_k = amp^2 P(k) / dx^3
    (Eq. varFandDFgeneral with Upsilon = 1, scaled so that amp = N^(3/2)
    reproduces the paper's physical variance and amp = 1 the per-mode
    variance 1/(2 w_k dx^3) at a = 1).  The real and imaginary parts of the
    left- and right-movers are each Gaussian with variance S_k / 2.
    Eqs. fpr_influct, fpr_influct2:
      df  = (f_l + f_r) / sqrt(2)
      df' = a^(alpha-1) (i w_k / sqrt(2)) (f_l - f_r) - H df
    and dp = a^(3-alpha) df'.  Modes 0 < |n| <= cutoff are kept; the pair
    partner -n gets the complex conjugate so the real-space field is real.
    omega2 here is a^2 m^2 (the mass term of w_k^2)."""
    n = mode_numbers(N)
    nx, ny, nz = np.meshgrid(n, n, n, indexing="ij")
    n2 = (nx * nx + ny * ny + nz * nz).astype(np.float64)
    keep = representative_mask(N) & (n2 > 0) & (n2 <= cutoff * cutoff)
    k = k_ir * np.sqrt(n2)
    w2 = k * k + omega2
    keep &= w2 > 0
    idx = np.nonzero(keep)
    ix, iy, iz = idx
    m = (ix.astype(np.uint64) * np.uint64(N) + iy.astype(np.uint64)) * np.uint64(N) + iz.astype(np.uint64)
    base = (np.uint64(j) * np.uint64(N) ** np.uint64(3) + m) * np.uint64(4)
    g = [gaussian(seed, np.uint64(2) * (base + np.uint64(d)) + np.uint64(1)) for d in range(4)]
    w = np.sqrt(w2[idx])
    Pk = 1.0 / (2.0 * a0 ** 2 * w)
    S = amp ** 2 * Pk / dx ** 3
    sig = np.sqrt(0.5 * S)
    fl = sig * (g[0] + 1j * g[1])
    fr = sig * (g[2] + 1j * g[3])
    df_rep = (fl + fr) / math.sqrt(2.0)
    dfp_rep = a0 ** (alpha - 1.0) * (1j * w / math.sqrt(2.0)) * (fl - fr) - H_hom * df_rep
    dp_rep = a0 ** (3.0 - alpha) * dfp_rep
    DF = np.zeros((N, N, N), dtype=np.complex128)
    DP = np.zeros((N, N, N), dtype=np.complex128)
    DF[idx] = df_rep
    DP[idx] = dp_rep
    # pair partner: index (-i) mod N
    jx, jy, jz = (-ix) % N, (-iy) % N, (-iz) % N
    DF[jx, jy, jz] = np.conj(df_rep)
    DP[jx, jy, jz] = np.conj(dp_rep)
    return DF, DP


def inverse_dft(G):
    """f(n) = N^-3 sum_n' exp(+i 2 pi n'.n / N) f(n') (Sect. 4.3)."""
    return np.fft.ifftn(G)


def seed_state(P: L.Params, k_ir: float, fbar, pbar, seed: int, a0: float = 1.0,
               cutoff: float | None = None, amp: float = 1.0, return_imag: bool = False):
    """Homogeneous values plus vacuum fluctuations (Sect. 2.3), then the
    initial b = a' from the lattice energy density so that the Hubble
    constraint holds exactly at the start.

    The -H df term of Eq. fpr_influct2 uses the homogeneous Hubble rate,
    from rho_hom = sum_j pbar_j^2 / (2 a^6) + V(fbar)."""
    N = P.N
    if cutoff is None:
        cutoff = N / 4.0
    nf = P.n_fields
    fb = np.array(list(fbar)[:nf] + [0.0] * (2 - nf))
    pb = np.array(list(pbar)[:nf] + [0.0] * (2 - nf))
    m2 = L.mass2_eff(fb, P)
    if P.expansion == "static":
        H_hom = 0.0
    else:
        f1 = fb[:nf].reshape(nf, 1, 1, 1)
        V_hom = float(L.potential(f1, P).ravel()[0])
        rho_hom = sum(pb[j] ** 2 for j in range(nf)) / (2.0 * a0 ** 6) + V_hom
        H_hom = math.sqrt(a0 ** (2.0 * P.alpha) * rho_hom / (3.0 * P.mp ** 2))
    f = np.empty((nf, N, N, N))
    p = np.empty((nf, N, N, N))
    imag = 0.0
    for j in range(nf):
        DF, DP = fourier_fluctuations(N, P.dx, k_ir, j, seed, a0 ** 2 * m2[j], a0, P.alpha,
                                      H_hom, cutoff, amp)
        df = inverse_dft(DF)
        dp = inverse_dft(DP)
        imag = max(imag, float(np.max(np.abs(df.imag))), float(np.max(np.abs(dp.imag))))
        f[j] = fb[j] + df.real
        p[j] = pb[j] + dp.real
    E = L.energies(f, p, a0, P)
    rho, _ = L.rho_pressure(*E)
    b0 = L.hubble_from_rho(a0, rho, P)
    s = L.State(f, p, a0, b0, 0.0)
    return (s, imag) if return_imag else s
