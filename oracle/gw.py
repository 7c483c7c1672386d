"""Oracle (test infrastructure only): gravitational waves sourced by the
scalar fields, in FP64, by the five-component traceless method.

Sect. 2.2 (Eq. EoMGWs) and Sect. 4.2: the tensor perturbation obeys
    h_ij'' + (3 - alpha) H h_ij' - a^(-2(1-alpha)) Lap h_ij
        = 2 / (m_p^2 a^(2(1-alpha))) Pi_ij^TT,
sourced for real scalars by Pi^eff_ij = sum over fields of d_i f d_j f
(Eq. anitensor).  The method evolves instead five auxiliary fields
v_11, v_12, v_13, v_22, v_23 (v_33 = -v_11 - v_22) with the same left-hand
side and the traceless part of the unprojected source,
    S_ij = Pi^eff_ij - delta_ij Pi^eff_kk / 3,
and obtains the physical waves only when they are measured, by the local
transverse-traceless projection in Fourier space,
    h_ij(k) = Lambda_ij,lm(k^) v_lm(k),
    Lambda_ij,lm = P_il P_jm - P_ij P_lm / 2,  P_ij = delta_ij - k^_i k^_j.
The energy density of the waves is rho_GW = m_p^2 <h'_ij h'_ij> / (4 a^(2 alpha))
(the integral over log k of the spectrum of Sect. 4.2).

Readings of what the paper leaves to its companion review (shared with the
library, written out here):
  * Time stepping.  With the conjugate momentum u_ij = a^(3-alpha) v_ij' the
    equation is the scalar one without a potential: drift v' = a^(alpha-3) u,
    kick u' = a^(1+alpha) (Lap v + (2/m_p^2) S).  v and u are advanced in the
    same velocity-Verlet sub-steps as the scalar fields (kick with the source
    at the same time level, drift with the midpoint a); they start at zero.
  * Source discretisation.  Pi^eff_ij at a site is the average of the
    products of forward differences and of backward differences,
    sum_fields [D+_i f D+_j f + D-_i f D-_j f] / (2 dx^2), symmetric in i, j
    and even under reflection of the lattice.
  * Projection.  k^ is the unit vector of the lattice momentum of the
    7-point Laplacian, k_i = (2/dx) sin(pi n_i / N); the mode n = 0 carries
    no waves.
  * Binned spectrum.  Bin l of width w (centred shells |n| in
    [l w - w/2, l w + w/2), as the scalar spectrum) holds
    rho_l = m_p^2 / (4 a^(2 alpha) N^6) sum over its modes of |h'_ij(n)|^2,
    so that the bins add up to rho_GW; d rho_GW / d log k at k_l = l w k_IR
    is taken as rho_l k_l / (w k_IR) = l rho_l, and
    Omega_GW = (d rho_GW / d log k) / rho_tot with rho_tot the lattice
    energy density.

Pins (tests/test_oracle_gw.py): tracelessness of the source, the free-wave
lattice dispersion, the projector against its closed form and its defining
properties, the absence of waves from an axis-aligned scalar plane wave, and
rho_GW of a prescribed transverse-traceless wave.
"""
from __future__ import annotations

import numpy as np

from . import lattice as L
from .spectrum import bin_index, mode_radii

# the five evolved components, as (i, j) index pairs
COMPONENTS = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2)]


def anisotropic_stress(f, P: L.Params):
    """Pi^eff_ij at every site, shape [3, 3, N, N, N] (source reading above)."""
    shape = f.shape[1:]
    Pi = np.zeros((3, 3) + shape)
    for j in range(P.n_fields):
        dp = [L.shift(f[j], ax, +1) - f[j] for ax in range(3)]
        dm = [f[j] - L.shift(f[j], ax, -1) for ax in range(3)]
        for a in range(3):
            for b in range(3):
                Pi[a, b] += 0.5 * (dp[a] * dp[b] + dm[a] * dm[b])
    return Pi / P.dx ** 2


def traceless_source(f, P: L.Params):
    """The five components of S_ij = Pi_ij - delta_ij Pi_kk / 3, shape [5, N, N, N]."""
    Pi = anisotropic_stress(f, P)
    tr = Pi[0, 0] + Pi[1, 1] + Pi[2, 2]
    return np.stack([Pi[i, j] - (tr / 3.0 if i == j else 0.0) for i, j in COMPONENTS])


def full_tensor(v):
    """[5, ...] components -> symmetric traceless [3, 3, ...] with v_33 = -v_11 - v_22."""
    t = np.zeros((3, 3) + v.shape[1:], dtype=v.dtype)
    for c, (i, j) in enumerate(COMPONENTS):
        t[i, j] = v[c]
        t[j, i] = v[c]
    t[2, 2] = -v[0] - v[3]
    return t


def gw_force(v, f, a: float, P: L.Params):
    """u' = a^(1+alpha) (Lap v + (2/m_p^2) S) for the five components."""
    S = traceless_source(f, P)
    out = np.empty_like(v)
    for c in range(5):
        out[c] = a ** (1.0 + P.alpha) * (L.laplacian(v[c], P.dx) + 2.0 / P.mp ** 2 * S[c])
    return out


def vv2(s: L.State, v, u, h: float, P: L.Params):
    """One velocity-Verlet sub-step of the scalar lattice (the lattice
    oracle's) with the five tensor components carried along: half kick of u
    with the source of the fields before the drift, drift of v with the
    midpoint a, half kick with the drifted fields and the new a."""
    u = u + 0.5 * h * gw_force(v, s.f, s.a, P)
    s1 = L.vv2(s, h, P)
    abar = 0.5 * (s.a + s1.a)
    v = v + h * abar ** (P.alpha - 3.0) * u
    u = u + 0.5 * h * gw_force(v, s1.f, s1.a, P)
    return s1, v, u


def step(s: L.State, v, u, dt: float, P: L.Params, integrator: str = "leapfrog"):
    """One full step (leapfrog = VV2(dt); vv4 = VV2(w1 dt) VV2(w0 dt) VV2(w1 dt))."""
    subs = [L.W1, L.W0, L.W1] if integrator == "vv4" else [1.0]
    for c in subs:
        s, v, u = vv2(s, v, u, c * dt, P)
    return s, v, u


def run(s: L.State, v, u, dt: float, n: int, P: L.Params, integrator: str = "leapfrog"):
    for _ in range(n):
        s, v, u = step(s, v, u, dt, P, integrator)
    return s, v, u


def lattice_khat(N: int):
    """Unit vectors of the lattice momentum sin(pi n_i / N) per DFT index,
    shape [3, N, N, N]; zero at n = 0."""
    m = np.arange(N)
    n = np.where(m <= N // 2, m, m - N).astype(np.float64)
    s = np.sin(np.pi * n / N)
    K = np.stack(np.meshgrid(s, s, s, indexing="ij"))
    norm = np.sqrt(np.sum(K * K, axis=0))
    return np.divide(K, norm, out=np.zeros_like(K), where=norm > 0)


def tt_project(T, khat):
    """Lambda_ij,lm(k^) T_lm for a field of 3x3 tensors [3, 3, ...] and unit
    vectors khat [3, ...] (zero vectors give zero)."""
    d = np.eye(3).reshape((3, 3) + (1,) * (T.ndim - 2))
    Pm = d - khat[:, None] * khat[None, :]
    PT = np.einsum("il...,lm...->im...", Pm, T)
    PTP = np.einsum("im...,mj...->ij...", PT, Pm)
    trPT = np.einsum("lm...,lm...->...", Pm, T)
    out = PTP - 0.5 * Pm * trPT
    zero = np.sum(khat * khat, axis=0) == 0
    out[..., zero] = 0.0
    return out


def gw_spectrum(u, a: float, P: L.Params, rho_tot: float, width: float = 1.0, nbins: int | None = None):
    """Binned energy density of the waves (reading above) from the tensor
    momenta u: returns (counts, rho_l, omega_l, rho_GW)."""
    N = P.N
    hp = a ** (P.alpha - 3.0) * full_tensor(u)
    Hk = np.fft.fftn(hp, axes=(2, 3, 4))
    TT = tt_project(Hk, lattice_khat(N))
    p = np.sum(TT.real ** 2 + TT.imag ** 2, axis=(0, 1)).ravel()
    lb = bin_index(mode_radii(N), width).ravel()
    if nbins is None:
        nbins = int(lb.max()) + 1
    keep = lb < nbins
    counts = np.bincount(lb[keep], minlength=nbins)[:nbins]
    sums = np.bincount(lb[keep], weights=p[keep], minlength=nbins)[:nbins]
    scale = P.mp ** 2 / (4.0 * a ** (2.0 * P.alpha) * float(N) ** 6)
    rho_l = scale * sums
    omega = np.arange(nbins) * rho_l / rho_tot
    return counts, rho_l, omega, scale * float(np.sum(p))
