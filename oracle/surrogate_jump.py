"""Oracle (test infrastructure only): one jump of the learned surrogate in FP64.

The paper has no learned component.  What a jump computes is a design of
this build, taken here from its written reading and restated plainly, so
that the library's jump can be checked step by step:

  1. The network's output y (per site and field channel, normalised) is an
     increment of the fluctuations about the volume means.
  2. Predictor: the homogeneous modes (the field means f_j and momentum
     means p_j) and the background (a, a') advance over the jump's n steps
     with the integrator's sub-step pattern, as the uniform-lattice equations
     of Sect. 2.1 (Eq. singletEOM without gradients, Eq. Friedmann1), where
     the force and the potential are averaged over Gaussian fluctuations of
     the start variances (the Hartree average), and the energy of the
     fluctuations beyond that potential average rides along as radiation:
     rho_r = rho_r0 (a_ref / a)^4, p_r = rho_r / 3.
  3. The new state: f = f_new_mean + (f - f_old_mean) + out_scale * y per
     field and momentum channel.
  4. Corrector: (a, a') are re-integrated from their start values with the
     same sub-step pattern, with rho and p from the a-independent volume
     sums S = (<pi^2>/2, <(grad f)^2>/2, <V>) at each kick (K = S_K / a^6,
     G = S_G / a^2, Eq. rhoLocal).  S is split into the homogeneous part
     (sum_j pbar_j^2 / 2, 0, Hartree average of V) taken along the
     predictor's trajectory at that kick, and the rest -- the fluctuations'
     share -- which moves linearly in time from its value at the start to
     that of the new state.
  5. The Hubble-constraint residual (Eq. Friedmann2) of the new state gates
     the jump.

Parity unpinned against the paper (none of this is in it); the pins fix
the pieces: the Gaussian averages against the Gaussian moments, the
predictor against the lattice oracle on a uniform lattice and against the
radiation closed form a = a0 + a'_0 eta, the corrector against the de Sitter
and kination closed forms.
"""
from __future__ import annotations

import math

import numpy as np

from . import lattice as L


def gaussian_average(fn, fbar, var, P: L.Params, order: int = 5):
    """E[fn(fbar + delta)] over independent Gaussian delta_j of variance
    var_j (one per field), by a tensor-product Gauss-Hermite rule of `order`
    points per field (exact for the polynomial potential of degree 4)."""
    x, w = np.polynomial.hermite_e.hermegauss(order)
    w = w / w.sum()
    nf = P.n_fields
    grids = np.meshgrid(*([x] * nf), indexing="ij")
    wts = np.ones_like(grids[0])
    for j in range(nf):
        wts = wts * w.reshape([-1 if k == j else 1 for k in range(nf)])
    pts = np.stack([fbar[j] + math.sqrt(max(var[j], 0.0)) * grids[j] for j in range(nf)])
    vals = fn(pts)
    return np.tensordot(vals, wts, axes=(list(range(vals.ndim - nf, vals.ndim)), list(range(nf))))


def hartree_force(fbar, var, P):
    """Mean of dV/df_j over the Gaussian fluctuations (shape [n_fields])."""
    return gaussian_average(lambda f: L.dpotential(f, P), fbar, var, P)


def hartree_potential(fbar, var, P):
    """Mean of V over the Gaussian fluctuations."""
    return float(gaussian_average(lambda f: L.potential(f, P), fbar, var, P))


def predictor(fbar, pbar, a, b, var, rho_r0, a_ref, dt, n, integrator, P: L.Params, record=None, trace=None):
    """Step 2: (fbar, pbar, a, b) after n steps of dt (leapfrog = VV2(dt),
    vv4 = VV2(w1 dt) VV2(w0 dt) VV2(w1 dt)), each VV2 sub-step in the order
    of the lattice step: half kick of p and b (b's from the energies before
    the kick, at the synchronised momenta), drift of a and f with the
    midpoint a, half kick of p and b (b's from the energies after it).
    If `record` is a list, the homogeneous sums (sum_j p_j^2 / 2, Hartree
    average of V) at every evaluation of b's kick are appended to it.  If
    `trace` is a list, every field half kick appends ("kick", h/2, a, f) and
    every drift ("drift", h abar^(alpha-3)), in order."""
    f = np.array(fbar, dtype=np.float64)
    p = np.array(pbar, dtype=np.float64)
    al, nf = P.alpha, P.n_fields
    expand = P.expansion != "static"

    def accel(aa):
        if not expand:
            return 0.0
        K = float(np.sum(p ** 2)) / (2.0 * aa ** 6)
        V = hartree_potential(f, var, P)
        if record is not None:
            record.append((float(np.sum(p ** 2)) / 2.0, V))
        rr = rho_r0 * (a_ref / aa) ** 4
        rho, pr = K + V + rr, K - V + rr / 3.0
        return aa ** (2.0 * al + 1.0) * ((2.0 * al - 1.0) * rho - 3.0 * pr) / (6.0 * P.mp ** 2)

    def vv2(h):
        nonlocal f, p, a, b
        A0 = accel(a)  # energies at the synchronised momenta, as the lattice step takes them
        if trace is not None:
            trace.append(("kick", 0.5 * h, a, f.copy()))
        p = p - 0.5 * h * a ** (3.0 + al) * hartree_force(f, var, P)
        b = b + 0.5 * h * A0
        a_new = a + h * b if expand else a
        if trace is not None:
            trace.append(("drift", h * (0.5 * (a + a_new)) ** (al - 3.0)))
        f = f + h * (0.5 * (a + a_new)) ** (al - 3.0) * p
        a = a_new
        if trace is not None:
            trace.append(("kick", 0.5 * h, a, f.copy()))
        p = p - 0.5 * h * a ** (3.0 + al) * hartree_force(f, var, P)
        b = b + 0.5 * h * accel(a)

    subs = [L.W1, L.W0, L.W1] if integrator == "vv4" else [1.0]
    for _ in range(n):
        for c in subs:
            vv2(c * dt)
    return f[:nf], p[:nf], a, b


def volume_sums(f, p, P: L.Params):
    """a-independent sums (<pi^2>/2, <(grad f)^2>/(2 dx^2), <V>) of a state,
    so that K = S_K / a^6 and G = S_G / a^2 (Eq. energy-contrib)."""
    EK, EG, EV = L.energies(f, p, 1.0, P)
    return np.array([sum(EK), sum(EG), EV])


def corrector(a, b, S0, S1, dt, n, integrator, P: L.Params, hom=None):
    """Step 4: (a, b) after n steps of dt.  Without `hom` the sums move
    linearly in time from S0 to S1; with `hom` (the predictor's record, one
    (S_K, S_V) pair per kick of b, in order) the homogeneous part follows it
    and only the remainder S - hom moves linearly between its start and end
    values."""
    if P.expansion == "static":
        return a, b
    al, T = P.alpha, dt * n
    tau = 0.0
    S0, S1 = np.asarray(S0, dtype=np.float64), np.asarray(S1, dtype=np.float64)
    if hom is not None:
        H = [np.array([k, 0.0, v]) for k, v in hom]
        R0, R1 = S0 - H[0], S1 - H[-1]
    calls = iter(range(10 ** 9))

    def accel(aa, t):
        w = t / T if T > 0 else 0.0
        if hom is None:
            S = (1.0 - w) * S0 + w * S1
        else:
            S = H[next(calls)] + (1.0 - w) * R0 + w * R1
        K, G, V = S[0] / aa ** 6, S[1] / aa ** 2, S[2]
        rho, pr = K + G + V, K - G / 3.0 - V
        return aa ** (2.0 * al + 1.0) * ((2.0 * al - 1.0) * rho - 3.0 * pr) / (6.0 * P.mp ** 2)

    subs = [L.W1, L.W0, L.W1] if integrator == "vv4" else [1.0]
    for _ in range(n):
        for c in subs:
            h = c * dt
            b = b + 0.5 * h * accel(a, tau)
            a = a + h * b
            tau = tau + h
            b = b + 0.5 * h * accel(a, tau)
    return a, b


def jump(s: L.State, y, out_scale, dt, n, integrator, P: L.Params):
    """Steps 2-5 for a lattice state s and a network output y[channel]
    (channels f_0 .. f_{nf-1}, pi_0 .. pi_{nf-1}, normalised).  Returns the
    new state (eta advanced by n dt) and its Hubble-constraint residual."""
    nf = P.n_fields
    fbar = np.array([np.mean(s.f[j]) for j in range(nf)])
    pbar = np.array([np.mean(s.p[j]) for j in range(nf)])
    var = np.array([np.mean((s.f[j] - fbar[j]) ** 2) for j in range(nf)])
    E0 = L.energies(s.f, s.p, s.a, P)
    rho_lat = sum(E0[0]) + sum(E0[1]) + E0[2]
    rho_hom_K = float(np.sum(pbar ** 2)) / (2.0 * s.a ** 6)
    rho_r0 = max(0.0, rho_lat - rho_hom_K - hartree_potential(fbar, var, P))
    hom = []
    fn, pn, a1, b1 = predictor(fbar, pbar, s.a, s.b, var, rho_r0, s.a, dt, n, integrator, P, record=hom)
    f = np.empty_like(s.f)
    p = np.empty_like(s.p)
    for j in range(nf):
        f[j] = fn[j] + (s.f[j] - fbar[j]) + out_scale[j] * y[j]
        p[j] = pn[j] + (s.p[j] - pbar[j]) + out_scale[nf + j] * y[nf + j]
    S0 = volume_sums(s.f, s.p, P)
    S1 = volume_sums(f, p, P)
    a1, b1 = corrector(s.a, s.b, S0, S1, dt, n, integrator, P, hom=hom if hom else None)
    new = L.State(f, p, a1, b1, s.eta + n * dt)
    r = L.hubble_residual(a1, b1, L.energies(f, p, a1, P), P)
    return new, r
