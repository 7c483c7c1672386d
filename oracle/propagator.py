"""Oracle (test infrastructure only): a jump by linear propagation of the
fluctuations, in FP64.

About the homogeneous background, the lattice equations of Sect. 2.1
(Eq. singletEOM in program variables: f' = a^(alpha-3) pi,
pi' = a^(1+alpha) Lap f - a^(3+alpha) dV/df) are linear in the fluctuations
to first order.  The 7-point Laplacian is diagonal in the lattice Fourier
modes, with eigenvalue -kappa^2, kappa^2 = sum_i (2/dx)^2 sin^2(pi n_i / N);
the force's first-order part is the mass matrix d^2V/df_i df_j at the
homogeneous values, taken here Hartree-averaged over Gaussian fluctuations of
the start variances (the background predictor's own average).  A jump:

  1. means, momentum means and variances of the state; the radiation share
     rho_r0 as in the network jump (surrogate_jump.jump);
  2. the background predictor over the n steps (surrogate_jump.predictor),
     which reports every half kick (h/2, a, fbar) and drift (h abar^(alpha-3))
     of its sub-steps;
  3. the fluctuations of every field and momentum go to Fourier space
     (numpy's FFT), every mode takes the same half kicks
     pi -= (h/2) (a^(1+alpha) kappa^2 f + a^(3+alpha) M(fbar) f) and drifts,
     and comes back;
  4. new state = predicted means + propagated fluctuations; (a, a') from the
     corrector (surrogate_jump.corrector) and the Hubble residual, as for the
     network jump.

This is a design of this build, not of the paper; the pins fix it against
the lattice oracle itself: for free fields on a static background the jump
equals the lattice integrator's steps; with interactions, its error against
them is second order in the fluctuation amplitude.
"""
from __future__ import annotations

import numpy as np

from . import lattice as L
from . import surrogate_jump as J


def laplacian_eigenvalues(N: int, dx: float, d: int = 3):
    """kappa^2(n) = sum_i (2/dx)^2 sin^2(pi n_i / N) on the d-dimensional
    grid of mode indices (shape [N] * d)."""
    s2 = (2.0 / dx) ** 2 * np.sin(np.pi * np.arange(N) / N) ** 2
    k2 = np.zeros([N] * d)
    for axis in range(d):
        shape = [1] * d
        shape[axis] = N
        k2 = k2 + s2.reshape(shape)
    return k2


def hartree_mass_matrix(fbar, var, P: L.Params):
    """Mean of d^2V/df_i df_j over independent Gaussian fluctuations of
    variance var_j about fbar ([n_fields, n_fields])."""
    nf = P.n_fields
    M = np.zeros((nf, nf))
    for j in range(nf):
        M[j, j] = P.m2[j] + 3.0 * P.lam[j] * (fbar[j] ** 2 + var[j])
    if nf == 2:
        M[0, 0] += P.g2 * (fbar[1] ** 2 + var[1])
        M[1, 1] += P.g2 * (fbar[0] ** 2 + var[0])
        M[0, 1] = M[1, 0] = 2.0 * P.g2 * fbar[0] * fbar[1]
    return M


def propagate_modes(F, Pm, trace, var, k2, P: L.Params):
    """Step 3 on the Fourier modes F[j], Pm[j] (complex arrays) with the
    predictor's trace."""
    al, nf = P.alpha, P.n_fields
    F, Pm = [x.copy() for x in F], [x.copy() for x in Pm]
    for item in trace:
        if item[0] == "kick":
            _, hh, a, fbar = item
            M = hartree_mass_matrix(fbar, var, P)
            F0 = [x.copy() for x in F]
            for j in range(nf):
                force = a ** (1.0 + al) * k2 * F0[j]
                for l in range(nf):
                    force = force + a ** (3.0 + al) * M[j, l] * F0[l]
                Pm[j] = Pm[j] - hh * force
        else:
            cd = item[1]
            for j in range(nf):
                F[j] = F[j] + cd * Pm[j]
    return F, Pm


def linear_jump(s: L.State, dt, n, integrator, P: L.Params):
    """Steps 1-4 for a lattice state s.  Returns the new state (eta advanced
    by n dt) and its Hubble-constraint residual."""
    nf = P.n_fields
    fbar = np.array([np.mean(s.f[j]) for j in range(nf)])
    pbar = np.array([np.mean(s.p[j]) for j in range(nf)])
    var = np.array([np.mean((s.f[j] - fbar[j]) ** 2) for j in range(nf)])
    E0 = L.energies(s.f, s.p, s.a, P)
    rho_lat = sum(E0[0]) + sum(E0[1]) + E0[2]
    rho_hom_K = float(np.sum(pbar ** 2)) / (2.0 * s.a ** 6)
    rho_r0 = max(0.0, rho_lat - rho_hom_K - J.hartree_potential(fbar, var, P))
    hom, trace = [], []
    fn, pn, a1, b1 = J.predictor(fbar, pbar, s.a, s.b, var, rho_r0, s.a, dt, n, integrator, P, record=hom,
                                 trace=trace)
    k2 = laplacian_eigenvalues(s.f.shape[1], P.dx, s.f.ndim - 1)
    F = [np.fft.fftn(s.f[j] - fbar[j]) for j in range(nf)]
    Pm = [np.fft.fftn(s.p[j] - pbar[j]) for j in range(nf)]
    F, Pm = propagate_modes(F, Pm, trace, var, k2, P)
    f = np.stack([fn[j] + np.fft.ifftn(F[j]).real for j in range(nf)])
    p = np.stack([pn[j] + np.fft.ifftn(Pm[j]).real for j in range(nf)])
    S0 = J.volume_sums(s.f, s.p, P)
    S1 = J.volume_sums(f, p, P)
    a1, b1 = J.corrector(s.a, s.b, S0, S1, dt, n, integrator, P, hom=hom if hom else None)
    new = L.State(f, p, a1, b1, s.eta + n * dt)
    r = L.hubble_residual(a1, b1, L.energies(f, p, a1, P), P)
    return new, r
