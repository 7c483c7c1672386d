"""Pins of the surrogate-jump oracle (oracle/surrogate_jump.py): each piece
against a closed form or an independent computation.  CPU only."""
import math

import numpy as np
import pytest

from oracle import lattice as L
from oracle import surrogate_jump as J


def test_gaussian_averages_match_gaussian_moments():
    """E[dV/df_j] and E[V] over independent Gaussian fluctuations, from the
    moments E[d] = E[d^3] = 0, E[d^2] = s^2, E[d^4] = 3 s^4 written out by hand
    for V = sum(m^2 f^2/2 + lam f^4/4) + g^2 f0^2 f1^2/2 + V0, and against a
    large Monte-Carlo sample."""
    P = L.Params(N=2, dx=1.0, n_fields=2, m2=(0.3, 0.7), lam=(1.2, 0.4), g2=2.5, V0=0.05)
    f = np.array([0.8, -0.35])
    v = np.array([0.04, 0.09])
    F = J.hartree_force(f, v, P)
    m2, lam, g2 = P.m2, P.lam, P.g2
    want0 = m2[0] * f[0] + lam[0] * (f[0] ** 3 + 3 * f[0] * v[0]) + g2 * f[0] * (f[1] ** 2 + v[1])
    want1 = m2[1] * f[1] + lam[1] * (f[1] ** 3 + 3 * f[1] * v[1]) + g2 * f[1] * (f[0] ** 2 + v[0])
    assert abs(F[0] - want0) <= 1e-14 * abs(want0) and abs(F[1] - want1) <= 1e-14 * abs(want1)
    Vw = P.V0
    for j in range(2):
        Vw += 0.5 * m2[j] * (f[j] ** 2 + v[j]) + 0.25 * lam[j] * (f[j] ** 4 + 6 * f[j] ** 2 * v[j] + 3 * v[j] ** 2)
    Vw += 0.5 * g2 * (f[0] ** 2 + v[0]) * (f[1] ** 2 + v[1])
    assert abs(J.hartree_potential(f, v, P) - Vw) <= 1e-14 * Vw
    rng = np.random.default_rng(0)
    n = 2_000_000
    pts = f[:, None] + np.sqrt(v)[:, None] * rng.standard_normal((2, n))
    mc = L.dpotential(pts.reshape(2, n, 1, 1), P).reshape(2, n)
    for j in range(2):
        assert abs(mc[j].mean() - F[j]) < 5 * mc[j].std() / math.sqrt(n)


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_predictor_without_fluctuations_is_the_uniform_lattice(integrator):
    """With zero variances and no radiation the predictor is the lattice
    equations on a uniform lattice: it must follow the lattice oracle run on
    uniform fields (two fields, expanding space) to rounding."""
    P = L.Params(N=2, dx=1.0, n_fields=2, lam=(1.0, 0.0), g2=30.0, m2=(0.1, 0.0))
    f0, p0 = np.array([0.9, 0.05]), np.array([0.02, -0.01])
    E = L.energies(np.broadcast_to(f0[:, None, None, None], (2, 2, 2, 2)).copy(),
                   np.broadcast_to(p0[:, None, None, None], (2, 2, 2, 2)).copy(), 1.0, P)
    b0 = L.hubble_from_rho(1.0, L.rho_pressure(*E)[0], P)
    dt, n = 0.01, 48
    fp, pp, a, b = J.predictor(f0, p0, 1.0, b0, np.zeros(2), 0.0, 1.0, dt, n, integrator, P)
    s = L.State(np.broadcast_to(f0[:, None, None, None], (2, 2, 2, 2)).copy(),
                np.broadcast_to(p0[:, None, None, None], (2, 2, 2, 2)).copy(), 1.0, b0)
    s, _ = L.run(s, dt, n, P, integrator)
    assert np.max(np.abs(fp - s.f[:, 0, 0, 0])) <= 1e-13
    assert np.max(np.abs(pp - s.p[:, 0, 0, 0])) <= 1e-13 * np.max(np.abs(s.p))
    assert abs(a - s.a) <= 1e-14 * s.a and abs(b - s.b) <= 1e-13 * abs(s.b)


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_predictor_radiation_closed_form(integrator):
    """Radiation alone in conformal time (alpha = 1): rho_r ~ a^-4 and
    p_r = rho_r / 3 make (2 alpha - 1) rho - 3 p vanish, so a'' = 0 and
    a = a0 + a'_0 eta exactly; a' stays on the constraint
    a'^2 = a^4 rho_r / 3 (m_p = 1)."""
    P = L.Params(N=2, dx=1.0, n_fields=1, lam=(0.0, 0.0))
    a0, rho_r0 = 1.3, 0.02
    b0 = a0 * math.sqrt(a0 ** 2 * rho_r0 / 3.0)
    dt, n = 0.05, 40
    _, _, a, b = J.predictor(np.zeros(1), np.zeros(1), a0, b0, np.zeros(1), rho_r0, a0, dt, n, integrator, P)
    assert abs(a - (a0 + b0 * dt * n)) <= 1e-14 * a
    assert abs(b - b0) <= 1e-14 * b0
    assert abs(b ** 2 - a ** 4 * rho_r0 * (a0 / a) ** 4 / 3.0) <= 1e-13 * b ** 2


@pytest.mark.parametrize("integrator,order", [("leapfrog", 2), ("vv4", 4)])
def test_predictor_radiation_cosmic_time(integrator, order):
    """Radiation alone in cosmic time (alpha = 0): H^2 = rho_r / 3 with
    rho_r = rho_r0 (a0 / a)^4 gives a = a0 sqrt(1 + 2 H0 t), H0^2 = rho_r0 / 3;
    the predictor converges to it at the scheme's order (a matter-like
    redshift a^-3 would give a ~ t^(2/3) instead)."""
    P = L.Params(N=2, dx=1.0, n_fields=1, lam=(0.0, 0.0), alpha=0.0)
    a0, rho_r0, T = 1.0, 0.3, 4.0
    H0 = math.sqrt(rho_r0 / 3.0)
    errs = []
    for dt in (0.1, 0.05):
        n = int(round(T / dt))
        _, _, a, b = J.predictor(np.zeros(1), np.zeros(1), a0, a0 * H0, np.zeros(1), rho_r0, a0, dt, n,
                                 integrator, P)
        errs.append(abs(a - a0 * math.sqrt(1.0 + 2.0 * H0 * T)))
    assert abs(errs[0] / errs[1] / 2 ** order - 1) < 0.15, errs


@pytest.mark.parametrize("integrator,order", [("leapfrog", 2), ("vv4", 4)])
def test_corrector_closed_forms(integrator, order):
    """Constant sums reduce the corrector to the background equations:
    (i) vacuum energy S = (0, 0, V0): a = 1/(1 - H0 eta), H0^2 = V0/3;
    (ii) kination S = (pbar^2/2, 0, 0) (K = S_K/a^6): a^2 = 1 + 2 H0 eta,
    H0^2 = pbar^2/6; convergence at the scheme's order (m_p = 1)."""
    P = L.Params(N=2, dx=1.0)
    cases = []
    V0 = 0.3
    H0 = math.sqrt(V0 / 3)
    cases.append(((0.0, 0.0, V0), H0, 1.5, lambda e: 1.0 / (1.0 - H0 * e)))
    pbar = 0.7
    Hk = math.sqrt(pbar ** 2 / 6)
    cases.append(((pbar ** 2 / 2, 0.0, 0.0), Hk, 3.0, lambda e: math.sqrt(1.0 + 2.0 * Hk * e)))
    for S, H, T, exact in cases:
        errs = []
        for dt in (0.05, 0.025):
            n = int(round(T / dt))
            a, b = J.corrector(1.0, H, S, S, dt, n, integrator, P)
            errs.append(abs(a - exact(T)))
        assert abs(errs[0] / errs[1] / 2 ** order - 1) < 0.15, errs


def test_corrector_interpolates_from_start_to_end():
    """Sums that change during the jump: the corrector converges at order 4
    (VV4) to an independent fine RK4 solution of a'' = A(a, S(t)) with S
    moving linearly from S0 (start) to S1 (end); the reversed direction is a
    different trajectory."""
    P = L.Params(N=2, dx=1.0)
    S0, S1 = np.array([0.05, 0.02, 0.2]), np.array([0.01, 0.08, 0.35])
    T, a0, b0 = 1.2, 1.0, 0.3

    def A(a, t):
        S = S0 + (t / T) * (S1 - S0)
        K, G, V = S[0] / a ** 6, S[1] / a ** 2, S[2]
        rho, p = K + G + V, K - G / 3 - V
        return a ** 3 * (rho - 3 * p) / 6

    y, t, h = np.array([a0, b0]), 0.0, T / 4000
    for _ in range(4000):
        k1 = np.array([y[1], A(y[0], t)])
        k2 = np.array([y[1] + h / 2 * k1[1], A(y[0] + h / 2 * k1[0], t + h / 2)])
        k3 = np.array([y[1] + h / 2 * k2[1], A(y[0] + h / 2 * k2[0], t + h / 2)])
        k4 = np.array([y[1] + h * k3[1], A(y[0] + h * k3[0], t + h)])
        y, t = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4), t + h
    errs = []
    for n in (12, 24):
        a, b = J.corrector(a0, b0, S0, S1, T / n, n, "vv4", P)
        errs.append(max(abs(a - y[0]), abs(b - y[1])))
    assert abs(errs[0] / errs[1] / 16 - 1) < 0.2, errs
    ar, _ = J.corrector(a0, b0, S1, S0, T / 24, 24, "vv4", P)
    assert abs(ar - y[0]) > 100 * errs[1]


def test_jump_with_zero_increment_moves_only_the_means():
    """A zero network output keeps every fluctuation about the mean and moves
    the means to the predictor's values; with no fluctuations at all the jump
    equals n lattice steps of the uniform state."""
    P = L.Params(N=4, dx=0.5, n_fields=2, lam=(1.0, 0.0), g2=5.0)
    rng = np.random.default_rng(3)
    f = np.stack([1.0 + 1e-3 * rng.standard_normal((4, 4, 4)), 0.1 + 1e-3 * rng.standard_normal((4, 4, 4))])
    p = 1e-3 * rng.standard_normal((2, 4, 4, 4))
    E = L.energies(f, p, 1.0, P)
    s = L.State(f, p, 1.0, L.hubble_from_rho(1.0, L.rho_pressure(*E)[0], P))
    new, r = J.jump(s, np.zeros((4, 4, 4, 4)), np.ones(4), 0.01, 16, "vv4", P)
    for j in range(2):
        assert np.allclose(new.f[j] - new.f[j].mean(), f[j] - f[j].mean(), rtol=0, atol=1e-15)
        assert np.allclose(new.p[j] - new.p[j].mean(), p[j] - p[j].mean(), rtol=0, atol=1e-15)
    assert new.eta == pytest.approx(0.16) and new.a > s.a
    # frozen small fluctuations: the background follows the lattice run closely
    ref, recs = L.run(s, 0.01, 16, P, "vv4")
    assert r < 1e-7 and abs(new.a - ref.a) < 1e-7 * ref.a and abs(new.b - ref.b) < 1e-5 * ref.b
    u = L.State(np.ones_like(f) * np.array([1.0, 0.1])[:, None, None, None], np.zeros_like(p), 1.0, 0.0)
    u.b = L.hubble_from_rho(1.0, L.rho_pressure(*L.energies(u.f, u.p, 1.0, P))[0], P)
    new, _ = J.jump(u, np.zeros((4, 4, 4, 4)), np.ones(4), 0.01, 16, "vv4", P)
    ref, _ = L.run(u, 0.01, 16, P, "vv4")
    assert np.max(np.abs(new.f - ref.f)) <= 1e-13 and abs(new.a - ref.a) <= 1e-13


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_corrector_follows_the_predictor_without_fluctuations(integrator):
    """With no fluctuations the sums are the homogeneous ones at both ends,
    the remainder the corrector interpolates is zero, and it must reproduce
    the predictor's (a, a') to rounding."""
    P = L.Params(N=2, dx=1.0, n_fields=2, lam=(1.0, 0.0), g2=30.0)
    f0, p0 = np.array([0.9, 0.05]), np.array([0.02, -0.01])
    V = J.hartree_potential(f0, np.zeros(2), P)
    b0 = L.hubble_from_rho(1.0, float(np.sum(p0 ** 2)) / 2 + V, P)
    hom = []
    fn, pn, a, b = J.predictor(f0, p0, 1.0, b0, np.zeros(2), 0.0, 1.0, 0.01, 32, integrator, P, record=hom)
    assert len(hom) == 32 * (3 if integrator == "vv4" else 1) * 2
    S0 = np.array([np.sum(p0 ** 2) / 2, 0.0, V])
    S1 = np.array([np.sum(pn ** 2) / 2, 0.0, J.hartree_potential(fn, np.zeros(2), P)])
    ac, bc = J.corrector(1.0, b0, S0, S1, 0.01, 32, integrator, P, hom=hom)
    assert abs(ac - a) <= 1e-15 * a and abs(bc - b) <= 1e-14 * abs(b)
    # linear interpolation of the whole sums is a worse reading here
    al, bl = J.corrector(1.0, b0, S0, S1, 0.01, 32, integrator, P)
    assert abs(bl - b) > 1e3 * abs(bc - b) + 1e-12
