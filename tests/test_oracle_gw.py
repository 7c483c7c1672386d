"""Pins of the gravitational-wave oracle (oracle/gw.py) against closed forms
and the defining properties of the transverse-traceless projection.  CPU only."""
import math

import numpy as np
import pytest

from oracle import gw as G
from oracle import lattice as L

from test_oracle_pins import cos_mode, kdk_matrix, lattice_omega2


def test_stress_converges_to_gradient_products():
    """Pi^eff_ij -> d_i f d_j f for a smooth field, at second order in dx
    (a dropped 1/dx^2, a wrong index pairing or a sign would not converge)."""
    errs = []
    for N in (16, 32):
        L_ = 2 * math.pi
        dx = L_ / N
        x = np.arange(N) * dx
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        f = np.sin(X + 0.3) * np.cos(2 * Y) + 0.5 * np.sin(Z - X)
        grad = [np.cos(X + 0.3) * np.cos(2 * Y) - 0.5 * np.cos(Z - X), -2 * np.sin(X + 0.3) * np.sin(2 * Y),
                0.5 * np.cos(Z - X)]
        P = L.Params(N=N, dx=dx, n_fields=1)
        Pi = G.anisotropic_stress(f[None], P)
        e = max(float(np.max(np.abs(Pi[i, j] - grad[i] * grad[j]))) for i in range(3) for j in range(3))
        errs.append(e)
        assert np.array_equal(Pi, np.swapaxes(Pi, 0, 1))
    assert abs(errs[0] / errs[1] / 4 - 1) < 0.1, errs


def test_source_is_traceless_and_sums_fields():
    """S_ij = Pi_ij - delta_ij Pi_kk / 3: the full tensor built with
    v_33 = -v_11 - v_22 equals Pi - delta tr/3 in every entry; two fields add."""
    P1 = L.Params(N=8, dx=0.7, n_fields=1)
    P2 = L.Params(N=8, dx=0.7, n_fields=2)
    rng = np.random.default_rng(1)
    f = rng.standard_normal((2, 8, 8, 8))
    S = G.full_tensor(G.traceless_source(f, P2))
    Pi = G.anisotropic_stress(f[:1], P1) + G.anisotropic_stress(f[1:], P1)
    tr = Pi[0, 0] + Pi[1, 1] + Pi[2, 2]
    want = Pi - np.eye(3)[:, :, None, None, None] * tr / 3.0
    assert np.max(np.abs(S - want)) <= 1e-13 * np.max(np.abs(Pi))


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_free_wave_dispersion(integrator):
    """Homogeneous scalar fields source nothing; a single cos-mode of one
    tensor component is a free wave with the massless lattice dispersion
    w^2 = sum_i (2/dx)^2 sin^2(k_i dx/2): leapfrog gives cos(n theta), VV4 the
    product of kick-drift-kick matrices (static space)."""
    N, dx, nvec = 8, 0.7, (1, 2, 3)
    P = L.Params(N=N, dx=dx, n_fields=2, expansion="static", lam=(1.0, 0.0), g2=2.0)
    g = cos_mode(N, dx, nvec)
    w2 = lattice_omega2(N, dx, nvec, 0.0)
    s = L.State(np.stack([np.full((N, N, N), 0.8), np.zeros((N, N, N))]), np.zeros((2, N, N, N)), 1.0, 0.0)
    v = np.zeros((5, N, N, N))
    v[1] = 1e-3 * g
    u = np.zeros_like(v)
    dt, n = 0.2, 1500
    s, v, u = G.run(s, v, u, dt, n, P, integrator)
    if integrator == "leapfrog":
        M = np.linalg.matrix_power(kdk_matrix(dt, w2), n)
    else:
        M = np.linalg.matrix_power(kdk_matrix(L.W1 * dt, w2) @ kdk_matrix(L.W0 * dt, w2) @ kdk_matrix(L.W1 * dt, w2), n)
    assert np.max(np.abs(v[1] / 1e-3 - M[0, 0] * g)) <= 1e-11
    assert np.max(np.abs(u[1] / 1e-3 - M[1, 0] * g)) <= 1e-11 * math.sqrt(w2)
    assert np.max(np.abs(v[[0, 2, 3, 4]])) == 0.0


def test_projector_closed_form_and_properties():
    """Lambda for k^ = z picks the (x, y) block's traceless part,
    [[(T11 - T22)/2, T12, 0], [T12, (T22 - T11)/2, 0], [0, 0, 0]]; for any k^
    the result is symmetric, traceless, transverse, idempotent, and leaves a
    transverse-traceless polarisation unchanged."""
    rng = np.random.default_rng(4)
    A = rng.standard_normal((3, 3))
    T = (A + A.T)[:, :, None]
    z = np.array([0.0, 0.0, 1.0])[:, None]
    out = G.tt_project(T, z)[:, :, 0]
    t = T[:, :, 0]
    want = np.array([[(t[0, 0] - t[1, 1]) / 2, t[0, 1], 0], [t[0, 1], (t[1, 1] - t[0, 0]) / 2, 0], [0, 0, 0]])
    assert np.max(np.abs(out - want)) <= 1e-15
    k = rng.standard_normal((3, 1))
    k /= np.linalg.norm(k)
    h = G.tt_project(T, k)
    assert np.max(np.abs(h - np.swapaxes(h, 0, 1))) <= 1e-15
    assert abs(np.trace(h[:, :, 0])) <= 1e-15
    assert np.max(np.abs(np.einsum("i...,ij...->j...", k, h))) <= 1e-15
    assert np.max(np.abs(G.tt_project(h, k) - h)) <= 1e-15
    e1 = np.cross(k[:, 0], [1.0, 0.0, 0.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(k[:, 0], e1)
    ep = (np.outer(e1, e1) - np.outer(e2, e2))[:, :, None]
    ex = (np.outer(e1, e2) + np.outer(e2, e1))[:, :, None]
    for e in (ep, ex):
        assert np.max(np.abs(G.tt_project(e, k) - e)) <= 1e-15


@pytest.mark.parametrize("nvec", [(2, 0, 0), (0, 0, 3), (1, 1, 0)])
def test_axis_or_diagonal_scalar_wave_sources_no_waves(nvec):
    """A scalar plane wave along a lattice axis or a face diagonal has a
    stress tensor along k k (plus a multiple of delta): its projection, and
    that of everything it sources, vanishes -- while the unprojected v and u
    do not (expanding two-field lattice, both fields carrying the wave)."""
    N = 8
    P = L.Params(N=N, dx=0.6, n_fields=2, lam=(1.0, 0.0), g2=3.0)
    g = cos_mode(N, 0.6, nvec)
    f = np.stack([1.0 + 0.2 * g, 0.1 + 0.1 * g])
    p = np.stack([0.05 * g, 0.02 * g])
    E = L.energies(f, p, 1.0, P)
    s = L.State(f, p, 1.0, L.hubble_from_rho(1.0, L.rho_pressure(*E)[0], P))
    v = np.zeros((5, N, N, N))
    s, v, u = G.run(s, v, np.zeros_like(v), 0.05, 30, P, "vv4")
    assert np.max(np.abs(v)) > 1e-4
    kh = G.lattice_khat(N)
    for x in (v, u):
        Tk = np.fft.fftn(G.full_tensor(x), axes=(2, 3, 4))
        assert np.max(np.abs(G.tt_project(Tk, kh))) <= 1e-12 * np.max(np.abs(Tk))
    _, rho_l, _, rho = G.gw_spectrum(u, s.a, P, 1.0)
    assert rho <= 1e-24 * np.max(np.abs(u)) ** 2 * 1e6


@pytest.mark.parametrize("nvec,alpha", [((0, 0, 3), 1.0), ((1, 2, 3), 1.0), ((2, 1, 0), 0.0)])
def test_energy_of_a_prescribed_wave(nvec, alpha):
    """u = a^(3-alpha) A cos(k.x) e, with e = e1 e1 - e2 e2 a polarisation
    transverse to the lattice momentum: h' = A cos(k.x) e, so
    <h'_ij h'_ij> = A^2 and rho_GW = m_p^2 A^2 / (4 a^(2 alpha)), all of it in the
    bin of |n|; Omega there is |n| rho_GW / rho_tot (canonical bins)."""
    N, A, a, mp = 8, 0.3, 1.7, 0.8
    P = L.Params(N=N, dx=0.5, n_fields=1, alpha=alpha, mp=mp)
    s = np.sin(np.pi * np.array(nvec) / N)
    k = s / np.linalg.norm(s)
    e1 = np.cross(k, [1.0, 0.0, 0.0] if abs(k[0]) < 0.9 else [0.0, 1.0, 0.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(k, e1)
    e = np.outer(e1, e1) - np.outer(e2, e2)
    g = cos_mode(N, 0.5, nvec)
    u = np.stack([a ** (3 - alpha) * A * e[i, j] * g for i, j in G.COMPONENTS])
    counts, rho_l, omega, rho = G.gw_spectrum(u, a, P, rho_tot=2.0)
    want = mp ** 2 * A ** 2 / (4 * a ** (2 * alpha))
    b = int(math.floor(math.sqrt(sum(c * c for c in nvec)) + 0.5))
    assert abs(rho - want) <= 1e-13 * want
    assert abs(rho_l[b] - want) <= 1e-13 * want and abs(np.sum(rho_l) - want) <= 1e-13 * want
    assert abs(omega[b] - b * want / 2.0) <= 1e-13 * want
    assert counts.sum() == N ** 3


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_time_reversibility_with_waves(integrator):
    """n steps, negate every momentum (fields, a', tensor), n steps: back at
    the start (the tensor sub-steps are kick-drift-kick symmetric too)."""
    N = 8
    P = L.Params(N=N, dx=0.6, n_fields=2, lam=(1.0, 0.0), g2=5.0)
    rng = np.random.default_rng(8)
    f = np.stack([1.0 + 0.05 * rng.standard_normal((N, N, N)), 0.1 + 0.05 * rng.standard_normal((N, N, N))])
    p = 0.02 * rng.standard_normal((2, N, N, N))
    E = L.energies(f, p, 1.0, P)
    s0 = L.State(f, p, 1.0, L.hubble_from_rho(1.0, L.rho_pressure(*E)[0], P))
    v0 = 1e-3 * rng.standard_normal((5, N, N, N))
    u0 = 1e-3 * rng.standard_normal((5, N, N, N))
    s, v, u = G.run(s0.copy(), v0.copy(), u0.copy(), 0.03, 25, P, integrator)
    s = L.State(s.f, -s.p, s.a, -s.b)
    s, v, u = G.run(s, v, -u, 0.03, 25, P, integrator)
    assert np.max(np.abs(v - v0)) <= 1e-12 * np.max(np.abs(v0))
    assert np.max(np.abs(-u - u0)) <= 1e-11 * np.max(np.abs(u0))
    assert np.max(np.abs(s.f - s0.f)) <= 1e-12


def test_stress_stencil_on_a_point_field():
    """A field that is 1 at the origin and 0 elsewhere, evaluated by hand:
    at the origin D+_x f = D+_y f = -1 and D-_x f = D-_y f = 1, so
    Pi_xy = ((-1)(-1) + (1)(1)) / (2 dx^2) = 1/dx^2 and Pi_xx = 1/dx^2 too;
    at n = (1, 0, 0) only D-_x f = -1 is non-zero (Pi_xx = 1/(2 dx^2),
    Pi_xy = 0); at n = (1, -1, 0) nothing is (Pi = 0).  The diagonal entries
    are sums of squares, never negative."""
    N, dx = 6, 0.5
    f = np.zeros((1, N, N, N))
    f[0, 0, 0, 0] = 1.0
    Pi = G.anisotropic_stress(f, L.Params(N=N, dx=dx, n_fields=1))
    assert Pi[0, 1, 0, 0, 0] == 1.0 / dx ** 2 and Pi[0, 0, 0, 0, 0] == 1.0 / dx ** 2
    assert Pi[0, 0, 1, 0, 0] == 0.5 / dx ** 2 and Pi[0, 1, 1, 0, 0] == 0.0
    assert np.all(Pi[:, :, 1, N - 1, 0] == 0.0)
    assert np.all(Pi[[0, 1, 2], [0, 1, 2]] >= 0.0)


@pytest.mark.parametrize("alpha,a0", [(1.0, 1.0), (1.0, 1.6), (0.0, 1.6)])
def test_short_time_response_follows_the_wave_equation(alpha, a0):
    """From v = v' = 0, Eq. EoMGWs for the auxiliary fields gives
    v''(0) = 2 S / (m_p^2 a^(2(1-alpha))): after one step h,
    v(h) / (h^2 / 2) tends to that source term at first order in h (the
    Laplacian and the friction act only through v and v', which start at
    zero).  Pins the factor 2/m_p^2 and the powers of a of the tensor kick."""
    N, mp = 8, 0.7
    P = L.Params(N=N, dx=0.6, n_fields=2, lam=(1.0, 0.0), g2=3.0, alpha=alpha, mp=mp)
    rng = np.random.default_rng(12)
    f = np.stack([1.0 + 0.1 * rng.standard_normal((N, N, N)), 0.1 * rng.standard_normal((N, N, N))])
    p = 0.01 * rng.standard_normal((2, N, N, N))
    E = L.energies(f, p, a0, P)
    s0 = L.State(f, p, a0, L.hubble_from_rho(a0, L.rho_pressure(*E)[0], P))
    want = 2.0 * G.traceless_source(f, P) / (mp ** 2 * a0 ** (2 * (1 - alpha)))
    errs = []
    for h in (1e-3, 5e-4):
        _, v, _ = G.step(s0.copy(), np.zeros((5, N, N, N)), np.zeros((5, N, N, N)), h, P, "leapfrog")
        errs.append(np.max(np.abs(v / (0.5 * h * h) - want)) / np.max(np.abs(want)))
    assert errs[1] < 1e-2 and abs(errs[0] / errs[1] / 2 - 1) < 0.2, errs
