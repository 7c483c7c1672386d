"""Pins of the linear-propagation jump oracle (oracle/propagator.py) against
the lattice oracle itself and closed forms.  CPU only."""
import numpy as np
import pytest

from oracle import lattice as L
from oracle import propagator as PR


def _state(N, P, amp, seed, fbar=(0.9, 0.05), pbar=(0.02, -0.01)):
    rng = np.random.default_rng(seed)
    nf = P.n_fields
    f = np.stack([fbar[j] + amp * rng.standard_normal((N, N, N)) for j in range(nf)])
    p = np.stack([pbar[j] + amp * rng.standard_normal((N, N, N)) for j in range(nf)])
    if P.expansion == "static":
        return L.State(f, p, 1.0, 0.0)
    E = L.energies(f, p, 1.0, P)
    return L.State(f, p, 1.0, L.hubble_from_rho(1.0, L.rho_pressure(*E)[0], P))


def test_laplacian_eigenvalues_are_those_of_the_lattice_operator():
    """L.laplacian applied to a plane wave exp(2 pi i n.x / N) returns
    -kappa^2(n) times it, for every n of a 6^3 lattice (brute force)."""
    N, dx = 6, 0.7
    k2 = PR.laplacian_eigenvalues(N, dx)
    x = np.indices((N, N, N))
    for n in np.ndindex(N, N, N):
        ph = 2 * np.pi * sum(n[i] * x[i] for i in range(3)) / N
        lap = L.laplacian(np.cos(ph), dx) + 1j * L.laplacian(np.sin(ph), dx)
        assert np.allclose(lap, -k2[n] * np.exp(1j * ph), atol=1e-12)


def test_hartree_mass_matrix_is_the_gaussian_mean_of_the_hessian():
    """M against the Gaussian mean of the Hessian written out by hand and a
    finite-difference Hessian of the Gaussian-averaged force."""
    from oracle import surrogate_jump as J
    P = L.Params(N=2, dx=1.0, n_fields=2, m2=(0.3, 0.7), lam=(1.2, 0.4), g2=2.5)
    f, v = np.array([0.8, -0.35]), np.array([0.04, 0.09])
    M = PR.hartree_mass_matrix(f, v, P)
    want = np.array([[0.3 + 3 * 1.2 * (0.64 + 0.04) + 2.5 * (0.1225 + 0.09), 2 * 2.5 * 0.8 * -0.35],
                     [2 * 2.5 * 0.8 * -0.35, 0.7 + 3 * 0.4 * (0.1225 + 0.09) + 2.5 * (0.64 + 0.04)]])
    assert np.allclose(M, want, rtol=1e-14)
    # d/df_l of the Gaussian-averaged force: equal to the averaged Hessian (the
    # average commutes with the derivative for fixed variances)
    h = 1e-6
    for l in range(2):
        e = np.zeros(2)
        e[l] = h
        col = (J.hartree_force(f + e, v, P) - J.hartree_force(f - e, v, P)) / (2 * h)
        assert np.allclose(col, M[:, l], rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_free_fields_on_a_static_background_equal_the_lattice_integrator(integrator):
    """lambda = g = 0: the lattice equations are linear, so the jump's modes
    must reproduce n lattice-oracle steps of the same integrator (two fields
    of different masses, 12^3) to rounding -- every coefficient, the kick and
    drift order and the Laplacian's eigenvalues enter."""
    P = L.Params(N=12, dx=0.4, n_fields=2, expansion="static", m2=(0.6, 2.3), lam=(0.0, 0.0), g2=0.0)
    s = _state(12, P, 0.3, seed=3)
    dt, n = 0.05, 16
    ref, _ = L.run(s.copy(), dt, n, P, integrator)
    new, r = PR.linear_jump(s, dt, n, integrator, P)
    assert np.max(np.abs(new.f - ref.f)) <= 1e-12 * np.max(np.abs(ref.f))
    assert np.max(np.abs(new.p - ref.p)) <= 1e-12 * np.max(np.abs(ref.p))
    assert new.eta == pytest.approx(s.eta + n * dt)


def test_interacting_error_is_second_order_in_the_amplitude():
    """lambphi^4 + g^2 phi^2 chi^2 on a static background, two fields: the
    jump's deviation from the lattice integrator, relative to the change of
    the fluctuations over the jump, halves when the amplitude halves (the
    neglected terms are quadratic in the fluctuations); a wrong mass matrix
    or eigenvalue would leave a relative error that does not shrink."""
    P = L.Params(N=10, dx=0.5, n_fields=2, expansion="static", m2=(0.2, 0.0), lam=(1.0, 0.0), g2=3.0)
    dt, n = 0.04, 16
    rel = []
    for amp in (2e-3, 1e-3, 5e-4):
        s = _state(10, P, amp, seed=5)
        ref, _ = L.run(s.copy(), dt, n, P, "vv4")
        new, _ = PR.linear_jump(s, dt, n, "vv4", P)
        fb0 = s.f.mean(axis=(1, 2, 3), keepdims=True)
        fb1 = ref.f.mean(axis=(1, 2, 3), keepdims=True)
        change = np.max(np.abs((ref.f - fb1) - (s.f - fb0)))
        err = np.max(np.abs((new.f - new.f.mean(axis=(1, 2, 3), keepdims=True)) - (ref.f - fb1)))
        rel.append(err / change)
    assert rel[0] < 0.05
    for k in range(2):
        assert 1.6 < rel[k] / rel[k + 1] < 2.4, rel


def test_expanding_free_fields_follow_the_lattice_closely():
    """Free fields in a self-consistently expanding space (alpha = 1): the
    background here is the predictor's, not the lattice's own sums, so the
    jump is not exact; the fields must still follow the lattice oracle to the
    predictor's background error (small fluctuations)."""
    P = L.Params(N=8, dx=0.5, n_fields=2, m2=(0.6, 2.3), lam=(0.0, 0.0), g2=0.0, mp=1.0)
    s = _state(8, P, 1e-3, seed=7, fbar=(0.9, 0.05))
    dt, n = 0.02, 16
    ref, _ = L.run(s.copy(), dt, n, P, "vv4")
    new, r = PR.linear_jump(s, dt, n, "vv4", P)
    assert abs(new.a - ref.a) <= 1e-8 * ref.a
    dev = np.max(np.abs(new.f - ref.f))
    assert dev <= 1e-7 * np.max(np.abs(ref.f))
    assert r < 1e-6
