"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against a closed form, an invariant or an
independent solver written here, never against a retyped copy of the
oracle's own formulas.  CPU only.
"""
import math

import numpy as np
import pytest

from oracle import lattice as L
from oracle import seed as S
import workloads as W


def cos_mode(N, dx, nvec, amp=1.0):
    """amp * cos(k.x) on the lattice for integer mode vector nvec."""
    i = np.arange(N)
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    phase = 2 * math.pi * (nvec[0] * X + nvec[1] * Y + nvec[2] * Z) / N
    return amp * np.cos(phase)


def lattice_omega2(N, dx, nvec, m2):
    """Lattice dispersion w^2 = m^2 + sum_i (2/dx)^2 sin^2(k_i dx / 2), k_i = 2 pi n_i / (N dx)."""
    return m2 + sum((2.0 / dx) ** 2 * math.sin(math.pi * n / N) ** 2 for n in nvec)


def kdk_matrix(h, w2):
    """Kick(h/2) Drift(h) Kick(h/2) acting on (f, p) of one harmonic mode."""
    K = np.array([[1.0, 0.0], [-0.5 * h * w2, 1.0]])
    D = np.array([[1.0, h], [0.0, 1.0]])
    return K @ D @ K


# ---------------------------------------------------------------- P7, P9
def test_laplacian_eigenmode():
    """P7: the 7-point Laplacian has eigenvalue -k_lat^2 on every Fourier mode."""
    N, dx = 16, 0.37
    for nvec in [(1, 0, 0), (1, 2, 3), (8, 0, 5), (7, 7, 7)]:
        g = cos_mode(N, dx, nvec)
        lap = L.laplacian(g, dx)
        w2 = lattice_omega2(N, dx, nvec, 0.0)
        assert np.max(np.abs(lap + w2 * g)) <= 1e-12 * w2


def test_laplacian_sums_to_zero_and_mean_momentum_law():
    """P9: sum_n L[f](n) = 0, so the kicks change <p> only through <dV/df>."""
    N = 8
    f, p = W.random_state(N, 1, seed=5, famp=0.3)
    dx = 0.5
    assert abs(np.sum(L.laplacian(f[0], dx))) <= 1e-12 * np.sum(np.abs(L.laplacian(f[0], dx)))
    P = L.Params(N=N, dx=dx, n_fields=1, expansion="static", lam=(1.0, 0.0), m2=(0.3, 0.0))
    s0 = L.State(f, p, 1.0, 0.0)
    h = 0.05
    s1 = L.vv2(s0, h, P)
    # static space: dV/df = m^2 f + lambda f^3, evaluated independently here
    dV0 = 0.3 * s0.f[0] + s0.f[0] ** 3
    dV1 = 0.3 * s1.f[0] + s1.f[0] ** 3
    expect = np.mean(s0.p) - 0.5 * h * (np.mean(dV0) + np.mean(dV1))
    assert abs(np.mean(s1.p) - expect) <= 1e-14


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_single_mode_dispersion(integrator):
    """P1: one Fourier mode of a free massive field in static space follows
    the discrete map of the lattice dispersion w^2 = m^2 + sum_i (2/dx)^2
    sin^2(k_i dx/2): f_n = A cos(n theta), sin(theta/2) = w dt/2 for leapfrog,
    and the product of kick-drift-kick matrices for the 4th-order scheme."""
    N, dx, m2 = 8, 0.7, 0.8
    nvec = (1, 2, 3)
    P = L.Params(N=N, dx=dx, n_fields=1, expansion="static", m2=(m2, 0.0), lam=(0.0, 0.0))
    g = cos_mode(N, dx, nvec)
    w2 = lattice_omega2(N, dx, nvec, m2)
    dt = 0.2
    n = 2000
    s = L.State(g[None].copy(), np.zeros((1, N, N, N)), 1.0, 0.0)
    for _ in range(n):
        s = L.step(s, dt, P, integrator)
    if integrator == "leapfrog":
        theta = 2.0 * math.asin(math.sqrt(w2) * dt / 2.0)
        c = math.cos(n * theta)
        M = np.linalg.matrix_power(kdk_matrix(dt, w2), n)
        assert abs(M[0, 0] - c) < 1e-11  # the closed form and the matrix agree
    else:
        M1 = kdk_matrix(L.W1 * dt, w2)
        M0 = kdk_matrix(L.W0 * dt, w2)
        M = np.linalg.matrix_power(M1 @ M0 @ M1, n)
        c = M[0, 0]
    assert np.max(np.abs(s.f[0] - c * g)) <= 1e-11
    assert np.max(np.abs(s.p[0] - M[1, 0] * g)) <= 1e-11 * math.sqrt(w2)


# ---------------------------------------------------------------- P2
def test_free_lattice_exact_mode_evolution():
    """P2: a whole free massive lattice in static space, evolved mode by mode
    with exact 2x2 transfer matrices in Fourier space, equals the oracle."""
    N, dx, m2, dt, n = 8, 0.6, 1.3, 0.15, 60
    P = L.Params(N=N, dx=dx, n_fields=1, expansion="static", m2=(m2, 0.0), lam=(0.0, 0.0))
    f, p = W.random_state(N, 1, seed=7, fbar=(0.2, 0.0), famp=0.5, pamp=0.5)
    s = L.State(f.copy(), p.copy(), 1.0, 0.0)
    for _ in range(n):
        s = L.step(s, dt, P, "leapfrog")
    Fk = np.fft.fftn(f[0])
    Pk = np.fft.fftn(p[0])
    kk = np.fft.fftfreq(N) * N
    KX, KY, KZ = np.meshgrid(kk, kk, kk, indexing="ij")
    w2 = m2 + (2.0 / dx) ** 2 * (np.sin(math.pi * KX / N) ** 2 + np.sin(math.pi * KY / N) ** 2
                                 + np.sin(math.pi * KZ / N) ** 2)
    Ff = np.empty_like(Fk)
    Pf = np.empty_like(Pk)
    for idx in np.ndindex(N, N, N):
        M = np.linalg.matrix_power(kdk_matrix(dt, w2[idx]), n)
        Ff[idx] = M[0, 0] * Fk[idx] + M[0, 1] * Pk[idx]
        Pf[idx] = M[1, 0] * Fk[idx] + M[1, 1] * Pk[idx]
    fe = np.fft.ifftn(Ff).real
    pe = np.fft.ifftn(Pf).real
    assert np.max(np.abs(s.f[0] - fe)) <= 1e-12 * np.max(np.abs(fe))
    assert np.max(np.abs(s.p[0] - pe)) <= 1e-12 * np.max(np.abs(pe))


# ---------------------------------------------------------------- P3
def rk4_homogeneous(f0, p0, a0, b0, T, h, alpha, mp, lam):
    """Fine RK4 of the homogeneous ODE written from the paper:
    f' = a^(alpha-3) p (momentum definition), p' = -a^(3+alpha) lambda f^3
    (Eq. singletEOM without gradients), a' = b,
    b' = a^(2 alpha+1)[(2 alpha-1) rho - 3 P]/(6 mp^2) (Eq. Friedmann1), with
    rho = K + V, P = K - V, K = f'^2/(2 a^(2 alpha)), V = lambda f^4/4."""
    def rhs(y):
        f, p, a, b = y
        fp = a ** (alpha - 3) * p
        K = fp ** 2 / (2 * a ** (2 * alpha))
        V = lam * f ** 4 / 4
        rho, P = K + V, K - V
        return np.array([fp, -a ** (3 + alpha) * lam * f ** 3, b,
                         a ** (2 * alpha + 1) * ((2 * alpha - 1) * rho - 3 * P) / (6 * mp ** 2)])
    y = np.array([f0, p0, a0, b0], dtype=np.float64)
    n = int(round(T / h))
    for _ in range(n):
        k1 = rhs(y)
        k2 = rhs(y + 0.5 * h * k1)
        k3 = rhs(y + 0.5 * h * k2)
        k4 = rhs(y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


@pytest.mark.parametrize("integrator,order", [("leapfrog", 2), ("vv4", 4), ("rk2", 2), ("rk3", 3), ("rk34", 3), ("rk4", 4),
                                               ("rk4_classic", 4)])
@pytest.mark.parametrize("alpha", [1.0, 0.0])
def test_homogeneous_mode_against_rk4(integrator, order, alpha):
    """P3: a uniform lattice reduces to the ODE of (f, p, a, b); the oracle
    converges to a fine RK4 solution at the scheme's order."""
    N, lam, mp = 4, 1.0, 1.0
    P = L.Params(N=N, dx=1.0, n_fields=1, alpha=alpha, mp=mp, lam=(lam, 0.0))
    f0, p0, a0 = 1.0, 0.0, 1.0
    rho0 = lam * f0 ** 4 / 4
    b0 = a0 * math.sqrt(a0 ** (2 * alpha) * rho0 / (3 * mp ** 2))
    T = 4.0
    ref = rk4_homogeneous(f0, p0, a0, b0, T, 1e-3, alpha, mp, lam)
    errs = []
    # the Runge-Kutta schemes reach their asymptotic rate at smaller steps
    for dt in ((0.1, 0.05) if integrator in ("leapfrog", "vv4") else (0.05, 0.025)):
        s = L.State(np.full((1, N, N, N), f0), np.full((1, N, N, N), p0), a0, b0)
        for _ in range(int(round(T / dt))):
            s = L.step(s, dt, P, integrator)
        got = np.array([s.f[0, 0, 0, 0], s.p[0, 0, 0, 0], s.a, s.b])
        errs.append(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3)))
    ratio = errs[0] / errs[1]
    assert_order(integrator, order, ratio, 0.15, errs)


def assert_order(integrator, order, ratio, tol, info):
    """Error ratio on halving the step equals 2^order.  RK3-4 was chosen to
    minimise its order-4 error terms, so where its order-3 term is small the
    h^4 term still dominates at these steps: for it the pin asks for at least
    order 3 (a wrong coefficient drops the order and fails either way)."""
    if integrator == "rk34":
        assert ratio / 2 ** order > 1 - tol, (info, ratio)
    else:
        assert abs(ratio / 2 ** order - 1) < tol, (info, ratio)


# ---------------------------------------------------------------- P11
@pytest.mark.parametrize("integrator,order", [("leapfrog", 2), ("vv4", 4), ("rk2", 2), ("rk3", 3), ("rk34", 3), ("rk4", 4),
                                               ("rk4_classic", 4)])
def test_closed_form_expansion(integrator, order):
    """P11: (i) vacuum energy V0 with alpha = 1 gives a = 1/(1 - H0 eta),
    H0^2 = V0/(3 mp^2); alpha = 0 gives a = exp(H0 t); (ii) kination
    (V = 0, constant homogeneous momentum) with alpha = 1 gives
    a^2 = 1 + 2 H0 eta with H0^2 = pbar^2/(6 mp^2).  Convergence at the
    scheme's order."""
    N = 2
    cases = []
    V0 = 0.3
    H0 = math.sqrt(V0 / 3)
    cases.append((L.Params(N=N, dx=1.0, alpha=1.0, lam=(0.0, 0.0), V0=V0), 0.0, 1.5,
                  lambda e: 1.0 / (1.0 - H0 * e)))
    cases.append((L.Params(N=N, dx=1.0, alpha=0.0, lam=(0.0, 0.0), V0=V0), 0.0, 3.0,
                  lambda e: math.exp(H0 * e)))
    pbar = 0.7
    Hk = math.sqrt(pbar ** 2 / 6)
    cases.append((L.Params(N=N, dx=1.0, alpha=1.0, lam=(0.0, 0.0)), pbar, 3.0,
                  lambda e: math.sqrt(1.0 + 2.0 * Hk * e)))
    # RK3-4's order-3 error term is small in the first case, whose error
    # changes sign near dt = 0.04: its pairs are taken where h^3 dominates
    steps = (0.00625, 0.003125) if integrator == "rk34" else (0.05, 0.025)
    for P, pb, T, exact in cases:
        errs = []
        for dt in steps:
            f = np.zeros((1, N, N, N))
            p = np.full((1, N, N, N), pb)
            E = L.energies(f, p, 1.0, P)
            b0 = L.hubble_from_rho(1.0, L.rho_pressure(*E)[0], P)
            s = L.State(f, p, 1.0, b0)
            for _ in range(int(round(T / dt))):
                s = L.step(s, dt, P, integrator)
            errs.append(abs(s.a - exact(s.eta)))
        ratio = errs[0] / errs[1]
        assert_order(integrator, order, ratio, 0.15, (P, errs))


# ---------------------------------------------------------------- P4
@pytest.mark.parametrize("integrator,order", [("leapfrog", 2), ("vv4", 4)])
def test_static_energy_bounded(integrator, order):
    """P4: in static space the total energy oscillates at O(dt^order) with no
    secular drift."""
    N = 8
    P = L.Params(N=N, dx=0.8, n_fields=2, expansion="static", lam=(1.0, 0.0), g2=2.0)
    f, p = W.random_state(N, 2, seed=3, fbar=(1.0, 0.1), famp=0.2, pamp=0.2)
    T = 40.0
    amps, slopes = [], []
    for dt in (0.08, 0.04):
        s = L.State(f.copy(), p.copy(), 1.0, 0.0)
        tot = []
        for _ in range(int(round(T / dt))):
            s = L.step(s, dt, P, integrator)
            EK, EG, EV = L.energies(s.f, s.p, 1.0, P)
            tot.append(sum(EK) + sum(EG) + EV)
        E0 = sum(sum(x) if isinstance(x, list) else x for x in L.energies(f, p, 1.0, P))
        dev = np.array(tot) - E0
        amps.append(np.max(np.abs(dev)))
        t = np.arange(len(dev))
        slopes.append(abs(np.polyfit(t / len(t), dev, 1)[0]))
    ratio = amps[0] / amps[1]
    assert ratio > 2 ** order * 0.7, (amps, ratio)
    # no secular drift: the fitted change over the whole run stays within the oscillation band
    assert slopes[1] < amps[1], (slopes, amps)


# ---------------------------------------------------------------- P5
@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_time_reversibility(integrator):
    """P5: n steps forward, negate momenta and a', n steps: back at the start."""
    w = W.C1.with_(N=8, k_ir=2.0)
    P = L.Params(N=8, dx=w.dx, n_fields=2, lam=(1.0, 0.0), g2=100.0)
    s0 = S.seed_state(P, w.k_ir, (1.0, 0.0), (0.0, 0.0), seed=4, amp=50.0)
    s = s0.copy()
    n, dt = 40, 0.02
    for _ in range(n):
        s = L.step(s, dt, P, integrator)
    assert s.a > 1.01 * s0.a
    s = L.State(s.f, -s.p, s.a, -s.b)
    for _ in range(n):
        s = L.step(s, dt, P, integrator)
    assert np.max(np.abs(s.f - s0.f)) <= 1e-12 * np.max(np.abs(s0.f))
    assert np.max(np.abs(-s.p - s0.p)) <= 1e-12 * np.max(np.abs(s0.p))
    assert abs(s.a - s0.a) <= 1e-12 * s0.a
    assert abs(-s.b - s0.b) <= 1e-12 * abs(s0.b)


# ---------------------------------------------------------------- P6
def test_gradient_energy_parseval():
    """P6: E_G from forward differences equals the Fourier-space sum
    (2 a^2 N^6)^-1 sum_n |f(n)|^2 sum_i (2/dx)^2 sin^2(pi n_i / N) (Eq. discretePSaux)."""
    N, dx, a = 12, 0.3, 1.7
    f, p = W.random_state(N, 1, seed=9, famp=1.0)
    P = L.Params(N=N, dx=dx, n_fields=1)
    _, EG, _ = L.energies(f, p, a, P)
    Fk = np.fft.fftn(f[0])
    kk = np.fft.fftfreq(N) * N
    KX, KY, KZ = np.meshgrid(kk, kk, kk, indexing="ij")
    s2 = (2.0 / dx) ** 2 * (np.sin(math.pi * KX / N) ** 2 + np.sin(math.pi * KY / N) ** 2
                            + np.sin(math.pi * KZ / N) ** 2)
    expect = np.sum(np.abs(Fk) ** 2 * s2) / (2 * a ** 2 * N ** 6)
    assert abs(EG[0] - expect) <= 1e-13 * expect


def test_kinetic_energy_definition():
    """E_K = <f'^2>/(2 a^(2 alpha)) with f' = a^(alpha-3) pi (Eq. energy-contrib),
    checked for two values of alpha on a uniform momentum."""
    N = 2
    for alpha in (0.0, 1.0):
        P = L.Params(N=N, dx=1.0, alpha=alpha)
        a, pi = 1.9, 0.4
        EK, _, _ = L.energies(np.zeros((1, N, N, N)), np.full((1, N, N, N), pi), a, P)
        fprime = a ** (alpha - 3) * pi
        assert abs(EK[0] - fprime ** 2 / (2 * a ** (2 * alpha))) <= 1e-15


# ---------------------------------------------------------------- P8
@pytest.mark.parametrize("integrator,order", [("leapfrog", 2), ("vv4", 4)])
def test_hubble_residual_order(integrator, order):
    """P8: r = 0 at the seeded start and O(dt^order) afterwards."""
    w = W.C0.with_(N=8)
    P = L.Params(N=8, dx=w.dx, n_fields=1, lam=(1.0, 0.0))
    s0 = S.seed_state(P, w.k_ir, (1.0,), (0.0,), seed=2)
    E0 = L.energies(s0.f, s0.p, s0.a, P)
    assert L.hubble_residual(s0.a, s0.b, E0, P) <= 1e-14
    T = 2.0
    rs = []
    for dt in (0.1, 0.05):
        s = s0.copy()
        for _ in range(int(round(T / dt))):
            s = L.step(s, dt, P, integrator)
        rs.append(L.observe(s, P)["r"])
    ratio = rs[0] / rs[1]
    assert abs(ratio / 2 ** order - 1) < 0.15, (rs, ratio)


# ---------------------------------------------------------------- RNG and seed (P10)
def test_splitmix64_known_answer():
    """First output of SplitMix64 from state 0 (published reference generator)."""
    want = int(open(__file__.replace("test_oracle_pins.py", "golden/splitmix64.txt")).read().split()[-1], 16)
    assert int(S.splitmix64(0, np.array([1], dtype=np.uint64))[0]) == want


def test_uniform_and_gaussian_statistics():
    k = np.arange(1, 400001, dtype=np.uint64)
    u = S.uniform(12345, k)
    assert u.min() > 0.0 and u.max() <= 1.0
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    expect = len(u) / 20
    chi2 = np.sum((hist - expect) ** 2 / expect)
    assert chi2 < 43.8  # 99.9% quantile, 19 dof
    g = S.gaussian(777, 2 * np.arange(200000, dtype=np.uint64) + 1)
    assert abs(np.mean(g)) < 5 / math.sqrt(len(g))
    assert abs(np.var(g) - 1) < 5 * math.sqrt(2 / len(g))
    assert abs(np.mean(g ** 4) - 3) < 0.06


def test_seed_statistics():
    """P10: the seed is real, zero-mean in its fluctuations, band-limited to
    0 < |n| <= N/4, and its Fourier amplitudes follow Eq. QuantumFlucts with
    the left/right-mover construction: <|df|^2> = S_k,
    <|dp|^2> = a^(2(3-alpha)) (a^(2(alpha-1)) w^2 + H^2) S_k and
    <Re(df* dp)> = -a^(3-alpha) H S_k, with S_k = 1/(2 a^2 w_k dx^3) (amp = 1)."""
    N, k_ir = 24, 0.2
    dx = 2 * math.pi / (k_ir * N)
    lam, phi0 = 1.0, 1.0
    P = L.Params(N=N, dx=dx, n_fields=1, lam=(lam, 0.0))
    s, imag = S.seed_state(P, k_ir, (phi0,), (0.0,), seed=99, return_imag=True)
    assert imag <= 1e-14 * np.max(np.abs(s.f[0] - phi0))
    df = s.f[0] - phi0
    dp = s.p[0]
    assert abs(np.mean(df)) <= 1e-16 * N ** 1.5
    Fk = np.fft.fftn(df)
    Pk = np.fft.fftn(dp)
    kk = np.fft.fftfreq(N) * N
    KX, KY, KZ = np.meshgrid(kk, kk, kk, indexing="ij")
    n2 = KX ** 2 + KY ** 2 + KZ ** 2
    inside = (n2 > 0) & (n2 <= (N / 4) ** 2)
    assert np.max(np.abs(Fk[~inside])) <= 1e-12 * np.max(np.abs(Fk))
    H = math.sqrt(lam * phi0 ** 4 / 4 / 3)
    w = np.sqrt(k_ir ** 2 * n2[inside] + 3 * lam * phi0 ** 2)
    Sk = 1.0 / (2 * w * dx ** 3)
    zf = np.abs(Fk[inside]) ** 2 / Sk
    M = zf.size / 2  # independent pairs
    assert abs(np.mean(zf) - 1) < 5 / math.sqrt(M)
    zp = np.abs(Pk[inside]) ** 2 / ((w ** 2 + H ** 2) * Sk)
    assert abs(np.mean(zp) - 1) < 5 / math.sqrt(M)
    cross = np.real(np.conj(Fk[inside]) * Pk[inside]) / (-H * Sk)
    assert abs(np.mean(cross) - 1) < 8 * math.sqrt((w ** 2).mean()) / H / math.sqrt(M)
    # real-space variance is the mode sum (Parseval, Eq. discretePSaux), within sampling error
    assert abs(np.var(df) / (np.sum(Sk) / N ** 6) - 1) < 5 / math.sqrt(M)


def test_seed_amplitude_config0():
    """The 32^3 single-field workload seeds fluctuations of rms about 2.7e-4."""
    w = W.C0
    P = L.Params(N=w.N, dx=w.dx, n_fields=1, lam=w.lam)
    s = S.seed_state(P, w.k_ir, w.fbar, w.pbar, w.seed)
    assert 2.3e-4 < np.std(s.f[0]) < 3.1e-4
    assert abs(s.b - math.sqrt(0.25 / 3)) < 1e-6


# ---------------------------------------------------------------- targeted pins
def test_inverse_dft_convention():
    """Sect. 4.3: f(n) = N^-3 sum_n' exp(+i 2 pi n'.n / N) f(n').  A single
    Fourier amplitude must come back as that exponential, checked by a
    brute-force sum on a tiny lattice."""
    N = 6
    G = np.zeros((N, N, N), dtype=np.complex128)
    G[1, 4, 2] = 2.0 - 0.5j          # mode (1, -2, 2)
    out = S.inverse_dft(G)
    for x, y, z in [(0, 0, 0), (1, 2, 3), (5, 1, 4)]:
        want = (2.0 - 0.5j) * np.exp(2j * math.pi * (1 * x - 2 * y + 2 * z) / N) / N ** 3
        assert abs(out[x, y, z] - want) <= 1e-15


def test_seed_band_is_exactly_the_cutoff_sphere():
    """Reading of 'modes above N/4 k_IR zeroed': every mode with
    0 < |n| <= N/4 is drawn (including |n| = N/4 exactly) and every other
    mode is zero."""
    N, k_ir = 16, 0.3
    P = L.Params(N=N, dx=2 * math.pi / (k_ir * N), n_fields=1, lam=(1.0, 0.0))
    s = S.seed_state(P, k_ir, (1.0,), (0.0,), seed=5)
    Fk = np.fft.fftn(s.f[0] - 1.0)
    kk = np.fft.fftfreq(N) * N
    KX, KY, KZ = np.meshgrid(kk, kk, kk, indexing="ij")
    n2 = KX ** 2 + KY ** 2 + KZ ** 2
    inside = (n2 > 0) & (n2 <= (N / 4) ** 2)
    scale = np.max(np.abs(Fk))
    assert np.all(np.abs(Fk[inside]) > 1e-9 * scale)
    assert np.all(np.abs(Fk[~inside]) < 1e-12 * scale)
    assert np.any(inside & (n2 == (N / 4) ** 2))


def test_seed_momentum_hubble_term():
    """Eq. fpr_influct2 at a = 1: dp = i w Y - H df with Y independent of df,
    so <Re(df* dp)> = -H <|df|^2>.  A small Planck mass makes H comparable
    to w so that the sign of the Hubble term is resolved."""
    N, k_ir, mp = 32, 0.2, 0.05
    P = L.Params(N=N, dx=2 * math.pi / (k_ir * N), n_fields=1, lam=(1.0, 0.0), mp=mp)
    s = S.seed_state(P, k_ir, (1.0,), (0.0,), seed=8)
    H = math.sqrt(0.25 / (3 * mp ** 2))
    Fk = np.fft.fftn(s.f[0] - 1.0)
    Pk = np.fft.fftn(s.p[0])
    kk = np.fft.fftfreq(N) * N
    KX, KY, KZ = np.meshgrid(kk, kk, kk, indexing="ij")
    n2 = KX ** 2 + KY ** 2 + KZ ** 2
    inside = (n2 > 0) & (n2 <= (N / 4) ** 2) & ((KX > 0) | ((KX == 0) & (KY > 0)) | ((KX == 0) & (KY == 0) & (KZ > 0)))
    c = np.real(np.conj(Fk[inside]) * Pk[inside]) + H * np.abs(Fk[inside]) ** 2
    z = np.mean(c) / (np.std(c) / math.sqrt(c.size))
    assert abs(z) < 5
    # and the Hubble term carries the weight it should
    d = np.real(np.conj(Fk[inside]) * Pk[inside])
    assert np.mean(d) < 0 and abs(np.mean(d) / np.mean(-H * np.abs(Fk[inside]) ** 2) - 1) < 0.2


@pytest.mark.parametrize("integrator,order", [("leapfrog", 2), ("vv4", 4)])
def test_hubble_constraint_converges_with_gradients(integrator, order):
    """P8 on a strongly inhomogeneous two-field lattice: the Hubble constraint
    (Eq. Friedmann2) is preserved up to O(dt^order) only if the gradient,
    potential and kinetic terms of the field equation and of rho, p carry
    the right powers of a."""
    N = 8
    P = L.Params(N=N, dx=0.9, n_fields=2, lam=(1.0, 0.0), g2=3.0, mp=0.5)
    f, p = W.random_state(N, 2, seed=21, fbar=(1.0, 0.2), famp=0.4, pamp=0.2)
    E = L.energies(f, p, 1.0, P)
    b0 = L.hubble_from_rho(1.0, L.rho_pressure(*E)[0], P)
    T = 3.0
    rs = []
    for dt in (0.04, 0.02):
        s = L.State(f.copy(), p.copy(), 1.0, b0)
        for _ in range(int(round(T / dt))):
            s = L.step(s, dt, P, integrator)
        rs.append(L.observe(s, P)["r"])
    assert s.a > 1.5
    ratio = rs[0] / rs[1]
    assert abs(ratio / 2 ** order - 1) < 0.2, (rs, ratio)


# ---------------------------------------------------------------- low-storage Runge-Kutta
def butcher_from_low_storage(A, B):
    """Explicit Butcher tableau (a, b, c) equivalent to the 2N recurrence
    d_i = A_i d_(i-1) + h k_i, y_i = y_(i-1) + B_i d_i, k_i = F(y_(i-1)):
    track y_i and d_i as combinations of h k_1 .. h k_s."""
    s = len(A)
    D = np.zeros((s, s))
    Y = np.zeros((s + 1, s))
    for i in range(s):
        if i:
            D[i] = A[i] * D[i - 1]
        D[i, i] += 1.0
        Y[i + 1] = Y[i] + B[i] * D[i]
    a = Y[:s]
    b = Y[s]
    return a, b, a.sum(axis=1)


@pytest.mark.parametrize("scheme,order", [("rk2", 2), ("rk3", 3), ("rk34", 3), ("rk4", 4)])
def test_low_storage_order_conditions(scheme, order):
    """The published low-storage coefficients satisfy the Runge-Kutta order
    conditions of their order (Butcher's rooted-tree conditions up to order
    4), so a wrong digit in any of them fails here."""
    A, B = L.RK_SCHEMES[scheme]
    assert A[0] == 0.0
    a, b, c = butcher_from_low_storage(A, B)
    assert np.allclose(np.tril(a, -1), a)  # explicit
    conds = [b.sum() - 1.0, b @ c - 0.5]
    if order >= 3:
        conds += [b @ c ** 2 - 1.0 / 3.0, b @ (a @ c) - 1.0 / 6.0]
    if order >= 4:
        conds += [b @ c ** 3 - 0.25, (b * c) @ (a @ c) - 0.125, b @ (a @ c ** 2) - 1.0 / 12.0,
                  b @ (a @ (a @ c)) - 1.0 / 24.0]
    assert np.max(np.abs(conds)) < 1e-13, conds


def test_rk2_is_the_explicit_midpoint_rule():
    """The two-stage low-storage scheme is exactly the explicit midpoint rule
    y1 = y0 + h F(y0 + h/2 F(y0)), written out here for the (f, pi, a, a')
    system of a two-field lattice in expanding space."""
    w = W.C1.with_(N=8, k_ir=2.0)
    P = L.Params(N=w.N, dx=w.dx, n_fields=2, m2=w.m2, lam=w.lam, g2=w.g2)
    f, p = W.random_state(w.N, 2, seed=5, fbar=(1.0, 0.05), famp=0.05, pamp=0.05)
    a, b, h = 1.3, 0.4, 0.02

    def F(f, p, a, b):
        E = L.energies(f, p, a, P)
        return (a ** (P.alpha - 3.0) * p, L.force(f, a, P), b, L.accel(a, E, P))

    k1 = F(f, p, a, b)
    mid = (f + 0.5 * h * k1[0], p + 0.5 * h * k1[1], a + 0.5 * h * k1[2], b + 0.5 * h * k1[3])
    k2 = F(*mid)
    s = L.rk_step(L.State(f.copy(), p.copy(), a, b), h, P, "rk2")
    assert np.max(np.abs(s.f - (f + h * k2[0]))) <= 1e-14 * np.max(np.abs(f))
    assert np.max(np.abs(s.p - (p + h * k2[1]))) <= 1e-13 * np.max(np.abs(p + h * k2[1]))
    assert abs(s.a - (a + h * k2[2])) <= 1e-15 * a
    assert abs(s.b - (b + h * k2[3])) <= 1e-14 * abs(b)


# ---------------------------------------------------------------- two-field coupling, seed masses, moments
@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
@pytest.mark.parametrize("moving", [0, 1])
def test_coupled_field_dispersion(integrator, moving):
    """P1 for the phi^2 chi^2 coupling (Sect. 5.1, lphi4 shape; Eq. singletEOM
    with V = g^2 f_0^2 f_1^2 / 2): in static space with no self couplings and
    no bare masses, one field held at the homogeneous value 1 gives the other
    an effective mass g^2, so a single tiny cos-mode of the other field obeys
    the lattice dispersion w^2 = g^2 + sum_i (2/dx)^2 sin^2(k_i dx/2).  Both
    directions are checked (moving = 0: phi oscillates in a chi background;
    moving = 1: chi in a phi background), so the coupling term of each
    component of dV/df is pinned, and with the static energy pin (P4) the
    factor 1/2 of the potential term as well.  The amplitude is small enough
    that the quadratic back-reaction on the background (of order g^2 A^2 t^2)
    stays below round-off."""
    N, dx, g2, A = 8, 0.7, 2.5, 1e-10
    nvec = (1, 2, 3)
    P = L.Params(N=N, dx=dx, n_fields=2, expansion="static", m2=(0.0, 0.0), lam=(0.0, 0.0), g2=g2)
    g = cos_mode(N, dx, nvec)
    w2 = lattice_omega2(N, dx, nvec, g2)
    dt, n = 0.2, 2000
    f = np.zeros((2, N, N, N))
    f[moving] = A * g
    f[1 - moving] = 1.0
    s = L.State(f, np.zeros((2, N, N, N)), 1.0, 0.0)
    for _ in range(n):
        s = L.step(s, dt, P, integrator)
    if integrator == "leapfrog":
        M = np.linalg.matrix_power(kdk_matrix(dt, w2), n)
        theta = 2.0 * math.asin(math.sqrt(w2) * dt / 2.0)
        assert abs(M[0, 0] - math.cos(n * theta)) < 1e-11
    else:
        M1 = kdk_matrix(L.W1 * dt, w2)
        M0 = kdk_matrix(L.W0 * dt, w2)
        M = np.linalg.matrix_power(M1 @ M0 @ M1, n)
    assert np.max(np.abs(s.f[moving] / A - M[0, 0] * g)) <= 1e-11
    assert np.max(np.abs(s.p[moving] / A - M[1, 0] * g)) <= 1e-11 * math.sqrt(w2)
    assert np.max(np.abs(s.f[1 - moving] - 1.0)) <= 1e-14


def _seed_mode_statistics(s, j, fbar_j, m2_j, k_ir, dx, H, N):
    """Normalised Fourier statistics of field j of a seeded state against the
    vacuum spectrum of Eq. QuantumFlucts with mass m2_j (a = 1, alpha = 1):
    returns (mean |df|^2 / S_k, mean |dp|^2 / ((w^2 + H^2) S_k),
    mean Re(df* dp) / (-H S_k), independent pairs)."""
    Fk = np.fft.fftn(s.f[j] - fbar_j)
    Pk = np.fft.fftn(s.p[j] - np.mean(s.p[j]))
    kk = np.fft.fftfreq(N) * N
    KX, KY, KZ = np.meshgrid(kk, kk, kk, indexing="ij")
    n2 = KX ** 2 + KY ** 2 + KZ ** 2
    inside = (n2 > 0) & (n2 <= (N / 4) ** 2)
    assert np.max(np.abs(Fk[~inside])) <= 1e-12 * np.max(np.abs(Fk))
    w = np.sqrt(k_ir ** 2 * n2[inside] + m2_j)
    Sk = 1.0 / (2 * w * dx ** 3)
    zf = np.mean(np.abs(Fk[inside]) ** 2 / Sk)
    zp = np.mean(np.abs(Pk[inside]) ** 2 / ((w ** 2 + H ** 2) * Sk))
    cross = np.mean(np.real(np.conj(Fk[inside]) * Pk[inside]) / (-H * Sk))
    return zf, zp, cross, inside.sum() / 2


def test_two_field_seed_statistics():
    """P10 for both fields of the two-field potential
    V = lambda phi^4/4 + g^2 phi^2 chi^2/2: each field's fluctuations follow
    Eq. QuantumFlucts with its own effective mass d^2V/df_j^2 at the
    homogeneous values (Eq. QuantumFlucts, m^2 = V''), i.e.
    m_phi^2 = 3 lambda phi0^2 + g^2 chi0^2 and m_chi^2 = g^2 phi0^2; the
    homogeneous Hubble rate of the -H df term comes from
    rho = lambda phi0^4/4 + g^2 phi0^2 chi0^2/2.  A non-zero chi0 makes both
    coupling terms of the masses visible; a factor 2 in either changes
    S_k by far more than the sampling error."""
    N, k_ir, lam, g2 = 48, 0.2, 1.0, 100.0
    dx = 2 * math.pi / (k_ir * N)
    phi0, chi0 = 1.0, 0.3
    P = L.Params(N=N, dx=dx, n_fields=2, lam=(lam, 0.0), g2=g2)
    s, imag = S.seed_state(P, k_ir, (phi0, chi0), (0.0, 0.0), seed=123, return_imag=True)
    assert imag <= 1e-14 * max(np.max(np.abs(s.f[0] - phi0)), np.max(np.abs(s.f[1] - chi0)))
    rho = lam * phi0 ** 4 / 4 + g2 * phi0 ** 2 * chi0 ** 2 / 2
    H = math.sqrt(rho / 3)
    masses = (3 * lam * phi0 ** 2 + g2 * chi0 ** 2, g2 * phi0 ** 2)
    for j, (fb, m2) in enumerate(zip((phi0, chi0), masses)):
        zf, zp, cross, M = _seed_mode_statistics(s, j, fb, m2, k_ir, dx, H, N)
        tol = 5 / math.sqrt(M)
        assert abs(zf - 1) < tol, (j, zf, tol)
        assert abs(zp - 1) < tol, (j, zp, tol)
        # the cross term has a large variance relative to its mean (w >> H)
        assert abs(cross - 1) < 8 * math.sqrt(m2 + (k_ir * N / 4) ** 2) / H / math.sqrt(M), (j, cross)
        # a mass off by the coupling factor 2 would be rejected at this size
        w_lo = np.sqrt(m2)
        w_hi = np.sqrt(m2 + (g2 * (chi0 ** 2 if j == 0 else phi0 ** 2)))
        assert w_hi / w_lo - 1 > 3 * tol


def test_two_field_seed_independent_streams():
    """The two fields draw from independent random streams (the field index
    is part of the counter): their Fourier amplitudes are uncorrelated."""
    N, k_ir = 16, 0.3
    P = L.Params(N=N, dx=2 * math.pi / (k_ir * N), n_fields=2, lam=(1.0, 0.0), g2=1.0)
    s = S.seed_state(P, k_ir, (1.0, 0.0), (0.0, 0.0), seed=77)
    a = np.fft.fftn(s.f[0] - 1.0).ravel()
    b = np.fft.fftn(s.f[1]).ravel()
    keep = np.abs(a) > 0
    c = np.abs(np.vdot(a[keep], b[keep])) / (np.linalg.norm(a[keep]) * np.linalg.norm(b[keep]))
    assert c < 5 / math.sqrt(keep.sum() / 2)


@pytest.mark.parametrize("nvec,half", [((1, 0, 0), True), ((2, 3, 5), True), ((8, 0, 0), False),
                                       ((8, 8, 8), False), ((3, 8, 0), True)])
def test_moments_plane_wave(nvec, half):
    """Volume mean and variance (Sect. 4.3 volume averages,
    <(f - <f>)^2>_V) of m + A cos(k.x): mean m, variance A^2/2 for a mode
    with a component off {0, N/2}, and A^2 for a mode made only of 0 and
    N/2 components (cos = +-1 on every site).  A large offset m makes a
    variance taken about zero, or divided by N^3 - 1, fail."""
    N = 16
    g = cos_mode(N, 1.0, nvec)
    for m, A in ((3.0, 0.25), (-1.5, 2.0)):
        f = np.stack([m + A * g, -m + 0.5 * A * g])
        P = L.Params(N=N, dx=1.0, n_fields=2)
        means, vars_ = L.moments(f, P)
        v = A ** 2 / 2 if half else A ** 2
        assert abs(means[0] - m) <= 1e-14 * abs(m)
        assert abs(means[1] + m) <= 1e-14 * abs(m)
        assert abs(vars_[0] - v) <= 1e-13 * v
        assert abs(vars_[1] - v / 4) <= 1e-13 * v
