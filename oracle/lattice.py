"""Oracle (test infrastructure only): real scalar fields on a periodic N^3
lattice in a self-consistently expanding FLRW background, in FP64.

Every function follows a passage of the paper (CosmoLattice 2.0); the
discrete-time readings the paper leaves to its companion review are stated
in the docstrings.  Arrays are indexed [x, y, z] with z fastest; a state of
n fields is an array of shape [n, N, N, N].
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Yoshida triple-jump weights for the 4th-order composition of velocity
# Verlet (Sect. 4.1 names Yoshida methods for orders 4 and above):
# w1 = 1 / (2 - 2^(1/3)), w0 = 1 - 2 w1.
W1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
W0 = 1.0 - 2.0 * W1


@dataclass
class Params:
    """Lattice, background and potential parameters (Sect. 2, Eq. FLRWmetric,
    Eq. FieldSpaceTimeNaturalVariables).  expansion is "self" (Friedmann
    equations) or "static" (a == 1, b == 0).  dim: spatial dimension of the
    lattice (Sect. 3, scalar dynamics in 1+1 and 2+1 dimensions: the same
    equations with the Laplacian and the gradient energy summed over dim
    directions and volume averages over N^dim sites); fields then have shape
    [n_fields] + [N] * dim."""
    N: int
    dx: float
    n_fields: int = 1
    alpha: float = 1.0
    mp: float = 1.0
    expansion: str = "self"
    m2: tuple = (0.0, 0.0)
    lam: tuple = (1.0, 0.0)
    g2: float = 0.0
    V0: float = 0.0
    dim: int = 3


@dataclass
class State:
    f: np.ndarray   # [n, N, N, N] fields
    p: np.ndarray   # [n, N, N, N] conjugate momenta pi = a^(3-alpha) f'
    a: float        # scale factor
    b: float        # pi_a = a' (Eq. SchemeContVirgin1)
    eta: float = 0.0

    def copy(self) -> "State":
        return State(self.f.copy(), self.p.copy(), self.a, self.b, self.eta)


# ---------------------------------------------------------------- potential
def potential(f, P: Params):
    """V = sum_j (m_j^2 f_j^2 / 2 + lambda_j f_j^4 / 4) + g^2 f_1^2 f_2^2 / 2 + V0.
    The quartic mother field and the phi^2 chi^2 daughter coupling are those of
    the lphi4 model (Sect. 5.1)."""
    V = np.full(f.shape[1:], P.V0, dtype=np.float64)
    for j in range(P.n_fields):
        V = V + 0.5 * P.m2[j] * f[j] ** 2 + 0.25 * P.lam[j] * f[j] ** 4
    if P.n_fields == 2:
        V = V + 0.5 * P.g2 * f[0] ** 2 * f[1] ** 2
    return V


def dpotential(f, P: Params):
    """Partial derivatives dV/df_j of `potential`, shape [n, N, N, N]."""
    out = np.empty_like(f)
    for j in range(P.n_fields):
        out[j] = P.m2[j] * f[j] + P.lam[j] * f[j] ** 3
    if P.n_fields == 2:
        out[0] = out[0] + P.g2 * f[0] * f[1] ** 2
        out[1] = out[1] + P.g2 * f[0] ** 2 * f[1]
    return out


def mass2_eff(fbar, P: Params):
    """m_j^2 = d^2V / df_j^2 at the homogeneous values (Eq. QuantumFlucts)."""
    out = []
    for j in range(P.n_fields):
        m = P.m2[j] + 3.0 * P.lam[j] * fbar[j] ** 2
        if P.n_fields == 2:
            m += P.g2 * fbar[1 - j] ** 2
        out.append(m)
    return out


# ------------------------------------------------------- lattice operators
def shift(g, axis: int, step: int):
    """g(n + step * e_axis) with periodic boundaries."""
    return np.roll(g, -step, axis=axis)


def laplacian(g, dx: float):
    """(2d+1)-point periodic Laplacian of one field on a d-dimensional
    lattice (d = g.ndim; 7 points in three dimensions):
    L[g](n) = sum_i [g(n + e_i) + g(n - e_i) - 2 g(n)] / dx^2."""
    out = np.zeros_like(g)
    for ax in range(g.ndim):
        out = out + shift(g, ax, +1) + shift(g, ax, -1) - 2.0 * g
    return out / dx ** 2


def grad_sq_sum(g):
    """sum_i (g(n + e_i) - g(n))^2 at every site (forward differences, over
    the g.ndim directions of the lattice)."""
    out = np.zeros_like(g)
    for ax in range(g.ndim):
        out = out + (shift(g, ax, +1) - g) ** 2
    return out


def force(f, a: float, P: Params):
    """Kick kernel of a canonical real scalar in alpha-time.  With
    pi = a^(3-alpha) f', Eq. singletEOM becomes
    pi' = a^(1+alpha) Lap f - a^(3+alpha) dV/df."""
    dV = dpotential(f, P)
    F = np.empty_like(f)
    for j in range(P.n_fields):
        F[j] = a ** (1.0 + P.alpha) * laplacian(f[j], P.dx) - a ** (3.0 + P.alpha) * dV[j]
    return F


# ---------------------------------------------------------------- energies
def energies(f, p, a: float, P: Params):
    """Volume averages (Sect. 4.3, <g>_V = N^-3 sum_n g(n); N^-dim on a
    reduced lattice) of the scalar
    energy contributions of Eq. energy-contrib:
      K_j = f_j'^2 / (2 a^(2 alpha)) = pi_j^2 / (2 a^6),
      G_j = sum_i (d_i f_j)^2 / (2 a^2), with forward differences,
      V   = potential.
    Returns (EK[n], EG[n], EV)."""
    N3 = float(P.N) ** P.dim
    EK = [float(np.sum(p[j] ** 2)) / (2.0 * a ** 6 * N3) for j in range(P.n_fields)]
    EG = [float(np.sum(grad_sq_sum(f[j]))) / (2.0 * a ** 2 * P.dx ** 2 * N3)
          for j in range(P.n_fields)]
    EV = float(np.sum(potential(f, P))) / N3
    return EK, EG, EV


def rho_pressure(EK, EG, EV):
    """rho = sum K + sum G + V and p = sum K - sum G / 3 - V (Eq. rhoLocal,
    scalar-singlet terms only)."""
    K = sum(EK)
    G = sum(EG)
    return K + G + EV, K - G / 3.0 - EV


def accel(a: float, E, P: Params) -> float:
    """b' = a'' = a^(2 alpha + 1) [(2 alpha - 1) rho - 3 p] / (6 m_p^2)
    (Eq. Friedmann1 multiplied by a).  Zero in static space."""
    if P.expansion == "static":
        return 0.0
    rho, pr = rho_pressure(*E)
    return a ** (2.0 * P.alpha + 1.0) * ((2.0 * P.alpha - 1.0) * rho - 3.0 * pr) / (6.0 * P.mp ** 2)


def hubble_residual(a: float, b: float, E, P: Params) -> float:
    """|H^2 - a^(2 alpha) rho / (3 m_p^2)| / (a^(2 alpha) rho / (3 m_p^2)) with
    H = a'/a (Eq. Friedmann2, the accuracy monitor of Sect. 2.1).  Zero in
    static space."""
    if P.expansion == "static":
        return 0.0
    rho, _ = rho_pressure(*E)
    rhs = a ** (2.0 * P.alpha) * rho / (3.0 * P.mp ** 2)
    return abs((b / a) ** 2 - rhs) / rhs


def hubble_from_rho(a: float, rho: float, P: Params) -> float:
    """Positive root of Eq. Friedmann2 for b = a' = a * sqrt(a^(2 alpha) rho / (3 m_p^2))."""
    if P.expansion == "static":
        return 0.0
    return a * math.sqrt(a ** (2.0 * P.alpha) * rho / (3.0 * P.mp ** 2))


def moments(f, P: Params):
    """Per-field volume mean and variance <(f - <f>)^2>."""
    means, vars_ = [], []
    for j in range(P.n_fields):
        m = float(np.mean(f[j]))
        means.append(m)
        vars_.append(float(np.mean((f[j] - m) ** 2)))
    return means, vars_


# --------------------------------------------------------------- time steps
def vv2(s: State, h: float, P: Params) -> State:
    """One velocity-Verlet sub-step of size h for fields and scale factor
    together (Sect. 4.1: scale factor as a homogeneous dof with
    pi_a' = K_a[a, E], drift D_i and field-only kick K_i for canonical
    fields).  Reading of the discrete form: energies are taken at the
    synchronised momenta, and the drift uses the midpoint scale factor
    abar = (a_old + a_new) / 2.
      1. E = energies(f, p, a); F = force(f, a)
      2. p += h/2 F;  b += h/2 A(a, E)
      3. a_new = a + h b;  f += h abar^(alpha-3) p;  a = a_new
      4. F = force(f, a);  p += h/2 F
      5. E = energies(f, p, a);  b += h/2 A(a, E)"""
    f, p, a, b = s.f.copy(), s.p.copy(), s.a, s.b
    E = energies(f, p, a, P)
    p = p + 0.5 * h * force(f, a, P)
    b = b + 0.5 * h * accel(a, E, P)
    a_new = a + h * b if P.expansion != "static" else a
    abar = 0.5 * (a + a_new)
    f = f + h * abar ** (P.alpha - 3.0) * p
    a = a_new
    p = p + 0.5 * h * force(f, a, P)
    E = energies(f, p, a, P)
    b = b + 0.5 * h * accel(a, E, P)
    return State(f, p, a, b, s.eta + h)


# ---------------------------------------------------------------- Runge-Kutta
# Low-storage ("2N") Runge-Kutta schemes (Sect. 4.1: the RK family of the
# release, with one auxiliary field per degree of freedom).  With
# y = (f, pi, a, a') and y' = F(y), one step of s stages is
#     d <- A_i d + h F(y);   y <- y + B_i d      (i = 1..s, A_1 = 0).
# Coefficients: RK2 -- the explicit midpoint rule written in this form;
# RK3-3 -- Williamson (1980); RK4-5 -- Carpenter and Kennedy (1994), five
# stages, fourth order.
RK_SCHEMES = {
    "rk2": ([0.0, -0.5], [0.5, 1.0]),
    "rk3": ([0.0, -5.0 / 9.0, -153.0 / 128.0], [1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0]),
    # RK3-4: the paper names a four-stage third-order low-storage scheme
    # without coefficients; this member of the 2N family satisfies the order-3
    # conditions and minimises the order-4 error terms.
    "rk34": ([0.0, -0.35643988236064206, -0.9681295617245512, -1.7681569348912718],
             [0.16095368082904207, 0.32750970610000874, 0.759520141721668, 1.0254284658050152]),
    "rk4": ([0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
             -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0],
            [1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
             1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
             2277821191437.0 / 14882151754819.0]),
}


def rhs(f, p, a: float, b: float, P: Params):
    """Right-hand side of the first-order system for (f, pi, a, a'):
    f' = a^(alpha-3) pi (the drift), pi' = force (the kick kernel),
    a' = b, b' = A(a, E(f, pi, a)) (Eq. Friedmann1 times a; zero in static
    space).  Canonical fields: the kernel does not depend on pi."""
    df = a ** (P.alpha - 3.0) * p
    dp = force(f, a, P)
    if P.expansion == "static":
        return df, dp, 0.0, 0.0
    return df, dp, b, accel(a, energies(f, p, a, P), P)


def rk_step(s: State, h: float, P: Params, scheme: str) -> State:
    """One step of a low-storage Runge-Kutta scheme (see RK_SCHEMES)."""
    A, B = RK_SCHEMES[scheme]
    f, p, a, b = s.f.copy(), s.p.copy(), s.a, s.b
    df = np.zeros_like(f)
    dp = np.zeros_like(p)
    da = db = 0.0
    for Ai, Bi in zip(A, B):
        rf, rp, ra, rb = rhs(f, p, a, b, P)
        df = Ai * df + h * rf
        dp = Ai * dp + h * rp
        da = Ai * da + h * ra
        db = Ai * db + h * rb
        f = f + Bi * df
        p = p + Bi * dp
        a = a + Bi * da
        b = b + Bi * db
    return State(f, p, a, b, s.eta + h)


def rk4_classic_step(s: State, h: float, P: Params) -> State:
    """One step of the standard fourth-order Runge-Kutta method (the RK
    family's O(dt^4) standard scheme, Sect. 4.1) for (f, pi, a, a'):
    k1 = F(y), k2 = F(y + h/2 k1), k3 = F(y + h/2 k2), k4 = F(y + h k3),
    y + h/6 (k1 + 2 k2 + 2 k3 + k4)."""
    y = (s.f, s.p, s.a, s.b)

    def shifted(c, k):
        return tuple(yi + c * h * ki for yi, ki in zip(y, k))

    k1 = rhs(*y, P)
    k2 = rhs(*shifted(0.5, k1), P)
    k3 = rhs(*shifted(0.5, k2), P)
    k4 = rhs(*shifted(1.0, k3), P)
    f, p, a, b = (yi + h / 6.0 * (q1 + 2.0 * q2 + 2.0 * q3 + q4) for yi, q1, q2, q3, q4 in zip(y, k1, k2, k3, k4))
    return State(f, p, a, b, s.eta + h)


def step(s: State, dt: float, P: Params, integrator: str = "leapfrog") -> State:
    """One full time step.  leapfrog is velocity Verlet of size dt (its field
    trajectory is the staggered leapfrog one); vv4 is the Yoshida triple jump
    VV2(w1 dt) o VV2(w0 dt) o VV2(w1 dt), accurate to O(dt^4) (Sect. 4.1)."""
    if integrator == "leapfrog":
        return vv2(s, dt, P)
    if integrator == "vv4":
        s = vv2(s, W1 * dt, P)
        s = vv2(s, W0 * dt, P)
        return vv2(s, W1 * dt, P)
    if integrator in RK_SCHEMES:
        return rk_step(s, dt, P, integrator)
    if integrator == "rk4_classic":
        return rk4_classic_step(s, dt, P)
    raise ValueError(integrator)


def observe(s: State, P: Params) -> dict:
    """Per-step record: eta, a, H = a'/a, EK/EG per field, EV, moments, and
    the Hubble-constraint residual."""
    E = energies(s.f, s.p, s.a, P)
    means, vars_ = moments(s.f, P)
    return dict(eta=s.eta, a=s.a, H=s.b / s.a, EK=E[0], EG=E[1], EV=E[2],
                mean=means, var=vars_, r=hubble_residual(s.a, s.b, E, P))


def run(s: State, dt: float, n: int, P: Params, integrator: str = "leapfrog"):
    """Advance n full steps; return the final state and the n per-step records."""
    recs = []
    for _ in range(n):
        s = step(s, dt, P, integrator)
        recs.append(observe(s, P))
    return s, recs
