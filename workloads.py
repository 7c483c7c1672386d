"""Seeded synthetic workloads for the lattice scalar-field path.

This module is shared by the tests, the bench and the oracle.  It holds
only *inputs*: lattice sizes, couplings, time steps and seeds of the
workloads, plus seeded random field states for single-pass checks.  It
holds none of the method's arithmetic (no Laplacian, potential, energy,
scale-factor or seeding formula); those live separately in the oracle and
in the HIP library.

Workload shapes follow the paper's preheating setting (the lphi4 model of
Sect. 5.1: a mother field with a quartic potential and a daughter field
coupled through phi^2 chi^2), in program units with lambda = 1
(Eq. FieldSpaceTimeNaturalVariables), conformal time (alpha = 1,
Eq. FLRWmetric) and lattice geometry dx = L/N, k_IR = 2 pi / L (Sect. 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    N: int                  # sites per dimension
    k_ir: float             # infrared momentum 2 pi / L
    n_fields: int           # 1 (phi) or 2 (phi, chi)
    lam: tuple = (1.0, 0.0)  # quartic self couplings lambda_j
    m2: tuple = (0.0, 0.0)   # bare masses m_j^2
    g2: float = 0.0          # phi^2 chi^2 coupling g^2 (V term g^2 f1^2 f2^2 / 2)
    V0: float = 0.0          # constant vacuum energy
    fbar: tuple = (1.0, 0.0)  # homogeneous field values
    pbar: tuple = (0.0, 0.0)  # homogeneous momenta (pi = a^(3-alpha) f')
    alpha: float = 1.0
    mp: float = 1.0          # reduced Planck mass in program units
    expansion: str = "self"  # "self" (self-consistent) or "static" (a == 1)
    a0: float = 1.0
    integrator: str = "leapfrog"  # "leapfrog" or "vv4"
    dt_over_dx: float = 0.1
    steps: int = 200
    seed: int = 1
    precision: str = "fp64"  # "fp64" or "fp32"
    cutoff: float | None = None  # seeded modes kept for 0 < |n| <= cutoff; default N/4
    amp: float = 1.0

    @property
    def L(self) -> float:
        return 2.0 * math.pi / self.k_ir

    @property
    def dx(self) -> float:
        return self.L / self.N

    @property
    def dt(self) -> float:
        return self.dt_over_dx * self.dx

    @property
    def cutoff_modes(self) -> float:
        return float(self.N // 4) if self.cutoff is None else float(self.cutoff)

    @property
    def sites(self) -> int:
        return self.N ** 3

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# Single real scalar, V = phi^4/4, 32^3, k_IR = 0.1, FP64, leapfrog, dt = 0.1 dx, 200 steps.
C0 = Workload(name="lphi4-1field-32^3-fp64-leapfrog", N=32, k_ir=0.1, n_fields=1,
              lam=(1.0, 0.0), fbar=(1.0, 0.0), integrator="leapfrog",
              dt_over_dx=0.1, steps=200, seed=1, precision="fp64")

# Two-field preheating, V = phi^4/4 + q phi^2 chi^2 / 2 with q = g^2/lambda = 100,
# 256^3, k_IR = 0.5, 4th-order velocity Verlet, dt = 0.05 dx, 5000 steps, FP32 fields.
C1 = Workload(name="lphi4-2field-q100-256^3-fp32-vv4", N=256, k_ir=0.5, n_fields=2,
              lam=(1.0, 0.0), g2=100.0, fbar=(1.0, 0.0), integrator="vv4",
              dt_over_dx=0.05, steps=5000, seed=11, precision="fp32")

# Same physics at 1024^3, leapfrog, FP32 fields, k_IR = 0.25 (dt = 0.05 dx).
C3 = Workload(name="lphi4-2field-q100-1024^3-fp32-leapfrog", N=1024, k_ir=0.25, n_fields=2,
              lam=(1.0, 0.0), g2=100.0, fbar=(1.0, 0.0), integrator="leapfrog",
              dt_over_dx=0.05, steps=200, seed=31, precision="fp32")


def ensemble_members() -> list[Workload]:
    """96 independent realisations of the single-field physics with uneven sizes:
    48 x 32^3, 32 x 64^3 and 16 x 128^3, k_IR = 0.1 for every size, dt = 0.1 dx,
    FP32 fields, leapfrog, seeds 1000 + r."""
    out = []
    r = 0
    for count, N in ((48, 32), (32, 64), (16, 128)):
        for _ in range(count):
            out.append(C0.with_(name=f"ens-{r}-{N}^3", N=N, seed=1000 + r,
                                precision="fp32", steps=1000))
            r += 1
    return out


def random_state(N: int, n_fields: int, seed: int, fbar=(1.0, 0.0), pbar=(0.0, 0.0),
                 famp: float = 1e-2, pamp: float = 1e-2, dim: int = 3):
    """Seeded random field state (f, p), each of shape [n_fields] + [N] * dim
    FP64, last index fastest.  Homogeneous values plus independent uniform
    noise of the given amplitudes.  Used for checks that do not need a
    physical seed (and for the reduced lattices, which take their fields
    from the caller)."""
    rng = np.random.default_rng(seed)
    shape = (N,) * dim
    f = np.empty((n_fields,) + shape)
    p = np.empty((n_fields,) + shape)
    for j in range(n_fields):
        f[j] = fbar[j] + famp * rng.uniform(-1.0, 1.0, shape)
        p[j] = pbar[j] + pamp * rng.uniform(-1.0, 1.0, shape)
    return f, p


# Reduced (2+1)-dimensional lattice of the two-field preheating physics:
# 4096^2 sites, FP32 fields, VV4, dt = 0.05 dx, k_IR = 0.5 * 256 / 4096 (the
# same dx as the 256^3 workload); seeded noise states.
C4 = Workload(name="lphi4-2field-q100-4096^2-fp32-vv4", N=4096, k_ir=0.5 * 256 / 4096, n_fields=2,
              lam=(1.0, 0.0), g2=100.0, fbar=(1.0, 0.0), integrator="vv4",
              dt_over_dx=0.05, steps=2000, seed=51, precision="fp32")
