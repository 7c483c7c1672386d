"""Pins of the oracle on reduced (1+1)- and (2+1)-dimensional lattices
(CPU only).  The reduced lattice solves the same field and Friedmann
equations with the Laplacian and the gradient energy summed over d
directions and volume averages over N^d sites, so (i) its Laplacian has the
d-dimensional lattice eigenvalues, and (ii) a three-dimensional state that
does not depend on the remaining 3 - d coordinates is an exact solution of
the three-dimensional lattice that stays equal to the reduced run -- which
ties the reduced oracle to the pinned three-dimensional one."""
import math

import numpy as np
import pytest

from oracle import lattice as L
import workloads as W


@pytest.mark.parametrize("d", [1, 2])
def test_laplacian_eigenmodes(d):
    """cos(2 pi k.n / N) is an eigenvector of the d-dimensional lattice
    Laplacian with eigenvalue -sum_i (2/dx)^2 sin^2(pi k_i / N)."""
    N, dx = 12, 0.37
    k = (3, 5)[:d]
    idx = np.meshgrid(*[np.arange(N)] * d, indexing="ij")
    phase = sum(2 * np.pi * ki * ni / N for ki, ni in zip(k, idx))
    g = np.cos(phase)
    lam = -sum((2.0 / dx) ** 2 * math.sin(math.pi * ki / N) ** 2 for ki in k)
    assert np.max(np.abs(L.laplacian(g, dx) - lam * g)) <= 1e-12 * abs(lam)


def _embed(f, d):
    """A 3-D array that repeats the d-dimensional one along the trailing
    3 - d axes."""
    N = f.shape[-1]
    out = f
    for _ in range(3 - d):
        out = np.repeat(out[..., None], N, axis=-1)
    return np.ascontiguousarray(out)


@pytest.mark.parametrize("d", [1, 2])
@pytest.mark.parametrize("integrator", ["leapfrog", "vv4"])
def test_reduced_lattice_equals_embedded_3d(d, integrator):
    """Two-field preheating potential in self-consistent expansion: n steps
    of the d-dimensional oracle equal n steps of the 3-D oracle started from
    the embedded state, fields and per-step records, to rounding."""
    N, nf = 8, 2
    w = W.C1.with_(N=N, k_ir=2.0)
    f, p = W.random_state(N, nf, seed=41, fbar=(1.0, 0.05), famp=0.3, pamp=0.2)
    sl = (slice(None),) + (slice(None),) * d + (0,) * (3 - d)
    fd, pd = np.ascontiguousarray(f[sl]), np.ascontiguousarray(p[sl])
    kw = dict(N=N, dx=w.dx, n_fields=nf, m2=w.m2, lam=w.lam, g2=w.g2)
    Pd, P3 = L.Params(dim=d, **kw), L.Params(**kw)
    E = L.energies(fd, pd, 1.0, Pd)
    b0 = L.hubble_from_rho(1.0, L.rho_pressure(*E)[0], Pd)
    sd, rd = L.run(L.State(fd, pd, 1.0, b0), w.dt, 12, Pd, integrator)
    s3, r3 = L.run(L.State(_embed(fd, d), _embed(pd, d), 1.0, b0), w.dt, 12, P3, integrator)
    assert s3.a > 1.0 and sd.a == pytest.approx(s3.a, rel=1e-13)
    assert np.max(np.abs(_embed(sd.f, d) - s3.f)) <= 1e-12 * np.max(np.abs(s3.f))
    assert np.max(np.abs(_embed(sd.p, d) - s3.p)) <= 1e-12 * np.max(np.abs(s3.p))
    for a, b in zip(rd, r3):
        for k in ("a", "H", "EV"):
            assert a[k] == pytest.approx(b[k], rel=1e-12), k
        for k in ("EK", "EG"):
            assert np.allclose(a[k], b[k], rtol=1e-12, atol=1e-15), k


def test_reduced_gradient_energy_counts_d_directions():
    """A plane wave along the first axis has the same gradient energy on the
    1-, 2- and 3-dimensional lattice (the other directions add nothing), and
    on the 2-D lattice a wave along the second axis has it too (both
    directions are summed alike)."""
    N, dx = 10, 0.5
    n = np.arange(N)
    g1 = np.cos(2 * np.pi * 2 * n / N)
    vals = []
    for d in (1, 2, 3):
        g = g1.reshape((N,) + (1,) * (d - 1)) * np.ones((N,) * d)
        P = L.Params(N=N, dx=dx, n_fields=1, lam=(0.0, 0.0), dim=d)
        vals.append(L.energies(g[None], np.zeros((1,) + (N,) * d), 1.0, P)[1][0])
    assert vals[0] > 0 and np.allclose(vals, vals[0], rtol=1e-14)
    g2 = np.cos(2 * np.pi * 2 * n / N)[None, :] * np.ones((N, N))
    P2 = L.Params(N=N, dx=dx, n_fields=1, lam=(0.0, 0.0), dim=2)
    assert L.energies(g2[None], np.zeros((1, N, N)), 1.0, P2)[1][0] == pytest.approx(vals[0], rel=1e-14)
