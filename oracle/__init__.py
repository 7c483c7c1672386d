"""CPU FP64 oracle for the lattice scalar-field method -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously correct reference of what the
HIP path computes.  Only the tests, the smoke check of the entry module and
the CPU-baseline leg of the bench may import it.  The product library never
calls it, and it shares no code with the library: both are written
independently from the paper (CosmoLattice 2.0), and only the seeded input
module ``workloads`` is common to both sides.

Contents
  lattice    -- potential, 7-point Laplacian, force, drift, volume-averaged
                energies, Friedmann acceleration, Hubble residual, and the
                velocity-Verlet / leapfrog / 4th-order Yoshida time steps
                (Sect. 2.1 Eqs. singletEOM, Friedmann1, Friedmann2, rhoLocal,
                energy-contrib; Sect. 4.1 Eqs. SchemeContVirgin1-4), and the
                low-storage Runge-Kutta steps RK2, RK3-3, RK3-4, RK4-5
                and the standard RK4 of the (f, pi, a, a') system (Sect.
                4.1, RK family).
  seed       -- counter-based RNG and the vacuum-fluctuation initial
                condition (Sect. 2.3 Eqs. QuantumFlucts, fpr_influct,
                fpr_influct2; Sect. 4.3 DFT convention).
  surrogate  -- periodic 3D convolution net in FP64 (forward, backward,
                MSE, Adam) used to check the learned-surrogate kernels.
  spectrum   -- DFT power spectrum in spherical bins of arbitrary width
                (Sect. 4.3, Eqs. discretePSaux, discretePST2).

Parity unpinned (the paper is silent; the oracle and the library share a
written reading instead of a paper value): the reduced Planck mass in
program units, the seed amplitude normalisation, when the kinetic energy
enters the scale-factor kick, the midpoint scale factor in the drift, the
RNG stream, and every surrogate hyper-parameter.
"""
