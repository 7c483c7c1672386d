/*
 * cl_lattice.h -- C ABI of the MI355X lattice scalar-field library.
 *
 * The library evolves n_fields (1 or 2) interacting real scalar fields on a
 * periodic N^3 lattice in a spatially flat FLRW background, in alpha-time
 * (CosmoLattice 2.0, Sect. 2, Eq. FLRWmetric).  Each time step is a drift of
 * the fields, a kick of the conjugate momenta pi = a^(3-alpha) f' by the
 * 7-point Laplacian and the potential derivative (Sect. 2.1, Eq. singletEOM),
 * and volume averages of the kinetic, gradient and potential energies
 * (Eq. energy-contrib) that drive the scale-factor update through the
 * Friedmann equations (Eqs. Friedmann1, Friedmann2), all advanced together by
 * a symplectic kick-drift scheme (Sect. 4.1, Eqs. SchemeContVirgin1-4).
 *
 * Conventions
 *   - Every call returns cl_status: CL_OK (0) on success, a negative code on
 *     failure.  No C++ exception crosses this boundary.  cl_last_error()
 *     gives a human-readable message for the last failure.
 *   - Handles are opaque and not thread safe; one handle issues all its GPU
 *     work on one HIP stream (the null stream unless cl_set_stream is used).
 *   - Host arrays are copy-in / copy-out; the caller owns them.
 *   - Field arrays are structure-of-arrays, field-major: element
 *     [j][(x*N + y)*N + z] for field j, z fastest, n_fields * N^3 values.
 *   - Device memory is allocated and freed by the library unless the caller
 *     attaches its own buffers with cl_attach_device_buffers.
 *   - Passing NULL for a required pointer returns CL_EINVAL.
 */
#ifndef CL_LATTICE_H
#define CL_LATTICE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CL_OK = 0,
    CL_EINVAL = -1,       /* invalid argument */
    CL_ENOMEM = -2,       /* host or device allocation failed */
    CL_EDEVICE = -3,      /* a HIP runtime call failed */
    CL_ESTATE = -4,       /* call not valid in the handle's current state */
    CL_EUNSTABLE = -5,    /* non-finite values appeared, or the time step exceeds the scheme's stability bound */
    CL_EUNSUPPORTED = -6  /* valid request this build does not support */
} cl_status;

typedef enum { CL_FP64 = 0, CL_FP32 = 1 } cl_precision;

/* CL_STATIC: a == 1, a' == 0.  CL_SELF_CONSISTENT: a follows Eq. Friedmann1
 * sourced by the lattice volume averages of rho and p (Eq. rhoLocal). */
typedef enum { CL_STATIC = 0, CL_SELF_CONSISTENT = 1 } cl_expansion;

/* CL_LEAPFROG: staggered leapfrog, O(dt^2).  CL_VV4: 4th-order Yoshida
 * composition of velocity Verlet, O(dt^4) (Sect. 4.1).  CL_RK2, CL_RK3,
 * CL_RK34, CL_RK4: low-storage Runge-Kutta schemes of the (f, pi, a, a')
 * system with one auxiliary array per field and momentum (Sect. 4.1, RK
 * family): the explicit midpoint rule (2 stages, O(dt^2)), Williamson's
 * RK3-3 (3 stages, O(dt^3)), an RK3-4 (4 stages, O(dt^3); the paper names
 * the scheme without coefficients: ours meets the order-3 conditions and
 * minimises the order-4 error terms) and Carpenter-Kennedy's RK4-5 (5
 * stages, O(dt^4)).  CL_RK4_CLASSIC: the standard four-stage RK4 with
 * three auxiliary arrays per degree of freedom (Sect. 4.1: the RK
 * family's standard O(dt^4) method), each stage one fused pass.  A
 * Runge-Kutta step costs one fused pass per stage, each moving 32 B per
 * field and site in FP32 (64 B in FP64), against 16 (32) for a leapfrog pass;
 * the auxiliary arrays are allocated by the first Runge-Kutta step. */
typedef enum {
    CL_LEAPFROG = 0,
    CL_VV4 = 1,
    CL_RK2 = 2,
    CL_RK3 = 3,
    CL_RK4 = 4,
    CL_RK34 = 5,
    CL_RK4_CLASSIC = 6
} cl_integrator;

/* V = sum_j (m2[j] f_j^2 / 2 + lambda[j] f_j^4 / 4) + g2 f_0^2 f_1^2 / 2 + V0,
 * in program variables (Eq. FieldSpaceTimeNaturalVariables).  With two fields
 * this is the mother/daughter potential of the lphi4 model (Sect. 5.1). */
typedef struct {
    double m2[2];
    double lambda[2];
    double g2;
    double V0;
} cl_potential;

/* Homogeneous background state: scale factor a, its alpha-time derivative
 * b = a' (the scale-factor momentum of Eq. SchemeContVirgin1), time eta and
 * the number of completed time steps. */
typedef struct {
    double a;
    double b;
    double eta;
    int64_t step;
} cl_scalars;

/* Observables of one synchronised state.  EK, EG: kinetic and gradient
 * energy densities per field, EV: potential energy density (volume averages,
 * Eq. energy-contrib with <.>_V of Sect. 4.3).  H = a'/a.  mean, var: per-field
 * volume mean and variance of f.  hubble_residual:
 * |H^2 - a^(2 alpha) rho/(3 m_p^2)| / (a^(2 alpha) rho/(3 m_p^2)) (Eq. Friedmann2),
 * 0 in static space.  nonfinite: 1 if any lattice sum was NaN or Inf. */
typedef struct {
    double eta;
    double a;
    double H;
    double EK[2];
    double EG[2];
    double EV;
    double mean[2];
    double var[2];
    double hubble_residual;
    int32_t nonfinite;
    int32_t reserved;
} cl_observables;

typedef struct cl_lattice cl_lattice;
typedef struct cl_ensemble cl_ensemble;

/* Message for the last failing call on h (or on any handle-less call when h
 * is NULL).  The string stays valid until the next call on the same handle. */
const char* cl_last_error(const cl_lattice* h);

/* Library version string (static storage). */
const char* cl_version(void);

/* Create a lattice of N^3 sites with spacing dx (Sect. 2: dx = L/N,
 * k_IR = 2 pi / L), n_fields in {1, 2}, field storage precision prec.  N must
 * be even and >= 8 (power of two for cl_seed), dx > 0.  Allocates the field,
 * momentum and ping-pong buffers on the current HIP device (4 * n_fields *
 * N^3 values of the chosen precision) plus a small scalar block.  Defaults:
 * alpha = 1, self-consistent expansion, m_p = 1, a0 = 1, V = lambda f^4/4 with
 * lambda = 1 for field 0, fields zero.  On failure *out is NULL. */
cl_status cl_create(int N, double dx, int n_fields, cl_precision prec, cl_lattice** out);

/* Reduced lattice (Sect. 3, scalar dynamics in 1+1 and 2+1 dimensions):
 * dim = 1 or 2 spatial directions of N sites (N a multiple of 4, at least
 * 8), the same field and Friedmann equations with the Laplacian and the
 * gradient energy summed over dim directions and volume averages over N^dim
 * sites; dim = 3 is cl_create.  Host arrays of cl_set_fields / cl_get_fields
 * hold n_fields * N^dim values per kind (the last index fastest); on the
 * device, array a of row x (dim = 2) starts at (x * 2 * n_fields + a) * N.
 * Reduced lattices step with CL_LEAPFROG and CL_VV4 and support
 * cl_read_observables, cl_get_state / cl_set_state and the buffer calls;
 * cl_seed, the Runge-Kutta schemes, tiles, the autotuner, the power
 * spectrum, ensembles and the surrogate return CL_EUNSUPPORTED. */
cl_status cl_create_dim(int dim, int N, double dx, int n_fields, cl_precision prec, cl_lattice** out);

/* Free everything the library allocated for h.  cl_destroy(NULL) is a no-op. */
cl_status cl_destroy(cl_lattice* h);

/* Issue all GPU work of h on the given hipStream_t (NULL = null stream).  The
 * caller keeps the stream alive while h uses it. */
cl_status cl_set_stream(cl_lattice* h, void* hip_stream);

/* Use caller-owned device memory instead of library-owned buffers.  Each of
 * the two buffers (the state and its ping-pong partner) holds
 * 2 * n_fields * N^3 values of the handle's precision, 16-byte aligned, in the
 * library's row-interleaved layout: for row (x, y) the arrays f_0 ..
 * f_{n_fields-1}, pi_0 .. pi_{n_fields-1} follow each other, N values each,
 * so array a at (x, y, z) is element ((x*N + y)*2*n_fields + a)*N + z.  The
 * current state is in `state`.  Library-owned buffers are freed.  The caller
 * keeps the memory alive until cl_destroy.  Field values are not copied: set
 * them afterwards. */
cl_status cl_attach_device_buffers(cl_lattice* h, void* state, void* state_pp);

/* Device address of the buffer that holds the current state (library-owned
 * or attached), in the row-interleaved layout above.  Every pass writes the
 * other buffer, so the address may change with each cl_step; it stays valid
 * until the next call that advances, attaches or destroys h.  Lets a caller
 * read or overwrite the fields in place on the device; after writing them,
 * call cl_set_state (a, a', eta) and cl_read_observables, which re-centres the
 * variance sums on the new means. */
cl_status cl_get_state_buffer(const cl_lattice* h, void** state);

/* Background: alpha-time exponent alpha (Eq. FLRWmetric; 0 cosmic, 1
 * conformal), expansion mode, reduced Planck mass m_p in program units, and
 * the initial scale factor a0 used by cl_seed / cl_set_fields. */
cl_status cl_set_background(cl_lattice* h, double alpha, cl_expansion mode, double m_p, double a0);

/* Potential coefficients (copied). */
cl_status cl_set_potential(cl_lattice* h, const cl_potential* pot);

/* Vacuum-fluctuation initial condition (Sect. 2.3, Eqs. QuantumFlucts,
 * fpr_influct, fpr_influct2): homogeneous values fbar[j], pbar[j] (momenta
 * pi) plus Gaussian fluctuations drawn in Fourier space on modes
 * 0 < |n| <= cutoff_modes with <|df(n)|^2> = amp^2 / (2 a0^2 w_k dx^3),
 * w_k^2 = k^2 + a0^2 d2V/df_j^2(fbar), transformed with the DFT convention of
 * Sect. 4.3.  Random numbers: SplitMix64 counter stream keyed by seed, field
 * and mode.  Afterwards a = a0 and a' is set from the lattice energy density
 * so that the Hubble constraint holds exactly (0 in static space); eta = 0,
 * step = 0.  Runs on the host in FP64 (N must be a power of two), then
 * uploads.  cutoff_modes <= 0 selects N/4. */
cl_status cl_seed(cl_lattice* h, uint64_t seed, const double* fbar, const double* pbar,
                  double cutoff_modes, double amp);

/* Copy host FP64 fields and momenta (n_fields * N^3 each, layout above) into
 * the current state, rounding to the handle's precision.  Sets a = a0,
 * eta = 0, step = 0 and a' from the Hubble constraint (0 in static space). */
cl_status cl_set_fields(cl_lattice* h, const double* f, const double* p);

/* Copy the current (synchronised) fields and momenta to host FP64 arrays. */
cl_status cl_get_fields(cl_lattice* h, double* f, double* p);

/* Read / overwrite the background state (checkpoint and resume).  Fields are
 * saved and restored with cl_get_fields / cl_set_fields followed by
 * cl_set_state. */
cl_status cl_get_state(const cl_lattice* h, cl_scalars* out);
cl_status cl_set_state(cl_lattice* h, const cl_scalars* in);

/* Advance n full time steps of size dt with the given integrator, starting
 * and ending in a synchronised state.  If per_step is not NULL it receives n
 * records, one after each full step.  Returns CL_EUNSTABLE if a lattice sum
 * became non-finite (the records then show where) or if w_max dt reaches the
 * integrator's stability limit on a harmonic mode, with
 * w_max^2 = 4 dim / dx^2 a^(2 alpha - 2) + a^(2 alpha) max_j d^2V/df_j^2
 * (the fastest lattice mode of Eq. singletEOM; the curvature of V taken at
 * the field means of the last synchronised state).  Limits: leapfrog 2,
 * VV4 1.5735, RK3-3 sqrt(3), RK3-4 2.823, RK4-5 3.341, classic RK4 2 sqrt(2)
 * (ends of the stability intervals on the imaginary axis); RK2, which has
 * none, is held to at most 1 % growth per step of the fastest mode
 * (w_max dt < 0.532).  The work is issued on the handle's stream and the
 * call returns after it completes. */
cl_status cl_step(cl_lattice* h, cl_integrator integ, double dt, int n, cl_observables* per_step);

/* cl_step without any allocation, for callers that cannot allocate memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The passes and results are those of cl_step; the passes are
 * issued directly on the handle's stream (no graph is built), and their
 * scratch -- the workgroup partial sums, the two scalar blocks that carry
 * the background between passes and the per-step record ring -- lives in a
 * fixed device array of the library (about 1.2 MB, held by every device the
 * library runs on until the process ends) instead of buffers the handle
 * allocates on first use.  Its address on a device is looked up on the
 * first call on that device.  Limits: n <= 4096 steps per call (CL_EINVAL
 * beyond), integrators CL_LEAPFROG and CL_VV4 (the Runge-Kutta schemes need
 * state-sized registers: CL_EUNSUPPORTED).  Every call on one device shares
 * that array and leaves it holding its own last contents (nothing in it is
 * read before it is written within a call), so calls that overlap in time on
 * one device -- from several threads, or on several streams -- race and
 * must not be issued.  On success nothing is allocated, host or device; a
 * failure stores its message in the handle as every call does. */
cl_status cl_step_noalloc(cl_lattice* h, cl_integrator integ, double dt, int n, cl_observables* per_step);

/* Observables of the current state (one reduction pass over the lattice). */
cl_status cl_read_observables(cl_lattice* h, cl_observables* out);

/* Gravitational waves (Sect. 2.2 Eq. EoMGWs, Sect. 4.2): with on != 0 the
 * state also carries the five components v_11, v_12, v_13, v_22, v_23 of a
 * traceless tensor (v_33 = -v_11 - v_22) and their momenta
 * u = a^(3-alpha) v', starting at zero.  Each step advances them with the
 * fields' own kick-drift scheme: drift v' = a^(alpha-3) u, kick
 * u' = a^(1+alpha) (Lap v + (2/m_p^2) S), where S is the traceless part of the
 * fields' anisotropic stress (Eq. anitensor) evaluated on the lattice as the
 * sum over fields of [D+_i f D+_j f + D-_i f D-_j f] / (2 dx^2) (forward and
 * backward differences) at the time level of the kick.  The physical waves
 * are the transverse-traceless projection of v in Fourier space
 * (cl_gw_spectrum).  The fields, momenta and background are kept; a step
 * then moves 2 (n_fields + 5) arrays per site (FP32: 16 (n_fields + 5) bytes
 * per site and pass).  Only the symplectic schemes run with the tensor;
 * ensembles and the surrogate take lattices without it.  Needs
 * library-owned buffers (attach buffers of 2 (n_fields + 5) N^3 values
 * afterwards if wanted: the layout is the one of cl_attach_device_buffers
 * with n_fields + 5 arrays of each kind, fields first, then v_11 .. v_23).
 * on == 0 drops the tensor.  Three-dimensional lattices only. */
cl_status cl_gw_enable(cl_lattice* h, int on);

/* Host FP64 copies of the tensor components and their momenta, component
 * major: [c][(x*N + y)*N + z] for c = 11, 12, 13, 22, 23 (5 N^3 values each;
 * either pointer of cl_gw_get may be NULL).  CL_ESTATE if the waves are off. */
cl_status cl_gw_set(cl_lattice* h, const double* v, const double* u);
cl_status cl_gw_get(cl_lattice* h, double* v, double* u);

/* Energy spectrum of the gravitational waves of the current state (Sect.
 * 4.2): the DFT of every component of u on the device (FP64), per mode the
 * projection h'_ij = a^(alpha-3) Lambda_ij,lm(k^) u_lm with
 * Lambda_ij,lm = P_il P_jm - P_ij P_lm / 2, P = 1 - k^ k^, and k^ the unit
 * lattice momentum (sin(pi n_i / N))_i (the mode n = 0 carries none), and
 * |h'_ij|^2 summed over centred shells of |n| of width `width` as the scalar
 * spectrum bins them.  Outputs (each may be NULL): counts[l] -- modes in bin
 * l; rho[l] = m_p^2 / (4 a^(2 alpha) N^6) sum over the bin of |h'_ij(n)|^2,
 * the bin's share of rho_GW = m_p^2 <h'_ij h'_ij> / (4 a^(2 alpha));
 * omega[l] = l rho[l] / rho_tot, the discretised (d rho_GW / d log k) / rho_tot
 * at k_l = l width k_IR with rho_tot the lattice energy density; *rho_gw --
 * rho_GW over every mode (bins beyond nbins included).  nbins <= 4096, N a
 * power of two; uses 80 N^3 bytes of device memory, allocated on first use. */
cl_status cl_gw_spectrum(cl_lattice* h, double width, int nbins, int64_t* counts, double* rho, double* omega,
                         double* rho_gw);

/* Power spectrum of one array of the current state (Sect. 4.3, Eqs.
 * discretePSaux, discretePST2): field `field`, what = 0 for f, 1 for pi.  The
 * DFT f(n~) = sum_n exp(-2 pi i n~.n / N) f(n) (n~_i in -N/2+1 .. N/2) is
 * computed on the device in FP64; the modes are binned by |n~| into centred
 * shells of width `width` (bin l: l w - w/2 <= |n~| < l w + w/2; w = 1 is the
 * canonical binning), bins l = 0 .. nbins-1 (nbins <= 4096; modes beyond are
 * dropped).  Outputs (host arrays of nbins, each may be NULL): counts[l] --
 * modes in the bin (exact); sums[l] -- sum of |f(n~)|^2 over the bin (FP64,
 * accumulated with atomics, so equal between calls to rounding only);
 * delta[l] = (k_l / 2 pi) (dx / N^5) sums[l] with k_l = k_IR l w, the
 * exact-multiplicity form of Eq. discretePST2.  N must be a power of two.
 * Uses a device buffer of 16 N^3 bytes, allocated on first use. */
cl_status cl_power_spectrum(cl_lattice* h, int field, int what, double width, int nbins, int64_t* counts,
                            double* sums, double* delta);

/* Work decomposition of the lattice passes: each workgroup owns a tz x ty
 * tile of (z, y) and marches over cx x-planes; ry is the number of y rows per
 * thread (1 or 2) and pd the number of x-planes whose loads are kept in
 * flight ahead of the plane being computed (1, 2, or 4 with ry = 1; 0 selects
 * 1).  tz, ty, cx
 * must divide N; tz is a multiple of 4 (FP32) or 2 (FP64) with at most 256
 * threads per workgroup.  An invalid tile returns CL_EINVAL and leaves the
 * current one in place. */
typedef struct {
    int tz;
    int ty;
    int cx;
    int ry;
    int pd;
} cl_tile;

cl_status cl_get_tile(const cl_lattice* h, cl_tile* out);
cl_status cl_set_tile(cl_lattice* h, const cl_tile* t);

/* Autotuner: times `reps` fused drift-kick passes of every candidate tile on
 * the current state (fields and background are left unchanged), then times
 * the four fastest again in three interleaved rounds of at least 40 passes
 * each, selects the finalist with the shortest round and writes a JSON
 * report ("candidates": the screening, "finalists", "best"; NUL-terminated,
 * truncated to report_cap) if report is not NULL.  If the environment variable
 * CL_TUNE_CACHE names a file, the result is appended there as one JSON line
 * and later cl_create calls for the same (N, n_fields, precision) start from
 * it. */
cl_status cl_autotune(cl_lattice* h, int reps, char* report, size_t report_cap);

/* Streaming-copy probe on the current device: copies `bytes` (rounded down
 * to 16) between two scratch buffers `reps` times and returns the achieved
 * read+write bandwidth in GB/s (1e9 bytes/s).  Allocates and frees its own
 * buffers. */
cl_status cl_copy_bandwidth(size_t bytes, int reps, double* gbps);

/* Ensembles: advance several independent lattices (equal precision and
 * n_fields, any N >= 32 accepted by cl_create) together, each pass of all members in one persistent
 * launch, the passes of a call captured in one HIP graph.  Members keep their
 * own potential, background, scale factor and time step; they must use the
 * null stream or a common one.  The ensemble does not own the members. */
cl_status cl_ensemble_create(int n_members, cl_lattice* const* members, cl_ensemble** out);
cl_status cl_ensemble_set_dt(cl_ensemble* e, int member, double dt);
/* out: NULL or n_steps * n_members records, step-major ([s][member]).
 * integ: CL_LEAPFROG or CL_VV4 (the Runge-Kutta schemes: CL_EUNSUPPORTED). */
cl_status cl_ensemble_step(cl_ensemble* e, cl_integrator integ, int n_steps, cl_observables* out);
/* Tile the ensemble kernel uses for one member (two rows per thread where
 * the lattice is tall enough).  A member stepped on its own with this tile
 * (cl_set_tile) gives bitwise the same result as inside the ensemble. */
cl_status cl_ensemble_get_tile(const cl_ensemble* e, int member, cl_tile* out);
/* Ensemble autotuner: times `reps` passes of every distinct work
 * decomposition (about 8k to 128k sites per work item, with and without two
 * rows per thread) on the members' current states, which are left unchanged
 * (fields bitwise, scalar blocks restored), and keeps the fastest.  Writes a
 * JSON report (NUL-terminated, truncated to report_cap) if report is not
 * NULL.  The decomposition changes the order of the lattice sums, not the
 * site updates. */
cl_status cl_ensemble_autotune(cl_ensemble* e, int reps, char* report, size_t report_cap);
cl_status cl_ensemble_destroy(cl_ensemble* e);

#ifdef __cplusplus
}
#endif

#endif /* CL_LATTICE_H */
