// Internal declarations shared by the library's host runtime and its HIP
// kernels.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/cl_lattice.h"

namespace cl {

constexpr int kMaxFields = 2;
// Lattice sums per pass: per field {sum p_sync^2, sum |forward grad f|^2,
// sum (f - shift), sum (f - shift)^2, sum p_new}, then sum V.
constexpr int kSumsPerField = 5;
constexpr int kMaxSums = kSumsPerField * kMaxFields + 1;
// Workgroups of a lattice pass: every workgroup of a pass sums the partials of
// all workgroups of the pass before it, so their number is bounded (and kept
// lower still for the tuned candidates).
constexpr int kMaxPassBlocks = 4096;
constexpr int kTunedPassBlocks = 1024;
// Largest lattice-pass workgroup (one row per thread); also the finishing
// kernel's launch bound.
constexpr int kMaxPassThreads = 512;
constexpr int nsums(int nf) { return kSumsPerField * nf + 1; }

// Background state and the coefficients of the next pass, in device memory.
// Written by the last workgroup of every pass, read by the next pass.
struct Scal {
    double a;          // scale factor of the field state produced last
    double b;          // a' (between the passes of one call: the half-step value)
    double eta;        // time of the state the next pass produces
    double cd;         // drift coefficient of the next pass: h abar^(alpha-3)
    double kL;         // a_next^(1+alpha) / dx^2
    double kV;         // a_next^(3+alpha)
    double a_next;     // scale factor after the next drift
    double shift[2];   // predicted mean of f after the next drift (variance shift)
    double mean_f[2];  // mean of f in the state produced last
    double mean_p[2];  // mean of the momenta written last
    double pa1, pa0;   // a_next^(2 alpha + 1), a_next^(2 alpha) (for the next Friedmann step)
    double pf;         // a_next^(alpha - 3) (the drift rate of a Runge-Kutta stage)
    double da, db;     // Runge-Kutta registers of a and a' (low-storage d; classic: the weighted sum of stages)
    double a0, b0;     // classic Runge-Kutta: a and a' at the start of the step
    int32_t nonfinite; // sticky: a lattice sum was NaN / Inf
    int32_t pad;
};

struct Phys {
    double m2[2], lam[2], g2, V0;
    double alpha, mp, dx, inv_vol;
    int nf;
    int expand;  // 1: self-consistent expansion, 0: static
    int fp32;    // 1: fields stored in FP32
    int pad;
};

// Tile of one workgroup: TZ z-values x TY y-rows, marching over CX x-planes.
struct Tile {
    int TZ = 0, TY = 0, CX = 0;  // tile extents
    int RY = 1;                  // y-rows per thread
    int NT = 0;                  // threads per workgroup
    int HI = 1;                  // halo items per thread (1 or 2)
    int PD = 1;                  // x-planes of loads kept in flight (1 or 2)
    int nbz = 0, nby = 0, nbx = 0;
    int nblocks() const { return nbz * nby * nbx; }
};

// One pass over the lattice: optional drift, kick, lattice sums and the
// last-workgroup background update.
//
// Device layout of a state buffer: for every (x, y) row, the 2*nf arrays
// f_0 .. f_{nf-1}, pi_0 .. pi_{nf-1} follow each other, each N values along z:
// element (a, x, y, z) at ((x*N + y)*2*nf + a)*N + z.  A pass then reads one
// contiguous address stream and writes another.
struct PassArgs {
    const void* in;   // state read by the pass
    void* out;        // state written by the pass (the ping-pong partner)
    int N;
    int TZ, TY, CX, nbz, nby, nbx;
    int drift;      // 1: drift f by cd * p before the kick
    int write_out;  // 0: reduction only (no field writes, no kick)
    int rec;        // observable slot for this pass, -1: none
    int flags;      // bit 0: nontemporal stores, bit 1: nontemporal loads
    double kt;      // kick multiplier for the stored momenta
    double kb;      // kick multiplier for the synchronised momenta (energies)
    double h_next;  // drift step of the following pass, 0: call ends here
    // Scalar flow.  A pass leaves its per-workgroup sums in `partials`; the
    // FP64 scalar step that consumes them (Friedmann update, observables,
    // coefficients of the next pass) runs at the start of the next pass, in
    // every workgroup alike, or in the closing finisher kernel.
    const Scal* sc_in;  // scalars before the pending step (or the pass's own, has_prev == 0)
    Scal* sc_out;       // where workgroup 0 leaves the scalars after the pending step
    double* partials;   // this pass: nsums(nf) * nblocks doubles
    const double* prev_partials;  // the previous pass's sums
    int prev_nslots;    // workgroups of the previous pass
    int has_prev;       // 1: finish the previous pass first
    int prev_rec;       // observable slot of the previous pass, -1: none
    int dim;            // spatial dimension of the lattice (1, 2 or 3)
    int ng;             // gravitational-wave tensor components carried in the state (0 or 5)
    double pkt, pkb, phn;  // kt, kb, h_next of the previous pass
    // Runge-Kutta stage, for the fields (registers in `aux`, state layout) and,
    // in the scalar step, for (a, a').  rk = 1, low storage: d <- rkA d +
    // rkh F(y); y <- y + rkB d (rk_first: rkA = 0, aux is not read).  rk = 2,
    // classic: k = rkh F(Y) at the stage input Y; output y0 + rkA s + rkB k,
    // s <- rkC s + rkD k with y0 the state at the start of the step (in `y0`;
    // the stage input itself when rk_first) and s the weighted sum of the
    // stages in `aux` (not read when rk_first, not written when rk_last).
    int rk, rk_first;
    int prev_rk, prev_rk_first;  // the pending step is a Runge-Kutta stage's
    int rk_last, pad3_;
    double rkA, rkB, rkC, rkD, rkh, rkdeta;      // rkdeta: time advanced by this stage
    double prkA, prkB, prkC, prkD, prkh, prkdeta;  // the previous pass's stage coefficients
    void* aux;
    const void* y0;
    cl_observables* obs;
    Phys ph;
};

// One member of an ensemble, as the persistent ensemble kernel sees it.
// Refreshed from the member handles before every ensemble call.
struct EnsMember {
    void* buf[2];        // state buffers; a pass reads buf[cur0 ^ parity]
    int N, TZ, TY, CX;   // tile (TZ * TY / (vector width * RY) == 256 threads)
    int nbz, nby, nbx, nitems;
    int cur0;            // buffer holding the state when the call starts
    int RY;              // rows per thread (1 or 2)
    double dt;
    Phys ph;
    Scal* sc;            // the member's scalar block (start and end of a call)
    Scal* scb;           // two scratch scalar blocks for the passes inside a call
    double* partials;    // two halves of nsums(nf) * nitems, slot = logical tile id
};

struct EnsItem {
    int member;
    int tile;  // logical tile id: bz + nbz * (by + nby * bx)
};

// One pass over every member, in one persistent launch.  Kick and drift
// steps are given in units of each member's dt.  As in a single lattice's
// pass sequence, pass p leaves per-tile partial sums (half p mod 2) and the
// scalar step that consumes them runs at the start of pass p + 1, in every
// work item of the member alike (the item of tile 0 keeps the result and the
// record), or in the closing finisher.
struct EnsArgs {
    const EnsMember* members;
    const EnsItem* items;
    int nitems, nmembers;
    int parity;  // pass index within the call
    int drift, write_out, flags, rec;
    int lds_bytes;  // dynamic shared memory: the largest member tile
    double ckt, ckb, chn;
    int prev_rec;                // record of the previous pass, -1: none
    double pckt, pckb, pchn;     // its kick and drift coefficients (units of dt); pass 0: unused
    unsigned* counter;    // [0] work items handed out, [1] workgroups finished
    cl_observables* obs;  // [rec][member]
};
// One workgroup per member: the scalar step of the last pass of a call.
hipError_t launch_ensemble_finish(const EnsArgs& a, int nf, hipStream_t s);

// Scratch of a sequence of lattice passes: the workgroup partial sums (two
// halves of `half` doubles, used by alternate passes), two scalar blocks that
// carry the background state between the passes of one call, and the ring of
// per-step observable records.  The handle's own buffers by default; the
// allocation-free entry point passes a fixed device array instead.
struct Work {
    double* partials;
    size_t half;
    Scal* scb;
    cl_observables* obs;
    int obs_cap;
};

// Kernel launchers (stencil.hip).  Return the HIP error of the launch.
hipError_t launch_ensemble_pass(const EnsArgs& a, cl_precision prec, int nf, int grid, int maxry, hipStream_t s);
size_t ensemble_lds_bytes(cl_precision prec, int nf, int maxTY, int maxTZ);
int ensemble_grid(cl_precision prec, int nf, size_t lds, int maxry);
hipError_t launch_pass(const PassArgs& a, const Tile& t, cl_precision prec, hipStream_t s);
// One workgroup of t.NT threads: the pending scalar step of the last pass.
hipError_t launch_finish(const PassArgs& a, const Tile& t, int nf, hipStream_t s);
// Power spectrum (spectrum.hip).
// One axis pass of the line FFT (in place); inverse: conjugate twiddles, no 1/N.
// P: stored z per (x, y) (0: N); a y or x pass may run over the first P z of
// an array of pitch P (a multiple of the lines per batch).
hipError_t launch_spec_fft(double2* data, const double2* tw, int N, int axis, hipStream_t s, bool inverse = false,
                           int P = 0);
// The same in FP32 (complex float values and twiddles), whole arrays.
hipError_t launch_fft_f32(float2* data, const float2* tw, int N, int axis, hipStream_t s, bool inverse);
// Pitch of the power spectrum's half array along z: z = 0 .. N / 2 rounded
// up to whole batches of the y and x passes (at most N).
int spec_half_pitch(int N);
// The power spectrum's fused first pass (extraction of array `arr` + the z
// transform, the first P values of each line stored with pitch P) and last
// pass (the x transform + binning into sums / counts, which the caller has
// cleared, of the half array along z, the mirrored modes counted twice).
// `zs`, `zc`: nzero sums and counts (the bins) that the first workgroup
// clears for the last pass (nullptr: none).
hipError_t launch_spec_extract_fftz(const void* state, bool fp32, int N, int na, int arr, const double2* tw,
                                   double2* F, int P, double* zs, unsigned long long* zc, int nzero,
                                   hipStream_t s);
hipError_t launch_spec_fftx_bin(const double2* F, const double2* tw, int N, int P, double width, int nbins,
                                double* sums, unsigned long long* counts, hipStream_t s);
// Gravitational-wave spectrum: projected |U|^2 per centred shell (sums has
// nbins + 1 slots, the last for the modes beyond the bins), U the half
// z <= N / 2 of the five transforms (pitch P, components N^3 apart).
hipError_t launch_gw_bin(const double2* U, int N, int P, double width, int nbins, double* sums,
                         unsigned long long* counts, hipStream_t s);
// Linear propagation of the fluctuations over a jump (propagator.hip): the
// 2 nf channels f_0..f_{nf-1}, pi_0..pi_{nf-1} of a site minus their means,
// packed pairwise into nf complex arrays (channel 2q real, 2q+1 imaginary),
// go through the three axis passes of the line FFT.  The z pass is fused
// with the packing (forward) and with the unpacking (inverse): one
// workgroup takes the line FFT's batch of consecutive rows of array q =
// blockIdx.y.  The complex arrays and the transforms are in the state's
// precision (double2 for FP64 lattices, float2 for FP32).
struct PropZArgs {
    const void* state;  // forward: the state read (row-interleaved)
    void* out;          // inverse: the state written (may not alias `state`)
    void* z[2];         // the packed complex arrays
    const void* tw;     // exp(-2 pi i k / N), k < N / 2
    int N, nf;
    int logN, L;        // filled by the launchers
    double mean[4];     // forward: subtracted; inverse: added back
};
struct PropStep {
    double ck0, m0[3], cd, ck1, m1[3];
};
struct PropModeArgs {
    const void* in[2];     // forward transforms of the packed arrays (state precision)
    void* out[2];          // propagated modes, packed again, times `scale`
    int N, nf;
    const double* kap2;    // [N]: (2/dx)^2 sin^2(pi n / N)
    const PropStep* steps;
    int nsteps;
    double scale;          // 1 / N^3 (the inverse transform's normalisation)
    void* table;           // [prop_table_entries(N)][(2 nf)^2]: transfer matrices, FP32 for FP32
                           // lattices, else FP64 (workspace of 16 doubles per entry)
    const uint32_t* triples;  // prop_triples(N) on the device
    size_t ntriples;
};
// Entries of the transfer-matrix table: sorted triples i0 <= i1 <= i2 of
// folded mode indices (each in [0, N/2]), and the list of them in table
// order, packed 10 bits each (N <= 1024).
size_t prop_table_entries(int N);
std::vector<uint32_t> prop_triples(int N);
// Packing + forward z pass; inverse z pass + unpacking into `out`.
hipError_t launch_prop_pack_fftz(const PropZArgs& a, bool fp32, hipStream_t s);
hipError_t launch_prop_ifftz_unpack(const PropZArgs& a, bool fp32, hipStream_t s);
// Transfer matrices (FP64) and their application to every mode; fp32: the
// arrays hold float2 values (converted to FP64 for the product).
hipError_t launch_prop_modes(const PropModeArgs& a, bool fp32, hipStream_t s);
hipError_t launch_init_scalars(Scal* sc, double a, double b, double eta, const Phys& ph,
                               const double* shift, hipStream_t s);
// Default tile for a lattice; valid for every N accepted by cl_create.
Tile default_tile(int N, cl_precision prec, int nf);
// Fill nbz/nby/nbx and check that the tile divides the lattice and fits the
// kernel's limits.  Returns false if not.
bool finalize_tile(Tile& t, int N, cl_precision prec);
// LDS of a pass for `arrays` stencil arrays (the fields, plus the tensor
// components when gravitational waves are on).
size_t pass_lds_bytes(const Tile& t, cl_precision prec, int arrays);
// All valid tiles the autotuner tries for a lattice.
void candidate_tiles(int N, cl_precision prec, int nf, Tile* out, int* count, int cap);
hipError_t launch_copy(const void* in, void* out, size_t bytes, hipStream_t s);

// Allocation-free stepping (lattice_api.cpp): checks the arguments as
// cl_step does, issues the passes of n steps of a symplectic scheme directly
// on the handle's stream (no graph) with the scratch `w`, copies the n
// records to per_step (if not NULL) and waits.  Allocates nothing.
cl_status step_in_work(cl_lattice* h, cl_integrator integ, double dt, int n, cl_observables* per_step, const Work& w);
// Records the failure message on h (or the handle-less message) and returns st.
cl_status set_error(cl_lattice* h, cl_status st, const char* msg);
// Overwrite the background of h on its stream without waiting: a, a', eta,
// the step count and the field means (the variance shift); the pass
// coefficients follow from a.
cl_status set_background_async(cl_lattice* h, double a, double b, double eta, int64_t step, const double* mean);
// One reduction pass of the current state, its observables and the scalar
// block copied to the host, one wait.  The variance sums are taken about the
// shift the scalar block holds (set_background_async's means), so the
// caller sets it at the state's expected means first.
cl_status observe_once(cl_lattice* h, cl_observables* o, Scal* sc);
// The line FFT's twiddle table of the lattice (allocated on first use).
cl_status spectral_twiddles(cl_lattice* h, const double2** tw);

// Host seed (host_seed.cpp): fills f, p (n_fields * N^3 FP64 each).
// Returns an empty string on success, an error message otherwise.
const char* host_seed(int N, double dx, int nf, const Phys& ph, double a0, uint64_t seed,
                      const double* fbar, const double* pbar, double cutoff, double amp,
                      double* f, double* p);

}  // namespace cl

#include <string>

struct GraphKey {
    int integ = -1;
    double dt = 0.0;
    int n = 0;
    int cur = 0;
    bool operator==(const GraphKey& o) const {
        return integ == o.integ && dt == o.dt && n == o.n && cur == o.cur;
    }
};

struct cl_lattice {
    int N = 0;
    double dx = 0.0;
    int nf = 1;
    cl_precision prec = CL_FP64;
    double alpha = 1.0, mp = 1.0, a0 = 1.0;
    cl_expansion mode = CL_SELF_CONSISTENT;
    cl_potential pot{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool own_buffers = true;
    int device = 0;
    void* buf[2] = {nullptr, nullptr};  // ping-pong state buffers (row-interleaved layout)
    void* aux = nullptr;                // Runge-Kutta registers of f and pi (same layout), on first use
    void* aux2 = nullptr;               // classic RK4: the third stage buffer, on first use
    int dim = 3;                        // spatial dimension (reduced lattices: 1 or 2)
    int ng = 0;                         // gravitational-wave tensor components in the state (0 or 5)
    double2* spec = nullptr;            // power spectrum: N^3 complex FP64, on first use
    double2* gw_spec = nullptr;         // gravitational-wave spectrum: 5 N^3 complex FP64, on first use
    double2* spec_tw = nullptr;         // its twiddle factors (N / 2)
    double* spec_sums = nullptr;        // per-bin sums and counts (spec_cap bins; two allocations:
    unsigned long long* spec_counts = nullptr;  // the last pass's atomics on both were slower in one)
    double* spec_host = nullptr;        // pinned host copy: spec_cap sums, then spec_cap counts
    int spec_cap = 0;
    int pass_flags = 1;                 // nontemporal stores
    int cur = 0;
    cl::Scal* sc = nullptr;
    double* partials = nullptr;  // two halves, used by alternate passes
    size_t partials_cap = 0;     // doubles (both halves)
    cl::Scal* scb = nullptr;     // two scratch scalar blocks for the passes inside a call
    cl_observables* obs = nullptr;
    int obs_cap = 0;
    cl::Tile tile;
    int64_t step = 0;
    // background last seen on the host (after a call synchronised with the
    // device): scale factor and field means, for the time-step stability check
    double host_a = 1.0;
    double host_mean[2] = {0.0, 0.0};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};  // one per starting buffer
    GraphKey gkey[2];
    bool use_graph = true;
    std::string err;
};


