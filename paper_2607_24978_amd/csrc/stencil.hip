// Lattice pass kernels for gfx950: fused drift + kick + lattice sums, with
// the scale-factor (Friedmann) update done by the last workgroup.
//
// Physics (CosmoLattice 2.0):
//   drift   f += cd * pi,            cd = h abar^(alpha-3)      (pi = a^(3-alpha) f')
//   kick    pi += k * F,  F = a^(1+alpha) Lap f - a^(3+alpha) dV/df   (Eq. singletEOM)
//   sums    pi_sync^2, forward-difference gradients, V, moments  (Eq. energy-contrib)
//   a''     = a^(2 alpha+1) [(2 alpha-1) rho - 3 p] / (6 m_p^2)  (Eq. Friedmann1)
// The scale factor rides along as a homogeneous degree of freedom with its
// own kick and drift (Sect. 4.1, Eqs. SchemeContVirgin1-2).
//
// Memory layout: per (x, y) row the arrays f_0.., pi_0.. follow each other,
// z fastest, so a pass reads one contiguous address stream and writes
// another.  A pass reads one state buffer and writes the other (ping-pong),
// since the drift of halo cells needs the old momenta of neighbouring tiles.
//
// Blocking: a workgroup owns a TZ x TY tile of (z, y) and marches over CX
// x-planes.  Each x-plane of drifted f (tile plus a one-cell y/z halo) is
// staged in LDS (double-buffered, one barrier per plane); the x-neighbours
// live in registers.  Each thread owns V consecutive z values (16-byte
// vector loads and stores) in RY rows.
#include "internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <type_traits>

// Every fused multiply-add below is written out; no other contraction, so
// all kernel instantiations (tiles, prefetch depths, the ensemble kernel)
// round every site update identically.
#pragma clang fp contract(off)

namespace cl {

__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> struct VecOf;
template <> struct VecOf<float> { using type = float4; static constexpr int V = 4; };
template <> struct VecOf<double> { using type = double2; static constexpr int V = 2; };

template <typename T>
__device__ __forceinline__ void vload(const T* p, T (&out)[VecOf<T>::V]) {
    using VT = typename VecOf<T>::type;
    VT v = *reinterpret_cast<const VT*>(p);
    if constexpr (VecOf<T>::V == 4) { out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w; }
    else { out[0] = v.x; out[1] = v.y; }
}

template <typename T> struct NatVec;
template <> struct NatVec<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct NatVec<double> { typedef double type __attribute__((ext_vector_type(2))); };

// Streaming variants: the nontemporal hint keeps data that is not reused in
// this pass from displacing the halo lines in the caches.
template <typename T>
__device__ __forceinline__ void vload_nt(const T* p, T (&out)[VecOf<T>::V]) {
    using NV = typename NatVec<T>::type;
    NV v = __builtin_nontemporal_load(reinterpret_cast<const NV*>(p));
#pragma unroll
    for (int i = 0; i < VecOf<T>::V; ++i) out[i] = v[i];
}

template <typename T>
__device__ __forceinline__ void vstore_nt(T* p, const T (&in)[VecOf<T>::V]) {
    using NV = typename NatVec<T>::type;
    NV v;
#pragma unroll
    for (int i = 0; i < VecOf<T>::V; ++i) v[i] = in[i];
    __builtin_nontemporal_store(v, reinterpret_cast<NV*>(p));
}

template <typename T>
__device__ __forceinline__ void vstore(T* p, const T (&in)[VecOf<T>::V]) {
    using VT = typename VecOf<T>::type;
    VT v;
    if constexpr (VecOf<T>::V == 4) { v.x = in[0]; v.y = in[1]; v.z = in[2]; v.w = in[3]; }
    else { v.x = in[0]; v.y = in[1]; }
    *reinterpret_cast<VT*>(p) = v;
}

// dV/df_j in the field precision.
template <typename T, int NF>
__device__ __forceinline__ void site_dV(const T (&f)[NF], const T (&m2)[2], const T (&lam)[2], T g2,
                                        T (&dV)[NF]) {
#pragma unroll
    for (int j = 0; j < NF; ++j) dV[j] = f[j] * fmad(lam[j], f[j] * f[j], m2[j]);
    if constexpr (NF == 2) {
        dV[0] = fmad(g2 * f[0], f[1] * f[1], dV[0]);
        dV[1] = fmad(g2 * f[1], f[0] * f[0], dV[1]);
    }
}

// Last workgroup of a pass: observables and the scale-factor kick/drift.
// `tot` holds the lattice sums.  Called by all 64 lanes of one wave: the
// powers of a are evaluated on separate lanes, lane 0 writes the results.
__device__ __forceinline__ void finish_pass(const Phys& P, Scal* sc, double kt, double kb, double h_next, cl_observables* rec_out,
                            const double* tot) {
    const int lane = threadIdx.x & 63;
    const int nf = P.nf;
    const double a = sc->a_next;  // scale factor of the state just produced
    const double a2 = a * a;
    const double a6 = a2 * a2 * a2;
    double EK[2] = {0.0, 0.0}, EG[2] = {0.0, 0.0}, mean[2] = {0.0, 0.0};
    double var[2] = {0.0, 0.0}, meanp[2] = {0.0, 0.0};
    int bad = 0;
    for (int j = 0; j < nf; ++j) {
        const double* t = tot + kSumsPerField * j;
        EK[j] = t[0] * P.inv_vol / (2.0 * a6);
        EG[j] = t[1] * P.inv_vol / (2.0 * a2 * P.dx * P.dx);
        const double m1 = t[2] * P.inv_vol;
        // the kernels subtract the shift rounded to the field precision
        const double c = P.fp32 ? static_cast<double>(static_cast<float>(sc->shift[j])) : sc->shift[j];
        mean[j] = c + m1;
        var[j] = t[3] * P.inv_vol - m1 * m1;
        meanp[j] = t[4] * P.inv_vol;
    }
    const double EV = tot[kSumsPerField * nf] * P.inv_vol + P.V0;
    for (int k = 0; k < nsums(nf); ++k) bad |= !isfinite(tot[k]);
    const double K = EK[0] + EK[1], G = EG[0] + EG[1];
    const double rho = K + G + EV;
    const double pr = K - G / 3.0 - EV;
    double acc = 0.0, r = 0.0;
    const double b_half = sc->b;
    // a^(2 alpha + 1) and a^(2 alpha), formed by the step that fixed a
    const double a_2al1 = sc->pa1, a_2al = sc->pa0;
    if (P.expand) {
        acc = a_2al1 * ((2.0 * P.alpha - 1.0) * rho - 3.0 * pr) / (6.0 * P.mp * P.mp);
    }
    const double bs = b_half + kb * acc;
    if (P.expand) {
        const double rhs = a_2al * rho / (3.0 * P.mp * P.mp);
        const double H = bs / a;
        r = fabs(H * H - rhs) / rhs;
    }
    const double b_new = b_half + kt * acc;
    const double an = (h_next != 0.0 && P.expand) ? a + h_next * b_new : a;
    const double abar = 0.5 * (a + an);
    // lane 0: abar^(alpha - 3), lanes 1..5: an^(1 + alpha), an^(3 + alpha),
    // an^(2 alpha + 1), an^(2 alpha), an^(alpha - 3)
    double ex = P.alpha - 3.0;
    if (lane == 1) ex = 1.0 + P.alpha;
    if (lane == 2) ex = 3.0 + P.alpha;
    if (lane == 3) ex = 2.0 * P.alpha + 1.0;
    if (lane == 4) ex = 2.0 * P.alpha;
    const double pw = (h_next != 0.0 && lane < 6) ? pow(lane == 0 ? abar : an, ex) : 0.0;
    const double abar_al3 = __shfl(pw, 0, 64), an_1al = __shfl(pw, 1, 64), an_3al = __shfl(pw, 2, 64);
    const double an_2al1 = __shfl(pw, 3, 64), an_2al = __shfl(pw, 4, 64), an_al3 = __shfl(pw, 5, 64);
    if (lane != 0) return;
    if (rec_out) {
        cl_observables o;
        o.eta = sc->eta;
        o.a = a;
        o.H = bs / a;
        for (int j = 0; j < 2; ++j) {
            o.EK[j] = EK[j];
            o.EG[j] = EG[j];
            o.mean[j] = mean[j];
            o.var[j] = var[j];
        }
        o.EV = EV;
        o.hubble_residual = r;
        o.nonfinite = bad;
        o.reserved = 0;
        *rec_out = o;
    }
    sc->a = a;
    sc->b = b_new;
    sc->nonfinite |= bad;
    for (int j = 0; j < 2; ++j) {
        sc->mean_f[j] = mean[j];
        sc->mean_p[j] = meanp[j];
    }
    if (h_next != 0.0) {
        sc->cd = h_next * abar_al3;
        sc->kL = an_1al / (P.dx * P.dx);
        sc->kV = an_3al;
        sc->a_next = an;
        sc->pa1 = an_2al1;
        sc->pa0 = an_2al;
        sc->pf = an_al3;
        sc->eta += h_next;
        for (int j = 0; j < 2; ++j) sc->shift[j] = mean[j] + sc->cd * meanp[j];
    } else {
        sc->cd = 0.0;
        sc->a_next = a;
        for (int j = 0; j < 2; ++j) sc->shift[j] = mean[j];
    }
}

// The scalar step after a Runge-Kutta stage.  The sums in `tot` describe the
// stage's input state y_i at scale factor a = sc->a (momenta and fields at
// the same time): record the observables of y_i (if rec_out), then advance
// (a, a') by the same recurrence as the fields -- low storage (mode 1):
//   d_a <- A d_a + h a',  d_b <- A d_b + h a''(a, E(y_i)),  a += B d_a, a' += B d_b;
// classic (mode 2), with k = h (a', a'') at the stage input, (a0, b0) the
// start of the step and s the weighted stage sum (first: a0 = a, s = 0):
//   (a, a') <- (a0, b0) + A s + B k,  s <- C s + D k --
// and form the next stage's coefficients at the new a (all 64 lanes of one
// wave call; the powers are spread over lanes; lane 0 writes).
__device__ __forceinline__ void finish_rk(const Phys& P, Scal* sc, int mode, int first, double rkA, double rkB,
                                          double rkC, double rkD, double h, double deta, cl_observables* rec_out,
                                          const double* tot) {
    const int lane = threadIdx.x & 63;
    const int nf = P.nf;
    const double a = sc->a, b = sc->b;
    const double a2 = a * a;
    const double a6 = a2 * a2 * a2;
    double EK[2] = {0.0, 0.0}, EG[2] = {0.0, 0.0}, mean[2] = {0.0, 0.0};
    double var[2] = {0.0, 0.0}, meanp[2] = {0.0, 0.0};
    int bad = 0;
    for (int j = 0; j < nf; ++j) {
        const double* t = tot + kSumsPerField * j;
        EK[j] = t[0] * P.inv_vol / (2.0 * a6);
        EG[j] = t[1] * P.inv_vol / (2.0 * a2 * P.dx * P.dx);
        const double m1 = t[2] * P.inv_vol;
        const double c = P.fp32 ? static_cast<double>(static_cast<float>(sc->shift[j])) : sc->shift[j];
        mean[j] = c + m1;
        var[j] = t[3] * P.inv_vol - m1 * m1;
        meanp[j] = t[4] * P.inv_vol;
    }
    const double EV = tot[kSumsPerField * nf] * P.inv_vol + P.V0;
    for (int k = 0; k < nsums(nf); ++k) bad |= !isfinite(tot[k]);
    const double K = EK[0] + EK[1], G = EG[0] + EG[1];
    const double rho = K + G + EV;
    const double pr = K - G / 3.0 - EV;
    double acc = 0.0, r = 0.0;
    if (P.expand) {
        acc = sc->pa1 * ((2.0 * P.alpha - 1.0) * rho - 3.0 * pr) / (6.0 * P.mp * P.mp);
        const double rhs = sc->pa0 * rho / (3.0 * P.mp * P.mp);
        const double H = b / a;
        r = fabs(H * H - rhs) / rhs;
    }
    double da, db, an, bn;
    const double a0 = (mode == 2 && !first) ? sc->a0 : a, b0 = (mode == 2 && !first) ? sc->b0 : b;
    if (mode == 2) {
        const double sa = first ? 0.0 : sc->da, sb = first ? 0.0 : sc->db;
        an = P.expand ? a0 + rkA * sa + rkB * (h * b) : a;
        bn = P.expand ? b0 + rkA * sb + rkB * (h * acc) : b;
        da = rkC * sa + rkD * (h * b);
        db = rkC * sb + rkD * (h * acc);
    } else {
        da = rkA * sc->da + h * b;
        db = rkA * sc->db + h * acc;
        an = P.expand ? a + rkB * da : a;
        bn = P.expand ? b + rkB * db : b;
    }
    // lanes 0..4: an^(alpha - 3), an^(1 + alpha), an^(3 + alpha), an^(2 alpha + 1), an^(2 alpha)
    double ex = P.alpha - 3.0;
    if (lane == 1) ex = 1.0 + P.alpha;
    if (lane == 2) ex = 3.0 + P.alpha;
    if (lane == 3) ex = 2.0 * P.alpha + 1.0;
    if (lane == 4) ex = 2.0 * P.alpha;
    const double pw = lane < 5 ? pow(an, ex) : 0.0;
    const double an_al3 = __shfl(pw, 0, 64), an_1al = __shfl(pw, 1, 64), an_3al = __shfl(pw, 2, 64);
    const double an_2al1 = __shfl(pw, 3, 64), an_2al = __shfl(pw, 4, 64);
    if (lane != 0) return;
    if (rec_out) {
        cl_observables o;
        o.eta = sc->eta;
        o.a = a;
        o.H = b / a;
        for (int j = 0; j < 2; ++j) {
            o.EK[j] = EK[j];
            o.EG[j] = EG[j];
            o.mean[j] = mean[j];
            o.var[j] = var[j];
        }
        o.EV = EV;
        o.hubble_residual = r;
        o.nonfinite = bad;
        o.reserved = 0;
        *rec_out = o;
    }
    sc->a = an;
    sc->a_next = an;
    sc->b = bn;
    sc->da = da;
    sc->db = db;
    sc->a0 = a0;
    sc->b0 = b0;
    sc->eta += deta;
    sc->nonfinite |= bad;
    sc->cd = 0.0;
    sc->kL = an_1al / (P.dx * P.dx);
    sc->kV = an_3al;
    sc->pf = an_al3;
    sc->pa1 = an_2al1;
    sc->pa0 = an_2al;
    for (int j = 0; j < 2; ++j) {
        sc->mean_f[j] = mean[j];
        sc->mean_p[j] = meanp[j];
        sc->shift[j] = mean[j];
    }
}

// Word-wise copy of the scalar block by the threads of a workgroup (no
// struct temporaries).
__device__ __forceinline__ void copy_scal(Scal* dst, const Scal* src, int nthreads) {
    static_assert(sizeof(Scal) % 8 == 0, "Scal is a whole number of 8-byte words");
    const unsigned long long* s = reinterpret_cast<const unsigned long long*>(src);
    unsigned long long* d = reinterpret_cast<unsigned long long*>(dst);
    for (int i = threadIdx.x; i < static_cast<int>(sizeof(Scal) / 8); i += nthreads) d[i] = s[i];
}

// Sum over the workgroup of NS per-thread FP64 values: a butterfly over the
// lanes of each wave, level by level so that the NS exchanges of one level
// are in flight together (levels at or above NT are skipped: tiny lattices
// run workgroups of fewer than 64 threads), then the waves in order by
// thread 0 into out[] (shared memory).  Every thread calls; out[] is valid
// for all threads on return.  The order depends on NT only.
template <int NS>
__device__ __forceinline__ void block_sum(double (&v)[NS], int NT, double* out) {
    __shared__ double wsum[kMaxPassThreads / 64][kMaxSums];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        if (off >= NT) continue;
#pragma unroll
        for (int k = 0; k < NS; ++k) v[k] += __shfl_xor(v[k], off, 64);
    }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NS; ++k) wsum[wave][k] = v[k];
    __syncthreads();
    if (tid == 0) {
        const int nw = (NT + 63) / 64;
        for (int k = 0; k < NS; ++k) {
            double s = wsum[0][k];
            for (int w = 1; w < nw; ++w) s += wsum[w][k];
            out[k] = s;
        }
    }
    __syncthreads();
}

// Totals of NS sums over `nslots` workgroup partials (partials[k * nslots +
// slot]) in a fixed order: thread t takes slots t, t + NT, ... with Neumaier
// compensation (all NS sums at once so that their loads overlap), then
// block_sum.  Deterministic for a fixed nslots and NT.
template <int NS>
__device__ __forceinline__ void slots_sum(const double* partials, int NT, int nslots, double* tot) {
    double s[NS], c[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] = c[k] = 0.0;
#pragma unroll 4
    for (int i = threadIdx.x; i < nslots; i += NT) {
        double x[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) x[k] = partials[(size_t)k * nslots + i];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const double t = s[k] + x[k];
            c[k] += (fabs(s[k]) >= fabs(x[k])) ? (s[k] - t) + x[k] : (x[k] - t) + s[k];
            s[k] = t;
        }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] += c[k];
    block_sum<NS>(s, NT, tot);
}

// Everything one workgroup does for one tile: march over CX x-planes of the
// TZ x TY tile at (z0, y0, x0), drifting, kicking and writing the new state
// and accumulating the per-thread lattice sums into `acc`.
struct TileJob {
    const void* in;
    void* out;
    int N, TZ, TY, CX;
    int z0, y0, x0;
    int drift, write_out, flags;
    double kt, kb;
    const Scal* sc;
    const Phys* ph;
    // Runge-Kutta stage (march_tile<..., RK = 1 low storage, 2 classic>)
    void* aux;
    const void* step0;  // classic: the state at the start of the step
    double rkA, rkB, rkC, rkD, rkh;
    int rk_first, rk_last;
};

// Calls f(integral_constant<int, B>), ..., f(integral_constant<int, E - 1>).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// RK = 0: fused drift + kick (the symplectic schemes).  RK = 1: one
// low-storage Runge-Kutta stage -- no drift (the plane staged in LDS is the
// stage's input f), F = h (a^(alpha-3) pi, a^(1+alpha) L f - a^(3+alpha) dV),
// d <- A d + F and y <- y + B d with the registers d of (f, pi) in `aux`
// (loaded one plane ahead), sums over the stage's input state.  RK = 2: one
// classic Runge-Kutta stage -- the same F at the stage input Y, output
// y0 + A s + B F and s <- C s + D F with the step's start y0 (in `step0`) and
// the weighted stage sum s (in `aux`), both loaded one plane ahead.
// NG > 0 (symplectic schemes only): the state also holds the NG = 5
// components v_11, v_12, v_13, v_22, v_23 of the traceless tensor whose
// transverse-traceless part is the gravitational-wave field (Sect. 4.2), and
// their momenta u = a^(3-alpha) v': each row holds f_0.., v_11.., pi_0..,
// u_11.. .  They drift with the fields' coefficient and are kicked by
// kL (L[v] + (1/m_p^2) S) where S is the traceless part of the sum over
// fields of the products of forward and of backward differences of the
// drifted fields (no lattice sums for them).
template <typename T, int NF, int RY, int HI, int PD, int RK, int HPD, int NG, typename Prelude>
__device__ __forceinline__ void march_tile(const TileJob& J, unsigned char* smem_raw, double (&acc)[kSumsPerField * NF + 1],
                           Prelude&& prelude) {
    constexpr int V = VecOf<T>::V;
    constexpr int NS = kSumsPerField * NF + 1;
    constexpr int NA = NF + NG;  // stencil arrays (fields and tensor components)
    static_assert(NG == 0 || (NG == 5 && RK == 0), "tensor components with the symplectic schemes only");
    const int N = J.N, TZ = J.TZ, TY = J.TY, CX = J.CX;
    const int z0 = J.z0, y0 = J.y0, x0 = J.x0;
    const int BZ = TZ / V;
    const int RL = TY / RY;
    const int NT = BZ * RL;
    const int tid = threadIdx.x;
    const int tz = tid % BZ;
    const int tr = tid / BZ;
    // Row-interleaved state: array a of row (x, y) starts at ((x*N + y)*2NA + a)*N.
    const int rs = 2 * NA * N;  // row stride (elements)
    const T* fin[NA];
    const T* pin[NA];
    T* fout[NA];
    T* pout[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        fin[j] = static_cast<const T*>(J.in) + j * N;
        pin[j] = static_cast<const T*>(J.in) + (NA + j) * N;
        fout[j] = static_cast<T*>(J.out) + j * N;
        pout[j] = static_cast<T*>(J.out) + (NA + j) * N;
    }
    const bool nt_store = J.flags & 1;
    const bool nt_load = J.flags & 2;
    T* auxf[NF];
    T* auxp[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        auxf[j] = RK ? static_cast<T*>(J.aux) + j * N : nullptr;
        auxp[j] = RK ? static_cast<T*>(J.aux) + (NF + j) * N : nullptr;
    }
    const bool rk_first = RK && J.rk_first;
    const bool rk_last = RK == 2 && J.rk_last;
    const T rA = static_cast<T>(J.rkA), rB = static_cast<T>(J.rkB);
    const T rC = static_cast<T>(J.rkC), rD = static_cast<T>(J.rkD);
    const T* y0f[NF];
    const T* y0p[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        y0f[j] = RK == 2 ? static_cast<const T*>(J.step0) + j * N : nullptr;
        y0p[j] = RK == 2 ? static_cast<const T*>(J.step0) + (NF + j) * N : nullptr;
    }

    // Pass coefficients; set once the prelude has produced the scalars.
    T cd = T(0), kL = T(0), kV = T(0), cF = T(0);
    const T kt = static_cast<T>(J.kt);
    const T kb = static_cast<T>(J.kb);
    // Variance shift in the field precision: f - c is exact for f near c.
    T shift[NF];
    const T m2[2] = {static_cast<T>(J.ph->m2[0]), static_cast<T>(J.ph->m2[1])};
    const T lam[2] = {static_cast<T>(J.ph->lam[0]), static_cast<T>(J.ph->lam[1])};
    const T g2 = static_cast<T>(J.ph->g2);
    const T hm2[2] = {T(0.5) * m2[0], T(0.5) * m2[1]};
    const T qlam[2] = {T(0.25) * lam[0], T(0.25) * lam[1]};
    const T hg2 = T(0.5) * g2;
    // tensor source weight: 2 / m_p^2 times the 1/2 of the difference average
    const T cS = static_cast<T>(1.0 / (J.ph->mp * J.ph->mp));

    T* lds = reinterpret_cast<T*>(smem_raw);
    const int S = TZ + 2 * V;        // LDS row stride (interior starts at column V)
    const int PL = (TY + 2) * S;     // one plane of one field
    // lds[buf][field][row][col]; row 0 = y0-1, row TY+1 = y0+TY.

    const int zc = z0 + tz * V;
    int yrow[RY];
#pragma unroll
    for (int k = 0; k < RY; ++k) yrow[k] = (y0 + tr + k * RL) * rs + zc;

    // Halo items of this thread (row halo: V values; z halo: 1 value).
    const int nhalo = 2 * BZ + 2 * TY;
    int h_goff[HI];   // offset within a plane (y*N + z), -1 if none
    int h_lds[HI];    // LDS offset within a plane
    bool h_vec[HI];   // vector item (row halo) or scalar item (z halo)
#pragma unroll
    for (int q = 0; q < HI; ++q) {
        const int item = tid + q * NT;
        h_goff[q] = -1;
        h_lds[q] = 0;
        h_vec[q] = false;
        if (item < nhalo) {
            if (item < 2 * BZ) {
                const int side = item / BZ, cz = item % BZ;
                const int y = side == 0 ? (y0 - 1 + N) % N : (y0 + TY) % N;
                h_goff[q] = y * rs + z0 + cz * V;
                h_lds[q] = (side == 0 ? 0 : TY + 1) * S + V + cz * V;
                h_vec[q] = true;
            } else {
                const int kk = item - 2 * BZ;
                const int row = kk >> 1, side = kk & 1;
                const int z = side == 0 ? (z0 - 1 + N) % N : (z0 + TZ) % N;
                h_goff[q] = (y0 + row) * rs + z;
                h_lds[q] = (row + 1) * S + (side == 0 ? V - 1 : V + TZ);
            }
        }
    }

    const size_t plane = static_cast<size_t>(N) * rs;
    // Raw (undrifted) loads of up to PD planes in flight: own values in a ring
    // of PD register sets, halo items in a ring of HPD sets (HPD = PD, or 2 <
    // PD where registers are short: few threads hold halo items, and a deep
    // halo ring costs every thread its registers), issued HPD planes ahead.
    // The prologue below fixes which plane travels in which set.
    static_assert(HPD == PD || (HPD == 2 && PD == 4), "halo ring depth");
    T rf[PD][NA][RY][V], rp[PD][NA][RY][V], hf[HPD][NA][HI][V], hp[HPD][NA][HI][V];
    // Loads of plane x0+ko (own values, into set S; ko may be -1) and of the
    // halo items of plane x0+kh (into halo set H, only for planes staged in
    // LDS, 0 <= kh < CX), field by field; kNone skips either part.
    constexpr int kNone = -1000000;
    auto issue = [&](auto Sc, auto Hc, int ko, int kh) {
        constexpr int S_ = decltype(Sc)::value;
        constexpr int H_ = decltype(Hc)::value;
        const bool own = ko != kNone;
        const bool halo = kh >= 0 && kh < CX;
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            if (own) {
                const size_t obase = static_cast<size_t>((x0 + ko + N) % N) * plane;
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    if (nt_load) {
                        vload_nt(fin[j] + obase + yrow[r], rf[S_][j][r]);
                        vload_nt(pin[j] + obase + yrow[r], rp[S_][j][r]);
                    } else {
                        vload(fin[j] + obase + yrow[r], rf[S_][j][r]);
                        vload(pin[j] + obase + yrow[r], rp[S_][j][r]);
                    }
                }
            }
            if (halo) {
                const size_t hbase = static_cast<size_t>((x0 + kh + N) % N) * plane;
#pragma unroll
                for (int q = 0; q < HI; ++q) {
                    if (h_goff[q] < 0) continue;
                    if (h_vec[q]) {
                        vload(fin[j] + hbase + h_goff[q], hf[H_][j][q]);
                        vload(pin[j] + hbase + h_goff[q], hp[H_][j][q]);
                    } else {
                        hf[H_][j][q][0] = fin[j][hbase + h_goff[q]];
                        hp[H_][j][q][0] = pin[j][hbase + h_goff[q]];
                    }
                }
            }
        }
    };
    // Drift the raw plane of set S: own values into fd / po, and (if
    // stage_buf >= 0) the drifted own values and halo into LDS buffer stage_buf.
    T prev[NA][RY][V], cur[NA][RY][V], nxt[NA][RY][V], pc[NA][RY][V], pn[NA][RY][V];
    auto consume = [&](auto Sc, auto Hc, T (&fd)[NA][RY][V], T (&po)[NA][RY][V], int stage_buf) {
        constexpr int S_ = decltype(Sc)::value;
        constexpr int H_ = decltype(Hc)::value;
#pragma unroll
        for (int j = 0; j < NA; ++j)
#pragma unroll
            for (int r = 0; r < RY; ++r)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    po[j][r][v] = rp[S_][j][r][v];
                    fd[j][r][v] = fmad(cd, rp[S_][j][r][v], rf[S_][j][r][v]);
                }
        if (stage_buf < 0) return;
        T* L0 = lds + static_cast<size_t>(stage_buf) * NA * PL;
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            T* Lj = L0 + j * PL;
#pragma unroll
            for (int r = 0; r < RY; ++r) vstore(Lj + (tr + r * RL + 1) * S + V + tz * V, fd[j][r]);
#pragma unroll
            for (int q = 0; q < HI; ++q) {
                if (h_goff[q] < 0) continue;
                if (h_vec[q]) {
                    T fv[V];
#pragma unroll
                    for (int v = 0; v < V; ++v) fv[v] = fmad(cd, hp[H_][j][q][v], hf[H_][j][q][v]);
                    vstore(Lj + h_lds[q], fv);
                } else {
                    Lj[h_lds[q]] = fmad(cd, hp[H_][j][q][0], hf[H_][j][q][0]);
                }
            }
        }
    };


    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, PD >= 2 ? 1 : 0>;
    // halo set of plane k: its own set (k + 1) mod PD when HPD = PD, else k mod 2
    auto hs = [](auto Kc) {
        constexpr int k = decltype(Kc)::value;
        return std::integral_constant<int, HPD == PD ? (k + 1) % PD : k % HPD>{};
    };
    using K0 = std::integral_constant<int, 0>;
    using K1 = std::integral_constant<int, 1>;
    using K2 = std::integral_constant<int, 2>;
    // Prologue: plane x0-1 (own only), plane x0 (own + halo into buffer 0),
    // then the loads of planes x0+1 .. x0+PD stay in flight into the loop.
    // With PD >= 2 the own values of plane k travel in set (k + 1) mod PD and
    // planes x0-1 .. x0+PD-2 are in flight while the prelude runs, with their
    // halo when HPD = PD; with HPD = 2 < PD only the halo of x0 is, and that
    // of x0+1, x0+2 goes out once plane x0 is staged (after the prelude,
    // whose sums need registers too).  With PD = 1 plane k >= 1 travels in
    // the one set.
    issue(S0{}, S0{}, -1, kNone);
    if constexpr (PD >= 2) {
        issue(S1{}, hs(K0{}), 0, 0);
        static_for<2, PD>([&](auto Sc) {
            constexpr int s_ = decltype(Sc)::value;
            using Km = std::integral_constant<int, s_ - 1>;
            if (s_ - 1 <= CX) issue(Sc, hs(Km{}), s_ - 1, HPD == PD ? s_ - 1 : kNone);
        });
    }
    // the scalars of this pass (the previous pass's scalar step may run here,
    // while the first loads are in flight)
    prelude();
    {
        const Scal* sc = J.sc;
        if constexpr (RK) {
            // h folded into the coefficients (formed in FP64, rounded once)
            cF = static_cast<T>(J.rkh * sc->pf);
            kL = static_cast<T>(J.rkh * sc->kL);
            kV = static_cast<T>(J.rkh * sc->kV);
        } else {
            cd = J.drift ? static_cast<T>(sc->cd) : T(0);
            kL = static_cast<T>(sc->kL);
            kV = static_cast<T>(sc->kV);
        }
#pragma unroll
        for (int j = 0; j < NF; ++j) shift[j] = static_cast<T>(sc->shift[j]);
    }
    // Runge-Kutta registers of (f, pi) for the current plane and the next one.
    // (classic stages: also the step's start y0 of (f, pi))
    T axc[RK ? 2 : 1][NF][RY][V], axn[RK ? 2 : 1][NF][RY][V];
    T y0c[RK == 2 ? 2 : 1][NF][RY][V], y0n[RK == 2 ? 2 : 1][NF][RY][V];
    auto aux_load = [&](int k, T (&dst)[RK ? 2 : 1][NF][RY][V], T (&ydst)[RK == 2 ? 2 : 1][NF][RY][V]) {
        if constexpr (RK) {
            const size_t base = static_cast<size_t>(x0 + k) * static_cast<size_t>(N) * rs;
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    vload(auxf[j] + base + yrow[r], dst[0][j][r]);
                    vload(auxp[j] + base + yrow[r], dst[RK ? 1 : 0][j][r]);
                    if constexpr (RK == 2) {
                        vload(y0f[j] + base + yrow[r], ydst[0][j][r]);
                        vload(y0p[j] + base + yrow[r], ydst[1][j][r]);
                    }
                }
        }
    };
    if (RK && !rk_first) aux_load(0, axc, y0c);
    consume(S0{}, S0{}, prev, pn, -1);
    if constexpr (PD >= 2) {
        consume(S1{}, hs(K0{}), cur, pc, 0);
        if constexpr (HPD == PD) {
            using Ka = std::integral_constant<int, PD - 1>;
            using Kb = std::integral_constant<int, PD>;
            if (PD - 1 <= CX) issue(S0{}, hs(Ka{}), PD - 1, PD - 1);
            if (PD <= CX) issue(S1{}, hs(Kb{}), PD, PD);
        } else {
            issue(S0{}, hs(K1{}), PD - 1 <= CX ? PD - 1 : kNone, 1);
            issue(S1{}, hs(K2{}), PD <= CX ? PD : kNone, 2);
        }
    } else {
        issue(S0{}, S0{}, 0, 0);
        consume(S0{}, S0{}, cur, pc, 0);
        issue(S0{}, S0{}, 1, 1);
    }
    __syncthreads();

    // One x-plane: plane x+1 arrives from set S and halo set H (drift,
    // stage), the own loads of plane x+1+PD go out into the same set and the
    // halo loads of plane x+1+HPD into the same halo set, then plane x is
    // computed.
    auto body = [&](auto Sc, auto Hc, int i) {
        const int x = x0 + i;
        const int buf = i & 1;
        consume(Sc, Hc, nxt, pn, i + 1 < CX ? (buf ^ 1) : -1);
        if constexpr (HPD == PD) {
            if (i + 1 + PD <= CX) issue(Sc, Hc, i + 1 + PD, i + 1 + PD);
        } else {
            issue(Sc, Hc, i + 1 + PD <= CX ? i + 1 + PD : kNone, i + 1 + HPD);
        }
        if (RK && !rk_first && i + 1 < CX) aux_load(i + 1, axn, y0n);

        const T* L0 = lds + static_cast<size_t>(buf) * NA * PL;
        const size_t base = static_cast<size_t>(x) * plane;
        // Per-plane partial sums in the field precision, promoted once.
        T part[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) part[q] = T(0);
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int row = tr + k * RL + 1;
            const int col = V + tz * V;
            T ym[NA][V], yp[NA][V], zm0[NA], zp0[NA];
#pragma unroll
            for (int j = 0; j < NA; ++j) {
                const T* Lj = L0 + j * PL;
                vload(Lj + (row - 1) * S + col, ym[j]);
                vload(Lj + (row + 1) * S + col, yp[j]);
                zm0[j] = Lj[row * S + col - 1];
                zp0[j] = Lj[row * S + col + V];
            }
            T pnew[NA][V], fnew[NF][V], dfo[NF][V], dpo[NF][V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                T fs[NF], dV[NF];
#pragma unroll
                for (int j = 0; j < NF; ++j) fs[j] = cur[j][k][v];
                site_dV<T, NF>(fs, m2, lam, g2, dV);
                {
                    T Vs = T(0);
#pragma unroll
                    for (int j = 0; j < NF; ++j) {
                        const T f2 = fs[j] * fs[j];
                        Vs = fmad(f2, fmad(qlam[j], f2, hm2[j]), Vs);
                    }
                    if constexpr (NF == 2) Vs = fmad(hg2 * (fs[0] * fs[0]), fs[1] * fs[1], Vs);
                    part[NS - 1] += Vs;
                }
#pragma unroll
                for (int j = 0; j < NF; ++j) {
                    const T f = fs[j];
                    const T zm = v == 0 ? zm0[j] : cur[j][k][v - 1];
                    const T zp = v == V - 1 ? zp0[j] : cur[j][k][v + 1];
                    const T xp = nxt[j][k][v];
                    const T nb = ((prev[j][k][v] + xp) + (ym[j][v] + yp[j][v])) + (zm + zp);
                    const T F = fmad(kL, fmad(T(-6), f, nb), -(kV * dV[j]));
                    const T po = pc[j][k][v];
                    const T gx = xp - f, gy = yp[j][v] - f, gz = zp - f;
                    const T d = f - shift[j];
                    T* q5 = part + kSumsPerField * j;
                    if constexpr (RK == 1) {
                        const T Ff = cF * po;
                        const T dfn = rk_first ? Ff : fmad(rA, axc[0][j][k][v], Ff);
                        const T dpn = rk_first ? F : fmad(rA, axc[RK ? 1 : 0][j][k][v], F);
                        dfo[j][v] = dfn;
                        dpo[j][v] = dpn;
                        fnew[j][v] = fmad(rB, dfn, f);
                        pnew[j][v] = fmad(rB, dpn, po);
                        q5[0] = fmad(po, po, q5[0]);
                        q5[4] += po;
                    } else if constexpr (RK == 2) {
                        const T Ff = cF * po;
                        const T sf = rk_first ? T(0) : axc[0][j][k][v];
                        const T sp = rk_first ? T(0) : axc[1][j][k][v];
                        const T yf = rk_first ? f : y0c[0][j][k][v];
                        const T yp = rk_first ? po : y0c[RK == 2 ? 1 : 0][j][k][v];
                        fnew[j][v] = fmad(rB, Ff, fmad(rA, sf, yf));
                        pnew[j][v] = fmad(rB, F, fmad(rA, sp, yp));
                        dfo[j][v] = fmad(rD, Ff, rC * sf);
                        dpo[j][v] = fmad(rD, F, rC * sp);
                        q5[0] = fmad(po, po, q5[0]);
                        q5[4] += po;
                    } else {
                        const T p1 = fmad(kt, F, po);
                        const T ps = fmad(kb, F, po);
                        pnew[j][v] = p1;
                        q5[0] = fmad(ps, ps, q5[0]);
                        q5[4] += p1;
                    }
                    q5[1] = fmad(gz, gz, fmad(gy, gy, fmad(gx, gx, q5[1])));
                    q5[2] += d;
                    q5[3] = fmad(d, d, q5[3]);
                }
                if constexpr (NG > 0) {
                    // sum over fields of D+_a f D+_b f + D-_a f D-_b f
                    T sxx = T(0), syy = T(0), szz = T(0), sxy = T(0), sxz = T(0), syz = T(0);
#pragma unroll
                    for (int j = 0; j < NF; ++j) {
                        const T f = cur[j][k][v];
                        const T zm = v == 0 ? zm0[j] : cur[j][k][v - 1];
                        const T zp = v == V - 1 ? zp0[j] : cur[j][k][v + 1];
                        const T ax = nxt[j][k][v] - f, bx = f - prev[j][k][v];
                        const T ay = yp[j][v] - f, by = f - ym[j][v];
                        const T az = zp - f, bz = f - zm;
                        sxx = fmad(ax, ax, fmad(bx, bx, sxx));
                        syy = fmad(ay, ay, fmad(by, by, syy));
                        szz = fmad(az, az, fmad(bz, bz, szz));
                        sxy = fmad(ax, ay, fmad(bx, by, sxy));
                        sxz = fmad(ax, az, fmad(bx, bz, sxz));
                        syz = fmad(ay, az, fmad(by, bz, syz));
                    }
                    const T tr3 = (sxx + syy + szz) * static_cast<T>(1.0 / 3.0);
                    const T src[5] = {sxx - tr3, sxy, sxz, syy - tr3, syz};
#pragma unroll
                    for (int c = 0; c < NG; ++c) {
                        const int j = NF + c;
                        const T w = cur[j][k][v];
                        const T zm = v == 0 ? zm0[j] : cur[j][k][v - 1];
                        const T zp = v == V - 1 ? zp0[j] : cur[j][k][v + 1];
                        const T nb = ((prev[j][k][v] + nxt[j][k][v]) + (ym[j][v] + yp[j][v])) + (zm + zp);
                        const T F = kL * fmad(cS, src[c], fmad(T(-6), w, nb));
                        pnew[j][v] = fmad(kt, F, pc[j][k][v]);
                    }
                }
            }
            if (J.write_out) {
#pragma unroll
                for (int j = 0; j < NA; ++j) {
                    if constexpr (RK) {
                        if (nt_store) {
                            vstore_nt(fout[j] + base + yrow[k], fnew[j]);
                            vstore_nt(pout[j] + base + yrow[k], pnew[j]);
                            if (!rk_last) {
                                vstore_nt(auxf[j] + base + yrow[k], dfo[j]);
                                vstore_nt(auxp[j] + base + yrow[k], dpo[j]);
                            }
                        } else {
                            vstore(fout[j] + base + yrow[k], fnew[j]);
                            vstore(pout[j] + base + yrow[k], pnew[j]);
                            if (!rk_last) {
                                vstore(auxf[j] + base + yrow[k], dfo[j]);
                                vstore(auxp[j] + base + yrow[k], dpo[j]);
                            }
                        }
                    } else if (nt_store) {
                        vstore_nt(fout[j] + base + yrow[k], cur[j][k]);
                        vstore_nt(pout[j] + base + yrow[k], pnew[j]);
                    } else {
                        vstore(fout[j] + base + yrow[k], cur[j][k]);
                        vstore(pout[j] + base + yrow[k], pnew[j]);
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) acc[q] += static_cast<double>(part[q]);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NA; ++j)
#pragma unroll
            for (int k = 0; k < RY; ++k)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    prev[j][k][v] = cur[j][k][v];
                    cur[j][k][v] = nxt[j][k][v];
                    pc[j][k][v] = pn[j][k][v];
                    if constexpr (RK) {
                        axc[0][j][k][v] = axn[0][j][k][v];
                        axc[RK ? 1 : 0][j][k][v] = axn[RK ? 1 : 0][j][k][v];
                    }
                    if constexpr (RK == 2) {
                        y0c[0][j][k][v] = y0n[0][j][k][v];
                        y0c[RK == 2 ? 1 : 0][j][k][v] = y0n[RK == 2 ? 1 : 0][j][k][v];
                    }
                }
    };
    for (int i = 0; i < CX; i += PD) {
        static_for<0, PD>([&](auto Sc) {
            constexpr int s_ = decltype(Sc)::value;
            // body(i) takes plane i + 1: set (i + 2) mod PD and halo set
            // hs(i + 1) (i is a multiple of PD here), the one set (PD = 1)
            using Set = std::integral_constant<int, PD >= 2 ? (s_ + 2) % PD : 0>;
            using HSet = decltype(hs(std::integral_constant<int, s_ + 1>{}));
            if (i + s_ < CX) body(Set{}, HSet{}, i + s_);
        });
    }
}

// NTB: the launch bound (256, or 512 for the tall one-row-per-thread tiles,
// whose register footprint fits two waves per SIMD).
template <typename T, int NF, int RY, int HI, int PD, int RK, int NTB, int NG = 0>
__global__ __launch_bounds__(NTB) void lattice_pass(PassArgs A) {
    constexpr int NS = kSumsPerField * NF + 1;
    const int nblocks = A.nbz * A.nby * A.nbx;
    // XCD-aware order: consecutive workgroup ids land on different XCDs
    // (round robin over 8), so give XCD k a contiguous range of tiles; its
    // co-resident workgroups then share y/z halos in their L2.
    int bid = blockIdx.x;
    {
        const int per = nblocks / 8, rem = nblocks % 8;
        const int xcd = bid % 8, slot = bid / 8;
        if (per > 0) bid = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + slot;
    }
    TileJob J;
    J.in = A.in;
    J.out = A.out;
    J.N = A.N;
    J.TZ = A.TZ;
    J.TY = A.TY;
    J.CX = A.CX;
    J.z0 = (bid % A.nbz) * A.TZ;
    J.y0 = ((bid / A.nbz) % A.nby) * A.TY;
    J.x0 = (bid / (A.nbz * A.nby)) * A.CX;
    J.drift = A.drift;
    J.write_out = A.write_out;
    J.flags = A.flags;
    J.kt = A.kt;
    J.kb = A.kb;
    J.ph = &A.ph;
    J.aux = A.aux;
    J.step0 = A.y0;
    J.rkA = A.rkA;
    J.rkB = A.rkB;
    J.rkC = A.rkC;
    J.rkD = A.rkD;
    J.rkh = A.rkh;
    J.rk_first = A.rk_first;
    J.rk_last = A.rk_last;
    __shared__ Scal s_sc;
    __shared__ double tot[kMaxSums];
    J.sc = &s_sc;
    const int NT = (A.TZ / VecOf<T>::V) * (A.TY / RY);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    // (the prelude takes copies of the arguments it needs: a reference to the
    // kernel argument block would force a private copy of it)
    const Phys* php = J.ph;
    const Scal* sc_in = A.sc_in;
    Scal* sc_out = bid == 0 ? A.sc_out : nullptr;
    const double* prev_part = A.prev_partials;
    const int prev_nslots = A.prev_nslots, has_prev = A.has_prev;
    const double pkt = A.pkt, pkb = A.pkb, phn = A.phn;
    const int prev_rk = A.prev_rk;
    const double prkA = A.prkA, prkB = A.prkB, prkC = A.prkC, prkD = A.prkD, prkh = A.prkh, prkdeta = A.prkdeta;
    const int prev_rk_first = A.prev_rk_first;
    cl_observables* prev_rec = (bid == 0 && A.prev_rec >= 0) ? A.obs + A.prev_rec : nullptr;
    Scal* ssc = &s_sc;
    double* stot = tot;
    auto prelude = [=]() {
        // the scalar block travels through registers so that its load overlaps
        // those of the partial sums (2 NT >= its words: NT >= 16)
        constexpr int NW = sizeof(Scal) / 8;
        static_assert(NW <= 32, "two words per thread at the smallest workgroup");
        const unsigned long long* src = reinterpret_cast<const unsigned long long*>(sc_in);
        unsigned long long* dst = reinterpret_cast<unsigned long long*>(ssc);
        const int t = threadIdx.x;
        const unsigned long long w0 = t < NW ? src[t] : 0ull;
        const unsigned long long w1 = t + NT < NW ? src[t + NT] : 0ull;
        if (has_prev) {
            // the previous pass's scalar step, identically in every workgroup
            slots_sum<NS>(prev_part, NT, prev_nslots, stot);
            if (t < NW) dst[t] = w0;
            if (t + NT < NW) dst[t + NT] = w1;
            __syncthreads();
            if (threadIdx.x < 64) {
                if (prev_rk) finish_rk(*php, ssc, prev_rk, prev_rk_first, prkA, prkB, prkC, prkD, prkh, prkdeta, prev_rec, stot);
                else finish_pass(*php, ssc, pkt, pkb, phn, prev_rec, stot);
            }
            __syncthreads();
            if (sc_out) copy_scal(sc_out, ssc, NT);
        } else {
            if (t < NW) dst[t] = w0;
            if (t + NT < NW) dst[t + NT] = w1;
            __syncthreads();
        }
    };
    // wide workgroups keep the halo ring at depth 2 (two waves per SIMD)
    march_tile<T, NF, RY, HI, PD, RK, (NTB > 256 && PD > 2) ? 2 : PD, NG>(J, smem_raw, acc, prelude);
    block_sum<NS>(acc, NT, tot);
    if (threadIdx.x == 0)
        for (int k = 0; k < NS; ++k) A.partials[(size_t)k * nblocks + bid] = tot[k];
}

// The pending scalar step of the last pass of a sequence (one workgroup of
// the passes' NT threads, so that the sums are formed in the same order).
template <int NS>
__global__ __launch_bounds__(kMaxPassThreads) void finish_kernel(PassArgs A) {
    __shared__ Scal s_sc;
    __shared__ double tot[kMaxSums];
    copy_scal(&s_sc, A.sc_in, blockDim.x);
    slots_sum<NS>(A.prev_partials, blockDim.x, A.prev_nslots, tot);
    cl_observables* rec = A.prev_rec >= 0 ? A.obs + A.prev_rec : nullptr;
    if (threadIdx.x < 64) {
        if (A.prev_rk)
            finish_rk(A.ph, &s_sc, A.prev_rk, A.prev_rk_first, A.prkA, A.prkB, A.prkC, A.prkD, A.prkh, A.prkdeta, rec,
                      tot);
        else finish_pass(A.ph, &s_sc, A.pkt, A.pkb, A.phn, rec, tot);
    }
    __syncthreads();
    copy_scal(A.sc_out, &s_sc, blockDim.x);
}

__global__ void init_scalars_kernel(Scal* sc, double a, double b, double eta, double alpha, double dx,
                                    double s0, double s1) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    Scal s;
    s.a = a;
    s.b = b;
    s.eta = eta;
    s.cd = 0.0;
    s.kL = pow(a, 1.0 + alpha) / (dx * dx);
    s.kV = pow(a, 3.0 + alpha);
    s.a_next = a;
    s.shift[0] = s0;
    s.shift[1] = s1;
    s.mean_f[0] = s0;
    s.mean_f[1] = s1;
    s.mean_p[0] = 0.0;
    s.mean_p[1] = 0.0;
    s.pa1 = pow(a, 2.0 * alpha + 1.0);
    s.pa0 = pow(a, 2.0 * alpha);
    s.pf = pow(a, alpha - 3.0);
    s.da = 0.0;
    s.db = 0.0;
    s.nonfinite = 0;
    s.pad = 0;
    *sc = s;
}

// Streaming copy: four 16-byte vectors per thread per iteration, loads
// first, nontemporal hints on both sides -- the best one-stream-in,
// one-stream-out pattern we found, used as the measured bandwidth ceiling.
__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ in, float4* __restrict__ out,
                                                   size_t n) {
    using NV = NatVec<float>::type;
    const NV* src = reinterpret_cast<const NV*>(in);
    NV* dst = reinterpret_cast<NV*>(out);
    constexpr int U = 4;
    const size_t chunk = static_cast<size_t>(blockDim.x) * U;
    for (size_t base = static_cast<size_t>(blockIdx.x) * chunk; base < n; base += static_cast<size_t>(gridDim.x) * chunk) {
        NV v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = base + u * blockDim.x + threadIdx.x;
            if (i < n) v[u] = __builtin_nontemporal_load(src + i);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = base + u * blockDim.x + threadIdx.x;
            if (i < n) __builtin_nontemporal_store(v[u], dst + i);
        }
    }
}

hipError_t launch_copy(const void* in, void* out, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    const int blocks = 4096;
    hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, s, static_cast<const float4*>(in),
                       static_cast<float4*>(out), n);
    return hipGetLastError();
}

hipError_t launch_init_scalars(Scal* sc, double a, double b, double eta, const Phys& ph,
                               const double* shift, hipStream_t s) {
    hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, s, sc, a, b, eta, ph.alpha, ph.dx,
                       shift[0], shift[1]);
    return hipGetLastError();
}

size_t pass_lds_bytes(const Tile& t, cl_precision prec, int nf) {
    const int V = prec == CL_FP32 ? 4 : 2;
    const size_t es = prec == CL_FP32 ? 4 : 8;
    return 2ull * nf * (t.TY + 2) * (t.TZ + 2 * V) * es;
}

static bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

bool finalize_tile(Tile& t, int N, cl_precision prec) {
    const int V = prec == CL_FP32 ? 4 : 2;
    if (t.TZ <= 0 || t.TY <= 0 || t.CX <= 0 || t.RY <= 0) return false;
    if (t.TZ % V || N % t.TZ || N % t.TY || N % t.CX || t.TY % t.RY) return false;
    const int BZ = t.TZ / V;
    const int RL = t.TY / t.RY;
    t.NT = BZ * RL;
    if (t.NT > kMaxPassThreads || !is_pow2(t.NT) || !is_pow2(BZ)) return false;
    if (t.RY != 1 && t.RY != 2) return false;
    if (t.NT > 256 && t.RY != 1) return false;  // two rows per thread do not fit two waves per SIMD
    if (t.PD != 1 && t.PD != 2 && t.PD != 4) return false;
    if (t.PD == 4 && t.RY != 1) return false;  // the deep ring is built for one row per thread
    const int nhalo = 2 * BZ + 2 * t.TY;
    t.HI = (nhalo + t.NT - 1) / t.NT;
    if (t.HI > 2) return false;
    if (t.HI < 1) t.HI = 1;
    if (t.NT > 256 && t.HI != 1) return false;  // the wide instance takes one halo item per thread
    t.nbz = N / t.TZ;
    t.nby = N / t.TY;
    t.nbx = N / t.CX;
    // every workgroup of a pass reads all partial sums of the pass before it
    if (t.nblocks() > kMaxPassBlocks) return false;
    return true;
}

Tile default_tile(int N, cl_precision prec, int nf) {
    const int V = prec == CL_FP32 ? 4 : 2;
    Tile t;
    t.TZ = N < 64 * V ? N : 64 * V;
    const int BZ = t.TZ / V;
    t.RY = 1;
    int RL = 256 / BZ;
    while (RL > 1 && (RL > N || N % RL)) RL >>= 1;
    t.TY = RL * t.RY;
    if ((N / t.TZ) * (N / t.TY) > kTunedPassBlocks && N % (2 * RL) == 0) {
        t.RY = 2;  // two rows per thread: half the workgroups
        t.TY = 2 * RL;
    }
    const int tiles = (N / t.TZ) * (N / t.TY);
    t.CX = N;
    while (t.CX > 4 && tiles * (N / t.CX) < 512 && (t.CX % 2 == 0)) t.CX /= 2;
    (void)nf;
    finalize_tile(t, N, prec);
    return t;
}

// Persistent ensemble pass: workgroups take tiles of all members from one
// work counter until none is left.  Each member has its own partial slots
// (two halves, alternate passes); a work item first runs the member's scalar
// step of the previous pass from those slots in fixed order (as the solo
// pass does, so there is no cross-workgroup ticket and no device-scope
// release per item), then marches its tile and leaves its sums.  The last
// workgroup to leave resets the counters for the next pass.  MAXRY: the
// largest rows per thread among the members; with one row everywhere the
// kernel has only that path, with its halo ring at depth 2, and fits two
// waves per SIMD.
// Scalar blocks of an ensemble member inside a call: pass p starts from the
// scalars pass p - 1 used (the member's own block for p = 1 and p = 0) and
// leaves its own in scratch block p mod 2.
__device__ __forceinline__ const Scal* ens_scal_before(const EnsMember& M, int pass) {
    return pass <= 0 ? M.sc : M.scb + (pass & 1);
}

template <typename T, int NF, int MAXRY>
__global__ __launch_bounds__(256, (NF == 1 && MAXRY == 1) ? 3 : 1) void ensemble_pass(EnsArgs E) {
    constexpr int NS = kSumsPerField * NF + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double tot[kMaxSums];
    __shared__ Scal s_sc;
    __shared__ int item_s;
    const int pass = E.parity;
    for (;;) {
        __syncthreads();  // the previous tile no longer reads shared memory
        if (threadIdx.x == 0)
            item_s = static_cast<int>(__hip_atomic_fetch_add(&E.counter[0], 1u, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT));
        __syncthreads();
        const int it = item_s;
        if (it >= E.nitems) break;
        const EnsItem I = E.items[it];
        const EnsMember& M = E.members[I.member];
        const double kt = E.ckt * M.dt, kb = E.ckb * M.dt;
        TileJob J;
        J.in = M.buf[M.cur0 ^ (pass & 1)];
        J.out = M.buf[M.cur0 ^ (pass & 1) ^ 1];
        J.N = M.N;
        J.TZ = M.TZ;
        J.TY = M.TY;
        J.CX = M.CX;
        J.z0 = (I.tile % M.nbz) * M.TZ;
        J.y0 = ((I.tile / M.nbz) % M.nby) * M.TY;
        J.x0 = (I.tile / (M.nbz * M.nby)) * M.CX;
        J.drift = E.drift;
        J.write_out = E.write_out;
        J.flags = E.flags;
        J.kt = kt;
        J.kb = kb;
        J.sc = &s_sc;
        J.ph = &M.ph;
        J.aux = nullptr;
        J.step0 = nullptr;
        J.rkA = J.rkB = J.rkC = J.rkD = J.rkh = 0.0;
        J.rk_first = J.rk_last = 0;
        const size_t half = static_cast<size_t>(NS) * M.nitems;
        // the member's scalars for this pass: the previous pass's scalar step
        // (deferred), identically in every item of the member
        auto prelude = [&]() {
            copy_scal(&s_sc, ens_scal_before(M, pass - 1), 256);
            if (pass > 0) {
                slots_sum<NS>(M.partials + ((pass - 1) & 1) * half, 256, M.nitems, tot);
                __syncthreads();
                if (threadIdx.x < 64) {
                    cl_observables* rec = (I.tile == 0 && E.prev_rec >= 0)
                                              ? E.obs + (size_t)E.prev_rec * E.nmembers + I.member
                                              : nullptr;
                    finish_pass(M.ph, &s_sc, E.pckt * M.dt, E.pckb * M.dt, E.pchn * M.dt, rec, tot);
                }
                __syncthreads();
                if (I.tile == 0) copy_scal(M.scb + (pass & 1), &s_sc, 256);
            } else {
                __syncthreads();
            }
        };
        double acc[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) acc[k] = 0.0;
        if constexpr (MAXRY == 2) {
            if (M.RY == 2) march_tile<T, NF, 2, 1, 4, 0, 4, 0>(J, smem_raw, acc, prelude);
            else march_tile<T, NF, 1, 1, 4, 0, 4, 0>(J, smem_raw, acc, prelude);
        } else {
            march_tile<T, NF, 1, 1, 4, 0, 2, 0>(J, smem_raw, acc, prelude);
        }
        block_sum<NS>(acc, 256, tot);
        if (threadIdx.x == 0) {
            double* part = M.partials + (pass & 1) * half;
            for (int k = 0; k < NS; ++k) part[(size_t)k * M.nitems + I.tile] = tot[k];
        }
    }
    if (threadIdx.x == 0) {
        const unsigned done = __hip_atomic_fetch_add(&E.counter[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            __hip_atomic_store(&E.counter[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&E.counter[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// The scalar step of the last pass of an ensemble call, member blockIdx.x:
// E.parity is that pass's index, E.prev_rec / E.pck* its record and
// coefficients.
template <int NS>
__global__ __launch_bounds__(256) void ensemble_finish(EnsArgs E) {
    __shared__ Scal s_sc;
    __shared__ double tot[kMaxSums];
    const int m = blockIdx.x;
    const EnsMember& M = E.members[m];
    const int pass = E.parity;
    const size_t half = static_cast<size_t>(NS) * M.nitems;
    copy_scal(&s_sc, ens_scal_before(M, pass), 256);
    slots_sum<NS>(M.partials + (pass & 1) * half, 256, M.nitems, tot);
    __syncthreads();
    if (threadIdx.x < 64) {
        cl_observables* rec = E.prev_rec >= 0 ? E.obs + (size_t)E.prev_rec * E.nmembers + m : nullptr;
        finish_pass(M.ph, &s_sc, E.pckt * M.dt, E.pckb * M.dt, E.pchn * M.dt, rec, tot);
    }
    __syncthreads();
    copy_scal(M.sc, &s_sc, 256);
}

hipError_t launch_ensemble_finish(const EnsArgs& a, int nf, hipStream_t s) {
    if (nf == 1) hipLaunchKernelGGL((ensemble_finish<kSumsPerField + 1>), dim3(a.nmembers), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((ensemble_finish<2 * kSumsPerField + 1>), dim3(a.nmembers), dim3(256), 0, s, a);
    return hipGetLastError();
}

size_t ensemble_lds_bytes(cl_precision prec, int nf, int maxTY, int maxTZ) {
    const int V = prec == CL_FP32 ? 4 : 2;
    const size_t es = prec == CL_FP32 ? 4 : 8;
    return 2ull * nf * (maxTY + 2) * (maxTZ + 2 * V) * es;
}

template <typename T, int NF, int MAXRY>
static int grid_for(size_t lds) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ensemble_pass<T, NF, MAXRY>, 256, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu * cus;
}

template <int MAXRY>
static int grid_ry(cl_precision prec, int nf, size_t lds) {
    if (prec == CL_FP32) return nf == 1 ? grid_for<float, 1, MAXRY>(lds) : grid_for<float, 2, MAXRY>(lds);
    return nf == 1 ? grid_for<double, 1, MAXRY>(lds) : grid_for<double, 2, MAXRY>(lds);
}

int ensemble_grid(cl_precision prec, int nf, size_t lds, int maxry) {
    return maxry == 2 ? grid_ry<2>(prec, nf, lds) : grid_ry<1>(prec, nf, lds);
}

template <int MAXRY>
static hipError_t launch_ens_ry(const EnsArgs& a, cl_precision prec, int nf, int grid, hipStream_t s) {
    const size_t lds = static_cast<size_t>(a.lds_bytes);
    if (prec == CL_FP32) {
        if (nf == 1) hipLaunchKernelGGL((ensemble_pass<float, 1, MAXRY>), dim3(grid), dim3(256), lds, s, a);
        else hipLaunchKernelGGL((ensemble_pass<float, 2, MAXRY>), dim3(grid), dim3(256), lds, s, a);
    } else {
        if (nf == 1) hipLaunchKernelGGL((ensemble_pass<double, 1, MAXRY>), dim3(grid), dim3(256), lds, s, a);
        else hipLaunchKernelGGL((ensemble_pass<double, 2, MAXRY>), dim3(grid), dim3(256), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_ensemble_pass(const EnsArgs& a, cl_precision prec, int nf, int grid, int maxry, hipStream_t s) {
    return maxry == 2 ? launch_ens_ry<2>(a, prec, nf, grid, s) : launch_ens_ry<1>(a, prec, nf, grid, s);
}

void candidate_tiles(int N, cl_precision prec, int nf, Tile* out, int* count, int cap) {
    const int V = prec == CL_FP32 ? 4 : 2;
    int n = 0;
    // candidates with at most kTunedPassBlocks workgroups; all valid ones
    // (up to kMaxPassBlocks) only if there is none
    for (int wide = 0; wide < 2 && n == 0; ++wide) {
        for (int tzm : {64, 32, 16}) {
            const int TZ = N < tzm * V ? N : tzm * V;
            if (tzm != 64 && TZ == N) continue;  // same as the full-row candidate
            const int BZ = TZ / V;
            for (int RY : {1, 2})
                for (int NT : {64, 128, 256, 512}) {
                    if (NT < BZ || (NT > 256 && RY != 1)) continue;
                    const int TY = (NT / BZ) * RY;
                    if (TY > N) continue;
                    for (int CX = 2; CX <= N; CX *= 2)
                        for (int PD : {1, 2, 4}) {
                            if (CX != N && (CX < 4 || CX > 256)) continue;
                            Tile t;
                            t.TZ = TZ;
                            t.TY = TY;
                            t.CX = CX;
                            t.RY = RY;
                            t.PD = PD;
                            if (!finalize_tile(t, N, prec)) continue;
                            if (pass_lds_bytes(t, prec, nf) > 60 * 1024) continue;
                            if (t.nblocks() > kTunedPassBlocks && !wide) continue;
                            if (n < cap) out[n++] = t;
                        }
                }
        }
    }
    *count = n;
}

template <typename T, int NF, int RY, int HI, int PD, int RK, int NTB>
static hipError_t launch_t(const PassArgs& a, const Tile& t, hipStream_t s, size_t lds) {
    hipLaunchKernelGGL((lattice_pass<T, NF, RY, HI, PD, RK, NTB>), dim3(t.nblocks()), dim3(t.NT), lds, s, a);
    return hipGetLastError();
}

template <typename T, int NF, int RY, int HI, int NTB = 256>
static hipError_t launch_pd(const PassArgs& a, const Tile& t, hipStream_t s, size_t lds) {
    // Runge-Kutta stages: prefetch depth 1 or 2 (a depth-4 tile runs them at
    // 2; the wide workgroups at 1, where the stage fits two waves per SIMD)
    // classic stages (two more register sets per plane) always at depth 1
    if (a.rk == 2) return launch_t<T, NF, RY, HI, 1, 2, NTB>(a, t, s, lds);
    if (a.rk) {
        if constexpr (NTB > 256) return launch_t<T, NF, RY, HI, 1, 1, NTB>(a, t, s, lds);
        else
            return t.PD == 1 ? launch_t<T, NF, RY, HI, 1, 1, NTB>(a, t, s, lds)
                             : launch_t<T, NF, RY, HI, 2, 1, NTB>(a, t, s, lds);
    }
    if constexpr (RY == 1) {
        if (t.PD == 4) return launch_t<T, NF, RY, HI, 4, 0, NTB>(a, t, s, lds);
    }
    return t.PD == 2 ? launch_t<T, NF, RY, HI, 2, 0, NTB>(a, t, s, lds)
                     : launch_t<T, NF, RY, HI, 1, 0, NTB>(a, t, s, lds);
}

template <typename T, int NF>
static hipError_t launch_nf(const PassArgs& a, const Tile& t, hipStream_t s, size_t lds) {
    if (a.ng) {
        // with the gravitational-wave tensor: one row per thread, depth 1,
        // at most 256 threads (seven stencil arrays of registers per thread)
        if (a.ng != 5 || a.rk || t.RY != 1 || t.PD != 1 || t.NT > 256) return hipErrorInvalidValue;
        if (t.HI == 1)
            hipLaunchKernelGGL((lattice_pass<T, NF, 1, 1, 1, 0, 256, 5>), dim3(t.nblocks()), dim3(t.NT), lds, s, a);
        else
            hipLaunchKernelGGL((lattice_pass<T, NF, 1, 2, 1, 0, 256, 5>), dim3(t.nblocks()), dim3(t.NT), lds, s, a);
        return hipGetLastError();
    }
    // (more than 256 threads: one row per thread, and 2 BZ + 2 TY <= NT)
    if (t.NT > 256) return launch_pd<T, NF, 1, 1, kMaxPassThreads>(a, t, s, lds);
    if (t.RY == 1) return t.HI == 1 ? launch_pd<T, NF, 1, 1>(a, t, s, lds) : launch_pd<T, NF, 1, 2>(a, t, s, lds);
    return t.HI == 1 ? launch_pd<T, NF, 2, 1>(a, t, s, lds) : launch_pd<T, NF, 2, 2>(a, t, s, lds);
}

hipError_t launch_finish(const PassArgs& a, const Tile& t, int nf, hipStream_t s) {
    if (nf == 1) hipLaunchKernelGGL((finish_kernel<kSumsPerField + 1>), dim3(1), dim3(t.NT), 0, s, a);
    else hipLaunchKernelGGL((finish_kernel<2 * kSumsPerField + 1>), dim3(1), dim3(t.NT), 0, s, a);
    return hipGetLastError();
}

// Pass over a reduced (1+1)- or (2+1)-dimensional lattice (Sect. 3, scalar
// dynamics in 1+1 and 2+1 dimensions): the same drift, kick and lattice sums
// as lattice_pass with the Laplacian and the gradient terms summed over D
// directions.  Layout: D = 2 has N rows (x) of N values (z), array a of row x
// at (x 2NF + a) N; D = 1 is one such row.  Grid-stride over groups of V
// consecutive z values; the x-neighbour rows and the two z-neighbours of a
// group are loaded directly (the rows of neighbouring groups share them in
// the caches).  The previous pass's scalar step runs first, as in
// lattice_pass.
template <typename T, int NF, int D>
__global__ __launch_bounds__(256) void lowdim_pass(PassArgs A) {
    constexpr int NS = kSumsPerField * NF + 1;
    constexpr int V = VecOf<T>::V;
    const int NT = 256;
    const int nblocks = gridDim.x;
    const int bid = blockIdx.x;
    __shared__ Scal s_sc;
    __shared__ double tot[kMaxSums];
    {
        constexpr int NW = sizeof(Scal) / 8;
        const unsigned long long* src = reinterpret_cast<const unsigned long long*>(A.sc_in);
        unsigned long long* dst = reinterpret_cast<unsigned long long*>(&s_sc);
        const int t = threadIdx.x;
        const unsigned long long w0 = t < NW ? src[t] : 0ull;
        if (A.has_prev) slots_sum<NS>(A.prev_partials, NT, A.prev_nslots, tot);
        if (t < NW) dst[t] = w0;
        __syncthreads();
        if (A.has_prev) {
            cl_observables* rec = (bid == 0 && A.prev_rec >= 0) ? A.obs + A.prev_rec : nullptr;
            if (threadIdx.x < 64) finish_pass(A.ph, &s_sc, A.pkt, A.pkb, A.phn, rec, tot);
            __syncthreads();
            if (bid == 0) copy_scal(A.sc_out, &s_sc, NT);
        }
    }
    const T cd = A.drift ? static_cast<T>(s_sc.cd) : T(0);
    const T kL = static_cast<T>(s_sc.kL), kV = static_cast<T>(s_sc.kV);
    const T kt = static_cast<T>(A.kt), kb = static_cast<T>(A.kb);
    T shift[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) shift[j] = static_cast<T>(s_sc.shift[j]);
    const T m2[2] = {static_cast<T>(A.ph.m2[0]), static_cast<T>(A.ph.m2[1])};
    const T lam[2] = {static_cast<T>(A.ph.lam[0]), static_cast<T>(A.ph.lam[1])};
    const T g2 = static_cast<T>(A.ph.g2);
    const T hm2[2] = {T(0.5) * m2[0], T(0.5) * m2[1]};
    const T qlam[2] = {T(0.25) * lam[0], T(0.25) * lam[1]};
    const T hg2 = T(0.5) * g2;
    const int N = A.N;
    const int rows = D == 2 ? N : 1;
    const int per_row = N / V;
    const size_t rs = static_cast<size_t>(2 * NF) * N;  // row stride
    const T* in = static_cast<const T*>(A.in);
    T* out = static_cast<T*>(A.out);
    double acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    const long groups = static_cast<long>(rows) * per_row;
    for (long g = static_cast<long>(bid) * NT + threadIdx.x; g < groups; g += static_cast<long>(nblocks) * NT) {
        const int x = static_cast<int>(g / per_row);
        const int zc = static_cast<int>(g % per_row) * V;
        const size_t row = static_cast<size_t>(x) * rs;
        const int zm_i = (zc - 1 + N) % N, zp_i = (zc + V) % N;
        T part[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) part[q] = T(0);
        T f[NF][V], po[NF][V], zm0[NF], zp0[NF], xm[NF][V], xp[NF][V];
#pragma unroll
        for (int j = 0; j < NF; ++j) {
            const T* fr = in + row + static_cast<size_t>(j) * N;
            const T* pr = in + row + static_cast<size_t>(NF + j) * N;
            T fv[V];
            vload(fr + zc, fv);
            vload(pr + zc, po[j]);
#pragma unroll
            for (int v = 0; v < V; ++v) f[j][v] = fmad(cd, po[j][v], fv[v]);
            zm0[j] = fmad(cd, pr[zm_i], fr[zm_i]);
            zp0[j] = fmad(cd, pr[zp_i], fr[zp_i]);
            if constexpr (D == 2) {
                const size_t rm = static_cast<size_t>((x - 1 + N) % N) * rs, rp = static_cast<size_t>((x + 1) % N) * rs;
                T a[V], b[V], c[V], d[V];
                vload(in + rm + static_cast<size_t>(j) * N + zc, a);
                vload(in + rm + static_cast<size_t>(NF + j) * N + zc, b);
                vload(in + rp + static_cast<size_t>(j) * N + zc, c);
                vload(in + rp + static_cast<size_t>(NF + j) * N + zc, d);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    xm[j][v] = fmad(cd, b[v], a[v]);
                    xp[j][v] = fmad(cd, d[v], c[v]);
                }
            }
        }
        T pnew[NF][V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T fs[NF], dV[NF];
#pragma unroll
            for (int j = 0; j < NF; ++j) fs[j] = f[j][v];
            site_dV<T, NF>(fs, m2, lam, g2, dV);
            {
                T Vs = T(0);
#pragma unroll
                for (int j = 0; j < NF; ++j) {
                    const T f2 = fs[j] * fs[j];
                    Vs = fmad(f2, fmad(qlam[j], f2, hm2[j]), Vs);
                }
                if constexpr (NF == 2) Vs = fmad(hg2 * (fs[0] * fs[0]), fs[1] * fs[1], Vs);
                part[NS - 1] += Vs;
            }
#pragma unroll
            for (int j = 0; j < NF; ++j) {
                const T fc = fs[j];
                const T zm = v == 0 ? zm0[j] : f[j][v - 1];
                const T zp = v == V - 1 ? zp0[j] : f[j][v + 1];
                T nb = zm + zp;
                T g = (zp - fc) * (zp - fc);
                if constexpr (D == 2) {
                    nb = (xm[j][v] + xp[j][v]) + nb;
                    g = fmad(xp[j][v] - fc, xp[j][v] - fc, g);
                }
                const T F = fmad(kL, fmad(T(-2 * D), fc, nb), -(kV * dV[j]));
                const T p0 = po[j][v];
                const T p1 = fmad(kt, F, p0);
                const T ps = fmad(kb, F, p0);
                const T dd = fc - shift[j];
                T* q5 = part + kSumsPerField * j;
                pnew[j][v] = p1;
                q5[0] = fmad(ps, ps, q5[0]);
                q5[1] += g;
                q5[2] += dd;
                q5[3] = fmad(dd, dd, q5[3]);
                q5[4] += p1;
            }
        }
        if (A.write_out) {
#pragma unroll
            for (int j = 0; j < NF; ++j) {
                vstore(out + row + static_cast<size_t>(j) * N + zc, f[j]);
                vstore(out + row + static_cast<size_t>(NF + j) * N + zc, pnew[j]);
            }
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) acc[q] += static_cast<double>(part[q]);
    }
    block_sum<NS>(acc, NT, tot);
    if (threadIdx.x == 0)
        for (int k = 0; k < NS; ++k) A.partials[(size_t)k * nblocks + bid] = tot[k];
}

// (2+1)-dimensional pass as a march: a work item is V consecutive z values
// of CX consecutive rows; its thread walks the rows keeping the drifted f of
// rows x-1, x, x+1 and pi of x, x+1 in registers, with the loads of row x+2
// in flight, so a row leaves HBM about once (the z-neighbours of a group
// come from the caches).  Items are dealt z-fastest, so a wave's loads are
// contiguous.  Sums, scalar step and writes as in lowdim_pass.
template <typename T, int NF>
__global__ __launch_bounds__(256) void lowdim2_march(PassArgs A) {
    constexpr int NS = kSumsPerField * NF + 1;
    constexpr int V = VecOf<T>::V;
    const int NT = 256;
    const int nblocks = gridDim.x;
    const int bid = blockIdx.x;
    __shared__ Scal s_sc;
    __shared__ double tot[kMaxSums];
    {
        constexpr int NW = sizeof(Scal) / 8;
        const unsigned long long* src = reinterpret_cast<const unsigned long long*>(A.sc_in);
        unsigned long long* dst = reinterpret_cast<unsigned long long*>(&s_sc);
        const int t = threadIdx.x;
        const unsigned long long w0 = t < NW ? src[t] : 0ull;
        if (A.has_prev) slots_sum<NS>(A.prev_partials, NT, A.prev_nslots, tot);
        if (t < NW) dst[t] = w0;
        __syncthreads();
        if (A.has_prev) {
            cl_observables* rec = (bid == 0 && A.prev_rec >= 0) ? A.obs + A.prev_rec : nullptr;
            if (threadIdx.x < 64) finish_pass(A.ph, &s_sc, A.pkt, A.pkb, A.phn, rec, tot);
            __syncthreads();
            if (bid == 0) copy_scal(A.sc_out, &s_sc, NT);
        }
    }
    const T cd = A.drift ? static_cast<T>(s_sc.cd) : T(0);
    const T kL = static_cast<T>(s_sc.kL), kV = static_cast<T>(s_sc.kV);
    const T kt = static_cast<T>(A.kt), kb = static_cast<T>(A.kb);
    T shift[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) shift[j] = static_cast<T>(s_sc.shift[j]);
    const T m2[2] = {static_cast<T>(A.ph.m2[0]), static_cast<T>(A.ph.m2[1])};
    const T lam[2] = {static_cast<T>(A.ph.lam[0]), static_cast<T>(A.ph.lam[1])};
    const T g2 = static_cast<T>(A.ph.g2);
    const T hm2[2] = {T(0.5) * m2[0], T(0.5) * m2[1]};
    const T qlam[2] = {T(0.25) * lam[0], T(0.25) * lam[1]};
    const T hg2 = T(0.5) * g2;
    const int N = A.N, CX = A.CX;
    const int per_row = N / V;
    const size_t rs = static_cast<size_t>(2 * NF) * N;
    const T* in = static_cast<const T*>(A.in);
    T* out = static_cast<T*>(A.out);
    double acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    // raw row loads: own V values of f and pi and the two z-neighbours
    struct Row {
        T f[NF][V], p[NF][V], zmf[NF], zmp[NF], zpf[NF], zpp[NF];
    };
    auto load_row = [&](Row& R, int x, int zc) {
        const size_t row = static_cast<size_t>((x + N) % N) * rs;
        const int zm_i = (zc - 1 + N) % N, zp_i = (zc + V) % N;
#pragma unroll
        for (int j = 0; j < NF; ++j) {
            const T* fr = in + row + static_cast<size_t>(j) * N;
            const T* pr = in + row + static_cast<size_t>(NF + j) * N;
            vload(fr + zc, R.f[j]);
            vload(pr + zc, R.p[j]);
            R.zmf[j] = fr[zm_i];
            R.zmp[j] = pr[zm_i];
            R.zpf[j] = fr[zp_i];
            R.zpp[j] = pr[zp_i];
        }
    };
    // drifted f of a row (own values and the z-neighbours)
    struct Drift {
        T f[NF][V], zm[NF], zp[NF];
    };
    auto drift = [&](const Row& R, Drift& D) {
#pragma unroll
        for (int j = 0; j < NF; ++j) {
#pragma unroll
            for (int v = 0; v < V; ++v) D.f[j][v] = fmad(cd, R.p[j][v], R.f[j][v]);
            D.zm[j] = fmad(cd, R.zmp[j], R.zmf[j]);
            D.zp[j] = fmad(cd, R.zpp[j], R.zpf[j]);
        }
    };
    const long items = static_cast<long>(per_row) * (N / CX);
    for (long it = static_cast<long>(bid) * NT + threadIdx.x; it < items; it += static_cast<long>(nblocks) * NT) {
        const int zc = static_cast<int>(it % per_row) * V;
        const int x0 = static_cast<int>(it / per_row) * CX;
        Row ra, rb;
        Drift dprev, dcur, dnxt;
        T pcur[NF][V], pnxt[NF][V];
        load_row(ra, x0 - 1, zc);
        load_row(rb, x0, zc);
        drift(ra, dprev);
        drift(rb, dcur);
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < V; ++v) pcur[j][v] = rb.p[j][v];
        load_row(ra, x0 + 1, zc);
        for (int i = 0; i < CX; ++i) {
            const int x = x0 + i;
            // row x+1 arrives (ra), the loads of row x+2 go out (rb)
            drift(ra, dnxt);
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int v = 0; v < V; ++v) pnxt[j][v] = ra.p[j][v];
            if (i + 1 < CX) load_row(rb, x + 2, zc);
            T part[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) part[q] = T(0);
            T pnew[NF][V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                T fs[NF], dV[NF];
#pragma unroll
                for (int j = 0; j < NF; ++j) fs[j] = dcur.f[j][v];
                site_dV<T, NF>(fs, m2, lam, g2, dV);
                {
                    T Vs = T(0);
#pragma unroll
                    for (int j = 0; j < NF; ++j) {
                        const T f2 = fs[j] * fs[j];
                        Vs = fmad(f2, fmad(qlam[j], f2, hm2[j]), Vs);
                    }
                    if constexpr (NF == 2) Vs = fmad(hg2 * (fs[0] * fs[0]), fs[1] * fs[1], Vs);
                    part[NS - 1] += Vs;
                }
#pragma unroll
                for (int j = 0; j < NF; ++j) {
                    const T fc = fs[j];
                    const T zm = v == 0 ? dcur.zm[j] : dcur.f[j][v - 1];
                    const T zp = v == V - 1 ? dcur.zp[j] : dcur.f[j][v + 1];
                    const T xm = dprev.f[j][v], xp = dnxt.f[j][v];
                    const T nb = (xm + xp) + (zm + zp);
                    const T F = fmad(kL, fmad(T(-4), fc, nb), -(kV * dV[j]));
                    const T p0 = pcur[j][v];
                    const T p1 = fmad(kt, F, p0);
                    const T ps = fmad(kb, F, p0);
                    const T dd = fc - shift[j];
                    T* q5 = part + kSumsPerField * j;
                    pnew[j][v] = p1;
                    q5[0] = fmad(ps, ps, q5[0]);
                    q5[1] = fmad(xp - fc, xp - fc, (zp - fc) * (zp - fc)) + q5[1];
                    q5[2] += dd;
                    q5[3] = fmad(dd, dd, q5[3]);
                    q5[4] += p1;
                }
            }
            if (A.write_out) {
                const size_t row = static_cast<size_t>(x) * rs;
#pragma unroll
                for (int j = 0; j < NF; ++j) {
                    vstore(out + row + static_cast<size_t>(j) * N + zc, dcur.f[j]);
                    vstore(out + row + static_cast<size_t>(NF + j) * N + zc, pnew[j]);
                }
            }
#pragma unroll
            for (int q = 0; q < NS; ++q) acc[q] += static_cast<double>(part[q]);
            dprev = dcur;
            dcur = dnxt;
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int v = 0; v < V; ++v) pcur[j][v] = pnxt[j][v];
            ra = rb;
        }
    }
    block_sum<NS>(acc, NT, tot);
    if (threadIdx.x == 0)
        for (int k = 0; k < NS; ++k) A.partials[(size_t)k * nblocks + bid] = tot[k];
}

template <typename T, int NF>
static hipError_t launch_lowdim(const PassArgs& a, int grid, hipStream_t s) {
    if (a.dim == 1) hipLaunchKernelGGL((lowdim_pass<T, NF, 1>), dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((lowdim2_march<T, NF>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pass(const PassArgs& a, const Tile& t, cl_precision prec, hipStream_t s) {
    if (a.dim < 3) {
        // one workgroup of 256 threads per tile slot (t.NT == 256)
        if (prec == CL_FP32)
            return a.ph.nf == 1 ? launch_lowdim<float, 1>(a, t.nblocks(), s) : launch_lowdim<float, 2>(a, t.nblocks(), s);
        return a.ph.nf == 1 ? launch_lowdim<double, 1>(a, t.nblocks(), s) : launch_lowdim<double, 2>(a, t.nblocks(), s);
    }
    const size_t lds = pass_lds_bytes(t, prec, a.ph.nf + a.ng);
    if (prec == CL_FP32)
        return a.ph.nf == 1 ? launch_nf<float, 1>(a, t, s, lds) : launch_nf<float, 2>(a, t, s, lds);
    return a.ph.nf == 1 ? launch_nf<double, 1>(a, t, s, lds) : launch_nf<double, 2>(a, t, s, lds);
}

}  // namespace cl
