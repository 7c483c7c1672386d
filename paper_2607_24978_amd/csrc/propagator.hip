// Linear propagation of the fluctuations over a jump, mode by mode.
//
// About a homogeneous background, the lattice equations of motion of
// Sect. 2.1 (Eq. singletEOM in program variables: f' = a^(alpha-3) pi,
// pi' = a^(1+alpha) Lap f - a^(3+alpha) dV/df) are linear in the
// fluctuations to first order, with the 7-point Laplacian diagonal in the
// lattice Fourier modes (eigenvalue -kappa^2, kappa^2 = sum_i (2/dx)^2
// sin^2(pi n_i / N)) and the mass matrix d^2V/df_i df_j at the homogeneous
// values.  Every mode then follows the integrator's own kick-drift-kick
// sub-steps with the background's (a, fbar) at each kick and drift, which
// the host takes from its FP64 background predictor.
//
// The propagation over a jump is linear with real coefficients that depend on
// a mode only through kappa^2, which is even in every index and symmetric in
// their order: one 2 nf x 2 nf transfer matrix per sorted triple of folded
// indices (about N^3 / 48) is built first, then applied to every mode.
//
// Layout: the 2 nf real channels of a site, in the order f_0..f_{nf-1},
// pi_0..pi_{nf-1}, are packed pairwise into nf complex arrays (channel 2q in
// the real and 2q+1 in the imaginary part of array q), each transformed with
// the line FFT; a mode's channels are recovered from the array at k and at
// -k (Hermitian symmetry of real fields).  The packing is fused with the
// forward z pass and the unpacking with the inverse z pass (the inverse runs
// x, y, z), so the state is read once and written once per jump.  The
// transforms run in the state's precision: FP32 lattices use float2 values,
// whose rounding (relative to the fluctuations, from which the means are
// removed) is far below that of the FP32 state itself; the transfer matrices
// and their product with a mode are FP64 for both.
#include "fft_lds.h"
#include "internal.h"

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>
#include <vector>

namespace cl {
namespace {

template <typename V2>
__device__ __forceinline__ V2 make_v2(double x, double y) {
    V2 v;
    v.x = static_cast<decltype(v.x)>(x);
    v.y = static_cast<decltype(v.y)>(y);
    return v;
}

// Element idx = l N + e of a batch of L consecutive rows starting at row0:
// channel c of site (row0 + l, z = e) in the row-interleaved state.
__device__ __forceinline__ size_t chan_index(size_t row0, int idx, int logN, int c, int na) {
    const size_t N = size_t{1} << logN;
    return ((row0 + (idx >> logN)) * na + c) * N + (idx & (N - 1));
}

// Fluctuations of channels 2q, 2q+1 of L rows -> LDS, bit-reversed along z
// (every global load of a thread before its LDS stores), forward z
// transform, out to z[q].  K = L N / 256 elements per thread (K = 1: L N <=
// 256, the rest of the threads idle).
template <typename T, typename V2, int K>
__global__ __launch_bounds__(256) void prop_pack_fftz(PropZArgs a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    V2* buf = reinterpret_cast<V2*>(lds_raw);
    const int N = a.N, logN = a.logN, L = a.L, total = L * N;
    const int q = blockIdx.y, na = 2 * a.nf;
    const size_t row0 = static_cast<size_t>(blockIdx.x) * L;
    const T* st = static_cast<const T*>(a.state);
    const double m0 = a.mean[2 * q], m1 = a.mean[2 * q + 1];
    T re[K], im[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int idx = static_cast<int>(threadIdx.x) + k * 256;
        if (K > 1 || idx < total) {
            const size_t i = chan_index(row0, idx, logN, 2 * q, na);
            re[k] = st[i];
            im[k] = st[i + N];
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int idx = static_cast<int>(threadIdx.x) + k * 256;
        if (K > 1 || idx < total) {
            const int l = idx >> logN, e = idx & (N - 1);
            buf[slot(l, bitrev(e, logN), N)] =
                make_v2<V2>(static_cast<double>(re[k]) - m0, static_cast<double>(im[k]) - m1);
        }
    }
    const V2* tws = stage_twiddles(buf, static_cast<const V2*>(a.tw), N, L);
    __syncthreads();
    fft_lds_stages(buf, tws, logN, L, false);
    V2* out = static_cast<V2*>(a.z[q]) + row0 * N;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) out[idx] = buf[slot(idx >> logN, idx & (N - 1), N)];
}

// Rows of z[q] -> LDS bit-reversed, inverse z transform, then the means
// added back and channels 2q, 2q+1 of the rows written to `out`.
template <typename T, typename V2, int K>
__global__ __launch_bounds__(256) void prop_ifftz_unpack(PropZArgs a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    V2* buf = reinterpret_cast<V2*>(lds_raw);
    const int N = a.N, logN = a.logN, L = a.L, total = L * N;
    const int q = blockIdx.y, na = 2 * a.nf;
    const size_t row0 = static_cast<size_t>(blockIdx.x) * L;
    const V2* in = static_cast<const V2*>(a.z[q]) + row0 * N;
    V2 v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int idx = static_cast<int>(threadIdx.x) + k * 256;
        if (K > 1 || idx < total) v[k] = in[idx];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int idx = static_cast<int>(threadIdx.x) + k * 256;
        if (K > 1 || idx < total) buf[slot(idx >> logN, bitrev(idx & (N - 1), logN), N)] = v[k];
    }
    const V2* tws = stage_twiddles(buf, static_cast<const V2*>(a.tw), N, L);
    __syncthreads();
    fft_lds_stages(buf, tws, logN, L, true);
    T* st = static_cast<T*>(a.out);
    const double m0 = a.mean[2 * q], m1 = a.mean[2 * q + 1];
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const V2 w = buf[slot(idx >> logN, idx & (N - 1), N)];
        const size_t i = chan_index(row0, idx, logN, 2 * q, na);
        st[i] = static_cast<T>(m0 + w.x);
        st[i + N] = static_cast<T>(m1 + w.y);
    }
}

// Index of a sorted triple i0 <= i1 <= i2 of folded mode indices (each in
// [0, N/2]): i2(i2+1)(i2+2)/6 + i1(i1+1)/2 + i0, dense in [0, C(N/2 + 3, 3)).
__device__ __forceinline__ size_t triple_index(size_t i0, size_t i1, size_t i2) {
    return i2 * (i2 + 1) * (i2 + 2) / 6 + i1 * (i1 + 1) / 2 + i0;
}

// The transfer matrix of the jump for kappa^2 = kap2[i0] + kap2[i1] +
// kap2[i2], one thread per sorted triple (a.triples lists them in index
// order, packed 10 bits each): the 2 NF x 2 NF real matrix that maps a mode's
// (f, pi) at the start to the end, built by applying every sub-step to the
// unit vectors (the same operations as on a mode's values; the columns are
// independent chains).  Layout T[row][col] with a stride of 16 per entry,
// rows and columns in the channel order f_0.., pi_0...
template <int NF, typename TT>
__global__ __launch_bounds__(256) void prop_transfer(PropModeArgs a) {
    constexpr int NC = 2 * NF;
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= a.ntriples) return;
    const uint32_t tr = a.triples[t];
    const double kap2 = a.kap2[tr & 1023u] + a.kap2[(tr >> 10) & 1023u] + a.kap2[(tr >> 20) & 1023u];
    double F[NC][NF], P[NC][NF];  // [column][field]
#pragma unroll
    for (int col = 0; col < NC; ++col)
#pragma unroll
        for (int j = 0; j < NF; ++j) {
            F[col][j] = (col == j) ? 1.0 : 0.0;
            P[col][j] = (col == NF + j) ? 1.0 : 0.0;
        }
    for (int i = 0; i < a.nsteps; ++i) {
        const PropStep& c = a.steps[i];
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const double ck = half ? c.ck1 : c.ck0;
            const double* mm = half ? c.m1 : c.m0;  // (h/2) a^(3+alpha) d2V: m00, m01, m11
            const double g0 = ck * kap2 + mm[0];
#pragma unroll
            for (int col = 0; col < NC; ++col) {
                if (NF == 1) {
                    P[col][0] -= g0 * F[col][0];
                } else {
                    const double g1 = ck * kap2 + mm[2];
                    const double f0 = F[col][0], f1 = F[col][NF - 1];
                    P[col][0] -= g0 * f0 + mm[1] * f1;
                    P[col][NF - 1] -= g1 * f1 + mm[1] * f0;
                }
                if (!half)
#pragma unroll
                    for (int j = 0; j < NF; ++j) F[col][j] += c.cd * P[col][j];
            }
        }
    }
    // stored in the lattice's precision (FP32 lattices: the matrices' rounding
    // is that of the FP32 transforms they act between), rounded once
    TT* T = static_cast<TT*>(a.table) + t * (NC * NC);
#pragma unroll
    for (int col = 0; col < NC; ++col)
#pragma unroll
        for (int j = 0; j < NF; ++j) {
            T[j * NC + col] = static_cast<TT>(F[col][j]);
            T[(NF + j) * NC + col] = static_cast<TT>(P[col][j]);
        }
}

// One thread per folded index triple (i0, i1, i2): the up to eight modes
// (+-i0, +-i1, +-i2) share kappa^2, hence the transfer matrix, and form up to
// four pairs (k, -k).  For a pair, the channels X = (A(k) + conj A(-k)) / 2,
// Y = (A(k) - conj A(-k)) / (2 i) of every packed array A (Hermitian symmetry
// of real fields) go through the matrix; then A'(k) = X' + i Y' and
// A'(-k) = conj X' + i conj Y', times the inverse transform's 1/N^3.  Every
// mode is read and written once (the planes i2 = 0 and N/2, which are their
// own mirrors, twice with the same values).  A thread issues the matrix's
// and all its pairs' loads before the first use.
template <int NF, typename V2>
__global__ __launch_bounds__(256) void prop_modes(PropModeArgs a) {
    constexpr int NC = 2 * NF;
    const int N = a.N;
    const size_t M = static_cast<size_t>(N) / 2 + 1;
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= M * M * M) return;
    const int i2 = static_cast<int>(t % M), i1 = static_cast<int>((t / M) % M), i0 = static_cast<int>(t / (M * M));
    int s0 = i0, s1 = i1, s2 = i2;  // sorted copy for the table
    if (s0 > s1) { const int x = s0; s0 = s1; s1 = x; }
    if (s1 > s2) { const int x = s1; s1 = s2; s2 = x; }
    if (s0 > s1) { const int x = s0; s0 = s1; s1 = x; }
    // the matrix in the table's precision (FP32 for FP32 lattices), 16-byte loads
    constexpr bool F32 = std::is_same<V2, float2>::value;
    using TS = typename std::conditional<F32, float, double>::type;
    using TV = typename std::conditional<F32, float4, double2>::type;
    constexpr int TPV = sizeof(TV) / sizeof(TS);  // table values per load
    const TV* T2 = reinterpret_cast<const TV*>(static_cast<const TS*>(a.table) + triple_index(s0, s1, s2) * (NC * NC));
    TV Tv[NC * NC / TPV];
#pragma unroll
    for (int e = 0; e < NC * NC / TPV; ++e) Tv[e] = T2[e];
    // representatives (sx, sy, +) of the pairs; an index equal to its mirror
    // (0 or N/2) has one sign only
    const bool x1 = i0 == 0 || 2 * i0 == N, y1 = i1 == 0 || 2 * i1 == N;
    size_t k[4], m[4];
    bool on[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int sx = p >> 1, sy = p & 1;
        on[p] = !(sx && x1) && !(sy && y1);
        const int kx = sx ? (N - i0) & (N - 1) : i0, ky = sy ? (N - i1) & (N - 1) : i1, kz = i2;
        k[p] = (static_cast<size_t>(kx) * N + ky) * N + kz;
        m[p] = (static_cast<size_t>((N - kx) & (N - 1)) * N + ((N - ky) & (N - 1))) * N + ((N - kz) & (N - 1));
    }
    V2 vk[4][NF], vm[4][NF];
#pragma unroll
    for (int p = 0; p < 4; ++p)
        if (on[p])
#pragma unroll
            for (int q = 0; q < NF; ++q) {
                vk[p][q] = static_cast<const V2*>(a.in[q])[k[p]];
                vm[p][q] = static_cast<const V2*>(a.in[q])[m[p]];
            }
    // the channel arithmetic in the table's precision: FP32 for FP32 lattices
    // (values and matrices are FP32 already; half the registers), FP64 else
    TS Tm[NC * NC];
#pragma unroll
    for (int e = 0; e < NC * NC / TPV; ++e) {
        const TS* tv = reinterpret_cast<const TS*>(&Tv[e]);
#pragma unroll
        for (int u = 0; u < TPV; ++u) Tm[TPV * e + u] = tv[u];
    }
    const TS half = TS(0.5), sc = static_cast<TS>(a.scale);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        if (!on[p]) continue;
        TS cx[NC], cy[NC];
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const TS ux = vk[p][q].x, uy = vk[p][q].y, rx = vm[p][q].x, ry = vm[p][q].y;
            cx[2 * q] = half * (ux + rx);
            cy[2 * q] = half * (uy - ry);
            cx[2 * q + 1] = half * (uy + ry);
            cy[2 * q + 1] = -half * (ux - rx);
        }
        TS ox[NC], oy[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            TS vx = TS(0), vy = TS(0);
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const TS tij = Tm[i * NC + j];
                vx += tij * cx[j];
                vy += tij * cy[j];
            }
            ox[i] = vx;
            oy[i] = vy;
        }
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const TS xx = ox[2 * q], xy = oy[2 * q], yx = ox[2 * q + 1], yy = oy[2 * q + 1];
            V2* o = static_cast<V2*>(a.out[q]);
            V2 vk2, vm2;
            vk2.x = sc * (xx - yy);
            vk2.y = sc * (xy + yx);
            vm2.x = sc * (xx + yy);
            vm2.y = sc * (yx - xy);
            o[k[p]] = vk2;
            o[m[p]] = vm2;
        }
    }
}

template <typename T, typename V2, int K>
void launch_zk(bool inverse, const PropZArgs& a, dim3 grid, size_t lds, hipStream_t s) {
    if (inverse) hipLaunchKernelGGL((prop_ifftz_unpack<T, V2, K>), grid, dim3(256), lds, s, a);
    else hipLaunchKernelGGL((prop_pack_fftz<T, V2, K>), grid, dim3(256), lds, s, a);
}

// K = L N / 256 exactly (L N a power of two), or 1 for L N <= 256
template <typename T, typename V2>
hipError_t launch_z(bool inverse, const PropZArgs& a, hipStream_t s) {
    const int total = a.L * a.N;
    const dim3 grid(static_cast<unsigned>(a.N) * a.N / a.L, a.nf);
    const size_t lds = fft_lds_bytes(a.N, a.L, sizeof(V2));
    switch (total) {
        case 2048: launch_zk<T, V2, 8>(inverse, a, grid, lds, s); break;
        case 1024: launch_zk<T, V2, 4>(inverse, a, grid, lds, s); break;
        case 512: launch_zk<T, V2, 2>(inverse, a, grid, lds, s); break;
        default: launch_zk<T, V2, 1>(inverse, a, grid, lds, s); break;
    }
    return hipGetLastError();
}

// Completes the z-pass shape (log2 N, rows per workgroup) and checks it: N a
// power of two <= 1024, L N <= 2048 elements (K <= 8 per thread).  z lines
// are contiguous, so both precisions take 2048-element batches (for float2
// half the LDS of the axis passes' batches, more workgroups per CU: measured
// faster than 4096 at 256^3).
bool z_shape(PropZArgs& a) {
    if (a.N < 2 || a.N > 1024 || (a.N & (a.N - 1)) != 0 || (a.nf != 1 && a.nf != 2)) return false;
    a.logN = 0;
    while ((1 << a.logN) < a.N) ++a.logN;
    a.L = fft_lines_per_block(a.N);
    return a.L * a.N <= 2048;
}

}  // namespace

hipError_t launch_prop_pack_fftz(const PropZArgs& args, bool fp32, hipStream_t s) {
    PropZArgs a = args;
    if (!z_shape(a)) return hipErrorInvalidValue;
    return fp32 ? launch_z<float, float2>(false, a, s) : launch_z<double, double2>(false, a, s);
}

hipError_t launch_prop_ifftz_unpack(const PropZArgs& args, bool fp32, hipStream_t s) {
    PropZArgs a = args;
    if (!z_shape(a)) return hipErrorInvalidValue;
    return fp32 ? launch_z<float, float2>(true, a, s) : launch_z<double, double2>(true, a, s);
}

size_t prop_table_entries(int N) {
    const size_t M = static_cast<size_t>(N) / 2 + 1;
    return M * (M + 1) * (M + 2) / 6;
}

std::vector<uint32_t> prop_triples(int N) {
    const uint32_t M = static_cast<uint32_t>(N) / 2 + 1;
    std::vector<uint32_t> out;
    out.reserve(prop_table_entries(N));
    for (uint32_t c = 0; c < M; ++c)
        for (uint32_t b = 0; b <= c; ++b)
            for (uint32_t a = 0; a <= b; ++a) out.push_back(a | (b << 10) | (c << 20));
    return out;
}

hipError_t launch_prop_modes(const PropModeArgs& a, bool fp32, hipStream_t s) {
    if (a.nf != 1 && a.nf != 2) return hipErrorInvalidValue;
    const unsigned tgrid = static_cast<unsigned>((a.ntriples + 255) / 256);
    const size_t M = a.N / 2 + 1;
    const unsigned mgrid = static_cast<unsigned>((M * M * M + 255) / 256);
    if (a.nf == 1) {
        if (fp32) {
            hipLaunchKernelGGL((prop_transfer<1, float>), dim3(tgrid), dim3(256), 0, s, a);
            hipLaunchKernelGGL((prop_modes<1, float2>), dim3(mgrid), dim3(256), 0, s, a);
        } else {
            hipLaunchKernelGGL((prop_transfer<1, double>), dim3(tgrid), dim3(256), 0, s, a);
            hipLaunchKernelGGL((prop_modes<1, double2>), dim3(mgrid), dim3(256), 0, s, a);
        }
    } else {
        if (fp32) {
            hipLaunchKernelGGL((prop_transfer<2, float>), dim3(tgrid), dim3(256), 0, s, a);
            hipLaunchKernelGGL((prop_modes<2, float2>), dim3(mgrid), dim3(256), 0, s, a);
        } else {
            hipLaunchKernelGGL((prop_transfer<2, double>), dim3(tgrid), dim3(256), 0, s, a);
            hipLaunchKernelGGL((prop_modes<2, double2>), dim3(mgrid), dim3(256), 0, s, a);
        }
    }
    return hipGetLastError();
}

}  // namespace cl
