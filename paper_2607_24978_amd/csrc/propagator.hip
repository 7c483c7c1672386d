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
// -k (Hermitian symmetry of real fields).
#include "internal.h"

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

namespace cl {
namespace {

// state channel c of site (row, z) in the row-interleaved layout
template <typename T>
__device__ __forceinline__ size_t chan_index(size_t row, int c, int na, size_t N, size_t z) {
    return (row * na + c) * N + z;
}

template <typename T>
__global__ void prop_pack(PropPackArgs a) {
    const size_t N = a.N, n3 = N * N * N;
    const int na = 2 * a.nf;
    const T* st = static_cast<const T*>(a.state);
    for (size_t s = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; s < n3;
         s += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const size_t z = s % N, row = s / N;
        for (int q = 0; q < a.nf; ++q) {
            const double re = static_cast<double>(st[chan_index<T>(row, 2 * q, na, N, z)]) - a.mean[2 * q];
            const double im = static_cast<double>(st[chan_index<T>(row, 2 * q + 1, na, N, z)]) - a.mean[2 * q + 1];
            a.z[q][s] = make_double2(re, im);
        }
    }
}

// Index of a sorted triple i0 <= i1 <= i2 of folded mode indices (each in
// [0, N/2]): i2(i2+1)(i2+2)/6 + i1(i1+1)/2 + i0, dense in [0, C(N/2 + 3, 3)).
__device__ __forceinline__ size_t triple_index(size_t i0, size_t i1, size_t i2) {
    return i2 * (i2 + 1) * (i2 + 2) / 6 + i1 * (i1 + 1) / 2 + i0;
}

// The transfer matrix of the jump for kappa^2 = kap2[i0] + kap2[i1] +
// kap2[i2], one thread per sorted triple (a.triples lists them in index
// order, packed 10 bits each): the 2 nf x 2 nf real matrix that maps a mode's
// (f, pi) at the start to the end, built by applying every sub-step to the
// unit vectors (the same operations as on a mode's values; the columns are
// independent chains).  Layout T[row][col], rows and columns in the channel
// order f_0.., pi_0...
__global__ void prop_transfer(PropModeArgs a) {
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= a.ntriples) return;
    const uint32_t tr = a.triples[t];
    const double kap2 = a.kap2[tr & 1023u] + a.kap2[(tr >> 10) & 1023u] + a.kap2[(tr >> 20) & 1023u];
    const int nf = a.nf, nc = 2 * nf;
    double F[4][2], P[4][2];  // [column][field]
#pragma unroll
    for (int col = 0; col < 4; ++col)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            F[col][j] = (col < nf && j == col) ? 1.0 : 0.0;
            P[col][j] = (col >= nf && j == col - nf) ? 1.0 : 0.0;
        }
    for (int i = 0; i < a.nsteps; ++i) {
        const PropStep& c = a.steps[i];
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const double ck = half ? c.ck1 : c.ck0;
            const double* mm = half ? c.m1 : c.m0;  // (h/2) a^(3+alpha) d2V: m00, m01, m11
            const double g0 = ck * kap2 + mm[0], g1 = ck * kap2 + mm[2];
#pragma unroll
            for (int col = 0; col < 4; ++col) {
                const double f0 = F[col][0], f1 = F[col][1];
                if (nf == 1) {
                    P[col][0] -= g0 * f0;
                } else {
                    P[col][0] -= g0 * f0 + mm[1] * f1;
                    P[col][1] -= g1 * f1 + mm[1] * f0;
                }
                if (!half) {
                    F[col][0] += c.cd * P[col][0];
                    F[col][1] += c.cd * P[col][1];
                }
            }
        }
    }
    double* T = a.table + t * 16;
    for (int col = 0; col < nc; ++col)
        for (int j = 0; j < nf; ++j) {
            T[j * nc + col] = F[col][j];
            T[(nf + j) * nc + col] = P[col][j];
        }
}

// One thread per folded index triple (i0, i1, i2): the up to eight modes
// (+-i0, +-i1, +-i2) share kappa^2, hence the transfer matrix, and form up to
// four pairs (k, -k).  For a pair, the channels X = (A(k) + conj A(-k)) / 2,
// Y = (A(k) - conj A(-k)) / (2 i) of every packed array A (Hermitian symmetry
// of real fields) go through the matrix; then A'(k) = X' + i Y' and
// A'(-k) = conj X' + i conj Y', times the inverse transform's 1/N^3.  Every
// mode is read and written once.
__global__ void prop_modes(PropModeArgs a) {
    const int N = a.N, nf = a.nf, nc = 2 * nf;
    const size_t M = static_cast<size_t>(N) / 2 + 1;
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= M * M * M) return;
    const int i2 = static_cast<int>(t % M), i1 = static_cast<int>((t / M) % M), i0 = static_cast<int>(t / (M * M));
    int s0 = i0, s1 = i1, s2 = i2;  // sorted copy for the table
    if (s0 > s1) { const int x = s0; s0 = s1; s1 = x; }
    if (s1 > s2) { const int x = s1; s1 = s2; s2 = x; }
    if (s0 > s1) { const int x = s0; s0 = s1; s1 = x; }
    const double* T = a.table + triple_index(s0, s1, s2) * 16;
    double Tm[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) Tm[e] = e < nc * nc ? T[e] : 0.0;
    // representatives (sx, sy, +) of the pairs; an index equal to its mirror
    // (0 or N/2) has one sign only
    const bool x1 = i0 == 0 || 2 * i0 == N, y1 = i1 == 0 || 2 * i1 == N;
    for (int sx = 0; sx < 2; ++sx) {
        if (sx && x1) break;
        for (int sy = 0; sy < 2; ++sy) {
            if (sy && y1) break;
            const int kx = sx ? (N - i0) & (N - 1) : i0, ky = sy ? (N - i1) & (N - 1) : i1, kz = i2;
            const size_t k = (static_cast<size_t>(kx) * N + ky) * N + kz;
            const size_t m = (static_cast<size_t>((N - kx) & (N - 1)) * N + ((N - ky) & (N - 1))) * N + ((N - kz) & (N - 1));
            double2 ch[4];
            for (int q = 0; q < nf; ++q) {
                const double2 p = a.in[q][k], r = a.in[q][m];
                ch[2 * q] = make_double2(0.5 * (p.x + r.x), 0.5 * (p.y - r.y));
                ch[2 * q + 1] = make_double2(0.5 * (p.y + r.y), -0.5 * (p.x - r.x));
            }
            double2 out[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                double2 v = make_double2(0.0, 0.0);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (i >= nc || j >= nc) continue;
                    const double tij = Tm[i * nc + j];
                    v.x += tij * ch[j].x;
                    v.y += tij * ch[j].y;
                }
                out[i] = v;
            }
            for (int q = 0; q < nf; ++q) {
                const double2 x = out[2 * q], y = out[2 * q + 1];
                a.out[q][k] = make_double2(a.scale * (x.x - y.y), a.scale * (x.y + y.x));
                a.out[q][m] = make_double2(a.scale * (x.x + y.y), a.scale * (y.x - x.y));
            }
        }
    }
}

template <typename T>
__global__ void prop_unpack(PropUnpackArgs a) {
    const size_t N = a.N, n3 = N * N * N;
    const int na = 2 * a.nf;
    T* st = static_cast<T*>(a.state);
    for (size_t s = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; s < n3;
         s += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const size_t z = s % N, row = s / N;
        for (int q = 0; q < a.nf; ++q) {
            const double2 v = a.z[q][s];
            st[chan_index<T>(row, 2 * q, na, N, z)] = static_cast<T>(a.mean[2 * q] + v.x);
            st[chan_index<T>(row, 2 * q + 1, na, N, z)] = static_cast<T>(a.mean[2 * q + 1] + v.y);
        }
    }
}

unsigned grid_for(size_t n) { return static_cast<unsigned>(n < 256 * 8192 ? (n + 255) / 256 : 8192); }

}  // namespace

hipError_t launch_prop_pack(const PropPackArgs& a, bool fp32, hipStream_t s) {
    const size_t n3 = static_cast<size_t>(a.N) * a.N * a.N;
    if (fp32) hipLaunchKernelGGL(prop_pack<float>, dim3(grid_for(n3)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(prop_pack<double>, dim3(grid_for(n3)), dim3(256), 0, s, a);
    return hipGetLastError();
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

hipError_t launch_prop_modes(const PropModeArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(prop_transfer, dim3(static_cast<unsigned>((a.ntriples + 255) / 256)), dim3(256), 0, s, a);
    const size_t M = a.N / 2 + 1;
    hipLaunchKernelGGL(prop_modes, dim3(static_cast<unsigned>((M * M * M + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_prop_unpack(const PropUnpackArgs& a, bool fp32, hipStream_t s) {
    const size_t n3 = static_cast<size_t>(a.N) * a.N * a.N;
    if (fp32) hipLaunchKernelGGL(prop_unpack<float>, dim3(grid_for(n3)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(prop_unpack<double>, dim3(grid_for(n3)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace cl
