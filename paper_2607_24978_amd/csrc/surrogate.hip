// Learned surrogate kernels for gfx950: periodic 3x3x3 convolutions as
// implicit GEMMs on BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulate),
// their input and weight gradients, GELU, MSE, Adam, and the packing of
// lattice states into network inputs.
//
// Activations are channels-last BF16, act[site][C] with C = 8 or 32 and
// site = (x*N + y)*N + z.  Weights for a convolution are BF16
// w[o][co][ci] (o = 27 stencil offsets, (dx+1)*9 + (dy+1)*3 + (dz+1); a 28th
// all-zero offset pads the 8-channel case), so that one MFMA operand
// fragment -- 8 consecutive input channels -- is one 16-byte load.
//
// MFMA 16x16x32 lane layout (gfx950): lane l holds A[m = l%16][k = 8g..8g+7]
// and B[k = 8g..8g+7][n = l%16] with g = l/16, and gets
// D[m = 4g + r][n = l%16], r = 0..3.  Here A = weights (m = output channel),
// B = inputs (n = site), so each lane ends with 4 consecutive output
// channels of one site.
#include "surrogate.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#pragma clang fp contract(off)

namespace cl {
namespace sg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// staging registers: a plain vector type, which (unlike uint4) is promoted to VGPRs
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest, ties to even (finite values)
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __builtin_bit_cast(float, static_cast<uint32_t>(h) << 16); }

// Two FP32 values to packed BF16 (round to nearest even) with the hardware
// conversion; the same rounding as f2bf.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t cvt2(float lo, float hi) {
    const bf16x2 v = {static_cast<__bf16>(lo), static_cast<__bf16>(hi)};
    return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ uint2 cvt4(const float* f) { return make_uint2(cvt2(f[0], f[1]), cvt2(f[2], f[3])); }

// 4 BF16 values packed in two words <-> FP32
__device__ __forceinline__ uint2 pack4(const uint16_t* h) {
    return make_uint2(static_cast<uint32_t>(h[0]) | (static_cast<uint32_t>(h[1]) << 16),
                      static_cast<uint32_t>(h[2]) | (static_cast<uint32_t>(h[3]) << 16));
}
__device__ __forceinline__ void unpack4(uint2 u, float* f) {
    f[0] = __builtin_bit_cast(float, u.x << 16);
    f[1] = __builtin_bit_cast(float, u.x & 0xFFFF0000u);
    f[2] = __builtin_bit_cast(float, u.y << 16);
    f[3] = __builtin_bit_cast(float, u.y & 0xFFFF0000u);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

// GELU(z) = z Phi(z) and GELU'(z) = Phi(z) + z phi(z) (Phi, phi: standard
// normal distribution and density).  The epilogues evaluate them for every
// output, so Phi goes through erfc(x), x = |z|/sqrt 2, in the Chebyshev-fitted
// form t exp(-x^2 + P(t)), t = 1/(1 + x/2), of Press et al. (Numerical Recipes,
// erfcc; relative error below 1.2e-7 for all x >= 0, so also in the negative
// tail where Phi is small), with the hardware reciprocal and exp2: one rcp, two
// exp2 and ten FMAs instead of the library's branchy erff and expf.
__device__ __forceinline__ float phi_cdf(float z, float* dens) {
    const float x = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
    float p = 0.17087277f;
    p = fmaf(p, t, -0.82215223f);
    p = fmaf(p, t, 1.48851587f);
    p = fmaf(p, t, -1.13520398f);
    p = fmaf(p, t, 0.27886807f);
    p = fmaf(p, t, -0.18628806f);
    p = fmaf(p, t, 0.09678418f);
    p = fmaf(p, t, 0.37409196f);
    p = fmaf(p, t, 1.00002368f);
    p = fmaf(p, t, -1.26551223f);
    constexpr float kLog2e = 1.4426950408889634f;
    const float mx2 = -x * x;
    const float half_erfc = 0.5f * t * __builtin_amdgcn_exp2f((mx2 + p) * kLog2e);
    if (dens) *dens = 0.39894228040143268f * __builtin_amdgcn_exp2f(mx2 * kLog2e);
    return z >= 0.f ? 1.0f - half_erfc : half_erfc;
}

__device__ __forceinline__ float gelu(float z) { return z * phi_cdf(z, nullptr); }

__device__ __forceinline__ float gelu_grad(float z) {
    float d;
    const float c = phi_cdf(z, &d);
    return c + z * d;
}

// Periodic neighbour of site (x, y, z) at stencil offset o.
__device__ __forceinline__ int neighbour(int x, int y, int z, int o, int N) {
    const int dx = o / 9 - 1, dy = (o / 3) % 3 - 1, dz = o % 3 - 1;
    int xx = x + dx, yy = y + dy, zz = z + dz;
    xx = xx < 0 ? xx + N : (xx >= N ? xx - N : xx);
    yy = yy < 0 ? yy + N : (yy >= N ? yy - N : yy);
    zz = zz < 0 ? zz + N : (zz >= N ? zz - N : zz);
    return (xx * N + yy) * N + zz;
}

// ---------------------------------------------------------------- forward
// One wave computes 16-site groups (consecutive z in one row) x NB*16
// output channels, GPW groups at a time sharing each weight fragment.
template <int CIN, int NB, int GPW>
__global__ __launch_bounds__(256) void conv_fwd(ConvArgs a) {
    constexpr int NO = CIN == 32 ? 27 : 28;       // stencil offsets stored (padded for CIN == 8)
    constexpr int KSTEPS = CIN == 32 ? 27 : 7;    // MFMAs along K per output block
    constexpr int WSZ = NO * NB * 16 * CIN;       // bf16 elements of the weights
    extern __shared__ __align__(16) uint16_t wlds[];
    const uint16_t* __restrict__ wg = reinterpret_cast<const uint16_t*>(a.w);
    for (int i = threadIdx.x * 8; i < WSZ; i += blockDim.x * 8)
        *reinterpret_cast<uint4*>(wlds + i) = *reinterpret_cast<const uint4*>(wg + i);
    __syncthreads();

    const uint16_t* __restrict__ in = reinterpret_cast<const uint16_t*>(a.in);
    const int N = a.N;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = lane & 15;     // site within the group / B column
    const int g = lane >> 4;     // k-group
    const int ngroups = a.nsites / 16;
    const int wave_id = blockIdx.x * 4 + wave;
    const int nwaves = gridDim.x * 4;
    for (int gb = wave_id * GPW; gb < ngroups; gb += nwaves * GPW) {
        int sx[GPW], sy[GPW], sz[GPW];
        bool valid[GPW];
#pragma unroll
        for (int q = 0; q < GPW; ++q) {
            const int grp = gb + q;
            valid[q] = grp < ngroups;
            const int site = (valid[q] ? grp : 0) * 16 + n;
            sz[q] = site % N;
            sy[q] = (site / N) % N;
            sx[q] = site / (N * N);
        }
        f32x4 acc[GPW][NB];
#pragma unroll
        for (int q = 0; q < GPW; ++q)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[q][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
        for (int s = 0; s < KSTEPS; ++s) {
            // weight fragments (A) of this K step for every output block
            const int o = CIN == 32 ? s : 4 * s + g;  // stencil offset this lane's k-group reads
            const int cbase = CIN == 32 ? 8 * g : 0;  // first input channel of the k-group
            bf16x8 wa[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) wa[b] = load8(wlds + ((o * NB * 16) + b * 16 + n) * CIN + cbase);
#pragma unroll
            for (int q = 0; q < GPW; ++q) {
                bf16x8 xb = zero8();
                if (valid[q] && o < 27) xb = load8(in + static_cast<size_t>(neighbour(sx[q], sy[q], sz[q], o, N)) * CIN + cbase);
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc[q][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[b], xb, acc[q][b], 0, 0, 0);
            }
        }
        // epilogue: lane holds output channels 16b + 4g + r of site (group, n)
#pragma unroll
        for (int q = 0; q < GPW; ++q) {
            if (!valid[q]) continue;
            const size_t site = static_cast<size_t>(gb + q) * 16 + n;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int c0 = 16 * b + 4 * g;
                if (c0 >= a.cout) continue;
                float v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = acc[q][b][r] + (a.bias ? a.bias[c0 + r] : 0.f);
                if (a.z_out) *reinterpret_cast<float4*>(a.z_out + site * a.z_stride + c0) = make_float4(v[0], v[1], v[2], v[3]);
                if (a.zh_out) {
                    const uint16_t zh[4] = {f2bf(v[0]), f2bf(v[1]), f2bf(v[2]), f2bf(v[3])};
                    *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(a.zh_out) + site * a.zh_stride + c0) = pack4(zh);
                }
                if (a.a_out) {
                    uint16_t h[4];
                    if (a.gz) {
                        float zv[4];
                        unpack4(*reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(a.gz) + site * a.gz_stride + c0), zv);
#pragma unroll
                        for (int r = 0; r < 4; ++r) h[r] = f2bf(v[r] * gelu_grad(zv[r]));
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r) h[r] = f2bf(a.gelu ? gelu(v[r]) : v[r]);
                    }
                    uint2 pk;
                    pk.x = static_cast<uint32_t>(h[0]) | (static_cast<uint32_t>(h[1]) << 16);
                    pk.y = static_cast<uint32_t>(h[2]) | (static_cast<uint32_t>(h[3]) << 16);
                    *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(a.a_out) + site * a.a_stride + c0) = pk;
                }
            }
        }
    }
}

// Register-blocked forward for 32 input channels and NB 16-wide output blocks
// (the hidden layers, the last layer, and the input gradient through the
// hidden layers).  A workgroup takes 4 x-planes
// (one per wave) x RY y-rows x 16 z-sites; the input block with its halo
// (6 x (RY+2) x 18 sites x 32 channels) is staged once in LDS.  For each dx
// the wave holds the 9 (dy, dz) weight fragments of its output blocks in
// registers, and every input fragment it reads from LDS feeds the
// three output rows it is a neighbour of.
template <int RY, int NB>
__global__ __launch_bounds__(256, 2) void conv32_fwd_tiled(ConvArgs a) {
    constexpr int ZR = 18, YR = RY + 2, PL = 6;
    __shared__ __align__(16) uint16_t tin[PL * YR * ZR * 32];
    const uint16_t* __restrict__ in = reinterpret_cast<const uint16_t*>(a.in);
    const uint16_t* __restrict__ wg = reinterpret_cast<const uint16_t*>(a.w);
    const int N = a.N;
    const int nzt = N / 16, nyt = N / RY;
    int t = blockIdx.x;
    const int tz = t % nzt;
    t /= nzt;
    const int ty = t % nyt;
    const int tx = t / nyt;
    const int x0 = tx * 4, y0 = ty * RY, z0 = tz * 16;
    constexpr int CHUNKS = PL * YR * ZR * 4;  // 16-byte chunks (8 channels)
    constexpr int ITER = (CHUNKS + 255) / 256;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    // the weights of dx = 0 first: they do not depend on the block and are in
    // flight with its loads
    bf16x8 wa[9][NB];
#pragma unroll
    for (int j = 0; j < 9; ++j)
#pragma unroll
        for (int b = 0; b < NB; ++b) wa[j][b] = load8(wg + static_cast<size_t>(j * NB * 16 + 16 * b + n) * 32 + 8 * g);
    // all loads of the tile first, then all LDS stores: the loads are in
    // flight together instead of one round trip per chunk
    u32x4 v[ITER];
    if (x0 >= 1 && x0 + PL - 1 <= N && y0 >= 1 && y0 + YR - 1 <= N && z0 >= 1 && z0 + ZR - 1 <= N) {
        // no periodic image in the block: offsets from its first site
        const uint16_t* base = in + static_cast<size_t>(((x0 - 1) * N + y0 - 1) * N + z0 - 1) * 32;
#pragma unroll
        for (int k = 0; k < ITER; ++k) {
            // past the last chunk a thread re-reads it (in bounds) and stores nothing
            const int i = min(static_cast<int>(threadIdx.x) + k * 256, CHUNKS - 1);
            const int r = i >> 2, zi = r % ZR, yi = (r / ZR) % YR, pi = r / (ZR * YR);
            v[k] = *reinterpret_cast<const u32x4*>(base + ((pi * N + yi) * N + zi) * 32 + (i & 3) * 8);
        }
    } else {
#pragma unroll
        for (int k = 0; k < ITER; ++k) {
            const int i = min(static_cast<int>(threadIdx.x) + k * 256, CHUNKS - 1);
            const int c4 = i & 3;
            int r = i >> 2;
            const int zi = r % ZR;
            r /= ZR;
            const int yi = r % YR, pi = r / YR;
            int xx = x0 - 1 + pi, yy = y0 - 1 + yi, zz = z0 - 1 + zi;
            xx = xx < 0 ? xx + N : (xx >= N ? xx - N : xx);
            yy = yy < 0 ? yy + N : (yy >= N ? yy - N : yy);
            zz = zz < 0 ? zz + N : (zz >= N ? zz - N : zz);
            v[k] = *reinterpret_cast<const u32x4*>(in + static_cast<size_t>((xx * N + yy) * N + zz) * 32 + c4 * 8);
        }
    }
    __builtin_amdgcn_sched_barrier(0);  // every load issued before the first store waits
#pragma unroll
    for (int k = 0; k < ITER; ++k) {
        const int i = threadIdx.x + k * 256;
        if (i < CHUNKS) *reinterpret_cast<u32x4*>(tin + static_cast<size_t>(i) * 8) = v[k];
    }
    __syncthreads();
    uint2 zg[RY][NB];
    f32x4 acc[RY][NB];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[r][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        // the next dx's weights load during this dx's MFMAs
        bf16x8 wn[9][NB];
        if (dx < 2) {
#pragma unroll
            for (int j = 0; j < 9; ++j)
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    wn[j][b] = load8(wg + static_cast<size_t>(((dx + 1) * 9 + j) * NB * 16 + 16 * b + n) * 32 + 8 * g);
        } else if (a.gz) {
            // the pre-activations the input gradient's epilogue needs (the
            // registers of the weight prefetch are free in the last dx)
#pragma unroll
            for (int r = 0; r < RY; ++r)
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    zg[r][b] = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(a.gz) +
                                                               static_cast<size_t>(((x0 + w) * N + y0 + r) * N + z0 + n) *
                                                                   a.gz_stride + 16 * b + 4 * g);
        }
        __builtin_amdgcn_sched_barrier(0);  // keep them ahead of the MFMAs
        const uint16_t* pl = tin + (w + dx) * YR * ZR * 32;
#pragma unroll
        for (int yi = 0; yi < YR; ++yi)
#pragma unroll
            for (int dz = 0; dz < 3; ++dz) {
                const bf16x8 xb = load8(pl + (yi * ZR + n + dz) * 32 + 8 * g);
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const int r = yi - dy;  // output row fed by input row yi at this dy
                    if (r < 0 || r >= RY) continue;
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        acc[r][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[dy * 3 + dz][b], xb, acc[r][b], 0, 0, 0);
                }
            }
        if (dx < 2) {
#pragma unroll
            for (int j = 0; j < 9; ++j)
#pragma unroll
                for (int b = 0; b < NB; ++b) wa[j][b] = wn[j][b];
        }
    }
    // this lane's bias values, all loaded before the first store (which the
    // compiler cannot prove does not alias them)
    float bias[NB][4];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = 16 * b + 4 * g + q;
            bias[b][q] = (a.bias && c < a.cout) ? a.bias[c] : 0.f;
        }
    // epilogue: every output value first, then all stores back to back (each
    // from registers of its own, so that no store waits for an earlier one)
    const int x = x0 + w;
    f32x4 zf[RY][NB];
    uint2 zh[RY][NB], ao[RY][NB];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = acc[r][b][q] + bias[b][q];
            zf[r][b] = f32x4{v[0], v[1], v[2], v[3]};
            if (a.zh_out) zh[r][b] = cvt4(v);
            if (a.a_out) {
                float h[4];
                if (a.gz) {
                    float zv[4];
                    unpack4(zg[r][b], zv);
#pragma unroll
                    for (int q = 0; q < 4; ++q) h[q] = v[q] * gelu_grad(zv[q]);
                } else if (a.gelu) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) h[q] = gelu(v[q]);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) h[q] = v[q];
                }
                ao[r][b] = cvt4(h);
            }
        }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const size_t site = static_cast<size_t>((x * N + y0 + r) * N + z0 + n);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int c0 = 16 * b + 4 * g;
            if (c0 >= a.cout) continue;
            if (a.z_out) *reinterpret_cast<f32x4*>(a.z_out + site * a.z_stride + c0) = zf[r][b];
            if (a.zh_out) *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(a.zh_out) + site * a.zh_stride + c0) = zh[r][b];
            if (a.a_out) *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(a.a_out) + site * a.a_stride + c0) = ao[r][b];
        }
    }
}

// The same blocking for 8 input channels and 32 outputs (the first layer, and
// the input gradient through the last one): one K = 32 step packs the
// 8 channels of 4 stencil offsets, lane group g taking offset 4s + g, so the
// whole weight set (7 steps x 2 output blocks) stays in registers.
template <int RY>
__global__ __launch_bounds__(256, 2) void conv8_fwd_tiled(ConvArgs a) {
    constexpr int ZR = 18, YR = RY + 2, PL = 6, KS = 7;
    __shared__ __align__(16) uint16_t tin[PL * YR * ZR * 8];
    const uint16_t* __restrict__ in = reinterpret_cast<const uint16_t*>(a.in);
    const uint16_t* __restrict__ wg = reinterpret_cast<const uint16_t*>(a.w);
    const int N = a.N;
    const int nzt = N / 16, nyt = N / RY;
    int t = blockIdx.x;
    const int tz = t % nzt;
    t /= nzt;
    const int ty = t % nyt;
    const int tx = t / nyt;
    const int x0 = tx * 4, y0 = ty * RY, z0 = tz * 16;
    constexpr int SITES = PL * YR * ZR;
    constexpr int ITER = (SITES + 255) / 256;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    // the weights (they do not depend on the tile) and all loads of the tile
    // first, then all LDS stores (past the last site a thread re-reads it, in
    // bounds, and stores nothing)
    bf16x8 wa[KS][2];
    int off[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int o = 4 * s + g;  // 27 is the all-zero padding offset
#pragma unroll
        for (int b = 0; b < 2; ++b) wa[s][b] = load8(wg + static_cast<size_t>(o * 32 + 16 * b + n) * 8);
        const int dx = o / 9, dy = (o / 3) % 3, dz = o % 3;
        off[s] = o < 27 ? (((w + dx) * YR + dy) * ZR + n + dz) * 8 : -1;
    }
    u32x4 v[ITER];
#pragma unroll
    for (int k = 0; k < ITER; ++k) {
        const int i = min(static_cast<int>(threadIdx.x) + k * 256, SITES - 1);
        const int zi = i % ZR, yi = (i / ZR) % YR, pi = i / (ZR * YR);
        int xx = x0 - 1 + pi, yy = y0 - 1 + yi, zz = z0 - 1 + zi;
        xx = xx < 0 ? xx + N : (xx >= N ? xx - N : xx);
        yy = yy < 0 ? yy + N : (yy >= N ? yy - N : yy);
        zz = zz < 0 ? zz + N : (zz >= N ? zz - N : zz);
        v[k] = *reinterpret_cast<const u32x4*>(in + static_cast<size_t>((xx * N + yy) * N + zz) * 8);
    }
    // pre-activations for the input gradient's epilogue, in flight with the tile
    const int x = x0 + w;
    uint2 zg[RY][2];
    if (a.gz) {
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                zg[r][b] = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(a.gz) +
                                                           static_cast<size_t>((x * N + y0 + r) * N + z0 + n) * a.gz_stride +
                                                           16 * b + 4 * g);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < ITER; ++k) {
        const int i = static_cast<int>(threadIdx.x) + k * 256;
        if (i < SITES) *reinterpret_cast<u32x4*>(tin + static_cast<size_t>(i) * 8) = v[k];
    }
    __syncthreads();
    f32x4 acc[RY][2];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[r][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const bf16x8 xb = off[s] >= 0 ? load8(tin + off[s] + r * ZR * 8) : zero8();
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[r][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[s][b], xb, acc[r][b], 0, 0, 0);
        }
    float bias[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) bias[b][q] = a.bias ? a.bias[16 * b + 4 * g + q] : 0.f;
    // every output value first, then all stores back to back
    f32x4 zf[RY][2];
    uint2 zh[RY][2], ao[RY][2];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = acc[r][b][q] + bias[b][q];
            zf[r][b] = f32x4{v[0], v[1], v[2], v[3]};
            if (a.zh_out) zh[r][b] = cvt4(v);
            if (a.a_out) {
                float h[4];
                if (a.gz) {
                    float zv[4];
                    unpack4(zg[r][b], zv);
#pragma unroll
                    for (int q = 0; q < 4; ++q) h[q] = v[q] * gelu_grad(zv[q]);
                } else if (a.gelu) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) h[q] = gelu(v[q]);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) h[q] = v[q];
                }
                ao[r][b] = cvt4(h);
            }
        }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const size_t site = static_cast<size_t>((x * N + y0 + r) * N + z0 + n);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int c0 = 16 * b + 4 * g;
            if (a.z_out) *reinterpret_cast<f32x4*>(a.z_out + site * a.z_stride + c0) = zf[r][b];
            if (a.zh_out) *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(a.zh_out) + site * a.zh_stride + c0) = zh[r][b];
            if (a.a_out) *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(a.a_out) + site * a.a_stride + c0) = ao[r][b];
        }
    }
}

// ---------------------------------------------------------------- weight gradient
// dW[o][co][ci] = sum_n dz[n][co] x[n + o][ci],  db[co] = sum_n dz[n][co],
// as MFMA products with K = 32 sites (one 32-site z segment of a row).  The
// MFMA operands need 8 consecutive sites of one channel per lane, the
// transpose of the channels-last layout: the staging threads load 8 sites x
// 8 channels, transpose them in registers and store channel-major rows in LDS
// with 16-byte writes.
//
// A workgroup owns BY y-rows x 32 z-sites and marches along x over L planes
// (a.L).  Step t has in LDS the x plane X0 - 1 + t (BY + 2 rows, each channel
// row holding z0 - 8 .. z0 + 39 so that the z halo sits at slots 7 and 40)
// and the dz plane X0 + t; the next step's planes are loaded from global
// memory before the MFMAs and stored to the other LDS buffer after them, one
// barrier per step.  Wave w takes one (output block b, input block c) pair and
// all 27 offsets (when the layer has only two pairs, two waves share a pair,
// each over half the rows, and write separate partial sums).  It keeps the dz
// fragments of planes X0 + t - 2 .. X0 + t in registers; every x fragment it
// reads (three shifts in z built from three aligned chunks) feeds each
// (dx, dy) offset whose segment lies in its rows.
template <int CIN, int COS, int BY>
__global__ __launch_bounds__(256, 2) void conv_wgrad(WgradArgs a) {
    constexpr int NBI = CIN == 32 ? 2 : 1, NB = COS == 32 ? 2 : 1;
    constexpr int NP = NB * NBI, WPP = 4 / NP, RW = BY / WPP;
    constexpr int CINP = 16 * NBI, COUTP = 16 * NB;
    constexpr int XR = BY + 2, ZS = 48;
    constexpr int CGX = CIN / 8, CGD = COS / 8;
    constexpr int NX = XR * 4 * CGX;  // 8 x 8 transposes of x per plane
    constexpr int ND = BY * 4 * CGD;  // of dz
    constexpr int NE = XR * 2 * CGX;  // z-halo loads of x (8 channels of one site)
    static_assert(NP * WPP == 4 && RW * WPP == BY, "wave split");
    static_assert(NX + ND + NE <= 256, "staging tasks exceed the workgroup");
    __shared__ __align__(16) uint16_t xs[2][XR][CIN][ZS];
    __shared__ __align__(16) uint16_t ds[2][BY][COS][32];
    __shared__ float dbs[ND][8];
    const uint16_t* __restrict__ dz = reinterpret_cast<const uint16_t*>(a.dz);
    const uint16_t* __restrict__ x = reinterpret_cast<const uint16_t*>(a.x);
    const int N = a.N, L = a.L;
    const int nyb = N / BY, nzb = N / 32;
    int blk = blockIdx.x;
    const int y0 = (blk % nyb) * BY;
    blk /= nyb;
    const int z0 = (blk % nzb) * 32;
    const int X0 = (blk / nzb) * L;

    // staging task of this thread, fixed over the march
    const int tid = threadIdx.x;
    int kind = -1, trow = 0, tk = 0, tcg = 0;
    if (tid < NX) {
        kind = 0;
        trow = tid / (4 * CGX);
        tk = (tid / CGX) % 4;
        tcg = tid % CGX;
    } else if (tid < NX + ND) {
        const int u = tid - NX;
        kind = 1;
        trow = u / (4 * CGD);
        tk = (u / CGD) % 4;
        tcg = u % CGD;
    } else if (tid >= 256 - NE) {
        const int u = tid - (256 - NE);
        kind = 2;
        trow = u / (2 * CGX);
        tk = (u / CGX) % 2;
        tcg = u % CGX;
    }
    const int xrow_y = (y0 - 1 + trow + N) % N;  // x rows (kinds 0 and 2)
    const int zedge = tk == 0 ? (z0 - 1 + N) % N : (z0 + 32) % N;
    uint4 pre[8];
    float dbacc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) dbacc[j] = 0.f;

    // global loads of the x plane px and the dz plane qd (periodic in x)
    auto load_stage = [&](int px, int qd) {
        px = px < 0 ? px + N : (px >= N ? px - N : px);
        qd = qd >= N ? qd - N : qd;
        if (kind == 0) {
            const uint16_t* src = x + (static_cast<size_t>(px * N + xrow_y) * N + z0 + 8 * tk) * CIN + 8 * tcg;
#pragma unroll
            for (int j = 0; j < 8; ++j) pre[j] = *reinterpret_cast<const uint4*>(src + j * CIN);
        } else if (kind == 1) {
            const uint16_t* src = dz + (static_cast<size_t>(qd * N + y0 + trow) * N + z0 + 8 * tk) * COS + 8 * tcg;
#pragma unroll
            for (int j = 0; j < 8; ++j) pre[j] = *reinterpret_cast<const uint4*>(src + j * COS);
        } else if (kind == 2) {
            pre[0] = *reinterpret_cast<const uint4*>(x + (static_cast<size_t>(px * N + xrow_y) * N + zedge) * CIN + 8 * tcg);
        }
    };
    // word d of site j: channels 2d (low half) and 2d + 1 (high half)
    auto word = [&](int j, int d) -> uint32_t {
        return d == 0 ? pre[j].x : d == 1 ? pre[j].y : d == 2 ? pre[j].z : pre[j].w;
    };
    // channel ch of sites 2i, 2i + 1 packed in one word
    auto tword = [&](int ch, int i) -> uint32_t {
        const uint32_t lo = word(2 * i, ch >> 1), hi = word(2 * i + 1, ch >> 1);
        return (ch & 1) ? ((lo >> 16) | (hi & 0xFFFF0000u)) : ((lo & 0xFFFFu) | (hi << 16));
    };
    auto store_stage = [&](int buf, bool dz_counts) {
        if (kind == 0) {
#pragma unroll
            for (int ch = 0; ch < 8; ++ch)
                *reinterpret_cast<uint4*>(&xs[buf][trow][8 * tcg + ch][8 + 8 * tk]) =
                    make_uint4(tword(ch, 0), tword(ch, 1), tword(ch, 2), tword(ch, 3));
        } else if (kind == 1) {
#pragma unroll
            for (int ch = 0; ch < 8; ++ch) {
                const uint4 v = make_uint4(tword(ch, 0), tword(ch, 1), tword(ch, 2), tword(ch, 3));
                *reinterpret_cast<uint4*>(&ds[buf][trow][8 * tcg + ch][8 * tk]) = v;
                if (dz_counts) {
                    float s = 0.f;
                    const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        s += bf2f(static_cast<uint16_t>(wv[i] & 0xFFFFu));
                        s += bf2f(static_cast<uint16_t>(wv[i] >> 16));
                    }
                    dbacc[ch] += s;
                }
            }
        } else if (kind == 2) {
            const int slot = tk == 0 ? 7 : 40;
#pragma unroll
            for (int ch = 0; ch < 8; ++ch) {
                const uint32_t wd = word(0, ch >> 1);
                xs[buf][trow][8 * tcg + ch][slot] = static_cast<uint16_t>((ch & 1) ? (wd >> 16) : (wd & 0xFFFFu));
            }
        }
    };

    const int lane = tid & 63, w = tid >> 6;
    const int n = lane & 15, g = lane >> 4;
    const int pr = w % NP, h = w / NP;
    const int b = pr / NBI, c = pr % NBI;
    const bool bl = CIN == 32 || n < 8;   // lane holds a real input channel
    const bool al = COS == 32 || n < 8;   // lane holds a real dz channel
    f32x4 acc[27];
#pragma unroll
    for (int o = 0; o < 27; ++o) acc[o] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 Ap[RW], Ac[RW], An[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) Ap[r] = Ac[r] = An[r] = zero8();

    load_stage(X0 - 1, X0);
    store_stage(0, true);
    __syncthreads();
    for (int t = 0; t < L + 2; ++t) {
        const int buf = t & 1;
        const bool more = t + 1 < L + 2;
        if (more) load_stage(X0 + t, X0 + t + 1);
        const bool qvalid = t < L;  // dz plane X0 + t lies in this chunk
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            Ap[r] = Ac[r];
            Ac[r] = An[r];
            An[r] = (qvalid && al) ? load8(&ds[buf][h * RW + r][16 * b + n][8 * g]) : zero8();
        }
#pragma unroll
        for (int yi = 0; yi < RW + 2; ++yi) {
            bf16x8 bm = zero8(), b0 = zero8(), bp = zero8();
            if (bl) {
                const uint16_t* base = &xs[buf][h * RW + yi][16 * c + n][8 * g];
                const uint4 c0 = *reinterpret_cast<const uint4*>(base);
                const uint4 c1 = *reinterpret_cast<const uint4*>(base + 8);
                const uint4 c2 = *reinterpret_cast<const uint4*>(base + 16);
                // z - 1: element 7 of c0, then elements 0..6 of c1; z + 1: 1..7 of c1, 0 of c2
                const uint4 m = make_uint4((c0.w >> 16) | (c1.x << 16), (c1.x >> 16) | (c1.y << 16),
                                           (c1.y >> 16) | (c1.z << 16), (c1.z >> 16) | (c1.w << 16));
                const uint4 p = make_uint4((c1.x >> 16) | (c1.y << 16), (c1.y >> 16) | (c1.z << 16),
                                           (c1.z >> 16) | (c1.w << 16), (c1.w >> 16) | (c2.x << 16));
                bm = __builtin_bit_cast(bf16x8, m);
                b0 = __builtin_bit_cast(bf16x8, c1);
                bp = __builtin_bit_cast(bf16x8, p);
            }
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const int ry = yi - 1 - dy;  // segment row fed by this x row at dy
                if (ry < 0 || ry >= RW) continue;
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const bf16x8 af = dx == 1 ? Ap[ry] : (dx == 0 ? Ac[ry] : An[ry]);
                    const int o = 9 * (dx + 1) + 3 * (dy + 1);
                    acc[o] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bm, acc[o], 0, 0, 0);
                    acc[o + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, b0, acc[o + 1], 0, 0, 0);
                    acc[o + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bp, acc[o + 2], 0, 0, 0);
                }
            }
        }
        if (more) store_stage(buf ^ 1, t + 1 < L);
        __syncthreads();
    }

    // partial sums: [o][co][ci] then [co] for the bias, one slot per wave group
    float* out = a.partials + static_cast<size_t>(blockIdx.x * WPP + h) * a.partial_stride;
#pragma unroll
    for (int o = 0; o < 27; ++o)
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(o * COUTP + 16 * b + 4 * g + r) * CINP + 16 * c + n] = acc[o][r];
    if (kind == 1) {
#pragma unroll
        for (int j = 0; j < 8; ++j) dbs[tid - NX][j] = dbacc[j];
    }
    __syncthreads();
    if (tid < COUTP) {
        float s = 0.f;
        if (tid < COS)
            for (int u = tid / 8; u < ND; u += CGD) s += dbs[u][tid % 8];
        out[27 * COUTP * CINP + tid] = s;
        if (WPP == 2) a.partials[static_cast<size_t>(blockIdx.x * WPP + 1) * a.partial_stride + 27 * COUTP * CINP + tid] = 0.f;
    }
}

// Fixed-order sum of the partials, then scatter into the flat gradient layout
// W[co][ci][dx][dy][dz] (FP32), b[co].  A block takes 64 consecutive
// elements; its four waves sum contiguous quarters of the partials in FP64
// (16 loads in flight per lane) and are combined in wave order.
__global__ __launch_bounds__(256) void wgrad_reduce(WgradReduceArgs a) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    const int nW = 27 * a.coutp * a.cinp;
    const int q = (a.nparts + 3) / 4;
    const int p0 = w * q, p1 = min(a.nparts, p0 + q);
    double s = 0.0;
    if (e < nW + a.coutp) {
        const float* src = a.partials + e;
        const size_t st = static_cast<size_t>(a.partial_stride);
        int p = p0;
        for (; p + 16 <= p1; p += 16) {
            float v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = src[static_cast<size_t>(p + j) * st];
#pragma unroll
            for (int j = 0; j < 16; ++j) s += static_cast<double>(v[j]);
        }
        for (; p < p1; ++p) s += static_cast<double>(src[static_cast<size_t>(p) * st]);
    }
    red[w][lane] = s;
    __syncthreads();
    if (w != 0 || e >= nW + a.coutp) return;
    const double tot = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    if (e < nW) {
        const int o = e / (a.coutp * a.cinp), co = (e / a.cinp) % a.coutp, ci = e % a.cinp;
        if (co < a.cout && ci < a.cin) a.gW[(static_cast<size_t>(co) * a.cin + ci) * 27 + o] = static_cast<float>(tot);
    } else {
        const int co = e - nW;
        if (co < a.cout) a.gb[co] = static_cast<float>(tot);
    }
}

// ---------------------------------------------------------------- elementwise
// MSE against the target: y is [site][ystride] FP32 (cout channels used),
// t is [c][site] FP32; writes d loss / d y as BF16 [site][8] (channels >= cout
// zero) and per-workgroup partial sums of squares.
__global__ __launch_bounds__(256) void mse_grad(const float* __restrict__ y, int ystride, const float* __restrict__ t,
                                                int cout, size_t nsites, double scale, uint16_t* __restrict__ dy,
                                                double* __restrict__ partial) {
    __shared__ double red[256];
    double acc = 0.0;
    for (size_t s = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; s < nsites;
         s += static_cast<size_t>(gridDim.x) * blockDim.x) {
        uint16_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int c = 0; c < cout; ++c) {
            const double d = static_cast<double>(y[s * ystride + c]) - static_cast<double>(t[c * nsites + s]);
            acc += d * d;
            h[c] = f2bf(static_cast<float>(2.0 * d * scale));
        }
        uint4 u;
        __builtin_memcpy(&u, h, 16);
        *reinterpret_cast<uint4*>(dy + s * 8) = u;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam on the FP32 master parameters (Kingma and Ba 2015, bias-corrected).
__global__ void adam_update(float* __restrict__ theta, const float* __restrict__ grad, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    theta[i] = theta[i] - lr * mh / (sqrtf(vh) + eps);
}

// FP32 flat parameters of one layer -> BF16 forward weights w[o][coutp][cinp]
// (zero padded, 28th offset zero) and BF16 input-gradient weights
// wd[o'][cinp'][coutp'] = w[flip(o')][co][ci] with roles swapped, plus FP32 bias.
__global__ void prepare_layer(PrepArgs a) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = a.no_f * a.coutp * a.cinp;
    if (e < nf) {
        const int o = e / (a.coutp * a.cinp), co = (e / a.cinp) % a.coutp, ci = e % a.cinp;
        float v = 0.f;
        if (o < 27 && co < a.cout && ci < a.cin) v = a.theta[(static_cast<size_t>(co) * a.cin + ci) * 27 + o];
        a.wf[e] = f2bf(v);
    }
    const int nd = a.no_d * a.cinp_d * a.coutp_d;  // input-gradient conv: inputs = co, outputs = ci
    if (a.wd && e < nd) {
        const int o = e / (a.coutp_d * a.cinp_d), ci = (e / a.cinp_d) % a.coutp_d, co = e % a.cinp_d;
        float v = 0.f;
        if (o < 27 && co < a.cout && ci < a.cin) {
            const int of = 26 - o;  // flipped offset: (-dx, -dy, -dz)
            v = a.theta[(static_cast<size_t>(co) * a.cin + ci) * 27 + of];
        }
        a.wd[e] = f2bf(v);
    }
    if (e < a.cout) a.bias[e] = a.theta[a.bias_offset + e];
}

// Lattice state (row-interleaved, T = float or double) -> network input,
// BF16 [site][8]: channels 0..2nf-1 = (field - mean) * inv_scale, then the
// broadcast features, the rest zero.  Also optionally stores the FP32
// fluctuations [c][site] (dataset recording).
template <typename T>
__global__ void pack_state(PackArgs a) {
    const size_t s = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t N = a.N, n3 = N * N * N;
    if (s >= n3) return;
    const size_t z = s % N, row = s / N;
    const T* st = static_cast<const T*>(a.state);
    const int na = 2 * a.nf;
    uint16_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = 0; c < na; ++c) {
        const double v = static_cast<double>(st[(row * na + c) * N + z]) - a.mean[c];
        if (a.fluct_out) a.fluct_out[c * n3 + s] = static_cast<float>(v);
        if (a.fluct_sub) a.fluct_sub[c * n3 + s] = static_cast<float>(v) - a.fluct_sub_ref[c * n3 + s];
        h[c] = f2bf(static_cast<float>(v * a.inv_scale[c]));
    }
    for (int k = 0; k < a.nextra; ++k) h[na + k] = f2bf(a.extra[k]);
    if (a.x_out) {
        uint4 u;
        __builtin_memcpy(&u, h, 16);
        *reinterpret_cast<uint4*>(a.x_out + s * 8) = u;
    }
}

// Normalised dataset sample -> BF16 input [site][8] and FP32 target [c][site].
__global__ void pack_sample(SampleArgs a) {
    const size_t s = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= a.n3) return;
    uint16_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = 0; c < a.nfc; ++c) {
        h[c] = f2bf(a.fluct[c * a.n3 + s] * a.inv_in[c]);
        a.target[c * a.n3 + s] = a.incr[c * a.n3 + s] * a.inv_out[c];
    }
    for (int k = 0; k < a.nextra; ++k) h[a.nfc + k] = f2bf(a.extra[k]);
    uint4 u;
    __builtin_memcpy(&u, h, 16);
    *reinterpret_cast<uint4*>(a.x + s * 8) = u;
}

// Apply a predicted jump to the lattice state: for every field channel c,
// state = new_mean[c] + (state - old_mean[c]) + out_scale[c] * y[site][c].
template <typename T>
__global__ void unpack_jump(UnpackArgs a) {
    const size_t s = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t N = a.N, n3 = N * N * N;
    if (s >= n3) return;
    const size_t z = s % N, row = s / N;
    const T* st = static_cast<const T*>(a.state);
    T* out = static_cast<T*>(a.out);
    const int na = 2 * a.nf;
    for (int c = 0; c < na; ++c) {
        const size_t i = (row * na + c) * N + z;
        const double old = static_cast<double>(st[i]);
        const double v = a.new_mean[c] + (old - a.old_mean[c]) + a.out_scale[c] * static_cast<double>(a.y[s * a.ystride + c]);
        out[i] = static_cast<T>(v);
    }
}

// Host-side launchers ------------------------------------------------------
hipError_t launch_conv_fwd(const ConvArgs& a, int cin, int nb, int grid, hipStream_t s) {
    const int no = cin == 32 ? 27 : 28;
    const size_t lds = static_cast<size_t>(no) * nb * 16 * cin * 2;
    if (cin == 32 && a.N >= 16 && a.N % 16 == 0 && a.cout <= 16 * nb) {
        // one workgroup per 4 x 8 x 16 block of output sites
        const int tiles = (a.N / 4) * (a.N / 8) * (a.N / 16);
        if (nb == 2) hipLaunchKernelGGL((conv32_fwd_tiled<8, 2>), dim3(tiles), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((conv32_fwd_tiled<8, 1>), dim3(tiles), dim3(256), 0, s, a);
    } else if (cin == 8 && nb == 2 && a.N >= 16 && a.N % 16 == 0 && a.cout == 32) {
        const int tiles = (a.N / 4) * (a.N / 8) * (a.N / 16);
        hipLaunchKernelGGL((conv8_fwd_tiled<8>), dim3(tiles), dim3(256), 0, s, a);
    } else if (cin == 32 && nb == 2) hipLaunchKernelGGL((conv_fwd<32, 2, 4>), dim3(grid), dim3(256), lds, s, a);
    else if (cin == 32 && nb == 1) hipLaunchKernelGGL((conv_fwd<32, 1, 4>), dim3(grid), dim3(256), lds, s, a);
    else if (cin == 8 && nb == 2) hipLaunchKernelGGL((conv_fwd<8, 2, 4>), dim3(grid), dim3(256), lds, s, a);
    else if (cin == 8 && nb == 1) hipLaunchKernelGGL((conv_fwd<8, 1, 4>), dim3(grid), dim3(256), lds, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

WgradShape wgrad_shape(int N, int cin, int cout_stride) {
    // x chunks double (L halves, kept >= 8) until about 512 workgroups
    const int base = (N / 4) * (N / 32);
    int L = N;
    while (base * (N / L) < 512 && L / 2 >= 8 && N % (L / 2) == 0) L /= 2;
    const int nbi = cin == 32 ? 2 : 1, nb = cout_stride == 32 ? 2 : 1;
    WgradShape sh;
    sh.L = L;
    sh.grid = base * (N / L);
    sh.parts = sh.grid * (4 / (nb * nbi));
    sh.stride = 27 * (16 * nb) * (16 * nbi) + 16 * nb;
    return sh;
}

hipError_t launch_conv_wgrad(const WgradArgs& a, int cin, hipStream_t s) {
    if (a.N % 32 || a.L < 1 || a.N % a.L) return hipErrorInvalidValue;
    const int grid = (a.N / 4) * (a.N / 32) * (a.N / a.L);
    if (cin == 32 && a.cout_stride == 32) hipLaunchKernelGGL((conv_wgrad<32, 32, 4>), dim3(grid), dim3(256), 0, s, a);
    else if (cin == 32 && a.cout_stride == 8) hipLaunchKernelGGL((conv_wgrad<32, 8, 4>), dim3(grid), dim3(256), 0, s, a);
    else if (cin == 8 && a.cout_stride == 32) hipLaunchKernelGGL((conv_wgrad<8, 32, 4>), dim3(grid), dim3(256), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_wgrad_reduce(const WgradReduceArgs& a, hipStream_t s) {
    const int n = 27 * a.coutp * a.cinp + a.coutp;
    hipLaunchKernelGGL(wgrad_reduce, dim3((n + 63) / 64), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mse_grad(const float* y, int ystride, const float* t, int cout, size_t nsites, double scale,
                           void* dy, double* partial, int grid, hipStream_t s) {
    hipLaunchKernelGGL(mse_grad, dim3(grid), dim3(256), 0, s, y, ystride, t, cout, nsites, scale,
                       static_cast<uint16_t*>(dy), partial);
    return hipGetLastError();
}

hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_update, dim3((n + 255) / 256), dim3(256), 0, s, theta, grad, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_prepare_layer(const PrepArgs& a, hipStream_t s) {
    int n = a.no_f * a.coutp * a.cinp;
    if (a.wd) n = n > a.no_d * a.cinp_d * a.coutp_d ? n : a.no_d * a.cinp_d * a.coutp_d;
    if (n < a.cout) n = a.cout;
    hipLaunchKernelGGL(prepare_layer, dim3((n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pack_state(const PackArgs& a, bool fp32, hipStream_t s) {
    const size_t n3 = static_cast<size_t>(a.N) * a.N * a.N;
    const dim3 grid(static_cast<unsigned>((n3 + 255) / 256));
    if (fp32) hipLaunchKernelGGL(pack_state<float>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(pack_state<double>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pack_sample(const SampleArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(pack_sample, dim3(static_cast<unsigned>((a.n3 + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_unpack_jump(const UnpackArgs& a, bool fp32, hipStream_t s) {
    const size_t n3 = static_cast<size_t>(a.N) * a.N * a.N;
    const dim3 grid(static_cast<unsigned>((n3 + 255) / 256));
    if (fp32) hipLaunchKernelGGL(unpack_jump<float>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(unpack_jump<double>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sg
}  // namespace cl
