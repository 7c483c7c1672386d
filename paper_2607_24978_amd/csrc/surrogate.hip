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

__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest, ties to even (finite values)
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __builtin_bit_cast(float, static_cast<uint32_t>(h) << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
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
                if (a.a_out) {
                    uint16_t h[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) h[r] = f2bf(a.gelu ? gelu(v[r]) : v[r]);
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
__global__ __launch_bounds__(256) void conv32_fwd_tiled(ConvArgs a) {
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
    // all loads of the tile first, then all LDS stores: the loads are in
    // flight together instead of one round trip per chunk
    uint4 v[ITER];
#pragma unroll
    for (int k = 0; k < ITER; ++k) {
        // past the last chunk a thread re-reads it (in bounds) and stores nothing
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
        v[k] = *reinterpret_cast<const uint4*>(in + static_cast<size_t>((xx * N + yy) * N + zz) * 32 + c4 * 8);
    }
#pragma unroll
    for (int k = 0; k < ITER; ++k) {
        const int i = threadIdx.x + k * 256;
        if (i < CHUNKS) *reinterpret_cast<uint4*>(tin + static_cast<size_t>(i) * 8) = v[k];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    f32x4 acc[RY][NB];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[r][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        bf16x8 wa[9][NB];
#pragma unroll
        for (int j = 0; j < 9; ++j)
#pragma unroll
            for (int b = 0; b < NB; ++b)
                wa[j][b] = load8(wg + static_cast<size_t>((dx * 9 + j) * NB * 16 + 16 * b + n) * 32 + 8 * g);
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
    }
    const int x = x0 + w;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const size_t site = static_cast<size_t>((x * N + y0 + r) * N + z0 + n);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int c0 = 16 * b + 4 * g;
            if (c0 >= a.cout) continue;
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = acc[r][b][q] + (a.bias ? a.bias[c0 + q] : 0.f);
            if (a.z_out) *reinterpret_cast<float4*>(a.z_out + site * a.z_stride + c0) = make_float4(v[0], v[1], v[2], v[3]);
            if (a.a_out) {
                uint16_t h[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) h[q] = f2bf(a.gelu ? gelu(v[q]) : v[q]);
                uint2 pk;
                pk.x = static_cast<uint32_t>(h[0]) | (static_cast<uint32_t>(h[1]) << 16);
                pk.y = static_cast<uint32_t>(h[2]) | (static_cast<uint32_t>(h[3]) << 16);
                *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(a.a_out) + site * a.a_stride + c0) = pk;
            }
        }
    }
}

// The same blocking for 8 input channels and 32 outputs (the first layer, and
// the input gradient through the last one): one K = 32 step packs the
// 8 channels of 4 stencil offsets, lane group g taking offset 4s + g, so the
// whole weight set (7 steps x 2 output blocks) stays in registers.
template <int RY>
__global__ __launch_bounds__(256) void conv8_fwd_tiled(ConvArgs a) {
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
    // all loads of the tile first, then all LDS stores (past the last site a
    // thread re-reads it, in bounds, and stores nothing)
    uint4 v[ITER];
#pragma unroll
    for (int k = 0; k < ITER; ++k) {
        const int i = min(static_cast<int>(threadIdx.x) + k * 256, SITES - 1);
        const int zi = i % ZR, yi = (i / ZR) % YR, pi = i / (ZR * YR);
        int xx = x0 - 1 + pi, yy = y0 - 1 + yi, zz = z0 - 1 + zi;
        xx = xx < 0 ? xx + N : (xx >= N ? xx - N : xx);
        yy = yy < 0 ? yy + N : (yy >= N ? yy - N : yy);
        zz = zz < 0 ? zz + N : (zz >= N ? zz - N : zz);
        v[k] = *reinterpret_cast<const uint4*>(in + static_cast<size_t>((xx * N + yy) * N + zz) * 8);
    }
#pragma unroll
    for (int k = 0; k < ITER; ++k) {
        const int i = static_cast<int>(threadIdx.x) + k * 256;
        if (i < SITES) *reinterpret_cast<uint4*>(tin + static_cast<size_t>(i) * 8) = v[k];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
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
    const int x = x0 + w;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const size_t site = static_cast<size_t>((x * N + y0 + r) * N + z0 + n);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int c0 = 16 * b + 4 * g;
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = acc[r][b][q] + (a.bias ? a.bias[c0 + q] : 0.f);
            if (a.z_out) *reinterpret_cast<float4*>(a.z_out + site * a.z_stride + c0) = make_float4(v[0], v[1], v[2], v[3]);
            if (a.a_out) {
                uint16_t h[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) h[q] = f2bf(a.gelu ? gelu(v[q]) : v[q]);
                uint2 pk;
                pk.x = static_cast<uint32_t>(h[0]) | (static_cast<uint32_t>(h[1]) << 16);
                pk.y = static_cast<uint32_t>(h[2]) | (static_cast<uint32_t>(h[3]) << 16);
                *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(a.a_out) + site * a.a_stride + c0) = pk;
            }
        }
    }
}

// ---------------------------------------------------------------- weight gradient
// dW[o][co][ci] = sum_n dz[n][co] x[n + o][ci],  db[co] = sum_n dz[n][co].
// A workgroup takes 32-site row segments; it stages dz^T and x^T (three
// copies shifted by dz = -1, 0, +1 so that every 8-site fragment is a
// 16-byte aligned read) of the 3 x 3 neighbour rows in LDS, then MFMAs with
// K = 32 sites.  Wave w owns offsets o = w, w+4, ...; each workgroup writes
// its partial sums, reduced later in a fixed order.
template <int CIN, int NB>
__global__ __launch_bounds__(256) void conv_wgrad(WgradArgs a) {
    constexpr int NBI = CIN == 32 ? 2 : 1;         // 16-wide input-channel blocks
    constexpr int CINP = NBI * 16;
    constexpr int COUTP = NB * 16;
    constexpr int MAXO = 7;                         // offsets per wave (27 over 4 waves)
    __shared__ __align__(16) uint16_t dzT[COUTP][32];
    __shared__ __align__(16) uint16_t xT[3][CINP][9][32];
    __shared__ float dbs[COUTP];
    const uint16_t* __restrict__ dz = reinterpret_cast<const uint16_t*>(a.dz);
    const uint16_t* __restrict__ x = reinterpret_cast<const uint16_t*>(a.x);
    const int N = a.N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    f32x4 acc[MAXO][NB][NBI];
#pragma unroll
    for (int i = 0; i < MAXO; ++i)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int c = 0; c < NBI; ++c) acc[i][b][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbacc = 0.f;
    const int nseg = a.nsites / 32;
    for (int seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
        const int site0 = seg * 32;
        const int z0 = site0 % N, y = (site0 / N) % N, xx = site0 / (N * N);
        __syncthreads();
        // dz^T: thread t -> (site t/8 ... ) load 8 channels of one site
        for (int it = threadIdx.x; it < 32 * (COUTP / 8); it += 256) {
            const int s = it / (COUTP / 8), c8 = (it % (COUTP / 8)) * 8;
            uint16_t v[8];
            if (c8 < a.cout_stride) {
                const uint4 u = *reinterpret_cast<const uint4*>(dz + static_cast<size_t>(site0 + s) * a.cout_stride + c8);
                __builtin_memcpy(v, &u, 16);
            } else {
                for (int j = 0; j < 8; ++j) v[j] = 0;
            }
            for (int j = 0; j < 8; ++j) dzT[c8 + j][s] = v[j];
        }
        // x^T for the 9 rows (dx, dy) and 34 z positions, stored as 3 shifted copies
        for (int it = threadIdx.x; it < 9 * 34 * (CINP / 8); it += 256) {
            const int c8 = (it % (CINP / 8)) * 8;
            const int rest = it / (CINP / 8);
            const int zi = rest % 34, row = rest / 34;
            const int dxr = row / 3 - 1, dyr = row % 3 - 1;
            int xr = xx + dxr, yr = y + dyr, zr = z0 + zi - 1;
            xr = (xr + N) % N;
            yr = (yr + N) % N;
            zr = (zr + N) % N;
            uint16_t v[8];
            if (c8 < CIN) {
                const uint4 u = *reinterpret_cast<const uint4*>(x + static_cast<size_t>((xr * N + yr) * N + zr) * CIN + c8);
                __builtin_memcpy(v, &u, 16);
            } else {
                for (int j = 0; j < 8; ++j) v[j] = 0;
            }
            // position zi (z0 - 1 + zi) goes to copy dzs at index zi - 1 - dzs... copy k holds z0 + k - 1 + i at i
            for (int k = 0; k < 3; ++k) {
                const int i = zi - k;  // copy k: element i is z = z0 + (k - 1) + i
                if (i >= 0 && i < 32)
                    for (int j = 0; j < 8; ++j) xT[k][c8 + j][row][i] = v[j];
            }
        }
        __syncthreads();
        if (threadIdx.x < COUTP) {
            float s = 0.f;
            for (int i = 0; i < 32; ++i) s += bf2f(dzT[threadIdx.x][i]);
            dbacc += s;
        }
        // A fragments: dz^T[co = 16b + n][sites 8g..8g+7]
        bf16x8 fa[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) fa[b] = load8(&dzT[16 * b + n][8 * g]);
#pragma unroll
        for (int i = 0; i < MAXO; ++i) {
            const int o = wave + 4 * i;
            if (o >= 27) break;
            const int row = (o / 9) * 3 + (o / 3) % 3, k = o % 3;
#pragma unroll
            for (int c = 0; c < NBI; ++c) {
                const bf16x8 fb = load8(&xT[k][16 * c + n][row][8 * g]);
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc[i][b][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[b], fb, acc[i][b][c], 0, 0, 0);
            }
        }
    }
    // partial sums of this workgroup: [o][co][ci] then [co] for the bias
    float* out = a.partials + static_cast<size_t>(blockIdx.x) * a.partial_stride;
#pragma unroll
    for (int i = 0; i < MAXO; ++i) {
        const int o = wave + 4 * i;
        if (o >= 27) break;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int c = 0; c < NBI; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int co = 16 * b + 4 * g + r, ci = 16 * c + n;
                    out[(o * COUTP + co) * CINP + ci] = acc[i][b][c][r];
                }
    }
    if (threadIdx.x < COUTP) out[27 * COUTP * CINP + threadIdx.x] = dbacc;
}

// Fixed-order sum of the workgroup partials, then scatter into the flat
// gradient layout W[co][ci][dx][dy][dz] (FP32), b[co].
__global__ void wgrad_reduce(WgradReduceArgs a) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;  // element of one partial
    const int nW = 27 * a.coutp * a.cinp;
    if (e >= nW + a.coutp) return;
    double s = 0.0;
    for (int p = 0; p < a.nparts; ++p) s += static_cast<double>(a.partials[static_cast<size_t>(p) * a.partial_stride + e]);
    if (e < nW) {
        const int o = e / (a.coutp * a.cinp), co = (e / a.cinp) % a.coutp, ci = e % a.cinp;
        if (co < a.cout && ci < a.cin) a.gW[(static_cast<size_t>(co) * a.cin + ci) * 27 + o] = static_cast<float>(s);
    } else {
        const int co = e - nW;
        if (co < a.cout) a.gb[co] = static_cast<float>(s);
    }
}

// ---------------------------------------------------------------- elementwise
// d(pre-activation) = d(activation) * GELU'(z), to BF16 channels-last.
__global__ void gelu_backward(const float* __restrict__ da, const float* __restrict__ z, uint16_t* __restrict__ dz,
                              size_t n) {
    const size_t i = (static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x);
    if (i < n) dz[i] = f2bf(da[i] * gelu_grad(z[i]));
}

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
    T* st = static_cast<T*>(a.state);
    const int na = 2 * a.nf;
    for (int c = 0; c < na; ++c) {
        const size_t i = (row * na + c) * N + z;
        const double old = static_cast<double>(st[i]);
        const double v = a.new_mean[c] + (old - a.old_mean[c]) + a.out_scale[c] * static_cast<double>(a.y[s * a.ystride + c]);
        st[i] = static_cast<T>(v);
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

hipError_t launch_conv_wgrad(const WgradArgs& a, int cin, int nb, int grid, hipStream_t s) {
    if (cin == 32 && nb == 2) hipLaunchKernelGGL((conv_wgrad<32, 2>), dim3(grid), dim3(256), 0, s, a);
    else if (cin == 32 && nb == 1) hipLaunchKernelGGL((conv_wgrad<32, 1>), dim3(grid), dim3(256), 0, s, a);
    else if (cin == 8 && nb == 2) hipLaunchKernelGGL((conv_wgrad<8, 2>), dim3(grid), dim3(256), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_wgrad_reduce(const WgradReduceArgs& a, hipStream_t s) {
    const int n = 27 * a.coutp * a.cinp + a.coutp;
    hipLaunchKernelGGL(wgrad_reduce, dim3((n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gelu_backward(const float* da, const float* z, void* dz, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(gelu_backward, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, da, z,
                       static_cast<uint16_t*>(dz), n);
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
