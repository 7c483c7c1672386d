// Device building blocks of the FP64 line FFT: L lines of N complex values
// (N a power of two) sit in LDS in bit-reversed order along each line, and
// the log2 N butterfly stages of an iterative decimation-in-time transform
// run over them, three stages per pass over LDS.  Used by the spectrum's
// axis passes and by the propagator's fused first and last passes.
#ifndef CL_FFT_LDS_H
#define CL_FFT_LDS_H

#include <hip/hip_runtime.h>

namespace cl {

// Lines per workgroup: L N = 2048 complex values (32 KB of LDS plus the pad
// slots) where N allows it, whole slabs below.
__host__ __device__ inline int fft_lines_per_block(int N) { return N <= 32 ? N : (N <= 2048 ? 2048 / N : 1); }

// The same for FP32 values (8 bytes): L N = 4096 (32 KB), so that a global
// access of the y and x passes still moves 16 consecutive values (128 bytes).
__host__ __device__ inline int fft_lines_per_block_f32(int N) { return N <= 64 ? N : (N <= 4096 ? 4096 / N : 1); }

// LDS slots of one line of N values: one pad slot per 16 values and one more
// per line (see slot()).
__host__ __device__ inline int fft_line_slots(int N) { return N + (N >> 4) + 1; }

// LDS bytes of a batch of L lines of N values of `vbytes` bytes each, with
// the pad slots of slot(), followed by the N / 2 twiddle factors.
__host__ __device__ inline size_t fft_lds_values(int N, int L) { return static_cast<size_t>(L) * fft_line_slots(N); }
inline size_t fft_lds_bytes(int N, int L, size_t vbytes = sizeof(double2)) {
    return (fft_lds_values(N, L) + (N / 2 > 0 ? N / 2 : 1)) * vbytes;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// LDS slot of element e of line l of a batch: one pad slot after every 16
// elements of a line, so that the bit-reversed stores (positions 16 apart)
// and the radix passes' groups fall in different banks, and one more slot
// per line, so that the y and x passes -- whose lanes store and read one
// element of 16 different lines -- do not stride the lines on one bank (the
// line stride is then odd in slots, 17 N / 16 + 1).
__device__ __forceinline__ int slot(int l, int e, int N) { return l * fft_line_slots(N) + e + (e >> 4); }

// Bit-reversed position of element e of a line of 2^logN values.
__device__ __forceinline__ int bitrev(int e, int logN) {
    return static_cast<int>(__brev(static_cast<unsigned>(e)) >> (32 - logN));
}

// S consecutive decimation-in-time stages (half-sizes m, 2m, .., 2^(S-1) m
// with m = 2^lm) in one pass over the L lines in LDS: each thread takes
// groups of 2^S elements i0 + j m (i0 = block of 2^S m + position < m),
// applies the stages' butterflies to them in registers -- the same
// butterflies, twiddles and operation order as S separate radix-2 stages --
// and writes them back.  tw[k] = exp(-2 pi i k / N), k < N / 2; inverse:
// conjugate twiddles.  V2: double2 (FP64) or float2 (FP32).
template <int S, typename V2>
__device__ __forceinline__ void fft_pass(V2* buf, const V2* __restrict__ tw, int logN, int L, int lm,
                                         bool inverse) {
    constexpr int R = 1 << S;
    const int N = 1 << logN, m = 1 << lm;
    const int groups = L << (logN - S);
    for (int t = threadIdx.x; t < groups; t += blockDim.x) {
        const int l = t >> (logN - S), q = t & ((N >> S) - 1);
        const int pos = q & (m - 1), i0 = ((q >> lm) << (lm + S)) + pos;
        V2 x[R];
#pragma unroll
        for (int j = 0; j < R; ++j) x[j] = buf[slot(l, i0 + j * m, N)];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int hk = 1 << k, sh = logN - 1 - lm - k;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (j & hk) continue;
                V2 w = tw[(pos + (j & (hk - 1)) * m) << sh];
                if (inverse) w.y = -w.y;
                const V2 u = x[j], v = cmul(x[j + hk], w);
                x[j].x = u.x + v.x;
                x[j].y = u.y + v.y;
                x[j + hk].x = u.x - v.x;
                x[j + hk].y = u.y - v.y;
            }
        }
#pragma unroll
        for (int j = 0; j < R; ++j) buf[slot(l, i0 + j * m, N)] = x[j];
    }
}

// Copies the N / 2 twiddle factors behind the batch in LDS (every thread of
// the block takes part; they are read after the caller's barrier that
// follows the batch's stores) and returns their LDS address.
template <typename V2>
__device__ __forceinline__ const V2* stage_twiddles(V2* buf, const V2* __restrict__ tw, int N, int L) {
    V2* t = buf + fft_lds_values(N, L);
    for (int i = threadIdx.x; i < N / 2; i += blockDim.x) t[i] = tw[i];
    return t;
}

// Every stage of the transform of the L bit-reversed lines in LDS, up to
// SMAX per pass (3: radix-8 passes; 4: radix-16, fewer LDS sweeps for more
// registers), a barrier after each pass (the caller has placed one after its
// stores).  The result is in natural order.
template <int SMAX = 3, typename V2>
__device__ __forceinline__ void fft_lds_stages(V2* buf, const V2* __restrict__ tw, int logN, int L, bool inverse) {
    for (int lm = 0; lm < logN;) {
        const int s = logN - lm >= SMAX ? SMAX : logN - lm;
        if (SMAX >= 4 && s == 4) fft_pass<(SMAX >= 4 ? 4 : 3)>(buf, tw, logN, L, lm, inverse);
        else if (s == 3) fft_pass<3>(buf, tw, logN, L, lm, inverse);
        else if (s == 2) fft_pass<2>(buf, tw, logN, L, lm, inverse);
        else fft_pass<1>(buf, tw, logN, L, lm, inverse);
        __syncthreads();
        lm += s;
    }
}

}  // namespace cl

#endif  // CL_FFT_LDS_H
