// Power spectrum of one lattice array (Sect. 4.3, Eqs. discretePSaux,
// discretePST2): the forward DFT f(n~) = sum_n exp(-2 pi i n~.n / N) f(n) in
// FP64 as three passes of line transforms (z, then y, then x), and
// the binning of |f(n~)|^2 into centred spherical shells of |n~|.  The
// extraction of the array from the state is fused with the z pass and the
// binning with the x pass, so the complex array is swept three times.
//
// Line transform: a workgroup stages L lines of N complex values in LDS
// (L N = 2048, 32 KB, for 64 <= N <= 2048), loaded in bit-reversed order,
// and runs the log2 N butterfly stages of an iterative decimation-in-time
// FFT, three stages per pass over LDS (radix-8 passes; radix-16 for FP32
// values) with a barrier between passes (fft_lds.h).  For the z axis the L
// lines are consecutive rows; for the y and x axes they are L consecutive z
// positions of one y-z (x-z) slab, so every global access moves L
// consecutive complex values.
#include "fft_lds.h"
#include "internal.h"

#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>

namespace cl {

template <typename V2>
struct FftArgs {
    V2* data;            // N^2 P complex, site (x N + y) P + z
    const V2* tw;        // exp(-2 pi i k / N), k < N / 2
    int N, logN, L, logL, axis;  // axis 0: z, 1: y, 2: x (N, L powers of two)
    int P, nzb;          // stored z per (x, y) (N, or fewer for the y and x passes over a half
                         // spectrum along z), batches of L z per slab (P / L)
    int inverse;         // 1: exp(+2 pi i k / N) (conjugate twiddles), no scaling
};

// Global index of element e of line l of batch b: for the y and x axes the
// batch fixes the outer coordinate and the first z of its L lines
// (`outer`, `z0`, formed once per workgroup).
template <typename V2>
__device__ __forceinline__ size_t line_elem(const FftArgs<V2>& a, int b, size_t outer, size_t z0, int l, int e) {
    const size_t N = a.N, P = a.P;
    if (a.axis == 0) return (static_cast<size_t>(b) * a.L + l) * N + e;  // P = N
    const size_t z = z0 + l;
    if (a.axis == 1) return (outer * N + e) * P + z;      // x = outer, y = e
    return (static_cast<size_t>(e) * N + outer) * P + z;  // x = e, y = outer
}

// Element idx of a batch -> (line l, element e): the z axis takes whole
// lines in turn, the y and x axes the L lines' element e side by side.
template <typename V2>
__device__ __forceinline__ void line_split(const FftArgs<V2>& a, int idx, int& l, int& e) {
    if (a.axis == 0) {
        l = idx >> a.logN;
        e = idx & (a.N - 1);
    } else {
        e = idx >> a.logL;
        l = idx & (a.L - 1);
    }
}

// A batch of K * 256 elements into LDS, bit-reversed along each line: every
// global load of a thread first, then its LDS stores.
template <int K, typename V2>
__device__ __forceinline__ void load_lines(const FftArgs<V2>& a, int b, size_t outer, size_t z0, V2* buf) {
    V2 v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int l, e;
        line_split(a, static_cast<int>(threadIdx.x) + k * 256, l, e);
        v[k] = a.data[line_elem(a, b, outer, z0, l, e)];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int l, e;
        line_split(a, static_cast<int>(threadIdx.x) + k * 256, l, e);
        const int r = bitrev(e, a.logN);
        buf[slot(l, r, a.N)] = v[k];
    }
}

template <typename V2>
__global__ __launch_bounds__(256) void fft_lines(FftArgs<V2> a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    V2* buf = reinterpret_cast<V2*>(lds_raw);  // [L][N] plus the pad slots of slot()
    const int N = a.N, L = a.L, b = blockIdx.x;
    const int logN = a.logN, logL = a.logL;
    const int total = L * N;
    const size_t outer = static_cast<size_t>(b) / a.nzb;  // a.nzb batches per slab
    const size_t z0 = (static_cast<size_t>(b) - outer * a.nzb) << logL;
    // load: consecutive threads take consecutive global addresses (powers of
    // two: shifts and masks instead of divisions).  Full batches (L N = 2048
    // or 4096: 8 or 16 elements per thread) issue all of a thread's loads
    // before its LDS stores.
    if (total == 2048 && blockDim.x == 256) load_lines<8>(a, b, outer, z0, buf);
    else if (total == 4096 && blockDim.x == 256) load_lines<16>(a, b, outer, z0, buf);
    else
        for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
            int l, e;
            line_split(a, idx, l, e);
            const int r = bitrev(e, logN);
            buf[slot(l, r, N)] = a.data[line_elem(a, b, outer, z0, l, e)];
        }
    const V2* tws = stage_twiddles(buf, a.tw, N, L);
    __syncthreads();
    // the log2 N butterfly stages, up to three per pass over LDS
    // FP32 values: radix-16 passes (two LDS sweeps at N = 256 instead of three)
    fft_lds_stages<sizeof(V2) == 8 ? 4 : 3>(buf, tws, logN, L, a.inverse != 0);
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        int l, e;
        if (a.axis == 0) {
            l = idx >> logN;
            e = idx & (N - 1);
        } else {
            e = idx >> logL;
            l = idx & (L - 1);
        }
        a.data[line_elem(a, b, outer, z0, l, e)] = buf[slot(l, e, N)];
    }
}

// Fused first pass of the power spectrum: array `arr` of L consecutive rows
// of the row-interleaved state, as complex (value, 0), into LDS bit-reversed
// along z, the z transform, out to F (the extraction's write and the z pass's
// read of the complex array are saved).  The first P of the N transformed
// values of a line are stored (row pitch P): the rest follow from Hermitian
// symmetry of a real array's transform.  K = L N / 256 values per thread.
// The first workgroup also clears the `nzero` sums and counts of the bins
// that the last pass, launched after this one on the same stream, adds to.
template <typename T, int K>
__global__ __launch_bounds__(256) void spec_extract_fftz(const T* __restrict__ state, int N, int logN, int L,
                                                         int na, int arr, const double2* __restrict__ tw,
                                                         double2* __restrict__ F, int P, double* __restrict__ zs,
                                                         unsigned long long* __restrict__ zc, int nzero) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double2* buf = reinterpret_cast<double2*>(lds_raw);
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < nzero; i += blockDim.x) {
            zs[i] = 0.0;
            zc[i] = 0ull;
        }
    const int total = L * N;
    const size_t row0 = static_cast<size_t>(blockIdx.x) * L;
    T v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int idx = static_cast<int>(threadIdx.x) + k * 256;
        if (K > 1 || idx < total) v[k] = state[((row0 + (idx >> logN)) * na + arr) * N + (idx & (N - 1))];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int idx = static_cast<int>(threadIdx.x) + k * 256;
        if (K > 1 || idx < total)
            buf[slot(idx >> logN, bitrev(idx & (N - 1), logN), N)] = make_double2(static_cast<double>(v[k]), 0.0);
    }
    const double2* tws = stage_twiddles(buf, tw, N, L);
    __syncthreads();
    fft_lds_stages(buf, tws, logN, L, false);
    double2* out = F + row0 * P;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int l = idx >> logN, e = idx & (N - 1);
        if (e < P) out[static_cast<size_t>(l) * P + e] = buf[slot(l, e, N)];
    }
}

// Fused last pass of the power spectrum: the x transform of each batch of L
// lines (L consecutive z of one y, as in fft_lines), then |F|^2 of every
// mode into centred shells l = floor(|n~| / w + 1/2) < nbins in LDS; a
// workgroup takes batches blockIdx.x, + gridDim.x, ... and adds its shells
// to the global sums and counts once (the x pass's write and the binning
// pass's read of the complex array are saved).  Only z <= N / 2 is held
// (row pitch P, nzb = P / L batches per y): a real array's transform has
// |F(-n~)| = |F(n~)|, so a mode with 0 < z < N / 2 also stands for its mirror
// (z' = N - z, same |n~|) and is counted twice; columns beyond N / 2 are
// padding of the last batch and are skipped.
template <int K>
__global__ __launch_bounds__(256) void spec_fftx_bin(const double2* __restrict__ F, int N, int logN, int L, int logL,
                                                     int P, int nzb, const double2* __restrict__ tw, double inv_w,
                                                     int nbins, double* __restrict__ sums,
                                                     unsigned long long* __restrict__ counts) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double2* buf = reinterpret_cast<double2*>(lds_raw);
    const size_t nv = fft_lds_values(N, L) + (N / 2 > 0 ? N / 2 : 1);
    double* s_sum = reinterpret_cast<double*>(buf + nv);
    unsigned* s_cnt = reinterpret_cast<unsigned*>(s_sum + nbins);
    const double2* tws = stage_twiddles(buf, tw, N, L);
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) {
        s_sum[i] = 0.0;
        s_cnt[i] = 0u;
    }
    const int total = L * N, hN = N / 2;
    const int batches = N * nzb;
    for (int b = blockIdx.x; b < batches; b += gridDim.x) {
        const size_t y = static_cast<size_t>(b / nzb);
        const int z0 = (b - static_cast<int>(y) * nzb) << logL;
        __syncthreads();  // the previous batch no longer reads LDS
        // element idx: x = idx >> logL, z = z0 + (idx & (L - 1)); L
        // consecutive z of a row per global access; every load of a thread
        // before its LDS stores (K = L N / 256 per thread, 1 below 256)
        double2 v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int idx = static_cast<int>(threadIdx.x) + k * 256;
            if (K > 1 || idx < total)
                v[k] = F[(static_cast<size_t>(idx >> logL) * N + y) * P + z0 + (idx & (L - 1))];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int idx = static_cast<int>(threadIdx.x) + k * 256;
            if (K > 1 || idx < total) buf[slot(idx & (L - 1), bitrev(idx >> logL, logN), N)] = v[k];
        }
        __syncthreads();
        fft_lds_stages(buf, tws, logN, L, false);
        // a thread walks the L modes of one x (consecutive z: mostly one
        // shell) and adds a run of equal shells to LDS once
        const int ny = static_cast<int>(y) <= hN ? static_cast<int>(y) : static_cast<int>(y) - N;
        for (int e = threadIdx.x; e < N; e += blockDim.x) {
            const int nx = e <= hN ? e : e - N;
            int cur = -1;
            double run = 0.0;
            unsigned cnt = 0u;
            for (int l = 0; l < L; ++l) {
                const int nz = z0 + l;
                if (nz > hN) break;  // padding columns (z grows with l)
                const double r = sqrt(static_cast<double>(nx * nx + ny * ny + nz * nz));
                const int lb = static_cast<int>(floor(r * inv_w + 0.5));
                if (lb != cur) {
                    if (cnt) {
                        atomicAdd(&s_sum[cur], run);
                        atomicAdd(&s_cnt[cur], cnt);
                    }
                    cur = lb;
                    run = 0.0;
                    cnt = 0u;
                }
                if (lb < nbins) {
                    const double2 v = buf[slot(l, e, N)];
                    const double p = fma(v.x, v.x, v.y * v.y);
                    const bool twice = nz != 0 && nz != hN;
                    run += twice ? 2.0 * p : p;
                    cnt += twice ? 2u : 1u;
                }
            }
            if (cnt) {
                atomicAdd(&s_sum[cur], run);
                atomicAdd(&s_cnt[cur], cnt);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) {
        if (s_cnt[i]) {
            atomicAdd(&sums[i], s_sum[i]);
            atomicAdd(&counts[i], static_cast<unsigned long long>(s_cnt[i]));
        }
    }
}

// Gravitational-wave spectrum (Sect. 4.2): U holds the DFTs of the five
// evolved tensor components (11, 12, 13, 22, 23; 33 = -11 - 22), N^3 each.
// Per mode: the transverse-traceless projection
// Lambda_ij,lm T_lm = (P T P)_ij - P_ij tr(P T) / 2 with P = 1 - k^ k^ and
// k^ the unit lattice momentum (sin(pi n_i / N)), then sum_ij |.|^2 into the
// centred shell of |n~| (slot nbins collects the modes beyond the last bin);
// the mode n~ = 0 carries no waves.
//
// U holds the half z <= N / 2 of each transform (row pitch P, components n3
// apart).  A mode with 0 < z < N / 2 also stands for its mirror (-x, -y,
// N - z), whose transform is the complex conjugate (a real tensor) and whose
// |n~| is the same: where neither x nor y is the Nyquist index N / 2 the
// mirror's lattice momentum is -k and the projector, even in k^, gives the
// same power, so the mode is counted twice; otherwise the mirror keeps +N/2
// in that component (the index convention of every mode) and its projection
// is evaluated on its own.
__device__ __forceinline__ double gw_mode_power(const int n[3], double pin, const double2 c11, const double2 c12,
                                                const double2 c13, const double2 c22, const double2 c23) {
    double k[3], kk = 0.0;
    for (int i = 0; i < 3; ++i) {
        k[i] = sin(pin * n[i]);
        kk += k[i] * k[i];
    }
    const double inv = 1.0 / sqrt(kk);
    for (int i = 0; i < 3; ++i) k[i] *= inv;
    double P[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) P[i][j] = (i == j ? 1.0 : 0.0) - k[i] * k[j];
    const double2 c33 = make_double2(-c11.x - c22.x, -c11.y - c22.y);
    const double2 T[3][3] = {{c11, c12, c13}, {c12, c22, c23}, {c13, c23, c33}};
    double2 PT[3][3], tr = make_double2(0.0, 0.0);
    for (int i = 0; i < 3; ++i)
        for (int m = 0; m < 3; ++m) {
            double2 a = make_double2(0.0, 0.0);
            for (int l = 0; l < 3; ++l) {
                a.x = fma(P[i][l], T[l][m].x, a.x);
                a.y = fma(P[i][l], T[l][m].y, a.y);
            }
            PT[i][m] = a;
            tr.x = fma(P[i][m], T[i][m].x, tr.x);
            tr.y = fma(P[i][m], T[i][m].y, tr.y);
        }
    double pw = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double hx = -0.5 * P[i][j] * tr.x, hy = -0.5 * P[i][j] * tr.y;
            for (int m = 0; m < 3; ++m) {
                hx = fma(PT[i][m].x, P[m][j], hx);
                hy = fma(PT[i][m].y, P[m][j], hy);
            }
            pw = fma(hx, hx, fma(hy, hy, pw));
        }
    return pw;
}

__global__ __launch_bounds__(256) void gw_bin(const double2* __restrict__ U, int N, int P, double inv_w, int nbins,
                                              double* __restrict__ sums, unsigned long long* __restrict__ counts) {
    extern __shared__ unsigned char raw[];
    double* s_sum = reinterpret_cast<double*>(raw);
    unsigned* s_cnt = reinterpret_cast<unsigned*>(s_sum + nbins + 1);
    for (int i = threadIdx.x; i <= nbins; i += blockDim.x) {
        s_sum[i] = 0.0;
        if (i < nbins) s_cnt[i] = 0u;
    }
    __syncthreads();
    const size_t n3 = static_cast<size_t>(N) * N * N;
    const int hN = N / 2, nz = hN + 1;
    const size_t modes = static_cast<size_t>(N) * N * nz;
    const double pin = M_PI / N;
    for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < modes;
         t += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const int z = static_cast<int>(t % nz), y = static_cast<int>((t / nz) % N),
                  x = static_cast<int>(t / (static_cast<size_t>(N) * nz));
        const size_t s = (static_cast<size_t>(x) * N + y) * P + z;
        const int n[3] = {x <= hN ? x : x - N, y <= hN ? y : y - N, z};
        const bool twice = z != 0 && z != hN;
        const double r = sqrt(static_cast<double>(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]));
        const int lb = min(static_cast<int>(floor(r * inv_w + 0.5)), nbins);
        double pw = 0.0;
        if (n[0] | n[1] | n[2]) {
            const double2 c11 = U[s], c12 = U[n3 + s], c13 = U[2 * n3 + s], c22 = U[3 * n3 + s],
                          c23 = U[4 * n3 + s];
            pw = gw_mode_power(n, pin, c11, c12, c13, c22, c23);
            if (twice) {
                if (x == hN || y == hN) {
                    const int m[3] = {x == hN ? hN : -n[0], y == hN ? hN : -n[1], -z};
                    pw += gw_mode_power(m, pin, c11, c12, c13, c22, c23);
                } else {
                    pw *= 2.0;
                }
            }
        }
        atomicAdd(&s_sum[lb], pw);
        if (lb < nbins) atomicAdd(&s_cnt[lb], twice ? 2u : 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= nbins; i += blockDim.x) {
        if (s_sum[i] != 0.0) atomicAdd(&sums[i], s_sum[i]);
        if (i < nbins && s_cnt[i]) atomicAdd(&counts[i], static_cast<unsigned long long>(s_cnt[i]));
    }
}

hipError_t launch_gw_bin(const double2* U, int N, int P, double width, int nbins, double* sums,
                         unsigned long long* counts, hipStream_t s) {
    if (P < N / 2 + 1 || P > N) return hipErrorInvalidValue;
    const size_t modes = static_cast<size_t>(N) * N * (N / 2 + 1);
    const unsigned grid = static_cast<unsigned>(std::min<size_t>((modes + 255) / 256, 2048));
    const size_t lds = static_cast<size_t>(nbins + 1) * sizeof(double) + static_cast<size_t>(nbins) * sizeof(unsigned);
    hipLaunchKernelGGL(gw_bin, dim3(grid), dim3(256), lds, s, U, N, P, 1.0 / width, nbins, sums, counts);
    return hipGetLastError();
}

namespace {
template <typename V2>
hipError_t launch_fft(V2* data, const V2* tw, int N, int L, int axis, hipStream_t s, bool inverse, int P) {
    // the z axis needs whole lines; a y or x pass may cover fewer z (P a
    // multiple of L, at most N)
    if (P <= 0 || P > N || P % L != 0 || (axis == 0 && P != N)) return hipErrorInvalidValue;
    FftArgs<V2> a;
    a.inverse = inverse ? 1 : 0;
    a.data = data;
    a.tw = tw;
    a.N = N;
    a.logN = 0;
    while ((1 << a.logN) < N) ++a.logN;
    a.L = L;
    a.logL = 0;
    while ((1 << a.logL) < a.L) ++a.logL;
    a.axis = axis;
    a.P = P;
    a.nzb = P / L;
    const int batches = axis == 0 ? N * N / L : N * a.nzb;
    const size_t lds = fft_lds_bytes(N, a.L, sizeof(V2));
    hipLaunchKernelGGL(fft_lines<V2>, dim3(batches), dim3(256), lds, s, a);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_spec_fft(double2* data, const double2* tw, int N, int axis, hipStream_t s, bool inverse, int P) {
    return launch_fft(data, tw, N, fft_lines_per_block(N), axis, s, inverse, P > 0 ? P : N);
}

hipError_t launch_fft_f32(float2* data, const float2* tw, int N, int axis, hipStream_t s, bool inverse) {
    return launch_fft(data, tw, N, fft_lines_per_block_f32(N), axis, s, inverse, N);
}

int spec_half_pitch(int N) {
    const int L = fft_lines_per_block(N), need = N / 2 + 1;
    return std::min(N, (need + L - 1) / L * L);
}


hipError_t launch_spec_extract_fftz(const void* state, bool fp32, int N, int na, int arr, const double2* tw,
                                   double2* F, int P, double* zs, unsigned long long* zc, int nzero,
                                   hipStream_t s) {
    if (!zs || !zc) nzero = 0;
    int logN = 0;
    while ((1 << logN) < N) ++logN;
    const int L = fft_lines_per_block(N), total = L * N;
    if ((1 << logN) != N || total > 2048 || P <= 0 || P > N) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(N) * N / L);
    const size_t lds = fft_lds_bytes(N, L);
#define CL_SPEC_XZ(T, K)                                                                                          \
    hipLaunchKernelGGL((spec_extract_fftz<T, K>), grid, dim3(256), lds, s, static_cast<const T*>(state), N, logN, L, \
                       na, arr, tw, F, P, zs, zc, nzero)
    if (fp32) {
        if (total == 2048) CL_SPEC_XZ(float, 8);
        else if (total == 1024) CL_SPEC_XZ(float, 4);
        else if (total == 512) CL_SPEC_XZ(float, 2);
        else CL_SPEC_XZ(float, 1);
    } else {
        if (total == 2048) CL_SPEC_XZ(double, 8);
        else if (total == 1024) CL_SPEC_XZ(double, 4);
        else if (total == 512) CL_SPEC_XZ(double, 2);
        else CL_SPEC_XZ(double, 1);
    }
#undef CL_SPEC_XZ
    return hipGetLastError();
}

hipError_t launch_spec_fftx_bin(const double2* F, const double2* tw, int N, int P, double width, int nbins,
                                double* sums, unsigned long long* counts, hipStream_t s) {
    int logN = 0;
    while ((1 << logN) < N) ++logN;
    const int L = fft_lines_per_block(N);
    int logL = 0;
    while ((1 << logL) < L) ++logL;
    if ((1 << logN) != N || (1 << logL) != L || P % L != 0 || P > N || P < N / 2 + 1) return hipErrorInvalidValue;
    const int nzb = P / L;
    const int batches = N * nzb;
    const unsigned grid = static_cast<unsigned>(std::min(batches, 2048));
    const size_t lds = fft_lds_bytes(N, L) + static_cast<size_t>(nbins) * (sizeof(double) + sizeof(unsigned));
    const int total = L * N;
#define CL_SPEC_XB(K) \
    hipLaunchKernelGGL((spec_fftx_bin<K>), dim3(grid), dim3(256), lds, s, F, N, logN, L, logL, P, nzb, tw, 1.0 / width, \
                       nbins, sums, counts)
    if (total == 2048) CL_SPEC_XB(8);
    else if (total == 1024) CL_SPEC_XB(4);
    else if (total == 512) CL_SPEC_XB(2);
    else if (total <= 256) CL_SPEC_XB(1);
    else return hipErrorInvalidValue;
#undef CL_SPEC_XB
    return hipGetLastError();
}


}  // namespace cl
