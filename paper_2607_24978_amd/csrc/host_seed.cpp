// Vacuum-fluctuation initial conditions on the host, in FP64.
//
// CosmoLattice 2.0, Sect. 2.3: fields start as homogeneous values plus
// Gaussian fluctuations set in Fourier space.  Each mode gets left- and
// right-moving complex amplitudes whose real and imaginary parts are normal
// with variance P(k)/2, P(k) = 1/(2 a^2 w_k), w_k^2 = k^2 + a^2 m^2 with m^2
// the curvature of the potential at the homogeneous values (Eq.
// QuantumFlucts); the field amplitude is their sum over sqrt(2) and the
// time derivative is i w (l - r)/sqrt(2) a^(alpha-1) minus H times the field
// amplitude (Eqs. fpr_influct, fpr_influct2).  The per-mode variance is
// scaled by amp^2 / dx^3 (Eq. varFandDFgeneral with Upsilon = 1, up to the
// N^3 of the DFT normalisation, which amp carries).  Modes 0 < |n| <= cutoff
// are drawn on half of mode space and mirrored by complex conjugation so the
// fields are real; the inverse DFT uses f(n) = N^-3 sum exp(+2 pi i n'.n/N)
// f(n') (Sect. 4.3).
//
// Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as a
// counter-based stream -- draw k is the finaliser applied to
// seed + k * 0x9E3779B97F4A7C15 -- so each mode's draws depend only on
// (seed, field, mode index, draw), independent of threading.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <thread>
#include <vector>

namespace cl {
namespace {

using cplx = std::complex<double>;

inline uint64_t sm64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

inline double unit(uint64_t seed, uint64_t k) {
    return (static_cast<double>(sm64(seed, k) >> 11) + 1.0) * 0x1p-53;
}

inline double normal(uint64_t seed, uint64_t k0) {
    const double u1 = unit(seed, k0);
    const double u2 = unit(seed, k0 + 1);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
}

inline int mode_of(int i, int N) { return i <= N / 2 ? i : i - N; }

int n_threads() {
    unsigned t = std::thread::hardware_concurrency();
    if (t == 0) t = 4;
    return static_cast<int>(std::min(t, 64u));
}

template <typename F>
void parallel_for(int64_t n, F&& body) {
    const int T = static_cast<int>(std::min<int64_t>(n_threads(), std::max<int64_t>(n, 1)));
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t)
        th.emplace_back([&, t] {
            const int64_t lo = n * t / T, hi = n * (t + 1) / T;
            for (int64_t i = lo; i < hi; ++i) body(i);
        });
    for (auto& x : th) x.join();
}

// In-place radix-2 transform of one line with exp(+2 pi i k n / N) (no scaling).
struct Radix2 {
    int N = 0, logN = 0;
    std::vector<cplx> w;  // w[k] = exp(+2 pi i k / N), k < N/2
    std::vector<int> rev;
    explicit Radix2(int n) : N(n) {
        while ((1 << logN) < N) ++logN;
        w.resize(N / 2);
        for (int k = 0; k < N / 2; ++k) {
            const double t = 2.0 * M_PI * k / N;
            w[k] = cplx(std::cos(t), std::sin(t));
        }
        rev.resize(N);
        for (int i = 0; i < N; ++i) {
            int r = 0;
            for (int b = 0; b < logN; ++b)
                if (i & (1 << b)) r |= 1 << (logN - 1 - b);
            rev[i] = r;
        }
    }
    void run(cplx* a) const {
        for (int i = 0; i < N; ++i)
            if (i < rev[i]) std::swap(a[i], a[rev[i]]);
        for (int len = 2; len <= N; len <<= 1) {
            const int half = len / 2, stride = N / len;
            for (int s = 0; s < N; s += len)
                for (int k = 0; k < half; ++k) {
                    const cplx u = a[s + k];
                    const cplx v = a[s + k + half] * w[k * stride];
                    a[s + k] = u + v;
                    a[s + k + half] = u - v;
                }
        }
    }
};

// Unscaled inverse 3D transform of a [N][N][N] array (z fastest) whose
// nonzero modes all satisfy n_x^2 + n_y^2 + n_z^2 <= c2: lines and planes
// that hold only zeros are skipped (their transform is zero).
void inverse_3d(cplx* a, int N, double c2) {
    const Radix2 fft(N);
    const int64_t NN = static_cast<int64_t>(N) * N;
    // z lines: contiguous; only (n_x, n_y) inside the disc carry data.
    parallel_for(NN, [&](int64_t line) {
        const int nx = mode_of(static_cast<int>(line / N), N), ny = mode_of(static_cast<int>(line % N), N);
        if (static_cast<double>(nx * nx + ny * ny) <= c2) fft.run(a + line * N);
    });
    // y and x lines: gather blocks of B neighbouring z columns to use whole cache lines.
    constexpr int B = 16;
    const int nb = (N + B - 1) / B;
    for (int axis = 1; axis >= 0; --axis) {
        const int64_t stride = axis == 1 ? N : NN;
        parallel_for(static_cast<int64_t>(N) * nb, [&](int64_t item) {
            const int other = static_cast<int>(item / nb);
            // y lines at fixed x: zero unless |n_x| lies inside the cutoff
            if (axis == 1) {
                const int nx = mode_of(other, N);
                if (static_cast<double>(nx) * nx > c2) return;
            }
            thread_local std::vector<cplx> tmp;
            tmp.resize(static_cast<size_t>(B) * N);
            const int zb = static_cast<int>(item % nb) * B;
            const int nz = std::min(B, N - zb);
            const int64_t base = (axis == 1 ? static_cast<int64_t>(other) * NN : static_cast<int64_t>(other) * N) + zb;
            for (int i = 0; i < N; ++i)
                for (int q = 0; q < nz; ++q) tmp[static_cast<size_t>(q) * N + i] = a[base + i * stride + q];
            for (int q = 0; q < nz; ++q) fft.run(tmp.data() + static_cast<size_t>(q) * N);
            for (int i = 0; i < N; ++i)
                for (int q = 0; q < nz; ++q) a[base + i * stride + q] = tmp[static_cast<size_t>(q) * N + i];
        });
    }
}

}  // namespace

const char* host_seed(int N, double dx, int nf, const Phys& ph, double a0, uint64_t seed, const double* fbar,
                      const double* pbar, double cutoff, double amp, double* f, double* p) {
    if (N & (N - 1)) return "seed needs N to be a power of two";
    const double k_ir = 2.0 * M_PI / (N * dx);
    const int64_t NN = static_cast<int64_t>(N) * N, N3 = NN * N;
    const double alpha = ph.alpha;
    // Curvature of V at the homogeneous values: d2V/df_j^2.
    double fb[2] = {fbar[0], nf > 1 ? fbar[1] : 0.0};
    double pb[2] = {pbar[0], nf > 1 ? pbar[1] : 0.0};
    double m2eff[2];
    for (int j = 0; j < nf; ++j) {
        m2eff[j] = ph.m2[j] + 3.0 * ph.lam[j] * fb[j] * fb[j];
        if (nf == 2) m2eff[j] += ph.g2 * fb[1 - j] * fb[1 - j];
    }
    // Hubble rate of the homogeneous background for the -H df term.
    double H = 0.0;
    if (ph.expand) {
        double V = ph.V0, K = 0.0;
        for (int j = 0; j < nf; ++j) {
            V += 0.5 * ph.m2[j] * fb[j] * fb[j] + 0.25 * ph.lam[j] * fb[j] * fb[j] * fb[j] * fb[j];
            K += pb[j] * pb[j] / (2.0 * std::pow(a0, 6.0));
        }
        if (nf == 2) V += 0.5 * ph.g2 * fb[0] * fb[0] * fb[1] * fb[1];
        const double rho = K + V;
        if (!(rho > 0.0)) return "homogeneous energy density is not positive";
        H = std::sqrt(std::pow(a0, 2.0 * alpha) * rho / (3.0 * ph.mp * ph.mp));
    }
    std::vector<cplx> Z;
    try {
        Z.assign(static_cast<size_t>(N3), cplx(0.0, 0.0));
    } catch (...) {
        return "out of host memory for the seed transform";
    }
    const double c2 = cutoff * cutoff;
    const double rs2 = std::sqrt(2.0);
    const double fa = std::pow(a0, alpha - 1.0), pa = std::pow(a0, 3.0 - alpha);
    for (int j = 0; j < nf; ++j) {
        std::fill(Z.begin(), Z.end(), cplx(0.0, 0.0));
        const double mass = a0 * a0 * m2eff[j];
        // Z = df + i dp: both are Hermitian, so one inverse transform gives
        // the two real fields as its real and imaginary parts.
        parallel_for(N, [&](int64_t ix) {
            const int nx = mode_of(static_cast<int>(ix), N);
            for (int iy = 0; iy < N; ++iy) {
                const int ny = mode_of(iy, N);
                for (int iz = 0; iz < N; ++iz) {
                    const int nz = mode_of(iz, N);
                    const bool rep = nx > 0 || (nx == 0 && (ny > 0 || (ny == 0 && nz > 0)));
                    if (!rep) continue;
                    const double n2 = static_cast<double>(nx * nx + ny * ny + nz * nz);
                    if (!(n2 > 0.0) || n2 > c2) continue;
                    const double k = k_ir * std::sqrt(n2);
                    const double w2 = k * k + mass;
                    if (!(w2 > 0.0)) continue;
                    const double w = std::sqrt(w2);
                    const double S = amp * amp * (1.0 / (2.0 * a0 * a0 * w)) / (dx * dx * dx);
                    const double sig = std::sqrt(0.5 * S);
                    const uint64_t m = (static_cast<uint64_t>(ix) * N + iy) * N + iz;
                    const uint64_t base = (static_cast<uint64_t>(j) * static_cast<uint64_t>(N3) + m) * 4;
                    double g[4];
                    for (int d = 0; d < 4; ++d) g[d] = normal(seed, 2 * (base + d) + 1);
                    const cplx fl(sig * g[0], sig * g[1]);
                    const cplx fr(sig * g[2], sig * g[3]);
                    const cplx df = (fl + fr) / rs2;
                    const cplx dfp = fa * (cplx(0.0, w / rs2) * (fl - fr)) - H * df;
                    const cplx dp = pa * dfp;
                    const int64_t id = static_cast<int64_t>(m);
                    const int64_t jd = ((static_cast<int64_t>((N - ix) % N) * N + (N - iy) % N) * N + (N - iz) % N);
                    Z[id] = df + cplx(0.0, 1.0) * dp;
                    Z[jd] = std::conj(df) + cplx(0.0, 1.0) * std::conj(dp);
                }
            }
        });
        inverse_3d(Z.data(), N, c2);
        const double inv = 1.0 / static_cast<double>(N3);
        double* fj = f + static_cast<size_t>(j) * N3;
        double* pj = p + static_cast<size_t>(j) * N3;
        parallel_for(N, [&](int64_t x) {
            for (int64_t i = x * NN; i < (x + 1) * NN; ++i) {
                fj[i] = fb[j] + Z[i].real() * inv;
                pj[i] = pb[j] + Z[i].imag() * inv;
            }
        });
    }
    return "";
}

}  // namespace cl
