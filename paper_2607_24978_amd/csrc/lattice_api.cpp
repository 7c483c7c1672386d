// Host runtime behind the C ABI of cl_lattice.h: handle state, pass
// schedules of the integrators, buffer management and error reporting.
//
// A call to cl_step issues one opening kick pass and then one fused
// drift-kick pass per velocity-Verlet sub-step, merging the two half kicks
// of adjacent sub-steps into one (Sect. 4.1: staggered leapfrog / velocity
// Verlet, and the 4th-order Yoshida composition).  The scale factor is
// advanced with the same kicks and drifts by the last workgroup of every
// pass, so no pass waits for the host.  The passes of a call are captured in
// a HIP graph and replayed while the call shape stays the same.
#include "internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <array>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using cl::PassArgs;
using cl::Phys;
using cl::Scal;
using cl::Tile;

namespace {

thread_local std::string g_err;

size_t elem_size(cl_precision p) { return p == CL_FP32 ? 4 : 8; }
size_t sites(const cl_lattice* h) {
    size_t n = 1;
    for (int d = 0; d < h->dim; ++d) n *= static_cast<size_t>(h->N);
    return n;
}
// rows of N values along z (N^2 in three dimensions, N or 1 on reduced lattices)
size_t rows(const cl_lattice* h) { return sites(h) / static_cast<size_t>(h->N); }
// Stencil arrays per row: the fields plus the gravitational-wave tensor
// components (each with its momentum: 2 na arrays per row).
int arrays(const cl_lattice* h) { return h->nf + h->ng; }
// One state buffer: 2 na arrays of N^3 values.
size_t state_bytes(const cl_lattice* h) { return 2 * static_cast<size_t>(arrays(h)) * sites(h) * elem_size(h->prec); }

cl_status fail(cl_lattice* h, cl_status st, const std::string& msg) {
    if (h) h->err = msg; else g_err = msg;
    return st;
}

#define HIPCHECK(h, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((h), CL_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

Phys make_phys(const cl_lattice* h) {
    Phys p{};
    for (int j = 0; j < 2; ++j) {
        p.m2[j] = h->pot.m2[j];
        p.lam[j] = h->pot.lambda[j];
    }
    p.g2 = h->pot.g2;
    p.V0 = h->pot.V0;
    p.alpha = h->alpha;
    p.mp = h->mp;
    p.dx = h->dx;
    p.inv_vol = 1.0 / static_cast<double>(sites(h));
    p.nf = h->nf;
    p.expand = h->mode == CL_SELF_CONSISTENT ? 1 : 0;
    p.fp32 = h->prec == CL_FP32 ? 1 : 0;
    return p;
}

// Background last seen on the host (the time-step stability check uses it).
void note_background(cl_lattice* h, double a, const double* mean) {
    h->host_a = a;
    for (int j = 0; j < 2; ++j) h->host_mean[j] = mean ? mean[j] : 0.0;
}

void drop_graph(cl_lattice* h) {
    for (int i = 0; i < 2; ++i) {
        if (h->gexec[i]) hipGraphExecDestroy(h->gexec[i]);
        h->gexec[i] = nullptr;
        h->gkey[i] = GraphKey{};
    }
}

bool valid_N(int N, cl_precision prec) {
    if (N < 8 || N > 1600 || (N % 2)) return false;
    const bool pow2 = (N & (N - 1)) == 0;
    const int big = prec == CL_FP32 ? 256 : 128;
    return pow2 || (N % big == 0);
}

// Two halves of nsums * nblocks doubles: consecutive passes alternate, as a
// pass reads the sums of the one before while writing its own.
cl_status ensure_partials(cl_lattice* h, int nblocks = 0) {
    if (nblocks <= 0) nblocks = h->tile.nblocks();
    const size_t need = 2 * static_cast<size_t>(cl::nsums(h->nf)) * nblocks;
    if (need <= h->partials_cap) return CL_OK;
    if (h->partials) hipFree(h->partials);
    h->partials = nullptr;
    h->partials_cap = 0;
    HIPCHECK(h, hipMalloc(&h->partials, need * sizeof(double)));
    h->partials_cap = need;
    drop_graph(h);
    return CL_OK;
}

cl_status ensure_obs(cl_lattice* h, int n) {
    if (n <= h->obs_cap) return CL_OK;
    if (h->obs) hipFree(h->obs);
    h->obs = nullptr;
    h->obs_cap = 0;
    int cap = 64;
    while (cap < n) cap *= 2;
    HIPCHECK(h, hipMalloc(&h->obs, static_cast<size_t>(cap) * sizeof(cl_observables)));
    h->obs_cap = cap;
    drop_graph(h);
    return CL_OK;
}

PassArgs base_args(cl_lattice* h, int in) {
    PassArgs a{};
    a.in = h->buf[in];
    a.out = h->buf[in ^ 1];
    a.flags = h->pass_flags;
    a.N = h->N;
    a.TZ = h->tile.TZ;
    a.TY = h->tile.TY;
    a.CX = h->tile.CX;
    a.nbz = h->tile.nbz;
    a.nby = h->tile.nby;
    a.nbx = h->tile.nbx;
    a.sc_in = h->sc;
    a.sc_out = nullptr;
    a.partials = h->partials;
    a.prev_partials = nullptr;
    a.has_prev = 0;
    a.prev_rec = -1;
    a.rk = a.rk_first = a.prev_rk = a.prev_rk_first = a.rk_last = 0;
    a.rkA = a.rkB = a.rkC = a.rkD = a.rkh = a.rkdeta = 0.0;
    a.prkA = a.prkB = a.prkC = a.prkD = a.prkh = a.prkdeta = 0.0;
    a.aux = h->aux;
    a.y0 = nullptr;
    a.dim = h->dim;
    a.ng = h->ng;
    a.obs = h->obs;
    a.ph = make_phys(h);
    a.rec = -1;
    return a;
}

cl::Work handle_work(cl_lattice* h) {
    return cl::Work{h->partials, h->partials_cap / 2, h->scb, h->obs, h->obs_cap};
}

// A sequence of passes on the handle's stream.  Each pass runs the scalar
// step of the one before it at its start; close() launches the step of the
// last one, which leaves the scalars in h->sc.  Inside the sequence the
// scalars travel through the two scratch blocks of the work area, and the
// partial sums alternate between its two halves.
struct PassSeq {
    cl_lattice* h;
    cl::Work w;
    int p = 0;
    PassArgs prev{};
    explicit PassSeq(cl_lattice* hh) : h(hh), w(handle_work(hh)) {}
    PassSeq(cl_lattice* hh, const cl::Work& ww) : h(hh), w(ww) {}
    double* part(int q) const { return w.partials + q * w.half; }
    const Scal* scal_before(int q) const { return q == 0 ? h->sc : w.scb + (q & 1); }
    void chain(PassArgs& a) const {
        a.has_prev = 1;
        a.sc_in = scal_before(p - 1);
        a.prev_partials = part((p - 1) & 1);
        a.prev_nslots = h->tile.nblocks();
        a.pkt = prev.kt;
        a.pkb = prev.kb;
        a.phn = prev.h_next;
        a.prev_rec = prev.rec;
        a.prev_rk = prev.rk;
        a.prev_rk_first = prev.rk_first;
        a.prkA = prev.rkA;
        a.prkB = prev.rkB;
        a.prkC = prev.rkC;
        a.prkD = prev.rkD;
        a.prkh = prev.rkh;
        a.prkdeta = prev.rkdeta;
    }
    hipError_t launch(PassArgs a) {
        a.partials = part(p & 1);
        a.obs = w.obs;
        if (p == 0) {
            a.has_prev = 0;
            a.sc_in = h->sc;
        } else {
            chain(a);
            a.sc_out = w.scb + (p & 1);
        }
        const hipError_t e = cl::launch_pass(a, h->tile, h->prec, h->stream);
        prev = a;
        ++p;
        return e;
    }
    hipError_t close() {
        if (p == 0) return hipSuccess;
        PassArgs f = prev;
        chain(f);
        f.sc_out = h->sc;
        return cl::launch_finish(f, h->tile, h->nf, h->stream);
    }
};

// Yoshida triple-jump weights of the 4th-order composition (Sect. 4.1):
// w1 = 1 / (2 - 2^(1/3)), w0 = 1 - 2 w1.
double yoshida_w1() { return 1.0 / (2.0 - std::cbrt(2.0)); }

// Drift steps per full step, and the size of drift step s in units of dt.
int substeps_per_step(cl_integrator integ) { return integ == CL_VV4 ? 3 : 1; }
double substep(cl_integrator integ, int s) {
    if (integ != CL_VV4) return 1.0;
    const double w1 = yoshida_w1();
    return s % 3 == 1 ? 1.0 - 2.0 * w1 : w1;
}

// Sub-step sizes of n full steps.
void substeps(cl_integrator integ, double dt, int n, std::vector<double>& h, int& per_step) {
    per_step = substeps_per_step(integ);
    h.resize(static_cast<size_t>(n) * per_step);
    for (size_t s = 0; s < h.size(); ++s) h[s] = substep(integ, static_cast<int>(s)) * dt;
}

bool is_rk(cl_integrator integ) {
    return integ == CL_RK2 || integ == CL_RK3 || integ == CL_RK34 || integ == CL_RK4 || integ == CL_RK4_CLASSIC;
}

// Low-storage Runge-Kutta coefficients (d <- A d + h F(y), y <- y + B d):
// the explicit midpoint rule; Williamson (1980) RK3-3; a four-stage
// third-order member of the same family (order-3 conditions met, order-4
// error terms minimised: the paper's RK3-4 comes without coefficients);
// Carpenter and Kennedy (1994) five-stage fourth-order scheme.
void rk_coefficients(cl_integrator integ, std::vector<double>& A, std::vector<double>& B) {
    if (integ == CL_RK2) {
        A = {0.0, -0.5};
        B = {0.5, 1.0};
    } else if (integ == CL_RK3) {
        A = {0.0, -5.0 / 9.0, -153.0 / 128.0};
        B = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    } else if (integ == CL_RK34) {
        A = {0.0, -0.35643988236064206, -0.9681295617245512, -1.7681569348912718};
        B = {0.16095368082904207, 0.32750970610000874, 0.759520141721668, 1.0254284658050152};
    } else {
        A = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
             -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
        B = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
             1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
             2277821191437.0 / 14882151754819.0};
    }
}

// Stage abscissae of a low-storage scheme: c_i = sum_j a_ij of the equivalent
// Butcher tableau, tracked as the coefficients of y_i and d_i in h k_j.
std::vector<double> rk_abscissae(const std::vector<double>& A, const std::vector<double>& B) {
    const size_t s = A.size();
    std::vector<double> c(s + 1, 0.0), D(s, 0.0), Y(s, 0.0);  // D, Y: coefficient rows
    for (size_t i = 0; i < s; ++i) {
        // d_i = A_i d_(i-1) + h k_i ; y_i = y_(i-1) + B_i d_i  (sum of coefficients suffices)
        double dsum = (i ? A[i] * D[i - 1] : 0.0) + 1.0;
        D[i] = dsum;
        c[i + 1] = c[i] + B[i] * dsum;
    }
    c[s] = 1.0;  // a consistent scheme ends at y(t + h)
    return c;
}

// ---------------------------------------------------------------- stability
// A scheme advances a harmonic mode y'' = -w^2 y of frequency w stably while
// y = w dt stays below a limit of its own: 2 for leapfrog (the kick-drift-kick
// matrix has trace 2 - y^2); for the 4th-order Yoshida composition, the y
// where the trace of the product of its three kick-drift-kick matrices
// reaches -2 (about 1.5735); for a Runge-Kutta scheme, the end of the
// interval of the imaginary axis where its stability polynomial
// R(z) = sum_k b^T A^(k-1) 1 z^k has |R| <= 1 (RK3-3: sqrt 3, RK3-4: 2.823,
// RK4-5: 3.341, classic RK4: 2 sqrt 2).  The explicit midpoint rule has no
// such interval (|R(iy)|^2 = 1 + y^4 / 4): it is held to a growth of at most
// 1 % per step of the fastest mode (y <= 0.532).

// |tr| of the Yoshida product at y (w = 1, step y).
double vv4_trace(double y) {
    const double w1 = yoshida_w1(), w0 = 1.0 - 2.0 * w1;
    double M[2][2] = {{1.0, 0.0}, {0.0, 1.0}};
    for (double c : {w1, w0, w1}) {
        const double h = c * y;
        // kick(h/2) drift(h) kick(h/2) on (f, p)
        const double K[2][2] = {{1.0 - 0.5 * h * h, h}, {-h * (1.0 - 0.25 * h * h), 1.0 - 0.5 * h * h}};
        double R[2][2];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) R[i][j] = K[i][0] * M[0][j] + K[i][1] * M[1][j];
        std::memcpy(M, R, sizeof M);
    }
    return std::fabs(M[0][0] + M[1][1]);
}

// |R(iy)| of a stability polynomial with coefficients g[0..s].
double rk_amplification(const std::vector<double>& g, double y) {
    double re = 0.0, im = 0.0;
    double pr = 1.0, pi = 0.0;  // (iy)^k
    for (double c : g) {
        re += c * pr;
        im += c * pi;
        const double nr = -pi * y, ni = pr * y;
        pr = nr;
        pi = ni;
    }
    return std::hypot(re, im);
}

// Stability polynomial of a low-storage scheme: its Butcher tableau is
// tracked as the coefficients of y_i and d_i in h k_1 .. h k_s.
std::vector<double> rk_polynomial(cl_integrator integ) {
    if (integ == CL_RK4_CLASSIC) return {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0};
    std::vector<double> A, B;
    rk_coefficients(integ, A, B);
    const size_t s = A.size();
    std::vector<std::vector<double>> a(s, std::vector<double>(s, 0.0));
    std::vector<double> D(s, 0.0), Y(s, 0.0);
    for (size_t i = 0; i < s; ++i) {
        a[i] = Y;  // stage i is evaluated at y_(i-1)
        for (size_t j = 0; j < s; ++j) D[j] *= (i ? A[i] : 0.0);
        D[i] += 1.0;
        for (size_t j = 0; j < s; ++j) Y[j] += B[i] * D[j];
    }
    // g_0 = 1, g_k = b^T a^(k-1) 1 with b = Y
    std::vector<double> g{1.0}, v(s, 1.0);
    for (size_t k = 1; k <= s; ++k) {
        double dot = 0.0;
        for (size_t j = 0; j < s; ++j) dot += Y[j] * v[j];
        g.push_back(dot);
        std::vector<double> nv(s, 0.0);
        for (size_t i = 0; i < s; ++i)
            for (size_t j = 0; j < s; ++j) nv[i] += a[i][j] * v[j];
        v = nv;
    }
    return g;
}

// First y > 0 where stable(y) fails, by a scan of step 1e-3 and bisection.
template <typename F>
double first_failure(F stable) {
    double lo = 0.0;
    for (double y = 1e-3; y < 8.0; y += 1e-3) {
        if (!stable(y)) {
            double hi = y;
            for (int it = 0; it < 60; ++it) {
                const double m = 0.5 * (lo + hi);
                (stable(m) ? lo : hi) = m;
            }
            return lo;
        }
        lo = y;
    }
    return lo;
}

double stability_limit(cl_integrator integ) {
    static const std::array<double, 7> all = [] {
        std::array<double, 7> L{};
        L[CL_LEAPFROG] = 2.0;
        L[CL_VV4] = first_failure([](double y) { return vv4_trace(y) < 2.0; });
        for (cl_integrator r : {CL_RK2, CL_RK3, CL_RK4, CL_RK34, CL_RK4_CLASSIC}) {
            const std::vector<double> g = rk_polynomial(r);
            double y = first_failure([&](double t) { return rk_amplification(g, t) <= 1.0 + 1e-12; });
            if (y < 0.1) y = first_failure([&](double t) { return rk_amplification(g, t) <= 1.01; });
            L[r] = y;
        }
        return L;
    }();
    return all[static_cast<int>(integ)];
}

// Fastest frequency of the lattice in the kick-drift dynamics
// f'' = a^(2 alpha - 2) Lap f - a^(2 alpha) V''(f) f (Eq. singletEOM with
// pi = a^(3 - alpha) f'): the largest Laplacian eigenvalue 4 dim / dx^2 plus
// the largest effective mass d^2V/df_j^2 at the homogeneous field values last
// seen on the host (the fluctuations about them are not included).
double omega_max(const cl_lattice* h) {
    const double a = h->mode == CL_SELF_CONSISTENT ? h->host_a : 1.0;
    double m2 = 0.0;
    for (int j = 0; j < h->nf; ++j) {
        const double f = h->host_mean[j];
        double m = h->pot.m2[j] + 3.0 * h->pot.lambda[j] * f * f;
        if (h->nf == 2) m += h->pot.g2 * h->host_mean[1 - j] * h->host_mean[1 - j];
        m2 = std::max(m2, m);
    }
    const double w2 = 4.0 * h->dim / (h->dx * h->dx) * std::pow(a, 2.0 * h->alpha - 2.0) +
                      std::pow(a, 2.0 * h->alpha) * m2;
    return std::sqrt(w2);
}

const char* integ_name(cl_integrator integ) {
    switch (integ) {
        case CL_LEAPFROG: return "leapfrog";
        case CL_VV4: return "VV4";
        case CL_RK2: return "RK2";
        case CL_RK3: return "RK3-3";
        case CL_RK4: return "RK4-5";
        case CL_RK34: return "RK3-4";
        default: return "RK4";
    }
}

// CL_OK, or CL_EUNSTABLE with a message if dt exceeds the scheme's limit.
cl_status check_stability(cl_lattice* h, cl_integrator integ, double dt, const std::string& who) {
    const double y = omega_max(h) * dt, lim = stability_limit(integ);
    if (y < lim) return CL_OK;
    char msg[256];
    std::snprintf(msg, sizeof msg,
                  "dt exceeds the stability bound of %s%s: omega_max dt = %.4g >= %.4g (omega_max^2 = 4 d / dx^2 "
                  "a^(2 alpha - 2) + a^(2 alpha) max V'' at the field means)",
                  integ_name(integ), who.c_str(), y, lim);
    return fail(h, CL_EUNSTABLE, msg);
}

// Passes of n classic RK4 steps (the standard scheme, three auxiliary arrays
// per degree of freedom): with y0 in buffer A = buf[cur], the stages read
// Y1 = y0 (A), Y2 (B = buf[cur^1]), Y3 (aux2), Y4 (B) and write Y2 = y0 + k1/2
// (to B), Y3 = y0 + k2/2 (aux2), Y4 = y0 + k3 (B) and finally
// y0 + (k1 + 2 k2 + 2 k3)/6 + k4/6 in place into A, reading y0 only at each
// thread's own sites; the weighted sum s of the k's lives in aux.  Then a
// reduction-only pass records the final state, as for the low-storage schemes.
cl_status issue_rk4_classic_steps(cl_lattice* h, double dt, int n, int cur, const cl::Work& w) {
    void* A = h->buf[cur];
    void* B = h->buf[cur ^ 1];
    void* X = h->aux2;
    // per stage: input, output; output = y0 + P s + Q k, s <- R s + S k
    void* in[4] = {A, B, X, B};
    void* out[4] = {B, X, B, A};
    const double P[4] = {0.0, 0.0, 0.0, 1.0}, Q[4] = {0.5, 0.5, 1.0, 1.0 / 6.0};
    const double R[4] = {0.0, 1.0, 1.0, 0.0}, S[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 0.0};
    const double deta[4] = {0.5, 0.0, 0.5, 0.0};  // time of each output past the input's
    PassSeq seq(h, w);
    for (int k = 0; k < n; ++k)
        for (int i = 0; i < 4; ++i) {
            PassArgs r = base_args(h, cur);
            r.in = in[i];
            r.out = out[i];
            r.y0 = A;
            r.drift = 0;
            r.write_out = 1;
            r.kt = r.kb = r.h_next = 0.0;
            r.rk = 2;
            r.rk_first = i == 0;
            r.rk_last = i == 3;
            r.rkA = P[i];
            r.rkB = Q[i];
            r.rkC = R[i];
            r.rkD = S[i];
            r.rkh = dt;
            r.rkdeta = deta[i] * dt;
            r.rec = (i == 0 && k > 0) ? k - 1 : -1;
            HIPCHECK(h, seq.launch(r));
        }
    PassArgs z = base_args(h, cur);
    z.drift = 0;
    z.write_out = 0;
    z.kt = z.kb = z.h_next = 0.0;
    z.rec = n - 1;
    HIPCHECK(h, seq.launch(z));
    HIPCHECK(h, seq.close());
    return CL_OK;
}

// Passes of n low-storage Runge-Kutta steps: one stage pass per stage, then
// a reduction-only pass whose scalar step records the final state.  The
// scalar step of stage 0 of step k records the end of step k - 1.
cl_status issue_rk_steps(cl_lattice* h, cl_integrator integ, double dt, int n, int cur, const cl::Work& w) {
    if (integ == CL_RK4_CLASSIC) return issue_rk4_classic_steps(h, dt, n, cur, w);
    std::vector<double> A, B;
    rk_coefficients(integ, A, B);
    const std::vector<double> c = rk_abscissae(A, B);
    const int S = static_cast<int>(A.size());
    PassSeq seq(h, w);
    for (int k = 0; k < n; ++k)
        for (int i = 0; i < S; ++i) {
            PassArgs r = base_args(h, cur);
            r.drift = 0;
            r.write_out = 1;
            r.kt = r.kb = r.h_next = 0.0;
            r.rk = 1;
            r.rk_first = i == 0;
            r.rkA = A[i];
            r.rkB = B[i];
            r.rkh = dt;
            r.rkdeta = (c[i + 1] - c[i]) * dt;
            r.rec = (i == 0 && k > 0) ? k - 1 : -1;
            HIPCHECK(h, seq.launch(r));
            cur ^= 1;
        }
    PassArgs z = base_args(h, cur);
    z.drift = 0;
    z.write_out = 0;
    z.kt = z.kb = z.h_next = 0.0;
    z.rec = n - 1;
    HIPCHECK(h, seq.launch(z));
    HIPCHECK(h, seq.close());
    return CL_OK;
}

// Issue the passes of n steps on the handle's stream, with the scratch w.
cl_status issue_steps(cl_lattice* h, cl_integrator integ, double dt, int n, int cur, const cl::Work& w) {
    if (is_rk(integ)) return issue_rk_steps(h, integ, dt, n, cur, w);
    // Sub-step sizes in units of dt; every kick and drift step is formed as
    // (coefficient) * dt, exactly as the ensemble kernel forms it per member.
    const int per = substeps_per_step(integ);
    const int M = n * per;
    PassSeq seq(h, w);
    // Opening half kick (no drift): pi += h_1/2 F(f, a), a' += h_1/2 a''.
    PassArgs k = base_args(h, cur);
    k.drift = 0;
    k.write_out = 1;
    k.kt = (0.5 * substep(integ, 0)) * dt;
    k.kb = 0.0;
    k.h_next = substep(integ, 0) * dt;
    HIPCHECK(h, seq.launch(k));
    cur ^= 1;
    for (int s = 0; s < M; ++s) {
        const double cs = substep(integ, s);
        const double cn = s + 1 < M ? substep(integ, s + 1) : 0.0;
        PassArgs d = base_args(h, cur);
        d.drift = 1;
        d.write_out = 1;
        d.kb = (0.5 * cs) * dt;
        d.kt = (s + 1 < M ? 0.5 * (cs + cn) : 0.5 * cs) * dt;
        d.h_next = s + 1 < M ? cn * dt : 0.0;
        d.rec = ((s + 1) % per == 0) ? (s + 1) / per - 1 : -1;
        HIPCHECK(h, seq.launch(d));
        cur ^= 1;
    }
    HIPCHECK(h, seq.close());
    return CL_OK;
}

cl_status init_scalars(cl_lattice* h, double a, double b, double eta, const double* shift) {
    const Phys ph = make_phys(h);
    HIPCHECK(h, cl::launch_init_scalars(h->sc, a, b, eta, ph, shift, h->stream));
    return CL_OK;
}

// One reduction-only pass over the current state into obs[0].
// sc_out (nullable): the scalar block after the pass, copied before the wait
cl_status reduce_pass(cl_lattice* h, cl_observables* out, Scal* sc_out = nullptr) {
    cl_status st = ensure_obs(h, 1);
    if (st) return st;
    PassArgs r = base_args(h, h->cur);
    r.drift = 0;
    r.write_out = 0;
    r.kt = 0.0;
    r.kb = 0.0;
    r.h_next = 0.0;
    r.rec = 0;
    PassSeq seq(h);
    HIPCHECK(h, seq.launch(r));
    HIPCHECK(h, seq.close());
    HIPCHECK(h, hipMemcpyAsync(out, h->obs, sizeof(cl_observables), hipMemcpyDeviceToHost, h->stream));
    if (sc_out) HIPCHECK(h, hipMemcpyAsync(sc_out, h->sc, sizeof(Scal), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return CL_OK;
}

// After new fields: a = a0, eta = 0, b from the Hubble constraint.
cl_status reset_background(cl_lattice* h, const double* mean) {
    cl_status st = init_scalars(h, h->a0, 0.0, 0.0, mean);
    if (st) return st;
    cl_observables o;
    st = reduce_pass(h, &o);
    if (st) return st;
    double b0 = 0.0;
    if (o.nonfinite) {
        init_scalars(h, h->a0, 0.0, 0.0, mean);
        h->step = 0;
        return fail(h, CL_EUNSTABLE, "non-finite field values");
    }
    if (h->mode == CL_SELF_CONSISTENT) {
        const double rho = o.EK[0] + o.EK[1] + o.EG[0] + o.EG[1] + o.EV;
        if (!(rho > 0.0)) return fail(h, CL_EINVAL, "lattice energy density is not positive; a' undefined");
        b0 = h->a0 * std::sqrt(std::pow(h->a0, 2.0 * h->alpha) * rho / (3.0 * h->mp * h->mp));
    }
    st = init_scalars(h, h->a0, b0, 0.0, o.mean);
    if (st) return st;
    h->step = 0;
    note_background(h, h->a0, o.mean);
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return CL_OK;
}

// Host SoA arrays (N^3 each) <-> device row-interleaved state: array a of
// row r sits at (r * 2 na + a) * N.  `count` consecutive host arrays go to
// (come from) device arrays first .. first + count - 1 of the current state.
template <typename T>
cl_status upload_arrays(cl_lattice* h, const double* src, int first, int count) {
    const size_t n = sites(h);
    const size_t N = static_cast<size_t>(h->N);
    std::vector<T> tmp;
    try {
        tmp.resize(n);
    } catch (const std::bad_alloc&) {
        return fail(h, CL_ENOMEM, "host staging buffer");
    }
    for (int k = 0; k < count; ++k) {
        const double* s = src + k * n;
        for (size_t i = 0; i < n; ++i) tmp[i] = static_cast<T>(s[i]);
        char* dst = static_cast<char*>(h->buf[h->cur]) + (first + k) * N * sizeof(T);
        HIPCHECK(h, hipMemcpy2DAsync(dst, 2 * arrays(h) * N * sizeof(T), tmp.data(), N * sizeof(T), N * sizeof(T),
                                     rows(h), hipMemcpyHostToDevice, h->stream));
        HIPCHECK(h, hipStreamSynchronize(h->stream));
    }
    return CL_OK;
}

template <typename T>
cl_status download_arrays(cl_lattice* h, double* dst, int first, int count) {
    const size_t n = sites(h);
    const size_t N = static_cast<size_t>(h->N);
    std::vector<T> tmp;
    try {
        tmp.resize(n);
    } catch (const std::bad_alloc&) {
        return fail(h, CL_ENOMEM, "host staging buffer");
    }
    for (int k = 0; k < count; ++k) {
        const char* src = static_cast<const char*>(h->buf[h->cur]) + (first + k) * N * sizeof(T);
        HIPCHECK(h, hipMemcpy2DAsync(tmp.data(), N * sizeof(T), src, 2 * arrays(h) * N * sizeof(T), N * sizeof(T),
                                     rows(h), hipMemcpyDeviceToHost, h->stream));
        HIPCHECK(h, hipStreamSynchronize(h->stream));
        double* d = dst + k * n;
        for (size_t i = 0; i < n; ++i) d[i] = static_cast<double>(tmp[i]);
    }
    return CL_OK;
}

// Fields f_j are arrays 0 .. nf-1, momenta pi_j arrays na .. na+nf-1.
template <typename T>
cl_status upload(cl_lattice* h, const double* f, const double* p) {
    cl_status st = upload_arrays<T>(h, f, 0, h->nf);
    return st ? st : upload_arrays<T>(h, p, arrays(h), h->nf);
}

template <typename T>
cl_status download(cl_lattice* h, double* f, double* p) {
    cl_status st = f ? download_arrays<T>(h, f, 0, h->nf) : CL_OK;
    return st || !p ? st : download_arrays<T>(h, p, arrays(h), h->nf);
}

void host_means(const cl_lattice* h, const double* f, double* mean) {
    const size_t n = sites(h);
    for (int j = 0; j < 2; ++j) mean[j] = 0.0;
    for (int j = 0; j < h->nf; ++j) {
        double s = 0.0;
        for (size_t i = 0; i < n; ++i) s += f[j * n + i];
        mean[j] = s / static_cast<double>(n);
    }
}

const char* prec_name(cl_precision p) { return p == CL_FP32 ? "fp32" : "fp64"; }

// Last cached tile for (N, n_fields, precision) in the CL_TUNE_CACHE file.
bool cached_tile(int N, int nf, cl_precision prec, Tile& t) {
    const char* path = std::getenv("CL_TUNE_CACHE");
    if (!path || !path[0]) return false;
    FILE* fp = std::fopen(path, "r");
    if (!fp) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, fp)) {
        int n = 0, f = 0, tz = 0, ty = 0, cx = 0, ry = 0, pd = 0;
        char pr[8] = {0};
        if (std::sscanf(line, "{\"arch\":\"gfx950\",\"N\":%d,\"nf\":%d,\"prec\":\"%4[^\"]\",\"tz\":%d,\"ty\":%d,\"cx\":%d,\"ry\":%d,\"pd\":%d",
                        &n, &f, pr, &tz, &ty, &cx, &ry, &pd) == 8 &&
            n == N && f == nf && std::strcmp(pr, prec_name(prec)) == 0) {
            Tile c;
            c.TZ = tz;
            c.TY = ty;
            c.CX = cx;
            c.RY = ry;
            c.PD = pd;
            if (cl::finalize_tile(c, N, prec)) {
                t = c;
                found = true;
            }
        }
    }
    std::fclose(fp);
    return found;
}

// Tile of a pass that carries the gravitational-wave tensor: one row per
// thread, 16 threads along z, 128-thread workgroups (seven stencil arrays of
// registers per thread; 40 KB of LDS in FP32), prefetch depth 1, and enough
// x-chunks for about a thousand workgroups.
Tile gw_tile(int N, cl_precision prec) {
    const int V = prec == CL_FP32 ? 4 : 2;
    Tile t;
    t.TZ = std::min(N, 16 * V);
    const int BZ = t.TZ / V;
    int TY = 128 / BZ;
    while (TY > 1 && (TY > N || N % TY)) TY >>= 1;
    t.TY = TY;
    t.RY = 1;
    t.PD = 1;
    const int tiles = (N / t.TZ) * (N / t.TY);
    t.CX = N;
    while (t.CX > 4 && tiles * (N / t.CX) < 1024 && t.CX % 2 == 0) t.CX /= 2;
    cl::finalize_tile(t, N, prec);
    return t;
}

// The tile a lattice starts from: the tuned cache entry or the default.
Tile start_tile(const cl_lattice* h) {
    if (h->ng) return gw_tile(h->N, h->prec);
    Tile t = cl::default_tile(h->N, h->prec, h->nf);
    cached_tile(h->N, h->nf, h->prec, t);
    return t;
}

// A tile the pass with the gravitational-wave tensor can run.
bool gw_tile_ok(const Tile& t, cl_precision prec, int na) {
    return t.RY == 1 && t.PD == 1 && t.NT <= 256 && cl::pass_lds_bytes(t, prec, na) <= 64 * 1024;
}

void free_buffers(cl_lattice* h) {
    if (!h->own_buffers) return;
    for (auto& b : h->buf) {
        if (b) hipFree(b);
        b = nullptr;
    }
}

// Argument checks shared by cl_step and the allocation-free entry point.
cl_status check_step(cl_lattice* h, cl_integrator integ, double dt, int n) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (integ != CL_LEAPFROG && integ != CL_VV4 && !is_rk(integ)) return fail(h, CL_EINVAL, "unknown integrator");
    if (h->dim != 3 && is_rk(integ))
        return fail(h, CL_EUNSUPPORTED, "reduced lattices run the symplectic schemes only");
    if (h->ng && is_rk(integ))
        return fail(h, CL_EUNSUPPORTED, "with gravitational waves on, the symplectic schemes only");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(h, CL_EINVAL, "dt must be positive and finite");
    if (n < 0) return fail(h, CL_EINVAL, "n must be >= 0");
    if (n == 0) return CL_OK;
    return check_stability(h, integ, dt, "");
}

// After the passes of n steps were issued: the state moved to the other
// buffer if the number of passes is odd; copy the records, wait, and note
// the background on the host.
cl_status finish_step(cl_lattice* h, cl_integrator integ, int n, cl_observables* per_step, const cl::Work& w) {
    // passes that move the state to the other buffer (the classic RK4 step
    // ends where it started)
    const int stages = integ == CL_RK2 ? 2 : integ == CL_RK3 ? 3 : integ == CL_RK34 ? 4 : integ == CL_RK4 ? 5 : 0;
    const int passes = integ == CL_RK4_CLASSIC ? 0 : is_rk(integ) ? n * stages : 1 + n * substeps_per_step(integ);
    if (passes % 2) h->cur ^= 1;
    if (per_step)
        HIPCHECK(h, hipMemcpyAsync(per_step, w.obs, static_cast<size_t>(n) * sizeof(cl_observables),
                                   hipMemcpyDeviceToHost, h->stream));
    Scal s;
    HIPCHECK(h, hipMemcpyAsync(&s, h->sc, sizeof(Scal), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    h->step += n;
    note_background(h, s.a, s.mean_f);
    if (s.nonfinite) return fail(h, CL_EUNSTABLE, "non-finite lattice sums (unstable evolution)");
    return CL_OK;
}

}  // namespace

namespace cl {

cl_status set_error(cl_lattice* h, cl_status st, const char* msg) { return fail(h, st, msg); }

cl_status set_background_async(cl_lattice* h, double a, double b, double eta, int64_t step, const double* mean) {
    cl_status st = init_scalars(h, a, b, eta, mean);
    if (st) return st;
    h->step = step;
    note_background(h, a, mean);
    return CL_OK;
}

cl_status observe_once(cl_lattice* h, cl_observables* o, Scal* sc) { return reduce_pass(h, o, sc); }

cl_status step_in_work(cl_lattice* h, cl_integrator integ, double dt, int n, cl_observables* per_step,
                       const Work& w) {
    cl_status st = check_step(h, integ, dt, n);
    if (st || n == 0) return st;
    if (is_rk(integ))
        return fail(h, CL_EUNSUPPORTED, "the allocation-free step runs the symplectic schemes only");
    if (n > w.obs_cap) return fail(h, CL_EINVAL, "n exceeds the record capacity of the work area");
    if (static_cast<size_t>(nsums(h->nf)) * h->tile.nblocks() > w.half)
        return fail(h, CL_EINVAL, "the lattice's tile has more workgroups than the work area holds");
    st = issue_steps(h, integ, dt, n, h->cur, w);
    if (st) return st;
    return finish_step(h, integ, n, per_step, w);
}

}  // namespace cl

extern "C" {

const char* cl_version(void) { return "cl_lattice 0.1 (gfx950)"; }

const char* cl_last_error(const cl_lattice* h) { return h ? h->err.c_str() : g_err.c_str(); }

cl_status cl_create(int N, double dx, int n_fields, cl_precision prec, cl_lattice** out) {
    return cl_create_dim(3, N, dx, n_fields, prec, out);
}

cl_status cl_create_dim(int dim, int N, double dx, int n_fields, cl_precision prec, cl_lattice** out) {
    if (!out) return fail(nullptr, CL_EINVAL, "out is NULL");
    *out = nullptr;
    if (prec != CL_FP32 && prec != CL_FP64) return fail(nullptr, CL_EINVAL, "precision must be CL_FP32 or CL_FP64");
    if (dim < 1 || dim > 3) return fail(nullptr, CL_EINVAL, "dim must be 1, 2 or 3");
    if (dim == 3 && !valid_N(N, prec))
        return fail(nullptr, CL_EINVAL,
                    "N must be a power of two in [8, 1024] or a multiple of 256 (FP32) / 128 (FP64) up to 1600");
    if (dim < 3 && (N < 8 || N % 4 || (dim == 2 && N > 32768) || (dim == 1 && N > (1 << 28))))
        return fail(nullptr, CL_EINVAL, "reduced lattice: N must be a multiple of 4, at least 8 (and N^dim < 2^30)");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(nullptr, CL_EINVAL, "dx must be positive and finite");
    if (n_fields != 1 && n_fields != 2) return fail(nullptr, CL_EINVAL, "n_fields must be 1 or 2");
    cl_lattice* h = new (std::nothrow) cl_lattice;
    if (!h) return fail(nullptr, CL_ENOMEM, "handle");
    h->N = N;
    h->dim = dim;
    h->dx = dx;
    h->nf = n_fields;
    h->prec = prec;
    h->pot.lambda[0] = 1.0;
    const char* ng = std::getenv("CL_NO_GRAPH");
    h->use_graph = !(ng && ng[0] == '1');
    auto bail = [&](cl_status st, const std::string& m) {
        g_err = m;
        cl_destroy(h);
        return st;
    };
    if (hipGetDevice(&h->device) != hipSuccess) return bail(CL_EDEVICE, "no HIP device");
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(CL_EDEVICE, "hipStreamCreate failed");
    h->own_stream = true;
    const size_t bytes = 2 * n_fields * sites(h) * elem_size(prec);
    for (int pp = 0; pp < 2; ++pp) {
        if (hipMalloc(&h->buf[pp], bytes) != hipSuccess) {
            h->buf[pp] = nullptr;
            return bail(CL_ENOMEM, "device state buffers (2 x " + std::to_string(bytes) + " bytes)");
        }
        hipMemsetAsync(h->buf[pp], 0, bytes, h->stream);
    }
    const char* nt = std::getenv("CL_PASS_FLAGS");
    if (nt && nt[0]) h->pass_flags = std::atoi(nt);
    if (hipMalloc(&h->sc, sizeof(Scal)) != hipSuccess) return bail(CL_ENOMEM, "scalar block");
    if (hipMalloc(&h->scb, 2 * sizeof(Scal)) != hipSuccess) return bail(CL_ENOMEM, "scalar blocks");
    if (dim == 3) {
        h->tile = start_tile(h);
    } else {
        // grid-stride pass: 256 threads per workgroup, each on V sites
        const size_t groups = sites(h) / (prec == CL_FP32 ? 4 : 2);
        Tile t;
        t.TZ = N;
        t.TY = t.CX = t.RY = t.PD = t.HI = 1;
        if (dim == 2) {
            // rows marched per work item, at most 32, while one item per
            // thread still fills 512 workgroups (two per CU): longer marches
            // re-read fewer halo rows (4096^2, two fields: 32 rows and 512
            // workgroups measured 4 % faster than 16 rows and 1024)
            t.CX = 1;
            while (t.CX < 32 && N % (2 * t.CX) == 0 && groups / (2 * t.CX) >= 256u * 512u) t.CX *= 2;
        }
        t.NT = 256;
        t.nbz = static_cast<int>(std::min<size_t>((groups / t.CX + 255) / 256, cl::kTunedPassBlocks));
        t.nby = t.nbx = 1;
        h->tile = t;
    }
    if (ensure_partials(h) != CL_OK) return bail(CL_ENOMEM, h->err);
    double zero[2] = {0.0, 0.0};
    if (init_scalars(h, 1.0, 0.0, 0.0, zero) != CL_OK) return bail(CL_EDEVICE, h->err);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(CL_EDEVICE, "sync");
    *out = h;
    return CL_OK;
}

cl_status cl_destroy(cl_lattice* h) {
    if (!h) return CL_OK;
    if (h->stream) hipStreamSynchronize(h->stream);
    drop_graph(h);
    free_buffers(h);
    if (h->aux) hipFree(h->aux);
    if (h->aux2) hipFree(h->aux2);
    if (h->spec_host) (void)hipHostFree(h->spec_host);
    for (void* q : {(void*)h->spec, (void*)h->gw_spec, (void*)h->spec_tw, (void*)h->spec_sums, (void*)h->spec_counts})
        if (q) hipFree(q);
    if (h->sc) hipFree(h->sc);
    if (h->partials) hipFree(h->partials);
    if (h->scb) hipFree(h->scb);
    if (h->obs) hipFree(h->obs);
    if (h->own_stream && h->stream) hipStreamDestroy(h->stream);
    delete h;
    return CL_OK;
}

cl_status cl_set_stream(cl_lattice* h, void* s) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    if (h->own_stream) hipStreamDestroy(h->stream);
    h->own_stream = false;
    h->stream = static_cast<hipStream_t>(s);
    drop_graph(h);
    return CL_OK;
}

cl_status cl_attach_device_buffers(cl_lattice* h, void* state, void* state_pp) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!state || !state_pp) return fail(h, CL_EINVAL, "device buffer pointer is NULL");
    if (state == state_pp) return fail(h, CL_EINVAL, "the two state buffers must differ");
    for (void* x : {state, state_pp})
        if (reinterpret_cast<uintptr_t>(x) % 16) return fail(h, CL_EINVAL, "device buffers must be 16-byte aligned");
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    free_buffers(h);
    h->own_buffers = false;
    h->cur = 0;
    h->buf[0] = state;
    h->buf[1] = state_pp;
    drop_graph(h);
    return CL_OK;
}

cl_status cl_get_state_buffer(const cl_lattice* h, void** state) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!state) return fail(const_cast<cl_lattice*>(h), CL_EINVAL, "state is NULL");
    *state = h->buf[h->cur];
    return CL_OK;
}

cl_status cl_set_background(cl_lattice* h, double alpha, cl_expansion mode, double m_p, double a0) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!std::isfinite(alpha)) return fail(h, CL_EINVAL, "alpha must be finite");
    if (mode != CL_STATIC && mode != CL_SELF_CONSISTENT) return fail(h, CL_EINVAL, "unknown expansion mode");
    if (!(m_p > 0.0) || !std::isfinite(m_p)) return fail(h, CL_EINVAL, "m_p must be positive");
    if (!(a0 > 0.0) || !std::isfinite(a0)) return fail(h, CL_EINVAL, "a0 must be positive");
    if (mode == CL_STATIC && a0 != 1.0) return fail(h, CL_EINVAL, "static space needs a0 = 1");
    h->alpha = alpha;
    h->mode = mode;
    h->mp = m_p;
    h->a0 = a0;
    drop_graph(h);
    return CL_OK;
}

cl_status cl_set_potential(cl_lattice* h, const cl_potential* pot) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!pot) return fail(h, CL_EINVAL, "potential is NULL");
    const double* v = &pot->m2[0];
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(v[i])) return fail(h, CL_EINVAL, "potential coefficients must be finite");
    h->pot = *pot;
    drop_graph(h);
    return CL_OK;
}

cl_status cl_set_fields(cl_lattice* h, const double* f, const double* p) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!f || !p) return fail(h, CL_EINVAL, "field arrays must not be NULL");
    cl_status st = h->prec == CL_FP32 ? upload<float>(h, f, p) : upload<double>(h, f, p);
    if (st) return st;
    double mean[2];
    host_means(h, f, mean);
    return reset_background(h, mean);
}

cl_status cl_get_fields(cl_lattice* h, double* f, double* p) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!f && !p) return fail(h, CL_EINVAL, "both output arrays are NULL");
    return h->prec == CL_FP32 ? download<float>(h, f, p) : download<double>(h, f, p);
}

cl_status cl_seed(cl_lattice* h, uint64_t seed, const double* fbar, const double* pbar, double cutoff,
                  double amp) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (h->dim != 3)
        return fail(h, CL_EUNSUPPORTED, "the seed is three-dimensional; set reduced lattices with cl_set_fields");
    if (!fbar || !pbar) return fail(h, CL_EINVAL, "fbar / pbar must not be NULL");
    if (h->N & (h->N - 1)) return fail(h, CL_EUNSUPPORTED, "cl_seed needs N to be a power of two");
    if (!std::isfinite(amp) || amp < 0.0) return fail(h, CL_EINVAL, "amp must be finite and >= 0");
    if (cutoff <= 0.0) cutoff = h->N / 4.0;
    const size_t n = sites(h) * h->nf;
    std::vector<double> f, p;
    try {
        f.resize(n);
        p.resize(n);
    } catch (const std::bad_alloc&) {
        return fail(h, CL_ENOMEM, "host seed arrays");
    }
    const Phys ph = make_phys(h);
    const char* e = cl::host_seed(h->N, h->dx, h->nf, ph, h->a0, seed, fbar, pbar, cutoff, amp, f.data(), p.data());
    if (e && e[0]) return fail(h, CL_EINVAL, e);
    return cl_set_fields(h, f.data(), p.data());
}

cl_status cl_get_state(const cl_lattice* hc, cl_scalars* out) {
    cl_lattice* h = const_cast<cl_lattice*>(hc);
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!out) return fail(h, CL_EINVAL, "out is NULL");
    Scal s;
    HIPCHECK(h, hipMemcpyAsync(&s, h->sc, sizeof(Scal), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    out->a = s.a;
    out->b = s.b;
    out->eta = s.eta;
    out->step = h->step;
    return CL_OK;
}

cl_status cl_set_state(cl_lattice* h, const cl_scalars* in) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!in) return fail(h, CL_EINVAL, "in is NULL");
    if (!(in->a > 0.0) || !std::isfinite(in->b) || !std::isfinite(in->eta) || in->step < 0)
        return fail(h, CL_EINVAL, "invalid background state");
    if (h->mode == CL_STATIC && (in->a != 1.0 || in->b != 0.0))
        return fail(h, CL_EINVAL, "static space needs a = 1, a' = 0");
    Scal s;
    HIPCHECK(h, hipMemcpyAsync(&s, h->sc, sizeof(Scal), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    cl_status st = init_scalars(h, in->a, in->b, in->eta, s.mean_f);
    if (st) return st;
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    h->step = in->step;
    note_background(h, in->a, s.mean_f);
    return CL_OK;
}

cl_status cl_step(cl_lattice* h, cl_integrator integ, double dt, int n, cl_observables* per_step) {
    cl_status st = check_step(h, integ, dt, n);
    if (st || n == 0) return st;
    st = ensure_obs(h, n);
    if (st) return st;
    if (is_rk(integ) && !h->aux) {
        // Runge-Kutta registers of (f, pi): one more state-sized buffer
        if (hipMalloc(&h->aux, state_bytes(h)) != hipSuccess) {
            h->aux = nullptr;
            return fail(h, CL_ENOMEM, "Runge-Kutta registers (" + std::to_string(state_bytes(h)) + " bytes)");
        }
        drop_graph(h);
    }
    if (integ == CL_RK4_CLASSIC && !h->aux2) {
        // the classic scheme's third stage buffer
        if (hipMalloc(&h->aux2, state_bytes(h)) != hipSuccess) {
            h->aux2 = nullptr;
            return fail(h, CL_ENOMEM, "RK4 stage buffer (" + std::to_string(state_bytes(h)) + " bytes)");
        }
        drop_graph(h);
    }
    const GraphKey key{static_cast<int>(integ), dt, n, h->cur};
    const cl::Work w = handle_work(h);
    if (h->use_graph && n > 1) {
        hipGraphExec_t& gx = h->gexec[h->cur];
        if (!(gx && h->gkey[h->cur] == key)) {
            if (gx) hipGraphExecDestroy(gx);
            gx = nullptr;
            hipGraph_t g = nullptr;
            HIPCHECK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
            st = issue_steps(h, integ, dt, n, h->cur, w);
            hipError_t e = hipStreamEndCapture(h->stream, &g);
            if (st) {
                if (g) hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) return fail(h, CL_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (e != hipSuccess) {
                gx = nullptr;
                return fail(h, CL_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
            }
            h->gkey[h->cur] = key;
        }
        HIPCHECK(h, hipGraphLaunch(gx, h->stream));
    } else {
        st = issue_steps(h, integ, dt, n, h->cur, w);
        if (st) return st;
    }
    return finish_step(h, integ, n, per_step, w);
}

cl_status cl_read_observables(cl_lattice* h, cl_observables* out) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!out) return fail(h, CL_EINVAL, "out is NULL");
    // Two passes: the first fixes the variance shift at the exact mean.
    cl_observables o;
    cl_status st = reduce_pass(h, &o);
    if (st) return st;
    return reduce_pass(h, out);
}

}  // extern "C"

namespace {

// Twiddle factors exp(-2 pi i k / N) of the line FFTs, formed in long double
// and rounded once; allocated on first use.
cl_status ensure_twiddles(cl_lattice* h) {
    if (h->spec_tw) return CL_OK;
    const int N = h->N;
    std::vector<double2> tw(N / 2);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < N / 2; ++k) {
        const long double t = -2.0L * pi * k / N;
        tw[k] = make_double2(static_cast<double>(std::cos(t)), static_cast<double>(std::sin(t)));
    }
    HIPCHECK(h, hipMalloc(&h->spec_tw, (N / 2 > 0 ? N / 2 : 1) * sizeof(double2)));
    HIPCHECK(h, hipMemcpyAsync(h->spec_tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return CL_OK;
}

}  // namespace

namespace cl {
cl_status spectral_twiddles(cl_lattice* h, const double2** tw) {
    const cl_status st = ensure_twiddles(h);
    if (st) return st;
    *tw = h->spec_tw;
    return CL_OK;
}
}  // namespace cl

namespace {

// Per-bin sums and counts for `slots` bins.
cl_status ensure_bins(cl_lattice* h, int slots) {
    if (h->spec_cap >= slots) return CL_OK;
    if (h->spec_sums) (void)hipFree(h->spec_sums);
    if (h->spec_counts) (void)hipFree(h->spec_counts);
    if (h->spec_host) (void)hipHostFree(h->spec_host);
    h->spec_sums = nullptr;
    h->spec_counts = nullptr;
    h->spec_host = nullptr;
    h->spec_cap = 0;
    HIPCHECK(h, hipMalloc(&h->spec_sums, slots * sizeof(double)));
    HIPCHECK(h, hipMalloc(&h->spec_counts, slots * sizeof(unsigned long long)));
    HIPCHECK(h, hipHostMalloc(&h->spec_host, 2 * static_cast<size_t>(slots) * sizeof(double)));
    h->spec_cap = slots;
    return CL_OK;
}

cl_status check_spectrum_args(cl_lattice* h, double width, int nbins) {
    if (h->dim != 3) return fail(h, CL_EUNSUPPORTED, "the power spectrum is three-dimensional");
    if (!(width > 0.0) || !std::isfinite(width)) return fail(h, CL_EINVAL, "bin width must be positive");
    if (nbins < 1 || nbins > 4096) return fail(h, CL_EINVAL, "nbins must be in [1, 4096]");
    if ((h->N & (h->N - 1)) != 0) return fail(h, CL_EUNSUPPORTED, "the spectrum needs N a power of two");
    return CL_OK;
}

// Device state buffers of the other layout (na_new stencil arrays per row):
// the fields and momenta of the current state are copied over, every other
// array starts at zero.
cl_status relayout(cl_lattice* h, int ng_new) {
    const size_t N = static_cast<size_t>(h->N), es = elem_size(h->prec);
    const int na_old = arrays(h), na_new = h->nf + ng_new;
    const size_t bytes = 2 * static_cast<size_t>(na_new) * sites(h) * es;
    void* nb[2] = {nullptr, nullptr};
    for (int pp = 0; pp < 2; ++pp) {
        if (hipMalloc(&nb[pp], bytes) != hipSuccess) {
            if (nb[0]) (void)hipFree(nb[0]);
            return fail(h, CL_ENOMEM, "device state buffers (2 x " + std::to_string(bytes) + " bytes)");
        }
        HIPCHECK(h, hipMemsetAsync(nb[pp], 0, bytes, h->stream));
    }
    for (int which = 0; which < 2; ++which)
        for (int j = 0; j < h->nf; ++j) {
            const char* src = static_cast<const char*>(h->buf[h->cur]) + (which * na_old + j) * N * es;
            char* dst = static_cast<char*>(nb[0]) + (which * na_new + j) * N * es;
            HIPCHECK(h, hipMemcpy2DAsync(dst, 2 * na_new * N * es, src, 2 * na_old * N * es, N * es, rows(h),
                                         hipMemcpyDeviceToDevice, h->stream));
        }
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    free_buffers(h);
    h->buf[0] = nb[0];
    h->buf[1] = nb[1];
    h->cur = 0;
    h->ng = ng_new;
    // Runge-Kutta registers have the state's layout
    for (void** q : {&h->aux, &h->aux2})
        if (*q) {
            (void)hipFree(*q);
            *q = nullptr;
        }
    h->tile = start_tile(h);
    cl_status st = ensure_partials(h);
    if (st) return st;
    drop_graph(h);
    return CL_OK;
}

}  // namespace

extern "C" {

cl_status cl_power_spectrum(cl_lattice* h, int field, int what, double width, int nbins, int64_t* counts,
                            double* sums, double* delta) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    cl_status st = check_spectrum_args(h, width, nbins);
    if (st) return st;
    if (field < 0 || field >= h->nf) return fail(h, CL_EINVAL, "field index out of range");
    if (what != 0 && what != 1) return fail(h, CL_EINVAL, "what must be 0 (f) or 1 (pi)");
    const int N = h->N;
    const size_t n3 = sites(h);
    if (!h->spec) {
        if (hipMalloc(&h->spec, n3 * sizeof(double2)) != hipSuccess) {
            h->spec = nullptr;
            return fail(h, CL_ENOMEM, "spectrum buffer (" + std::to_string(n3 * sizeof(double2)) + " bytes)");
        }
    }
    if ((st = ensure_twiddles(h)) || (st = ensure_bins(h, nbins))) return st;
    const int arr = what == 0 ? field : arrays(h) + field;
    // extraction fused with the z pass, the y pass, the x pass fused with the
    // binning: three sweeps of the complex array, the last two over the half
    // z <= N / 2 (pitch P) that a real array's transform needs
    // (the first pass clears the bins; they are copied to pinned memory)
    const int P = cl::spec_half_pitch(N), cap = h->spec_cap;
    HIPCHECK(h, cl::launch_spec_extract_fftz(h->buf[h->cur], h->prec == CL_FP32, N, 2 * arrays(h), arr, h->spec_tw,
                                             h->spec, P, h->spec_sums, h->spec_counts, nbins, h->stream));
    HIPCHECK(h, cl::launch_spec_fft(h->spec, h->spec_tw, N, 1, h->stream, false, P));
    HIPCHECK(h, cl::launch_spec_fftx_bin(h->spec, h->spec_tw, N, P, width, nbins, h->spec_sums, h->spec_counts,
                                         h->stream));
    HIPCHECK(h, hipMemcpyAsync(h->spec_host, h->spec_sums, nbins * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipMemcpyAsync(h->spec_host + cap, h->spec_counts, nbins * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    const double* s = h->spec_host;
    const unsigned long long* c = reinterpret_cast<const unsigned long long*>(h->spec_host + cap);
    const double k_ir = 2.0 * M_PI / (N * h->dx);
    const double n5 = std::pow(static_cast<double>(N), 5.0);
    for (int l = 0; l < nbins; ++l) {
        if (counts) counts[l] = static_cast<int64_t>(c[l]);
        if (sums) sums[l] = s[l];
        if (delta) delta[l] = (k_ir * width * l) / (2.0 * M_PI) * h->dx / n5 * s[l];
    }
    return CL_OK;
}

cl_status cl_gw_enable(cl_lattice* h, int on) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (h->dim != 3) return fail(h, CL_EUNSUPPORTED, "gravitational waves need a three-dimensional lattice");
    const int ng_new = on ? 5 : 0;
    if (ng_new == h->ng) return CL_OK;
    if (!h->own_buffers)
        return fail(h, CL_ESTATE, "switch gravitational waves on before attaching device buffers");
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return relayout(h, ng_new);
}

cl_status cl_gw_set(cl_lattice* h, const double* v, const double* u) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!h->ng) return fail(h, CL_ESTATE, "gravitational waves are off");
    if (!v || !u) return fail(h, CL_EINVAL, "tensor arrays must not be NULL");
    if (h->prec == CL_FP32) {
        cl_status st = upload_arrays<float>(h, v, h->nf, h->ng);
        return st ? st : upload_arrays<float>(h, u, arrays(h) + h->nf, h->ng);
    }
    cl_status st = upload_arrays<double>(h, v, h->nf, h->ng);
    return st ? st : upload_arrays<double>(h, u, arrays(h) + h->nf, h->ng);
}

cl_status cl_gw_get(cl_lattice* h, double* v, double* u) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!h->ng) return fail(h, CL_ESTATE, "gravitational waves are off");
    if (!v && !u) return fail(h, CL_EINVAL, "both output arrays are NULL");
    cl_status st = CL_OK;
    if (v) st = h->prec == CL_FP32 ? download_arrays<float>(h, v, h->nf, h->ng) : download_arrays<double>(h, v, h->nf, h->ng);
    if (st || !u) return st;
    return h->prec == CL_FP32 ? download_arrays<float>(h, u, arrays(h) + h->nf, h->ng)
                              : download_arrays<double>(h, u, arrays(h) + h->nf, h->ng);
}

cl_status cl_gw_spectrum(cl_lattice* h, double width, int nbins, int64_t* counts, double* rho, double* omega,
                         double* rho_gw) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!h->ng) return fail(h, CL_ESTATE, "gravitational waves are off");
    cl_status st = check_spectrum_args(h, width, nbins);
    if (st) return st;
    const int N = h->N;
    const size_t n3 = sites(h);
    if (!h->gw_spec) {
        if (hipMalloc(&h->gw_spec, 5 * n3 * sizeof(double2)) != hipSuccess) {
            h->gw_spec = nullptr;
            return fail(h, CL_ENOMEM, "gravitational-wave spectrum buffer (" + std::to_string(5 * n3 * sizeof(double2)) +
                                          " bytes)");
        }
    }
    if ((st = ensure_twiddles(h)) || (st = ensure_bins(h, nbins + 1))) return st;
    // the half z <= N / 2 of each transform (pitch P), as for the scalar
    // spectrum; the first extraction clears the bins
    const int P = cl::spec_half_pitch(N);
    for (int c = 0; c < 5; ++c) {
        double2* dst = h->gw_spec + c * n3;
        // extraction of the component fused with the z pass, then y and x
        HIPCHECK(h, cl::launch_spec_extract_fftz(h->buf[h->cur], h->prec == CL_FP32, N, 2 * arrays(h),
                                                 arrays(h) + h->nf + c, h->spec_tw, dst, P,
                                                 c == 0 ? h->spec_sums : nullptr, h->spec_counts, nbins + 1,
                                                 h->stream));
        for (int axis = 1; axis < 3; ++axis)
            HIPCHECK(h, cl::launch_spec_fft(dst, h->spec_tw, N, axis, h->stream, false, P));
    }
    HIPCHECK(h, cl::launch_gw_bin(h->gw_spec, N, P, width, nbins, h->spec_sums, h->spec_counts, h->stream));
    std::vector<double> s(nbins + 1);
    std::vector<unsigned long long> c(nbins);
    HIPCHECK(h, hipMemcpyAsync(s.data(), h->spec_sums, (nbins + 1) * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipMemcpyAsync(c.data(), h->spec_counts, nbins * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                               h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    cl_observables o;
    st = cl_read_observables(h, &o);
    if (st) return st;
    // h' = a^(alpha-3) u; rho_GW = m_p^2 <h'_ij h'_ij> / (4 a^(2 alpha)), <.> = N^-6 sum over modes
    const double a = o.a;
    const double scale = h->mp * h->mp / (4.0 * std::pow(a, 2.0 * h->alpha)) * std::pow(a, 2.0 * (h->alpha - 3.0)) /
                         std::pow(static_cast<double>(N), 6.0);
    const double rho_tot = o.EK[0] + o.EK[1] + o.EG[0] + o.EG[1] + o.EV;
    double total = 0.0;
    for (int l = 0; l <= nbins; ++l) total += s[l];
    for (int l = 0; l < nbins; ++l) {
        if (counts) counts[l] = static_cast<int64_t>(c[l]);
        if (rho) rho[l] = scale * s[l];
        if (omega) omega[l] = l * scale * s[l] / rho_tot;
    }
    if (rho_gw) *rho_gw = scale * total;
    return CL_OK;
}

cl_status cl_get_tile(const cl_lattice* h, cl_tile* out) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (!out) return fail(const_cast<cl_lattice*>(h), CL_EINVAL, "out is NULL");
    out->tz = h->tile.TZ;
    out->ty = h->tile.TY;
    out->cx = h->tile.CX;
    out->ry = h->tile.RY;
    out->pd = h->tile.PD;
    return CL_OK;
}

cl_status cl_set_tile(cl_lattice* h, const cl_tile* t) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (h->dim != 3) return fail(h, CL_EUNSUPPORTED, "reduced lattices have no tile choice");
    if (!t) return fail(h, CL_EINVAL, "tile is NULL");
    Tile c;
    c.TZ = t->tz;
    c.TY = t->ty;
    c.CX = t->cx;
    c.RY = t->ry;
    c.PD = t->pd == 0 ? 1 : t->pd;
    if (!cl::finalize_tile(c, h->N, h->prec)) return fail(h, CL_EINVAL, "tile does not fit this lattice");
    if (cl::pass_lds_bytes(c, h->prec, arrays(h)) > 60 * 1024) return fail(h, CL_EINVAL, "tile needs too much LDS");
    if (h->ng && !gw_tile_ok(c, h->prec, arrays(h)))
        return fail(h, CL_EINVAL, "with gravitational waves on, tiles take one row per thread, depth 1, <= 256 threads");
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    const Tile old = h->tile;
    h->tile = c;
    cl_status st = ensure_partials(h);
    if (st) {
        h->tile = old;
        return st;
    }
    drop_graph(h);
    return CL_OK;
}

cl_status cl_autotune(cl_lattice* h, int reps, char* report, size_t cap) {
    if (!h) return fail(nullptr, CL_EINVAL, "handle is NULL");
    if (h->dim != 3) return fail(h, CL_EUNSUPPORTED, "reduced lattices have no tile choice");
    if (reps < 1) reps = 3;
    std::vector<Tile> cands(1024);
    int nc = 0;
    cl::candidate_tiles(h->N, h->prec, h->nf, cands.data(), &nc, static_cast<int>(cands.size()));
    if (h->ng) {
        // the pass with the tensor: one-row, depth-1 tiles of at most 256 threads
        std::vector<Tile> keep;
        for (int i = 0; i < nc; ++i) {
            Tile c = cands[i];
            c.PD = 1;
            if (c.RY != 1 || !cl::finalize_tile(c, h->N, h->prec) || !gw_tile_ok(c, h->prec, arrays(h))) continue;
            bool dup = false;
            for (const Tile& k : keep) dup = dup || (k.TZ == c.TZ && k.TY == c.TY && k.CX == c.CX);
            if (!dup) keep.push_back(c);
        }
        nc = static_cast<int>(keep.size());
        for (int i = 0; i < nc; ++i) cands[i] = keep[i];
    }
    if (nc == 0) return fail(h, CL_EUNSUPPORTED, "no candidate tile");
    int maxb = 0;
    for (int i = 0; i < nc; ++i) maxb = std::max(maxb, cands[i].nblocks());
    cl_status st = ensure_partials(h, maxb);
    if (st) return st;
    Scal saved;
    HIPCHECK(h, hipMemcpyAsync(&saved, h->sc, sizeof(Scal), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    hipEvent_t e0, e1;
    HIPCHECK(h, hipEventCreate(&e0));
    HIPCHECK(h, hipEventCreate(&e1));
    std::string js = "{\"N\":" + std::to_string(h->N) + ",\"nf\":" + std::to_string(h->nf) + ",\"prec\":\"" +
                     prec_name(h->prec) + "\",\"reps\":" + std::to_string(reps) + ",\"candidates\":[";
    // With a zero drift coefficient, zero kicks and no drift step to follow, a
    // pass copies (f, pi) exactly and its scalar step leaves a, a' and the
    // (zero) drift coefficient as they are.  So the timed passes chain like a
    // real run -- each reads what the previous one wrote and runs its scalar
    // step first -- and an even number of them leaves the state bitwise
    // unchanged.
    Scal zero_drift = saved;
    zero_drift.cd = 0.0;
    const int pairs = (reps + 1) / 2;
    const Tile keep = h->tile;
    // passes of tile t, `np` timed pairs after a warm-up pair; < 0 if it
    // does not launch
    auto time_tile = [&](const Tile& t, int np) -> float {
        h->tile = t;
        if (hipMemcpyAsync(h->sc, &zero_drift, sizeof(Scal), hipMemcpyHostToDevice, h->stream) != hipSuccess)
            return -1.0f;
        PassArgs a[2];
        for (int q = 0; q < 2; ++q) {
            a[q] = base_args(h, h->cur ^ q);
            a[q].drift = 1;
            a[q].write_out = 1;
            a[q].kt = 0.0;
            a[q].kb = 0.0;
            a[q].h_next = 0.0;
            a[q].rec = -1;
        }
        PassSeq seq(h);
        if (seq.launch(a[0]) != hipSuccess || seq.launch(a[1]) != hipSuccess) {
            (void)hipGetLastError();
            (void)seq.close();
            return -1.0f;
        }
        hipEventRecord(e0, h->stream);
        for (int r = 0; r < np; ++r) {
            (void)seq.launch(a[0]);
            (void)seq.launch(a[1]);
        }
        hipEventRecord(e1, h->stream);
        if (seq.close() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0f;
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        return ms / (2 * np);
    };
    // screening: every candidate once
    std::vector<std::pair<float, int>> timed;
    for (int i = 0; i < nc; ++i) {
        const Tile& t = cands[i];
        const float ms = time_tile(t, pairs);
        if (ms < 0.0f) continue;
        timed.emplace_back(ms, i);
        char item[160];
        std::snprintf(item, sizeof item, "%s{\"tz\":%d,\"ty\":%d,\"cx\":%d,\"ry\":%d,\"pd\":%d,\"us\":%.2f}",
                      timed.size() > 1 ? "," : "", t.TZ, t.TY, t.CX, t.RY, t.PD, ms * 1e3);
        js += item;
    }
    // refinement: the fastest few again, three interleaved rounds of longer
    // runs, each finalist's best round counts (short screens are noisy at a
    // few per cent, the size of the gaps between the leading tiles)
    std::sort(timed.begin(), timed.end());
    const int nfin = std::min<int>(4, static_cast<int>(timed.size()));
    std::vector<float> fin_ms(nfin, -1.0f);
    for (int round = 0; round < 3; ++round)
        for (int k = 0; k < nfin; ++k) {
            const float ms = time_tile(cands[timed[k].second], std::max(pairs, 20));
            if (ms >= 0.0f && (fin_ms[k] < 0.0f || ms < fin_ms[k])) fin_ms[k] = ms;
        }
    int best = -1;
    float best_ms = 0.0f;
    js += "],\"finalists\":[";
    for (int k = 0; k < nfin; ++k) {
        const Tile& t = cands[timed[k].second];
        char item[160];
        std::snprintf(item, sizeof item, "%s{\"tz\":%d,\"ty\":%d,\"cx\":%d,\"ry\":%d,\"pd\":%d,\"us\":%.2f}",
                      k ? "," : "", t.TZ, t.TY, t.CX, t.RY, t.PD, fin_ms[k] * 1e3);
        js += item;
        if (fin_ms[k] >= 0.0f && (best < 0 || fin_ms[k] < best_ms)) {
            best = timed[k].second;
            best_ms = fin_ms[k];
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    h->tile = keep;
    HIPCHECK(h, hipMemcpyAsync(h->sc, &saved, sizeof(Scal), hipMemcpyHostToDevice, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    if (best < 0) return fail(h, CL_EDEVICE, "no candidate tile launched");
    h->tile = cands[best];
    drop_graph(h);
    char tail[200];
    std::snprintf(tail, sizeof tail, "],\"best\":{\"tz\":%d,\"ty\":%d,\"cx\":%d,\"ry\":%d,\"pd\":%d,\"us\":%.2f}}",
                  h->tile.TZ, h->tile.TY, h->tile.CX, h->tile.RY, h->tile.PD, best_ms * 1e3);
    js += tail;
    if (report && cap) {
        std::strncpy(report, js.c_str(), cap - 1);
        report[cap - 1] = '\0';
    }
    const char* path = std::getenv("CL_TUNE_CACHE");
    if (path && path[0]) {
        FILE* fp = std::fopen(path, "a");
        if (fp) {
            std::fprintf(fp, "{\"arch\":\"gfx950\",\"N\":%d,\"nf\":%d,\"prec\":\"%s\",\"tz\":%d,\"ty\":%d,\"cx\":%d,\"ry\":%d,\"pd\":%d,\"us\":%.2f}\n",
                         h->N, h->nf, prec_name(h->prec), h->tile.TZ, h->tile.TY, h->tile.CX, h->tile.RY,
                         h->tile.PD, best_ms * 1e3);
            std::fclose(fp);
        }
    }
    return CL_OK;
}

cl_status cl_copy_bandwidth(size_t bytes, int reps, double* gbps) {
    if (!gbps) return fail(nullptr, CL_EINVAL, "gbps is NULL");
    bytes &= ~static_cast<size_t>(15);
    if (bytes == 0 || reps < 1) return fail(nullptr, CL_EINVAL, "bytes and reps must be positive");
    void* a = nullptr;
    void* b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) return fail(nullptr, CL_ENOMEM, "copy probe buffer");
    if (hipMalloc(&b, bytes) != hipSuccess) {
        hipFree(a);
        return fail(nullptr, CL_ENOMEM, "copy probe buffer");
    }
    hipMemset(a, 0, bytes);
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    cl::launch_copy(a, b, bytes, nullptr);
    hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps; ++r) cl::launch_copy(a, b, bytes, nullptr);
    hipEventRecord(e1, nullptr);
    hipEventSynchronize(e1);
    float ms = 0.0f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(a);
    hipFree(b);
    if (!(ms > 0.0f)) return fail(nullptr, CL_EDEVICE, "copy probe timing failed");
    *gbps = 2.0 * static_cast<double>(bytes) * reps / (ms * 1e-3) / 1e9;
    return CL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- ensembles
//
// Independent lattices (uneven sizes allowed) advanced together: every pass
// of every member runs in one persistent launch that hands out tiles of all
// members from a work counter; the passes of a call are captured in one HIP
// graph.  Members keep their own potential, background, scale factor, time
// step and state buffers, so a member's handle stays usable on its own.

struct cl_ensemble {
    std::vector<cl_lattice*> m;
    cl_precision prec = CL_FP32;
    int nf = 1;
    std::vector<cl::EnsMember> table;
    cl::EnsMember* staging = nullptr;  // pinned host copy of the member table
    cl::EnsMember* d_table = nullptr;
    cl::EnsItem* d_items = nullptr;
    int nitems = 0;
    double* d_partials = nullptr;
    cl::Scal* d_scb = nullptr;      // two scratch scalar blocks per member
    unsigned* d_counter = nullptr;
    cl_observables* d_obs = nullptr;
    size_t obs_cap = 0;
    std::vector<double> dt;
    hipStream_t stream = nullptr;
    int grid = 0;
    size_t lds = 0;
    hipGraphExec_t gexec = nullptr;
    int g_integ = -1, g_n = -1;
    size_t partials_cap = 0, items_cap = 0;  // allocated slots
    int item_sites = 0;                      // layout parameters in use
    bool two_rows = true;
    int maxry = 1;                           // largest rows per thread among the members
    bool broken = false;                     // a layout change failed half way: no further steps
};

namespace {

cl_status efail(cl_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

#define EHIP(call)                                                                              \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) return efail(CL_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Default layout: about 32k sites per work item, two rows per thread where
// the lattice is tall enough.
constexpr int kEnsItemSites = 32768;

// Tile of one member: 256 threads, full rows when N <= 64 vectors, about
// item_sites sites per work item.
bool ensemble_tile(int N, cl_precision prec, cl::EnsMember& t, int item_sites, bool two_rows) {
    const int V = prec == CL_FP32 ? 4 : 2;
    t.TZ = N < 64 * V ? N : 64 * V;
    if (t.TZ % V || N % t.TZ) return false;
    const int BZ = t.TZ / V;
    if (256 % BZ) return false;
    // two rows per thread where the lattice is tall enough: twice the work
    // per plane against the same per-plane barriers and LDS round trips
    t.RY = (two_rows && 2 * 256 / BZ <= N && N % (2 * 256 / BZ) == 0) ? 2 : 1;
    t.TY = t.RY * 256 / BZ;
    if (t.TY > N || N % t.TY) return false;
    int cx = item_sites / (t.TZ * t.TY);
    if (cx < 2) cx = 2;
    while (cx > N || N % cx) cx /= 2;
    if (cx < 1) return false;
    t.CX = cx;
    t.nbz = N / t.TZ;
    t.nby = N / t.TY;
    t.nbx = N / t.CX;
    t.nitems = t.nbz * t.nby * t.nbx;
    // halo items must fit one per thread
    return 2 * BZ + 2 * t.TY <= 256;
}

// Work decomposition of all members for one (item size, rows per thread)
// choice: member tiles, the flat item list, partial-sum slots, LDS size and
// grid.  Device storage grows as needed; a captured graph is dropped.
cl_status ens_layout(cl_ensemble* e, int item_sites, bool two_rows) {
    const int n = static_cast<int>(e->m.size());
    std::vector<cl::EnsMember> table(n);
    std::vector<size_t> offs(n);
    std::vector<cl::EnsItem> items;
    size_t poff = 0;
    int maxTY = 0, maxTZ = 0;
    for (int i = 0; i < n; ++i) {
        cl::EnsMember t{};
        const int N = e->m[i]->N;
        if (!ensemble_tile(N, e->prec, t, item_sites, two_rows))
            return efail(CL_EUNSUPPORTED, "member " + std::to_string(i) + ": N = " + std::to_string(N) +
                                              " is too small for an ensemble tile (N >= 32 needed)");
        for (int k = 0; k < t.nitems; ++k) items.push_back({i, k});
        offs[i] = poff;
        poff += 2 * static_cast<size_t>(cl::nsums(e->nf)) * t.nitems;  // two halves
        maxTY = std::max(maxTY, t.TY);
        maxTZ = std::max(maxTZ, t.TZ);
        table[i] = t;
    }
    if (e->gexec) hipGraphExecDestroy(e->gexec);
    e->gexec = nullptr;
    EHIP(hipStreamSynchronize(e->stream));
    // from here on the old layout's device storage may be gone
    e->broken = true;
    if (poff > e->partials_cap) {
        if (e->d_partials) hipFree(e->d_partials);
        e->d_partials = nullptr;
        e->partials_cap = 0;
        if (hipMalloc(&e->d_partials, poff * sizeof(double)) != hipSuccess) {
            e->d_partials = nullptr;
            return efail(CL_ENOMEM, "ensemble partial sums");
        }
        e->partials_cap = poff;
    }
    if (items.size() > e->items_cap) {
        if (e->d_items) hipFree(e->d_items);
        e->d_items = nullptr;
        e->items_cap = 0;
        if (hipMalloc(&e->d_items, items.size() * sizeof(cl::EnsItem)) != hipSuccess) {
            e->d_items = nullptr;
            return efail(CL_ENOMEM, "ensemble work items");
        }
        e->items_cap = items.size();
    }
    for (int i = 0; i < n; ++i) {
        table[i].partials = e->d_partials + offs[i];
        table[i].scb = e->d_scb + 2 * i;
    }
    EHIP(hipMemcpyAsync(e->d_items, items.data(), items.size() * sizeof(cl::EnsItem), hipMemcpyHostToDevice,
                        e->stream));
    EHIP(hipStreamSynchronize(e->stream));
    e->table = table;
    e->nitems = static_cast<int>(items.size());
    e->lds = cl::ensemble_lds_bytes(e->prec, e->nf, maxTY, maxTZ);
    e->maxry = 1;
    for (const cl::EnsMember& t : e->table) e->maxry = std::max(e->maxry, t.RY);
    e->grid = std::min(cl::ensemble_grid(e->prec, e->nf, e->lds, e->maxry), e->nitems);
    e->item_sites = item_sites;
    e->two_rows = two_rows;
    e->broken = false;
    return CL_OK;
}

// The member table as the kernel reads it: the layout plus each member's
// buffers, current buffer, physics and scalar block, uploaded on the stream.
cl_status ens_upload_table(cl_ensemble* e, bool with_dt) {
    const int nm = static_cast<int>(e->m.size());
    for (int i = 0; i < nm; ++i) {
        cl::EnsMember t = e->table[i];
        cl_lattice* h = e->m[i];
        t.buf[0] = h->buf[0];
        t.buf[1] = h->buf[1];
        t.N = h->N;
        t.cur0 = h->cur;
        t.dt = with_dt ? e->dt[i] : 1.0;
        t.ph = make_phys(h);
        t.sc = h->sc;
        e->staging[i] = t;
    }
    EHIP(hipMemcpyAsync(e->d_table, e->staging, nm * sizeof(cl::EnsMember), hipMemcpyHostToDevice, e->stream));
    return CL_OK;
}

void ens_free(cl_ensemble* e) {
    if (e->stream) hipStreamSynchronize(e->stream);
    if (e->gexec) hipGraphExecDestroy(e->gexec);
    if (e->staging) hipHostFree(e->staging);
    for (void* p : {(void*)e->d_table, (void*)e->d_items, (void*)e->d_partials, (void*)e->d_scb,
                    (void*)e->d_counter, (void*)e->d_obs})
        if (p) hipFree(p);
    if (e->stream) hipStreamDestroy(e->stream);
    delete e;
}

}  // namespace

extern "C" {

cl_status cl_ensemble_create(int n, cl_lattice* const* members, cl_ensemble** out) {
    if (!out) return efail(CL_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !members) return efail(CL_EINVAL, "need at least one member");
    cl_ensemble* e = new (std::nothrow) cl_ensemble;
    if (!e) return efail(CL_ENOMEM, "ensemble handle");
    auto bail = [&](cl_status st, const std::string& msg) {
        ens_free(e);
        return efail(st, msg);
    };
    e->prec = members[0] ? members[0]->prec : CL_FP32;
    e->nf = members[0] ? members[0]->nf : 1;
    for (int i = 0; i < n; ++i) {
        cl_lattice* h = members[i];
        if (!h) return bail(CL_EINVAL, "member " + std::to_string(i) + " is NULL");
        for (int k = 0; k < i; ++k)
            if (members[k] == h) return bail(CL_EINVAL, "a lattice appears twice in the ensemble");
        if (h->prec != e->prec || h->nf != e->nf)
            return bail(CL_EINVAL, "all members need the same precision and number of fields");
        if (h->dim != 3) return bail(CL_EUNSUPPORTED, "ensemble members are three-dimensional lattices");
        if (h->ng) return bail(CL_EUNSUPPORTED, "ensemble members carry no gravitational-wave tensor");
        e->m.push_back(h);
    }
    e->dt.assign(n, 0.0);
    if (hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(CL_EDEVICE, "hipStreamCreate failed");
    if (hipMalloc(&e->d_scb, 2 * n * sizeof(cl::Scal)) != hipSuccess ||
        hipMalloc(&e->d_counter, 64) != hipSuccess ||
        hipMalloc(&e->d_table, n * sizeof(cl::EnsMember)) != hipSuccess ||
        hipHostMalloc(&e->staging, n * sizeof(cl::EnsMember)) != hipSuccess)
        return bail(CL_ENOMEM, "ensemble device tables");
    if (hipMemsetAsync(e->d_scb, 0, 2 * n * sizeof(cl::Scal), e->stream) != hipSuccess ||
        hipMemsetAsync(e->d_counter, 0, 64, e->stream) != hipSuccess ||
        hipStreamSynchronize(e->stream) != hipSuccess)
        return bail(CL_EDEVICE, "ensemble table upload");
    const cl_status st = ens_layout(e, kEnsItemSites, true);
    if (st) {
        const std::string msg = g_err;
        return bail(st, msg);
    }
    *out = e;
    return CL_OK;
}

cl_status cl_ensemble_set_dt(cl_ensemble* e, int i, double dt) {
    if (!e) return efail(CL_EINVAL, "ensemble is NULL");
    if (i < 0 || i >= static_cast<int>(e->m.size())) return efail(CL_EINVAL, "member index out of range");
    if (!(dt > 0.0) || !std::isfinite(dt)) return efail(CL_EINVAL, "dt must be positive and finite");
    // the loosest bound (leapfrog); cl_ensemble_step checks the scheme's own
    if (!(omega_max(e->m[i]) * dt < stability_limit(CL_LEAPFROG)))
        return efail(CL_EUNSTABLE, "dt exceeds the leapfrog stability bound omega_max dt < 2 of member " +
                                       std::to_string(i));
    e->dt[i] = dt;
    return CL_OK;
}

cl_status cl_ensemble_step(cl_ensemble* e, cl_integrator integ, int n, cl_observables* out) {
    if (!e) return efail(CL_EINVAL, "ensemble is NULL");
    if (e->broken) return efail(CL_ESTATE, "the ensemble's work layout could not be rebuilt; destroy it");
    if (is_rk(integ)) return efail(CL_EUNSUPPORTED, "ensembles run the symplectic schemes only");
    if (integ != CL_LEAPFROG && integ != CL_VV4) return efail(CL_EINVAL, "unknown integrator");
    if (n < 0) return efail(CL_EINVAL, "n must be >= 0");
    if (n == 0) return CL_OK;
    const int nm = static_cast<int>(e->m.size());
    for (int i = 0; i < nm; ++i) {
        if (!(e->dt[i] > 0.0)) return efail(CL_ESTATE, "dt of member " + std::to_string(i) + " not set");
        const double y = omega_max(e->m[i]) * e->dt[i];
        if (!(y < stability_limit(integ)))
            return efail(CL_EUNSTABLE, "dt of member " + std::to_string(i) + " exceeds the stability bound of " +
                                           integ_name(integ) + ": omega_max dt = " + std::to_string(y));
    }
    // members' own queued work finishes first
    for (cl_lattice* h : e->m) EHIP(hipStreamSynchronize(h->stream));
    cl_status ust = ens_upload_table(e, true);
    if (ust) return ust;
    const size_t need = static_cast<size_t>(n) * nm;
    if (need > e->obs_cap) {
        if (e->d_obs) hipFree(e->d_obs);
        e->d_obs = nullptr;
        e->obs_cap = 0;
        EHIP(hipMalloc(&e->d_obs, need * sizeof(cl_observables)));
        e->obs_cap = need;
        if (e->gexec) hipGraphExecDestroy(e->gexec);
        e->gexec = nullptr;
    }
    std::vector<double> c;
    int per = 1;
    substeps(integ, 1.0, n, c, per);
    const int M = static_cast<int>(c.size());
    const int passes = 1 + M;
    if (!(e->gexec && e->g_integ == static_cast<int>(integ) && e->g_n == n)) {
        if (e->gexec) hipGraphExecDestroy(e->gexec);
        e->gexec = nullptr;
        cl::EnsArgs a{};
        a.members = e->d_table;
        a.items = e->d_items;
        a.nitems = e->nitems;
        a.nmembers = nm;
        a.write_out = 1;
        a.flags = 1;
        a.counter = e->d_counter;
        a.obs = e->d_obs;
        a.lds_bytes = static_cast<int>(e->lds);
        hipGraph_t g = nullptr;
        EHIP(hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
        hipError_t err = hipSuccess;
        // Pass 0 is the opening half kick, pass s + 1 drift step s; each pass
        // runs the scalar step of the one before it at its start, and the
        // finisher that of the last.
        auto follow = [&](cl::EnsArgs& next, const cl::EnsArgs& prev) {
            next.prev_rec = prev.rec;
            next.pckt = prev.ckt;
            next.pckb = prev.ckb;
            next.pchn = prev.chn;
        };
        a.parity = 0;
        a.drift = 0;
        a.rec = -1;
        a.ckt = 0.5 * c[0];
        a.ckb = 0.0;
        a.chn = c[0];
        a.prev_rec = -1;
        a.pckt = a.pckb = a.pchn = 0.0;
        if (err == hipSuccess) err = cl::launch_ensemble_pass(a, e->prec, e->nf, e->grid, e->maxry, e->stream);
        for (int s = 0; s < M && err == hipSuccess; ++s) {
            cl::EnsArgs d = a;
            follow(d, a);
            d.parity = s + 1;
            d.drift = 1;
            d.ckb = 0.5 * c[s];
            d.ckt = s + 1 < M ? 0.5 * (c[s] + c[s + 1]) : 0.5 * c[s];
            d.chn = s + 1 < M ? c[s + 1] : 0.0;
            d.rec = ((s + 1) % per == 0) ? (s + 1) / per - 1 : -1;
            err = cl::launch_ensemble_pass(d, e->prec, e->nf, e->grid, e->maxry, e->stream);
            a = d;
        }
        if (err == hipSuccess) {
            cl::EnsArgs f = a;
            follow(f, a);
            err = cl::launch_ensemble_finish(f, e->nf, e->stream);
        }
        hipError_t e2 = hipStreamEndCapture(e->stream, &g);
        if (err != hipSuccess || e2 != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return efail(CL_EDEVICE, std::string("ensemble graph capture: ") +
                                         hipGetErrorString(err != hipSuccess ? err : e2));
        }
        err = hipGraphInstantiate(&e->gexec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (err != hipSuccess) {
            e->gexec = nullptr;
            return efail(CL_EDEVICE, std::string("ensemble graph instantiate: ") + hipGetErrorString(err));
        }
        e->g_integ = static_cast<int>(integ);
        e->g_n = n;
    }
    EHIP(hipGraphLaunch(e->gexec, e->stream));
    std::vector<cl_observables> tmp;
    cl_observables* dst = out;
    if (!dst) {
        tmp.resize(need);
        dst = tmp.data();
    }
    EHIP(hipMemcpyAsync(dst, e->d_obs, need * sizeof(cl_observables), hipMemcpyDeviceToHost, e->stream));
    EHIP(hipStreamSynchronize(e->stream));
    for (int i = 0; i < nm; ++i) {
        cl_lattice* h = e->m[i];
        if (passes % 2) h->cur ^= 1;
        h->step += n;
        const cl_observables& last = dst[static_cast<size_t>(n - 1) * nm + i];
        note_background(h, last.a, last.mean);
    }
    for (size_t k = 0; k < need; ++k)
        if (dst[k].nonfinite) return efail(CL_EUNSTABLE, "non-finite lattice sums in an ensemble member");
    return CL_OK;
}

cl_status cl_ensemble_get_tile(const cl_ensemble* e, int i, cl_tile* out) {
    if (!e || !out) return efail(CL_EINVAL, "ensemble or out is NULL");
    if (i < 0 || i >= static_cast<int>(e->m.size())) return efail(CL_EINVAL, "member index out of range");
    const cl::EnsMember& t = e->table[i];
    out->tz = t.TZ;
    out->ty = t.TY;
    out->cx = t.CX;
    out->ry = t.RY;
    out->pd = t.RY == 1 ? 4 : 2;  // the prefetch depth does not change the results
    return CL_OK;
}

cl_status cl_ensemble_autotune(cl_ensemble* e, int reps, char* report, size_t cap) {
    if (!e) return efail(CL_EINVAL, "ensemble is NULL");
    if (e->broken) return efail(CL_ESTATE, "the ensemble's work layout could not be rebuilt; destroy it");
    if (reps < 1) reps = 3;
    for (cl_lattice* h : e->m) EHIP(hipStreamSynchronize(h->stream));
    const int nm = static_cast<int>(e->m.size());
    // Passes without drift, with zero kicks and no scale-factor step copy
    // every member's (f, pi) exactly, so pairs of them leave the fields where
    // they were; their scalar steps rewrite the scalar blocks, which are
    // restored afterwards.
    std::vector<Scal> saved(nm);
    for (int i = 0; i < nm; ++i) EHIP(hipMemcpy(&saved[i], e->m[i]->sc, sizeof(Scal), hipMemcpyDeviceToHost));
    const int keep_sites = e->item_sites;
    const bool keep_rows = e->two_rows;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    EHIP(hipEventCreate(&e0));
    EHIP(hipEventCreate(&e1));
    std::string js = "{\"members\":" + std::to_string(nm) + ",\"reps\":" + std::to_string(reps) + ",\"candidates\":[";
    std::vector<std::vector<int>> seen;
    int best_sites = keep_sites;
    bool best_rows = keep_rows;
    float best_ms = -1.0f;
    cl_status st = CL_OK;
    bool first = true;
    const int pairs = (reps + 1) / 2;
    for (int sites : {8192, 16384, 32768, 65536, 131072}) {
        for (bool rows : {true, false}) {
            st = ens_layout(e, sites, rows);
            if (st) break;
            std::vector<int> sig;  // skip layouts equal to one already timed
            for (const cl::EnsMember& t : e->table) sig.insert(sig.end(), {t.TZ, t.TY, t.CX, t.RY});
            if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
            seen.push_back(sig);
            st = ens_upload_table(e, false);
            if (st) break;
            cl::EnsArgs a{};
            a.members = e->d_table;
            a.items = e->d_items;
            a.nitems = e->nitems;
            a.nmembers = nm;
            a.drift = 0;
            a.write_out = 1;
            a.flags = 1;
            a.rec = -1;
            a.prev_rec = -1;  // no records: the scalar steps of these passes are not kept
            a.counter = e->d_counter;
            a.obs = nullptr;
            a.lds_bytes = static_cast<int>(e->lds);
            a.ckt = a.ckb = a.chn = 0.0;
            a.pckt = a.pckb = a.pchn = 0.0;
            auto pair = [&]() {
                hipError_t r = hipSuccess;
                for (int q = 0; q < 2 && r == hipSuccess; ++q) {
                    a.parity = q;
                    r = cl::launch_ensemble_pass(a, e->prec, e->nf, e->grid, e->maxry, e->stream);
                }
                return r;
            };
            hipError_t r = pair();  // warm-up
            if (r == hipSuccess) r = hipEventRecord(e0, e->stream);
            for (int k = 0; k < pairs && r == hipSuccess; ++k) r = pair();
            if (r == hipSuccess) r = hipEventRecord(e1, e->stream);
            if (r == hipSuccess) r = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
            if (r != hipSuccess) {
                st = efail(CL_EDEVICE, std::string("ensemble autotune: ") + hipGetErrorString(r));
                break;
            }
            ms /= 2 * pairs;
            char item[128];
            std::snprintf(item, sizeof item, "%s{\"item_sites\":%d,\"two_rows\":%s,\"us\":%.2f}", first ? "" : ",",
                          sites, rows ? "true" : "false", ms * 1e3);
            js += item;
            first = false;
            if (best_ms < 0.0f || ms < best_ms) {
                best_ms = ms;
                best_sites = sites;
                best_rows = rows;
            }
        }
        if (st) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    for (int i = 0; i < nm; ++i) EHIP(hipMemcpy(e->m[i]->sc, &saved[i], sizeof(Scal), hipMemcpyHostToDevice));
    if (st) {
        const std::string msg = g_err;
        (void)ens_layout(e, keep_sites, keep_rows);
        return efail(st, msg);
    }
    st = ens_layout(e, best_sites, best_rows);
    if (st) return st;
    char tail[128];
    std::snprintf(tail, sizeof tail, "],\"best\":{\"item_sites\":%d,\"two_rows\":%s,\"us\":%.2f}}", best_sites,
                  best_rows ? "true" : "false", best_ms * 1e3);
    js += tail;
    if (report && cap) {
        std::strncpy(report, js.c_str(), cap - 1);
        report[cap - 1] = '\0';
    }
    return CL_OK;
}

cl_status cl_ensemble_destroy(cl_ensemble* e) {
    if (e) ens_free(e);
    return CL_OK;
}

}  // extern "C"
