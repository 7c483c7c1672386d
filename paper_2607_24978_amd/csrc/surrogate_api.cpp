// Host runtime of the learned surrogate (cl_surrogate.h): parameters,
// device buffers, the training loop (forward, MSE, backward, Adam) and the
// network jump with its Hubble-constraint fallback.
#include "../../include/cl_surrogate.h"
#include "internal.h"
#include "surrogate.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <random>
#include <string>
#include <vector>

using cl::sg::ConvArgs;

namespace {

thread_local std::string s_err;

cl_status sfail(cl_status st, const std::string& m) {
    s_err = m;
    return st;
}

#define SHIP(call)                                                                                   \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return sfail(CL_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct Layer {
    int cin = 0, cout = 0;     // real channels
    int cinp = 0, coutp = 0;   // padded (8 or 32 in; 16 or 32 out)
    int nb = 0;                // 16-wide output blocks
    size_t w_off = 0, b_off = 0;  // offsets in the flat parameter vector
    uint16_t* wf = nullptr;    // forward weights
    uint16_t* wd = nullptr;    // input-gradient weights (layers > 0)
    float* bias = nullptr;
    int cinp_d = 0, coutp_d = 0;  // input-gradient conv: inputs = cout (padded), outputs = cin
};

template <typename T>
T* dalloc(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) return nullptr;
    return static_cast<T*>(p);
}

}  // namespace

struct cl_surrogate {
    cl_surrogate_cfg cfg{};
    std::vector<Layer> L;
    int64_t nparams = 0;
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    int adam_t = 0;
    hipStream_t stream = nullptr;
    // activation buffers for one lattice size
    int bufN = 0;
    uint16_t* x0 = nullptr;               // [n3][8]
    std::vector<uint16_t*> act;           // [layers-1] x [n3][32]
    std::vector<uint16_t*> zpre;          // [layers-1] x [n3][32] BF16 pre-activations
    float* y = nullptr;                   // [n3][4..8]
    float* dA = nullptr;                  // [n3][32]
    uint16_t* dZ[2] = {nullptr, nullptr}; // [n3][32], layer gradients (ping-pong)
    uint16_t* dy = nullptr;               // [n3][8]
    float* target = nullptr;              // [c][n3]
    float* wpart = nullptr;               // wgrad partials
    double* lpart = nullptr;              // loss partials
    int lgrid = 2048;  // loss workgroups (8 per CU: the loop over sites is latency-bound)
    // dataset
    int dsN = 0, ds_cap = 0, ds_n = 0;
    bool pending = false;
    float* ds_fluct = nullptr;            // [cap][c][n3]
    float* ds_incr = nullptr;             // [cap][c][n3]
    std::vector<std::vector<double>> ds_extra;  // raw broadcast features per pair
    // normalisation
    bool scaled = false;
    double in_scale[4] = {1, 1, 1, 1}, out_scale[4] = {1, 1, 1, 1};
    double ex_mean[4] = {0, 0, 0, 0}, ex_std[4] = {1, 1, 1, 1};
    // second gate: largest relative change over a jump of each field's
    // variance and of the fluctuations' energy (against its redshifted start
    // value); <= 0 switches it off
    double fluct_tol = 0.25;
    // jump: network increment or linear propagation of the fluctuations
    cl_jump_mode jump_mode = CL_JUMP_NETWORK;
    int propN = 0;                              // lattice size, spacing and precision of the buffers below
    double propdx = 0.0;
    bool propfp32 = false;
    void* pz[2] = {nullptr, nullptr};           // packed fluctuations, forward transforms (double2 or float2)
    void* pw[2] = {nullptr, nullptr};           // propagated modes, inverse transforms
    float2* tw32 = nullptr;                     // FP32 twiddle factors (N / 2) for FP32 lattices
    double* kap2 = nullptr;                     // [N] lattice Laplacian eigenvalue per index
    double* ptable = nullptr;                   // transfer matrices per distinct kappa^2
    uint32_t* ptriples = nullptr;               // the sorted index triples of the table
    cl::PropStep* psteps = nullptr;             // sub-step coefficients of one jump
    cl::PropStep* psteps_host = nullptr;        // their pinned host staging copy
    int psteps_cap = 0;
    // pinned host landing place of a jump's reduction (both copies issued
    // back to back, one wait)
    struct JumpObs {
        cl_observables o;
        cl::Scal sc;
    }* jump_obs = nullptr;
};

namespace {

int nfc(const cl_surrogate* s) { return 2 * s->cfg.n_fields; }
int cin0(const cl_surrogate* s) { return nfc(s) + s->cfg.extra_inputs; }

void free_bufs(cl_surrogate* s) {
    auto f = [](void* p) {
        if (p) hipFree(p);
    };
    f(s->x0);
    for (auto p : s->act) f(p);
    for (auto p : s->zpre) f(p);
    f(s->y);
    f(s->dA);
    f(s->dZ[0]);
    f(s->dZ[1]);
    f(s->dy);
    f(s->target);
    f(s->wpart);
    f(s->lpart);
    s->x0 = nullptr;
    s->act.clear();
    s->zpre.clear();
    s->y = s->dA = s->target = s->wpart = nullptr;
    s->dZ[0] = s->dZ[1] = s->dy = nullptr;
    s->lpart = nullptr;
    s->bufN = 0;
}

cl_status ensure_bufs(cl_surrogate* s, int N, bool training) {
    if (s->bufN == N && (!training || !s->zpre.empty())) return CL_OK;
    free_bufs(s);
    const size_t n3 = static_cast<size_t>(N) * N * N;
    const int nl = static_cast<int>(s->L.size());
    s->x0 = dalloc<uint16_t>(n3 * 8);
    s->y = dalloc<float>(n3 * 8);
    bool ok = s->x0 && s->y;
    for (int l = 0; l + 1 < nl; ++l) {
        s->act.push_back(dalloc<uint16_t>(n3 * 32));
        ok = ok && s->act.back();
        if (training) {
            s->zpre.push_back(dalloc<uint16_t>(n3 * 32));
            ok = ok && s->zpre.back();
        }
    }
    if (training) {
        s->dA = dalloc<float>(n3 * 32);
        s->dZ[0] = dalloc<uint16_t>(n3 * 32);
        s->dZ[1] = dalloc<uint16_t>(n3 * 32);
        s->dy = dalloc<uint16_t>(n3 * 8);
        s->target = dalloc<float>(n3 * 8);
        // weight-gradient partial sums: the largest of the three layer shapes
        size_t wp = 0;
        const int shapes[3][2] = {{32, 32}, {32, 8}, {8, 32}};  // (input channels, dz stride)
        for (const auto& sh : shapes) {
            const cl::sg::WgradShape w = cl::sg::wgrad_shape(N, sh[0], sh[1]);
            wp = std::max(wp, static_cast<size_t>(w.parts) * w.stride);
        }
        s->wpart = dalloc<float>(wp);
        s->lpart = dalloc<double>(s->lgrid);
        ok = ok && s->dA && s->dZ[0] && s->dZ[1] && s->dy && s->target && s->wpart && s->lpart;
    }
    if (!ok) {
        free_bufs(s);
        return sfail(CL_ENOMEM, "surrogate activation buffers");
    }
    s->bufN = N;
    return CL_OK;
}

// FP32 master parameters -> BF16 forward / input-gradient weights, FP32 bias.
cl_status prepare(cl_surrogate* s) {
    for (size_t l = 0; l < s->L.size(); ++l) {
        const Layer& ly = s->L[l];
        cl::sg::PrepArgs a{};
        a.theta = s->theta + ly.w_off;
        a.bias_offset = static_cast<int>(ly.b_off - ly.w_off);
        a.cout = ly.cout;
        a.cin = ly.cin;
        a.coutp = ly.coutp;
        a.cinp = ly.cinp;
        a.no_f = ly.cinp == 32 ? 27 : 28;
        a.wf = ly.wf;
        a.wd = ly.wd;
        a.coutp_d = ly.coutp_d;
        a.cinp_d = ly.cinp_d;
        a.no_d = ly.cinp_d == 32 ? 27 : 28;
        a.bias = ly.bias;
        SHIP(cl::sg::launch_prepare_layer(a, s->stream));
    }
    return CL_OK;
}

// Network forward from s->x0; training keeps the pre-activations.
cl_status forward(cl_surrogate* s, int N, bool training) {
    const int nl = static_cast<int>(s->L.size());
    const int n3 = N * N * N;
    for (int l = 0; l < nl; ++l) {
        const Layer& ly = s->L[l];
        ConvArgs a{};
        a.in = l == 0 ? static_cast<const void*>(s->x0) : static_cast<const void*>(s->act[l - 1]);
        a.w = ly.wf;
        a.bias = ly.bias;
        a.N = N;
        a.nsites = n3;
        a.cout = ly.coutp == 16 ? 4 * ((ly.cout + 3) / 4) : 32;
        if (l + 1 < nl) {
            a.z_out = nullptr;
            a.zh_out = training ? s->zpre[l] : nullptr;
            a.zh_stride = 32;
            a.a_out = s->act[l];
            a.a_stride = 32;
            a.gelu = 1;
        } else {
            a.z_out = s->y;
            a.z_stride = a.cout;
            a.a_out = nullptr;
            a.gelu = 0;
        }
        const int groups = n3 / 16;
        const int grid = std::max(1, std::min(1024, (groups + 15) / 16));
        SHIP(cl::sg::launch_conv_fwd(a, ly.cinp, ly.nb, grid, s->stream));
    }
    return CL_OK;
}

int ystride(const cl_surrogate* s) { return 4 * ((s->L.back().cout + 3) / 4); }

// MSE and gradient of every parameter into s->grad; returns the loss.  With
// input_grad the gradient with respect to the network input is left in s->dA
// (FP32 [site][32], the first c_in channels).
cl_status loss_and_backward(cl_surrogate* s, int N, double* loss, bool input_grad = false) {
    const int nl = static_cast<int>(s->L.size());
    const size_t n3 = static_cast<size_t>(N) * N * N;
    const int co = s->L.back().cout;
    SHIP(cl::sg::launch_mse_grad(s->y, ystride(s), s->target, co, n3, 1.0 / (static_cast<double>(n3) * co), s->dy,
                                 s->lpart, s->lgrid, s->stream));
    const void* dz = s->dy;  // d loss / d z of layer l (BF16 channels-last)
    int dz_stride = 8;
    for (int l = nl - 1; l >= 0; --l) {
        const Layer& ly = s->L[l];
        const cl::sg::WgradShape sh = cl::sg::wgrad_shape(N, ly.cinp, dz_stride);
        cl::sg::WgradArgs w{};
        w.dz = dz;
        w.x = l == 0 ? static_cast<const void*>(s->x0) : static_cast<const void*>(s->act[l - 1]);
        w.partials = s->wpart;
        w.N = N;
        w.nsites = static_cast<int>(n3);
        w.cout_stride = dz_stride;
        w.partial_stride = sh.stride;
        w.L = sh.L;
        SHIP(cl::sg::launch_conv_wgrad(w, ly.cinp, s->stream));
        cl::sg::WgradReduceArgs r{};
        r.partials = s->wpart;
        r.nparts = sh.parts;
        r.partial_stride = sh.stride;
        r.coutp = dz_stride == 32 ? 32 : 16;
        r.cinp = ly.cinp == 32 ? 32 : 16;
        r.cout = ly.cout;
        r.cin = ly.cin;
        r.gW = s->grad + ly.w_off;
        r.gb = s->grad + ly.b_off;
        SHIP(cl::sg::launch_wgrad_reduce(r, s->stream));
        if (l > 0 || input_grad) {
            // input gradient: a convolution of dz with the flipped, transposed
            // weights; below a hidden layer it is multiplied by GELU'(z) of
            // that layer in the epilogue and becomes the next dz (BF16)
            ConvArgs a{};
            a.in = dz;
            a.w = ly.wd;
            a.bias = nullptr;
            a.N = N;
            a.nsites = static_cast<int>(n3);
            a.cout = 32;
            a.gelu = 0;
            uint16_t* next = s->dZ[(nl - 1 - l) & 1];
            if (l > 0) {
                a.z_out = nullptr;
                a.a_out = next;
                a.a_stride = 32;
                a.gz = s->zpre[l - 1];
                a.gz_stride = 32;
            } else {
                a.z_out = s->dA;
                a.z_stride = 32;
                a.a_out = nullptr;
            }
            const int groups = static_cast<int>(n3 / 16);
            const int grid2 = std::max(1, std::min(1024, (groups + 15) / 16));
            SHIP(cl::sg::launch_conv_fwd(a, ly.cinp_d, 2, grid2, s->stream));
            dz = next;
            dz_stride = 32;
        }
    }
    std::vector<double> lp(s->lgrid);
    SHIP(hipMemcpyAsync(lp.data(), s->lpart, s->lgrid * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    SHIP(hipStreamSynchronize(s->stream));
    double sum = 0.0;
    for (double x : lp) sum += x;
    *loss = sum / (static_cast<double>(n3) * co);
    return CL_OK;
}

// One Adam step (Kingma and Ba) of the FP32 master weights with the gradient
// in s->grad, bias-corrected with the handle's step count, then the BF16
// copies are refreshed.
cl_status adam_step(cl_surrogate* s, double lr) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    s->adam_t += 1;
    // bias corrections 1 - beta^t formed in FP64 from the FP32 betas and
    // rounded once: in FP32, 1 - beta2^t cancels to a few significant bits
    const float c1 = static_cast<float>(1.0 - std::pow(static_cast<double>(b1), s->adam_t));
    const float c2 = static_cast<float>(1.0 - std::pow(static_cast<double>(b2), s->adam_t));
    SHIP(cl::sg::launch_adam(s->theta, s->grad, s->m, s->v, static_cast<int>(s->nparams), static_cast<float>(lr), b1,
                             b2, eps, c1, c2, s->stream));
    return prepare(s);
}

bool valid_net_N(int N) { return N >= 16 && (N & (N - 1)) == 0; }
// The weight-gradient kernel takes 32-site segments of one z row.
bool valid_train_N(int N) { return N >= 32 && (N & (N - 1)) == 0; }

// Host FP32 [c][n3] -> BF16 [site][8] in s->x0 (through a staging upload).
cl_status upload_input(cl_surrogate* s, int N, const float* x) {
    const size_t n3 = static_cast<size_t>(N) * N * N;
    const int c = cin0(s);
    std::vector<uint16_t> h(n3 * 8, 0);
    for (int k = 0; k < c; ++k)
        for (size_t i = 0; i < n3; ++i) {
            uint32_t u;
            std::memcpy(&u, &x[k * n3 + i], 4);
            u += 0x7FFFu + ((u >> 16) & 1u);
            h[i * 8 + k] = static_cast<uint16_t>(u >> 16);
        }
    SHIP(hipMemcpyAsync(s->x0, h.data(), h.size() * 2, hipMemcpyHostToDevice, s->stream));
    SHIP(hipStreamSynchronize(s->stream));
    return CL_OK;
}

// Hartree-corrected lattice-mean force of the homogeneous modes, dV/df_j
// averaged over Gaussian fluctuations of variance var_k about fbar.
void mean_force(const cl_lattice* h, const double* f, const double* var, double* dv) {
    const cl_potential& p = h->pot;
    const int nf = h->nf;
    for (int j = 0; j < nf; ++j) dv[j] = p.m2[j] * f[j] + p.lambda[j] * (f[j] * f[j] * f[j] + 3.0 * f[j] * var[j]);
    if (nf == 2) {
        dv[0] += p.g2 * f[0] * (f[1] * f[1] + var[1]);
        dv[1] += p.g2 * f[1] * (f[0] * f[0] + var[0]);
    }
}

double hom_V(const cl_lattice* h, const double* f, const double* var) {
    const cl_potential& p = h->pot;
    double V = p.V0;
    for (int j = 0; j < h->nf; ++j) {
        const double f2 = f[j] * f[j];
        V += 0.5 * p.m2[j] * (f2 + var[j]) + 0.25 * p.lambda[j] * (f2 * f2 + 6.0 * f2 * var[j] + 3.0 * var[j] * var[j]);
    }
    if (h->nf == 2) V += 0.5 * p.g2 * (f[0] * f[0] + var[0]) * (f[1] * f[1] + var[1]);
    return V;
}

// Homogeneous volume sums at one kick of a': (sum_j pbar_j^2 / 2, Hartree
// average of V).
struct HomSums {
    double K, V;
};

// Advance (fbar, pbar, a, b) over n steps of dt with the integrator's
// sub-step pattern; the fluctuations' kinetic + gradient energy rides along
// as radiation, rho_r ~ a^-4, p_r = rho_r / 3.  The homogeneous sums at
// every kick of b are appended to `hom` (for the corrector).
// Hartree-averaged mass matrix d2V/df_i df_j (m00, m01, m11) at the
// homogeneous values f over Gaussian fluctuations of variance var.
void mass_matrix(const cl_lattice* h, const double* f, const double* var, double* M) {
    const cl_potential& p = h->pot;
    M[0] = p.m2[0] + 3.0 * p.lambda[0] * (f[0] * f[0] + var[0]);
    M[1] = 0.0;
    M[2] = 0.0;
    if (h->nf == 2) {
        M[0] += p.g2 * (f[1] * f[1] + var[1]);
        M[1] = 2.0 * p.g2 * f[0] * f[1];
        M[2] = p.m2[1] + 3.0 * p.lambda[1] * (f[1] * f[1] + var[1]) + p.g2 * (f[0] * f[0] + var[0]);
    }
}

void advance_homogeneous(const cl_lattice* h, cl_integrator integ, double dt, int n, double* f, double* pm, double& a,
                         double& b, const double* var, double rho_r0, double a_ref, std::vector<HomSums>& hom,
                         std::vector<cl::PropStep>* modes = nullptr) {
    const double al = h->alpha, mp = h->mp;
    const bool expand = h->mode == CL_SELF_CONSISTENT;
    auto accel = [&](double aa) {
        if (!expand) return 0.0;
        double K = 0.0, SK = 0.0;
        for (int j = 0; j < h->nf; ++j) {
            K += pm[j] * pm[j] / (2.0 * std::pow(aa, 6.0));
            SK += 0.5 * pm[j] * pm[j];
        }
        const double V = hom_V(h, f, var);
        hom.push_back({SK, V});
        const double rr = rho_r0 * std::pow(a_ref / aa, 4.0);
        const double rho = K + V + rr, pr = K - V + rr / 3.0;
        return std::pow(aa, 2.0 * al + 1.0) * ((2.0 * al - 1.0) * rho - 3.0 * pr) / (6.0 * mp * mp);
    };
    auto kick = [&](double hh, double aa) {
        double dv[2];
        mean_force(h, f, var, dv);
        for (int j = 0; j < h->nf; ++j) pm[j] -= hh * std::pow(aa, 3.0 + al) * dv[j];
    };
    // a mode's coefficients for a half kick at (a, f): (h/2) a^(1+alpha) for
    // kappa^2 and (h/2) a^(3+alpha) times the mass matrix
    auto mode_kick = [&](double hh, double aa, double& ck, double* m) {
        double M[3];
        mass_matrix(h, f, var, M);
        ck = 0.5 * hh * std::pow(aa, 1.0 + al);
        for (int i = 0; i < 3; ++i) m[i] = 0.5 * hh * std::pow(aa, 3.0 + al) * M[i];
    };
    auto vv2 = [&](double hh) {
        // the scale-factor half kick takes the energies at the synchronised
        // momenta (before the field half kick), as the lattice step does
        cl::PropStep ms{};
        if (modes) mode_kick(hh, a, ms.ck0, ms.m0);
        const double A0 = accel(a);
        kick(0.5 * hh, a);
        b += 0.5 * hh * A0;
        const double an = expand ? a + hh * b : a;
        const double abar = 0.5 * (a + an);
        for (int j = 0; j < h->nf; ++j) f[j] += hh * std::pow(abar, al - 3.0) * pm[j];
        a = an;
        if (modes) {
            ms.cd = hh * std::pow(abar, al - 3.0);
            mode_kick(hh, a, ms.ck1, ms.m1);
            modes->push_back(ms);
        }
        kick(0.5 * hh, a);
        b += 0.5 * hh * accel(a);
    };
    const double w1 = 1.0 / (2.0 - std::cbrt(2.0)), w0 = 1.0 - 2.0 * w1;
    for (int i = 0; i < n; ++i) {
        if (integ == CL_VV4) {
            vv2(w1 * dt);
            vv2(w0 * dt);
            vv2(w1 * dt);
        } else {
            vv2(dt);
        }
    }
}

// Corrector for the background over a jump: (a, b) re-integrated with the
// integrator's sub-step pattern, with rho and p at each kick from the
// a-independent volume sums S = (<pi^2>/2, <(grad f)^2>/2, <V>)
// (K = S_K/a^6, G = S_G/a^2; Eqs. Friedmann1, rhoLocal).  S is the
// homogeneous part along the predictor's trajectory (hom, one entry per kick
// in the same order) plus the fluctuations' share, which moves linearly in
// time from its value at the start (S0 - hom.front()) to that of the
// predicted endpoint (S1 - hom.back()).
void correct_background(const cl_lattice* h, cl_integrator integ, double dt, int n, const double* S0,
                        const double* S1, const std::vector<HomSums>& hom, double& a, double& b) {
    if (h->mode != CL_SELF_CONSISTENT || hom.empty()) return;
    const double al = h->alpha, mp = h->mp, T = dt * n;
    const double R0[3] = {S0[0] - hom.front().K, S0[1], S0[2] - hom.front().V};
    const double R1[3] = {S1[0] - hom.back().K, S1[1], S1[2] - hom.back().V};
    size_t k = 0;
    double tau = 0.0;
    auto accel = [&](double aa, double t) {
        const double w = T > 0 ? t / T : 0.0;
        const HomSums& H = hom[std::min(k++, hom.size() - 1)];
        const double SK = H.K + R0[0] + w * (R1[0] - R0[0]), SG = R0[1] + w * (R1[1] - R0[1]),
                     SV = H.V + R0[2] + w * (R1[2] - R0[2]);
        const double K = SK / std::pow(aa, 6.0), G = SG / (aa * aa);
        const double rho = K + G + SV, pr = K - G / 3.0 - SV;
        return std::pow(aa, 2.0 * al + 1.0) * ((2.0 * al - 1.0) * rho - 3.0 * pr) / (6.0 * mp * mp);
    };
    auto vv2 = [&](double hh) {
        b += 0.5 * hh * accel(a, tau);
        a += hh * b;
        tau += hh;
        b += 0.5 * hh * accel(a, tau);
    };
    const double w1 = 1.0 / (2.0 - std::cbrt(2.0)), w0 = 1.0 - 2.0 * w1;
    for (int i = 0; i < n; ++i) {
        if (integ == CL_VV4) {
            vv2(w1 * dt);
            vv2(w0 * dt);
            vv2(w1 * dt);
        } else {
            vv2(dt);
        }
    }
}

// a-independent volume sums of an observation taken at scale factor a.
void volume_sums(const cl_observables& o, double* S) {
    S[0] = (o.EK[0] + o.EK[1]) * std::pow(o.a, 6.0);
    S[1] = (o.EG[0] + o.EG[1]) * o.a * o.a;
    S[2] = o.EV;
}

// Raw broadcast features of a lattice state: (a, H, <f_0>, <pi_0>).
void raw_extra(const cl_observables& o, const cl::Scal& sc, double* e) {
    e[0] = o.a;
    e[1] = o.H;
    e[2] = o.mean[0];
    e[3] = sc.mean_p[0];
}

cl_status read_lattice(cl_lattice* h, cl_observables* o, cl::Scal* sc) {
    cl_status st = cl_read_observables(h, o);
    if (st) return sfail(st, std::string("reading lattice observables: ") + cl_last_error(h));
    SHIP(hipMemcpyAsync(sc, h->sc, sizeof(cl::Scal), hipMemcpyDeviceToHost, h->stream));
    SHIP(hipStreamSynchronize(h->stream));
    return CL_OK;
}

}  // namespace

extern "C" {

const char* cl_surrogate_last_error(void) { return s_err.c_str(); }

cl_status cl_surrogate_create(const cl_surrogate_cfg* cfg, cl_surrogate** out) {
    if (!out) return sfail(CL_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg) return sfail(CL_EINVAL, "cfg is NULL");
    if (cfg->n_fields < 1 || cfg->n_fields > 2) return sfail(CL_EINVAL, "n_fields must be 1 or 2");
    if (cfg->extra_inputs < 0 || 2 * cfg->n_fields + cfg->extra_inputs > 8)
        return sfail(CL_EINVAL, "at most 8 input channels");
    if (cfg->hidden != 32) return sfail(CL_EUNSUPPORTED, "hidden width must be 32");
    if (cfg->layers < 2 || cfg->layers > 16) return sfail(CL_EINVAL, "layers must be in [2, 16]");
    if (cfg->jump_steps < 1) return sfail(CL_EINVAL, "jump_steps must be >= 1");
    cl_surrogate* s = new (std::nothrow) cl_surrogate;
    if (!s) return sfail(CL_ENOMEM, "surrogate handle");
    s->cfg = *cfg;
    size_t off = 0;
    for (int l = 0; l < cfg->layers; ++l) {
        Layer ly;
        ly.cin = l == 0 ? cin0(s) : 32;
        ly.cout = l + 1 == cfg->layers ? nfc(s) : 32;
        ly.cinp = ly.cin <= 8 ? 8 : 32;
        ly.coutp = ly.cout <= 16 ? 16 : 32;
        if (l + 1 < cfg->layers) ly.coutp = 32;
        ly.nb = ly.coutp / 16;
        ly.cinp_d = ly.cout <= 8 ? 8 : 32;
        ly.coutp_d = 32;
        ly.w_off = off;
        off += static_cast<size_t>(ly.cout) * ly.cin * 27;
        ly.b_off = off;
        off += ly.cout;
        s->L.push_back(ly);
    }
    s->nparams = static_cast<int64_t>(off);
    auto bail = [&](cl_status st, const std::string& m) {
        cl_surrogate_destroy(s);
        return sfail(st, m);
    };
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) return bail(CL_EDEVICE, "stream");
    s->theta = dalloc<float>(off);
    s->grad = dalloc<float>(off);
    s->m = dalloc<float>(off);
    s->v = dalloc<float>(off);
    if (!s->theta || !s->grad || !s->m || !s->v) return bail(CL_ENOMEM, "parameters");
    for (auto& ly : s->L) {
        const int nof = ly.cinp == 32 ? 27 : 28;
        const int nod = ly.cinp_d == 32 ? 27 : 28;
        ly.wf = dalloc<uint16_t>(static_cast<size_t>(nof) * ly.coutp * ly.cinp);
        ly.wd = dalloc<uint16_t>(static_cast<size_t>(nod) * ly.coutp_d * ly.cinp_d);
        ly.bias = dalloc<float>(32);
        if (!ly.wf || !ly.wd || !ly.bias) return bail(CL_ENOMEM, "layer weights");
    }
    // He-style uniform initialisation on the host, biases zero
    std::vector<float> th(off, 0.0f);
    std::mt19937_64 rng(cfg->init_seed);
    for (const auto& ly : s->L) {
        const double bound = std::sqrt(6.0 / (27.0 * ly.cin));
        std::uniform_real_distribution<double> U(-bound, bound);
        for (size_t i = 0; i < static_cast<size_t>(ly.cout) * ly.cin * 27; ++i) th[ly.w_off + i] = static_cast<float>(U(rng));
    }
    cl_status st = cl_surrogate_set_params(s, th.data());
    if (st) return bail(st, s_err);
    *out = s;
    return CL_OK;
}

cl_status cl_surrogate_destroy(cl_surrogate* s) {
    if (!s) return CL_OK;
    if (s->stream) hipStreamSynchronize(s->stream);
    free_bufs(s);
    for (auto& ly : s->L) {
        if (ly.wf) hipFree(ly.wf);
        if (ly.wd) hipFree(ly.wd);
        if (ly.bias) hipFree(ly.bias);
    }
    for (void* p : {(void*)s->theta, (void*)s->grad, (void*)s->m, (void*)s->v, (void*)s->ds_fluct,
                    (void*)s->ds_incr, s->pz[0], s->pz[1], s->pw[0], s->pw[1], (void*)s->tw32,
                    (void*)s->kap2, (void*)s->ptable, (void*)s->ptriples, (void*)s->psteps})
        if (p) hipFree(p);
    if (s->psteps_host) hipHostFree(s->psteps_host);
    if (s->jump_obs) hipHostFree(s->jump_obs);
    if (s->stream) hipStreamDestroy(s->stream);
    delete s;
    return CL_OK;
}

cl_status cl_surrogate_num_params(const cl_surrogate* s, int64_t* n) {
    if (!s || !n) return sfail(CL_EINVAL, "NULL argument");
    *n = s->nparams;
    return CL_OK;
}

cl_status cl_surrogate_get_params(cl_surrogate* s, float* theta) {
    if (!s || !theta) return sfail(CL_EINVAL, "NULL argument");
    SHIP(hipMemcpyAsync(theta, s->theta, s->nparams * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    SHIP(hipStreamSynchronize(s->stream));
    return CL_OK;
}

cl_status cl_surrogate_set_params(cl_surrogate* s, const float* theta) {
    if (!s || !theta) return sfail(CL_EINVAL, "NULL argument");
    for (int64_t i = 0; i < s->nparams; ++i)
        if (!std::isfinite(theta[i])) return sfail(CL_EINVAL, "non-finite parameter");
    SHIP(hipMemcpyAsync(s->theta, theta, s->nparams * sizeof(float), hipMemcpyHostToDevice, s->stream));
    SHIP(hipMemsetAsync(s->m, 0, s->nparams * sizeof(float), s->stream));
    SHIP(hipMemsetAsync(s->v, 0, s->nparams * sizeof(float), s->stream));
    s->adam_t = 0;
    cl_status st = prepare(s);
    if (st) return st;
    SHIP(hipStreamSynchronize(s->stream));
    return CL_OK;
}

cl_status cl_surrogate_forward(cl_surrogate* s, int N, const float* x, float* y) {
    if (!s || !x || !y) return sfail(CL_EINVAL, "NULL argument");
    if (!valid_net_N(N)) return sfail(CL_EINVAL, "N must be a power of two >= 16");
    cl_status st = ensure_bufs(s, N, false);
    if (st) return st;
    st = upload_input(s, N, x);
    if (st) return st;
    st = forward(s, N, false);
    if (st) return st;
    const size_t n3 = static_cast<size_t>(N) * N * N;
    const int ys = ystride(s), co = s->L.back().cout;
    std::vector<float> h(n3 * ys);
    SHIP(hipMemcpyAsync(h.data(), s->y, h.size() * 4, hipMemcpyDeviceToHost, s->stream));
    SHIP(hipStreamSynchronize(s->stream));
    for (int c = 0; c < co; ++c)
        for (size_t i = 0; i < n3; ++i) y[c * n3 + i] = h[i * ys + c];
    return CL_OK;
}

cl_status cl_surrogate_loss_grad(cl_surrogate* s, int N, const float* x, const float* t, double* loss, float* grad,
                                 float* grad_x) {
    if (!s || !x || !t || !loss || !grad) return sfail(CL_EINVAL, "NULL argument");
    if (!valid_train_N(N)) return sfail(CL_EINVAL, "N must be a power of two >= 32");
    cl_status st = ensure_bufs(s, N, true);
    if (st) return st;
    st = upload_input(s, N, x);
    if (st) return st;
    const size_t n3 = static_cast<size_t>(N) * N * N;
    const int co = s->L.back().cout;
    SHIP(hipMemcpyAsync(s->target, t, n3 * co * sizeof(float), hipMemcpyHostToDevice, s->stream));
    st = forward(s, N, true);
    if (st) return st;
    st = loss_and_backward(s, N, loss, grad_x != nullptr);
    if (st) return st;
    SHIP(hipMemcpyAsync(grad, s->grad, s->nparams * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    std::vector<float> gx;
    if (grad_x) {
        gx.resize(n3 * 32);
        SHIP(hipMemcpyAsync(gx.data(), s->dA, gx.size() * 4, hipMemcpyDeviceToHost, s->stream));
    }
    SHIP(hipStreamSynchronize(s->stream));
    if (grad_x)
        for (int c = 0; c < cin0(s); ++c)
            for (size_t i = 0; i < n3; ++i) grad_x[c * n3 + i] = gx[i * 32 + c];
    return CL_OK;
}

cl_status cl_surrogate_apply_grad(cl_surrogate* s, const float* grad, double lr) {
    if (!s || !grad) return sfail(CL_EINVAL, "NULL argument");
    if (!(lr >= 0.0) || !std::isfinite(lr)) return sfail(CL_EINVAL, "lr must be finite and >= 0");
    for (int64_t i = 0; i < s->nparams; ++i)
        if (!std::isfinite(grad[i])) return sfail(CL_EINVAL, "non-finite gradient");
    SHIP(hipMemcpyAsync(s->grad, grad, s->nparams * sizeof(float), hipMemcpyHostToDevice, s->stream));
    cl_status st = adam_step(s, lr);
    if (st) return st;
    SHIP(hipStreamSynchronize(s->stream));
    return CL_OK;
}

cl_status cl_surrogate_get_normalisation(const cl_surrogate* s, cl_surrogate_norm* out) {
    if (!s || !out) return sfail(CL_EINVAL, "NULL argument");
    if (!s->scaled) return sfail(CL_ESTATE, "no normalisation fixed yet");
    for (int k = 0; k < 4; ++k) {
        out->in_scale[k] = s->in_scale[k];
        out->out_scale[k] = s->out_scale[k];
        out->extra_mean[k] = s->ex_mean[k];
        out->extra_std[k] = s->ex_std[k];
    }
    return CL_OK;
}

cl_status cl_surrogate_set_normalisation(cl_surrogate* s, const cl_surrogate_norm* in) {
    if (!s || !in) return sfail(CL_EINVAL, "NULL argument");
    for (int k = 0; k < 4; ++k)
        if (!(in->in_scale[k] > 0.0) || !(in->out_scale[k] > 0.0) || !(in->extra_std[k] > 0.0) ||
            !std::isfinite(in->in_scale[k]) || !std::isfinite(in->out_scale[k]) || !std::isfinite(in->extra_std[k]) ||
            !std::isfinite(in->extra_mean[k]))
            return sfail(CL_EINVAL, "scales must be positive and finite, means finite");
    for (int k = 0; k < 4; ++k) {
        s->in_scale[k] = in->in_scale[k];
        s->out_scale[k] = in->out_scale[k];
        s->ex_mean[k] = in->extra_mean[k];
        s->ex_std[k] = in->extra_std[k];
    }
    s->scaled = true;
    return CL_OK;
}

cl_status cl_surrogate_dataset_reserve(cl_surrogate* s, int N, int max_pairs) {
    if (!s) return sfail(CL_EINVAL, "NULL surrogate");
    if (!valid_train_N(N) || max_pairs < 1) return sfail(CL_EINVAL, "N must be a power of two >= 32, max_pairs >= 1");
    if (s->ds_fluct) hipFree(s->ds_fluct);
    if (s->ds_incr) hipFree(s->ds_incr);
    s->ds_fluct = s->ds_incr = nullptr;
    const size_t per = static_cast<size_t>(nfc(s)) * N * N * N;
    s->ds_fluct = dalloc<float>(per * max_pairs);
    s->ds_incr = dalloc<float>(per * max_pairs);
    if (!s->ds_fluct || !s->ds_incr) return sfail(CL_ENOMEM, "dataset (" + std::to_string(2 * per * max_pairs * 4) + " bytes)");
    s->dsN = N;
    s->ds_cap = max_pairs;
    s->ds_n = 0;
    s->pending = false;
    s->ds_extra.clear();
    return CL_OK;
}

static cl_status record(cl_surrogate* s, cl_lattice* h, bool input) {
    if (!s || !h) return sfail(CL_EINVAL, "NULL argument");
    if (h->dim != 3) return sfail(CL_EUNSUPPORTED, "the surrogate works on three-dimensional lattices");
    if (h->ng) return sfail(CL_EUNSUPPORTED, "the surrogate takes lattices without the gravitational-wave tensor");
    if (!s->ds_fluct) return sfail(CL_ESTATE, "no dataset reserved");
    if (h->N != s->dsN || h->nf != s->cfg.n_fields) return sfail(CL_EINVAL, "lattice does not match the dataset");
    if (input == s->pending) return sfail(CL_ESTATE, input ? "input already recorded" : "no input recorded");
    if (input && s->ds_n >= s->ds_cap) return sfail(CL_ESTATE, "dataset full");
    cl_observables o;
    cl::Scal sc;
    cl_status st = read_lattice(h, &o, &sc);
    if (st) return st;
    const size_t n3 = static_cast<size_t>(h->N) * h->N * h->N;
    const size_t per = static_cast<size_t>(nfc(s)) * n3;
    cl::sg::PackArgs a{};
    a.state = h->buf[h->cur];
    a.N = h->N;
    a.nf = h->nf;
    for (int j = 0; j < h->nf; ++j) {
        a.mean[j] = o.mean[j];
        a.mean[h->nf + j] = sc.mean_p[j];
    }
    for (int c = 0; c < 4; ++c) a.inv_scale[c] = 1.0;
    a.nextra = 0;
    if (input) {
        a.fluct_out = s->ds_fluct + per * s->ds_n;
        std::vector<double> e(4);
        raw_extra(o, sc, e.data());
        s->ds_extra.push_back(e);
    } else {
        a.fluct_sub = s->ds_incr + per * s->ds_n;
        a.fluct_sub_ref = s->ds_fluct + per * s->ds_n;
    }
    SHIP(cl::sg::launch_pack_state(a, h->prec == CL_FP32, h->stream));
    SHIP(hipStreamSynchronize(h->stream));
    if (input) {
        s->pending = true;
    } else {
        s->pending = false;
        s->ds_n += 1;
    }
    (void)n3;
    return CL_OK;
}

cl_status cl_surrogate_record_input(cl_surrogate* s, cl_lattice* h) { return record(s, h, true); }
cl_status cl_surrogate_record_target(cl_surrogate* s, cl_lattice* h) { return record(s, h, false); }

cl_status cl_surrogate_dataset_size(const cl_surrogate* s, int* pairs) {
    if (!s || !pairs) return sfail(CL_EINVAL, "NULL argument");
    *pairs = s->ds_n;
    return CL_OK;
}

// Per-channel RMS of the recorded fluctuations and increments, and the
// mean / spread of the broadcast features, over the first `count` pairs.
static cl_status fix_scales(cl_surrogate* s, int count) {
    const size_t n3 = static_cast<size_t>(s->dsN) * s->dsN * s->dsN;
    const int C = nfc(s);
    std::vector<float> h(n3);
    double sf[4] = {0, 0, 0, 0}, si[4] = {0, 0, 0, 0};
    const int stride = std::max(1, count / 16);  // a sample of the pairs is enough for the scales
    int used = 0;
    for (int p = 0; p < count; p += stride, ++used)
        for (int c = 0; c < C; ++c) {
            for (int which = 0; which < 2; ++which) {
                const float* src = (which == 0 ? s->ds_fluct : s->ds_incr) + (static_cast<size_t>(p) * C + c) * n3;
                SHIP(hipMemcpy(h.data(), src, n3 * 4, hipMemcpyDeviceToHost));
                double acc = 0.0;
                for (size_t i = 0; i < n3; ++i) acc += static_cast<double>(h[i]) * h[i];
                (which == 0 ? sf : si)[c] += acc / n3;
            }
        }
    for (int c = 0; c < C; ++c) {
        s->in_scale[c] = std::sqrt(sf[c] / used);
        s->out_scale[c] = std::sqrt(si[c] / used);
        if (!(s->in_scale[c] > 0)) s->in_scale[c] = 1.0;
        if (!(s->out_scale[c] > 0)) s->out_scale[c] = 1.0;
    }
    for (int k = 0; k < 4; ++k) {
        double m = 0.0, q = 0.0;
        for (int p = 0; p < count; ++p) m += s->ds_extra[p][k];
        m /= count;
        for (int p = 0; p < count; ++p) q += (s->ds_extra[p][k] - m) * (s->ds_extra[p][k] - m);
        s->ex_mean[k] = m;
        s->ex_std[k] = count > 1 && q > 0 ? std::sqrt(q / (count - 1)) : 1.0;
    }
    s->scaled = true;
    return CL_OK;
}

static cl_status load_sample(cl_surrogate* s, int p) {
    const size_t n3 = static_cast<size_t>(s->dsN) * s->dsN * s->dsN;
    const int C = nfc(s);
    cl::sg::SampleArgs a{};
    a.fluct = s->ds_fluct + static_cast<size_t>(p) * C * n3;
    a.incr = s->ds_incr + static_cast<size_t>(p) * C * n3;
    for (int c = 0; c < C; ++c) {
        a.inv_in[c] = static_cast<float>(1.0 / s->in_scale[c]);
        a.inv_out[c] = static_cast<float>(1.0 / s->out_scale[c]);
    }
    a.nextra = s->cfg.extra_inputs;
    for (int k = 0; k < a.nextra; ++k) a.extra[k] = static_cast<float>((s->ds_extra[p][k] - s->ex_mean[k]) / s->ex_std[k]);
    a.nfc = C;
    a.x = s->x0;
    a.target = s->target;
    a.n3 = n3;
    SHIP(cl::sg::launch_pack_sample(a, s->stream));
    return CL_OK;
}

cl_status cl_surrogate_train(cl_surrogate* s, const cl_train_cfg* cfg, cl_train_report* rep) {
    if (!s || !cfg) return sfail(CL_EINVAL, "NULL argument");
    if (s->pending) return sfail(CL_ESTATE, "an input is recorded without its target");
    const int ntrain = s->ds_n - std::max(0, cfg->holdout);
    if (ntrain < 1) return sfail(CL_ESTATE, "no training pairs");
    if (cfg->epochs < 1 || !(cfg->lr > 0.0)) return sfail(CL_EINVAL, "epochs >= 1 and lr > 0 needed");
    const auto t0 = std::chrono::steady_clock::now();
    const int N = s->dsN;
    cl_status st = ensure_bufs(s, N, true);
    if (st) return st;
    if (!s->scaled) {
        st = fix_scales(s, ntrain);
        if (st) return st;
    }
    std::vector<int> order(ntrain);
    std::iota(order.begin(), order.end(), 0);
    std::mt19937_64 rng(cfg->shuffle_seed);
    const int total = cfg->epochs * ntrain;
    double first = -1.0, epoch_sum = 0.0;
    int step = 0;
    for (int ep = 0; ep < cfg->epochs; ++ep) {
        std::shuffle(order.begin(), order.end(), rng);
        epoch_sum = 0.0;
        for (int k = 0; k < ntrain; ++k, ++step) {
            st = load_sample(s, order[k]);
            if (st) return st;
            st = forward(s, N, true);
            if (st) return st;
            double loss = 0.0;
            st = loss_and_backward(s, N, &loss);
            if (st) return st;
            if (!std::isfinite(loss)) return sfail(CL_EUNSTABLE, "non-finite training loss");
            if (first < 0) first = loss;
            epoch_sum += loss;
            const double lr = cfg->lr_final + 0.5 * (cfg->lr - cfg->lr_final) * (1.0 + std::cos(M_PI * step / total));
            st = adam_step(s, lr);
            if (st) return st;
        }
    }
    double hold = 0.0, zero = 0.0;
    const int nh = s->ds_n - ntrain;
    for (int p = ntrain; p < s->ds_n; ++p) {
        st = load_sample(s, p);
        if (st) return st;
        st = forward(s, N, true);
        if (st) return st;
        double loss = 0.0;
        st = loss_and_backward(s, N, &loss);
        if (st) return st;
        hold += loss;
        // zero-increment predictor: mean of the squared normalised target
        std::vector<float> t(static_cast<size_t>(nfc(s)) * N * N * N);
        SHIP(hipMemcpy(t.data(), s->target, t.size() * 4, hipMemcpyDeviceToHost));
        double z = 0.0;
        for (float x : t) z += static_cast<double>(x) * x;
        zero += z / t.size();
    }
    SHIP(hipStreamSynchronize(s->stream));
    if (rep) {
        rep->steps = step;
        rep->first_loss = first;
        rep->last_epoch_loss = epoch_sum / ntrain;
        rep->holdout_loss = nh ? hold / nh : 0.0;
        rep->holdout_zero = nh ? zero / nh : 0.0;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return CL_OK;
}

cl_status cl_surrogate_save(const cl_surrogate* cs, const char* path) {
    cl_surrogate* s = const_cast<cl_surrogate*>(cs);
    if (!s || !path) return sfail(CL_EINVAL, "NULL argument");
    std::vector<float> th(s->nparams);
    cl_status st = cl_surrogate_get_params(s, th.data());
    if (st) return st;
    FILE* f = std::fopen(path, "wb");
    if (!f) return sfail(CL_EINVAL, std::string("cannot open ") + path);
    const char magic[8] = {'C', 'L', 'S', 'G', '0', '0', '0', '1'};
    std::fwrite(magic, 1, 8, f);
    std::fwrite(&s->cfg, sizeof(s->cfg), 1, f);
    std::fwrite(&s->nparams, sizeof(s->nparams), 1, f);
    std::fwrite(th.data(), sizeof(float), th.size(), f);
    const int scaled = s->scaled ? 1 : 0;
    std::fwrite(&scaled, sizeof(int), 1, f);
    std::fwrite(s->in_scale, sizeof(double), 4, f);
    std::fwrite(s->out_scale, sizeof(double), 4, f);
    std::fwrite(s->ex_mean, sizeof(double), 4, f);
    std::fwrite(s->ex_std, sizeof(double), 4, f);
    const bool ok = std::fclose(f) == 0;
    return ok ? CL_OK : sfail(CL_EINVAL, "write failed");
}

cl_status cl_surrogate_load(cl_surrogate* s, const char* path) {
    if (!s || !path) return sfail(CL_EINVAL, "NULL argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return sfail(CL_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    cl_surrogate_cfg cfg;
    int64_t np = 0;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "CLSG0001", 8) == 0 &&
              std::fread(&cfg, sizeof(cfg), 1, f) == 1 && std::fread(&np, sizeof(np), 1, f) == 1;
    if (!ok || np != s->nparams || cfg.layers != s->cfg.layers || cfg.n_fields != s->cfg.n_fields ||
        cfg.extra_inputs != s->cfg.extra_inputs) {
        std::fclose(f);
        return sfail(CL_EINVAL, "file does not match this surrogate");
    }
    std::vector<float> th(np);
    int scaled = 0;
    ok = std::fread(th.data(), sizeof(float), np, f) == static_cast<size_t>(np) &&
         std::fread(&scaled, sizeof(int), 1, f) == 1 && std::fread(s->in_scale, sizeof(double), 4, f) == 4 &&
         std::fread(s->out_scale, sizeof(double), 4, f) == 4 && std::fread(s->ex_mean, sizeof(double), 4, f) == 4 &&
         std::fread(s->ex_std, sizeof(double), 4, f) == 4;
    std::fclose(f);
    if (!ok) return sfail(CL_EINVAL, "truncated surrogate file");
    s->scaled = scaled != 0;
    s->cfg.jump_steps = cfg.jump_steps;
    return cl_surrogate_set_params(s, th.data());
}

cl_status cl_surrogate_set_gate(cl_surrogate* s, double fluct_tol) {
    if (!s) return sfail(CL_EINVAL, "NULL surrogate");
    if (std::isnan(fluct_tol)) return sfail(CL_EINVAL, "fluct_tol is NaN");
    s->fluct_tol = fluct_tol;
    return CL_OK;
}

cl_status cl_surrogate_set_jump(cl_surrogate* s, cl_jump_mode mode) {
    if (!s) return sfail(CL_EINVAL, "NULL surrogate");
    if (mode != CL_JUMP_NETWORK && mode != CL_JUMP_LINEAR) return sfail(CL_EINVAL, "unknown jump mode");
    s->jump_mode = mode;
    return CL_OK;
}

namespace {

// Buffers of the linear propagation for an N^3 lattice of nf fields: nf
// packed complex arrays in and out, the Laplacian eigenvalues per index, the
// sub-step table.
// One axis pass of the line FFT over array q of the forward (pz) or
// propagated (pw) set, in the lattice's precision.
hipError_t prop_fft(cl_surrogate* s, int q, bool forward_set, const double2* tw64, int N, int axis, bool fp32,
                    bool inverse, hipStream_t st) {
    void* d = forward_set ? s->pz[q] : s->pw[q];
    if (fp32) return cl::launch_fft_f32(static_cast<float2*>(d), s->tw32, N, axis, st, inverse);
    return cl::launch_spec_fft(static_cast<double2*>(d), tw64, N, axis, st, inverse);
}

cl_status ensure_prop_bufs(cl_surrogate* s, const cl_lattice* h, int nsteps) {
    const int N = h->N;
    // the table's index triples are packed 10 bits per index
    if (N > 1024) return sfail(CL_EUNSUPPORTED, "the linear jump supports N <= 1024");
    const size_t n3 = static_cast<size_t>(N) * N * N;
    const bool fp32 = h->prec == CL_FP32;
    if (s->propN != N || s->propdx != h->dx || s->propfp32 != fp32) {
        for (void** p : {&s->pz[0], &s->pz[1], &s->pw[0], &s->pw[1]}) {
            if (*p) hipFree(*p);
            *p = nullptr;
        }
        if (s->tw32) hipFree(s->tw32);
        s->tw32 = nullptr;
        if (s->kap2) hipFree(s->kap2);
        if (s->ptable) hipFree(s->ptable);
        if (s->ptriples) hipFree(s->ptriples);
        s->kap2 = nullptr;
        s->ptable = nullptr;
        s->ptriples = nullptr;
        s->propN = 0;
        s->propdx = 0.0;
        for (int q = 0; q < h->nf; ++q) {
            if (fp32) {
                s->pz[q] = dalloc<float2>(n3);
                s->pw[q] = dalloc<float2>(n3);
            } else {
                s->pz[q] = dalloc<double2>(n3);
                s->pw[q] = dalloc<double2>(n3);
            }
            if (!s->pz[q] || !s->pw[q]) return sfail(CL_ENOMEM, "propagator buffers");
        }
        s->kap2 = dalloc<double>(N);
        s->ptable = dalloc<double>(cl::prop_table_entries(N) * 16);
        s->ptriples = dalloc<uint32_t>(cl::prop_table_entries(N));
        if (!s->kap2 || !s->ptable || !s->ptriples) return sfail(CL_ENOMEM, "propagator buffers");
        const std::vector<uint32_t> tri = cl::prop_triples(N);
        SHIP(hipMemcpy(s->ptriples, tri.data(), tri.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        std::vector<double> k2(N);
        const long double pi = 3.141592653589793238462643383279502884L;
        for (int n = 0; n < N; ++n) {
            const double sn = static_cast<double>(std::sin(pi * n / N));
            k2[n] = 4.0 / (h->dx * h->dx) * sn * sn;
        }
        SHIP(hipMemcpy(s->kap2, k2.data(), N * sizeof(double), hipMemcpyHostToDevice));
        if (fp32) {
            // exp(-2 pi i k / N) formed in long double, rounded once to FP32
            std::vector<float2> tw(std::max(N / 2, 1));
            for (int k = 0; k < N / 2; ++k) {
                const long double t = -2.0L * pi * k / N;
                tw[k] = make_float2(static_cast<float>(std::cos(t)), static_cast<float>(std::sin(t)));
            }
            s->tw32 = dalloc<float2>(tw.size());
            if (!s->tw32) return sfail(CL_ENOMEM, "propagator buffers");
            SHIP(hipMemcpy(s->tw32, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice));
        }
        s->propN = N;
        s->propdx = h->dx;
        s->propfp32 = fp32;
    }
    if (s->psteps_cap < nsteps) {
        if (s->psteps) hipFree(s->psteps);
        if (s->psteps_host) hipHostFree(s->psteps_host);
        s->psteps_host = nullptr;
        s->psteps = dalloc<cl::PropStep>(nsteps);
        if (s->psteps &&
            hipHostMalloc(reinterpret_cast<void**>(&s->psteps_host), nsteps * sizeof(cl::PropStep)) != hipSuccess)
            s->psteps_host = nullptr;
        s->psteps_cap = s->psteps && s->psteps_host ? nsteps : 0;
        if (!s->psteps_cap) return sfail(CL_ENOMEM, "propagator sub-step table");
    }
    return CL_OK;
}

}  // namespace

cl_status cl_surrogate_advance(cl_lattice* h, cl_surrogate* s, cl_integrator fallback, double dt, int n_jumps,
                               double threshold, cl_observables* per_jump, cl_surrogate_report* rep) {
    if (!h || !s) return sfail(CL_EINVAL, "NULL argument");
    if (h->dim != 3) return sfail(CL_EUNSUPPORTED, "the surrogate works on three-dimensional lattices");
    if (h->ng) return sfail(CL_EUNSUPPORTED, "the surrogate takes lattices without the gravitational-wave tensor");
    if (fallback != CL_LEAPFROG && fallback != CL_VV4)
        return sfail(CL_EINVAL, "the fallback integrator must be leapfrog or VV4");
    if (h->nf != s->cfg.n_fields) return sfail(CL_EINVAL, "lattice fields do not match the surrogate");
    if (!valid_net_N(h->N)) return sfail(CL_EINVAL, "lattice N must be a power of two >= 16");
    const bool linear = s->jump_mode == CL_JUMP_LINEAR;
    if (!linear && !s->scaled) return sfail(CL_ESTATE, "surrogate has no normalisation (train or load it first)");
    if (!(dt > 0.0) || n_jumps < 0) return sfail(CL_EINVAL, "dt > 0 and n_jumps >= 0 needed");
    const auto t0 = std::chrono::steady_clock::now();
    const int N = h->N, K = s->cfg.jump_steps;
    const bool expand = h->mode == CL_SELF_CONSISTENT;
    cl_status st = linear ? CL_OK : ensure_bufs(s, N, false);
    if (st) return st;
    const double2* tw = nullptr;
    const int sub = fallback == CL_VV4 ? 3 : 1;  // sub-steps per step
    if (linear) {
        if ((st = ensure_prop_bufs(s, h, sub * K))) return st;
        st = cl::spectral_twiddles(h, &tw);
        if (st) return sfail(st, cl_last_error(h));
    }
    int fallbacks = 0, fluct_rejects = 0;
    double maxr = 0.0, net_ms = 0.0;
    cl_observables o;
    cl::Scal sc;
    st = read_lattice(h, &o, &sc);
    if (st) return st;
    cl_scalars bg;
    st = cl_get_state(h, &bg);
    if (st) return sfail(st, cl_last_error(h));
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // network start / end (timing), packed input ready
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto& x : ev)
                if (x) hipEventDestroy(x);
            return sfail(CL_EDEVICE, "hipEventCreate");
        }
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard() {
            for (int i = 0; i < 3; ++i) hipEventDestroy(e[i]);
        }
    } ev_guard{ev};
    const double al = h->alpha, mp2 = h->mp * h->mp;
    const bool fp32 = h->prec == CL_FP32;
    // twiddles of the fused z passes, in the lattice's precision
    const void* const twz = fp32 ? static_cast<const void*>(s->tw32) : static_cast<const void*>(tw);
    if (!s->jump_obs &&
        hipHostMalloc(reinterpret_cast<void**>(&s->jump_obs), sizeof(cl_surrogate::JumpObs)) != hipSuccess) {
        s->jump_obs = nullptr;
        return sfail(CL_ENOMEM, "pinned host staging of the jump observables");
    }
    for (int j = 0; j < n_jumps; ++j) {
        // the jump writes the other state buffer; the current one is the
        // snapshot until the jump is kept
        const int cur0 = h->cur;
        void* const src = h->buf[cur0];
        void* const dst = h->buf[cur0 ^ 1];
        if (!linear) {
        // network input from the current state, then the network on the
        // surrogate's stream while the host runs the predictor
        cl::sg::PackArgs pa{};
        pa.state = src;
        pa.N = N;
        pa.nf = h->nf;
        double e[4];
        raw_extra(o, sc, e);
        for (int jf = 0; jf < h->nf; ++jf) {
            pa.mean[jf] = o.mean[jf];
            pa.mean[h->nf + jf] = sc.mean_p[jf];
        }
        for (int c = 0; c < 2 * h->nf; ++c) pa.inv_scale[c] = 1.0 / s->in_scale[c];
        pa.nextra = s->cfg.extra_inputs;
        for (int k = 0; k < pa.nextra; ++k) pa.extra[k] = static_cast<float>((e[k] - s->ex_mean[k]) / s->ex_std[k]);
        pa.x_out = s->x0;
        SHIP(cl::sg::launch_pack_state(pa, fp32, h->stream));
        SHIP(hipEventRecord(ev[2], h->stream));
        SHIP(hipStreamWaitEvent(s->stream, ev[2], 0));
        SHIP(hipEventRecord(ev[0], s->stream));
        st = forward(s, N, false);
        if (st) return st;
        SHIP(hipEventRecord(ev[1], s->stream));
        SHIP(hipStreamWaitEvent(h->stream, ev[1], 0));
        } else {
            // fluctuations -> modes (packing fused with the z pass, then y and
            // x) while the host runs the predictor
            SHIP(hipEventRecord(ev[0], h->stream));
            cl::PropZArgs pk{};
            pk.state = src;
            pk.N = N;
            pk.nf = h->nf;
            pk.tw = twz;
            for (int jf = 0; jf < h->nf; ++jf) {
                pk.mean[jf] = o.mean[jf];
                pk.mean[h->nf + jf] = sc.mean_p[jf];
            }
            for (int q = 0; q < h->nf; ++q) pk.z[q] = s->pz[q];
            SHIP(cl::launch_prop_pack_fftz(pk, fp32, h->stream));
            for (int q = 0; q < h->nf; ++q)
                for (int axis = 1; axis < 3; ++axis) SHIP(prop_fft(s, q, true, tw, N, axis, fp32, false, h->stream));
        }
        // predictor: homogeneous modes and background over the jump, in FP64
        double f[2] = {o.mean[0], o.mean[1]}, pm[2] = {sc.mean_p[0], sc.mean_p[1]}, var[2] = {o.var[0], o.var[1]};
        double rho_hom_K = 0.0;
        for (int jf = 0; jf < h->nf; ++jf) rho_hom_K += pm[jf] * pm[jf] / (2.0 * std::pow(o.a, 6.0));
        const double rho_lat = o.EK[0] + o.EK[1] + o.EG[0] + o.EG[1] + o.EV;
        const double rho_r0 = std::max(0.0, rho_lat - rho_hom_K - hom_V(h, f, var));
        double a = bg.a, b = bg.b;
        std::vector<HomSums> hom;
        std::vector<cl::PropStep> msteps;
        advance_homogeneous(h, fallback, dt, K, f, pm, a, b, var, rho_r0, bg.a, hom, linear ? &msteps : nullptr);
        if (linear) {
            // K steps of the linearised equations per mode, then back to sites
            // (x, y, then the z pass fused with the unpacking into dst)
            if (msteps.size() > static_cast<size_t>(s->psteps_cap))
                return sfail(CL_ESTATE, "propagator sub-step table too small");
            std::copy(msteps.begin(), msteps.end(), s->psteps_host);
            SHIP(hipMemcpyAsync(s->psteps, s->psteps_host, msteps.size() * sizeof(cl::PropStep),
                                hipMemcpyHostToDevice, h->stream));
            cl::PropModeArgs pmd{};
            for (int q = 0; q < h->nf; ++q) {
                pmd.in[q] = s->pz[q];
                pmd.out[q] = s->pw[q];
            }
            pmd.N = N;
            pmd.nf = h->nf;
            pmd.kap2 = s->kap2;
            pmd.steps = s->psteps;
            pmd.nsteps = static_cast<int>(msteps.size());
            pmd.scale = 1.0 / (static_cast<double>(N) * N * N);
            pmd.table = s->ptable;
            pmd.triples = s->ptriples;
            pmd.ntriples = cl::prop_table_entries(N);
            SHIP(cl::launch_prop_modes(pmd, fp32, h->stream));
            for (int q = 0; q < h->nf; ++q)
                for (int axis = 2; axis >= 1; --axis) SHIP(prop_fft(s, q, false, tw, N, axis, fp32, true, h->stream));
            cl::PropZArgs pu{};
            pu.out = dst;
            pu.N = N;
            pu.nf = h->nf;
            pu.tw = twz;
            for (int jf = 0; jf < h->nf; ++jf) {
                pu.mean[jf] = f[jf];
                pu.mean[h->nf + jf] = pm[jf];
            }
            for (int q = 0; q < h->nf; ++q) pu.z[q] = s->pw[q];
            SHIP(cl::launch_prop_ifftz_unpack(pu, fp32, h->stream));
            SHIP(hipEventRecord(ev[1], h->stream));
        } else {
            cl::sg::UnpackArgs ua{};
            ua.state = src;
            ua.out = dst;
            ua.N = N;
            ua.nf = h->nf;
            for (int jf = 0; jf < h->nf; ++jf) {
                ua.old_mean[jf] = o.mean[jf];
                ua.old_mean[h->nf + jf] = sc.mean_p[jf];
                ua.new_mean[jf] = f[jf];
                ua.new_mean[h->nf + jf] = pm[jf];
            }
            for (int c = 0; c < 2 * h->nf; ++c) ua.out_scale[c] = s->out_scale[c];
            ua.y = s->y;
            ua.ystride = ystride(s);
            SHIP(cl::sg::launch_unpack_jump(ua, fp32, h->stream));
        }
        const double eta1 = bg.eta + K * dt;
        const int64_t step1 = bg.step + K;
        // a prediction that leaves the background non-finite or a <= 0 is rejected outright
        bool ok = std::isfinite(a) && std::isfinite(b) && a > 0.0;
        cl_observables after{};
        cl::Scal sca{};
        const double a_pred = a;
        if (ok) {
            // one reduction of the new state (at the predicted a; the sums
            // that the corrector needs do not depend on a), its variances
            // about the predicted means
            h->cur = cur0 ^ 1;
            st = cl::set_background_async(h, a_pred, b, eta1, step1, f);
            if (!st) st = cl::observe_once(h, &s->jump_obs->o, &s->jump_obs->sc);
            if (st) {
                // the untouched state stays the current one
                h->cur = cur0;
                return sfail(st, cl_last_error(h));
            }
            after = s->jump_obs->o;
            sca = s->jump_obs->sc;
            ok = !after.nonfinite;
        } else {
            SHIP(hipStreamSynchronize(h->stream));
        }
        float ms = 0.0f;
        SHIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        net_ms += ms;
        double S1[3] = {0.0, 0.0, 0.0};
        if (ok) volume_sums(after, S1);
        if (ok && expand) {
            // corrector: background re-integrated against the start and endpoint sums
            double S0[3];
            volume_sums(o, S0);
            a = bg.a;
            b = bg.b;
            correct_background(h, fallback, dt, K, S0, S1, hom, a, b);
            ok = std::isfinite(a) && std::isfinite(b) && a > 0.0;
        }
        // the endpoint's observables at the corrected a, and its Hubble residual
        double r = std::nan("");
        cl_observables rec = after;
        if (ok) {
            const double sK = std::pow(a_pred / a, 6.0), sG = (a_pred / a) * (a_pred / a);
            for (int jf = 0; jf < 2; ++jf) {
                rec.EK[jf] = after.EK[jf] * sK;
                rec.EG[jf] = after.EG[jf] * sG;
            }
            rec.a = a;
            rec.H = expand ? b / a : 0.0;
            rec.eta = eta1;
            if (expand) {
                const double rho = S1[0] / std::pow(a, 6.0) + S1[1] / (a * a) + S1[2];
                const double rhs = std::pow(a, 2.0 * al) * rho / (3.0 * mp2);
                r = std::fabs((b / a) * (b / a) - rhs) / rhs;
            } else {
                r = 0.0;
            }
            rec.hubble_residual = r;
            maxr = std::max(maxr, r);
        }
        // second gate: the fluctuations' variance and energy may move only so
        // far over one jump (their physical change over 16 steps is a few per cent)
        bool fluct_ok = true;
        if (ok && s->fluct_tol > 0.0) {
            for (int jf = 0; jf < h->nf; ++jf)
                if (o.var[jf] > 0.0 && !(std::fabs(after.var[jf] / o.var[jf] - 1.0) <= s->fluct_tol)) fluct_ok = false;
            double pm1[2] = {sca.mean_p[0], sca.mean_p[1]}, f1[2] = {after.mean[0], after.mean[1]},
                   v1[2] = {after.var[0], after.var[1]};
            double K1 = 0.0;
            for (int jf = 0; jf < h->nf; ++jf) K1 += pm1[jf] * pm1[jf] / (2.0 * std::pow(a, 6.0));
            const double rho1 = rec.EK[0] + rec.EK[1] + rec.EG[0] + rec.EG[1] + rec.EV;
            const double fl1 = rho1 - K1 - hom_V(h, f1, v1);
            const double fl_pred = rho_r0 * std::pow(bg.a / a, 4.0);
            if (fl_pred > 0.0 && !(std::fabs(fl1 / fl_pred - 1.0) <= s->fluct_tol)) fluct_ok = false;
            if (!fluct_ok) ++fluct_rejects;
        }
        if (ok && r <= threshold && fluct_ok) {
            // accept: the corrected background goes to the device
            st = cl::set_background_async(h, a, b, eta1, step1, after.mean);
            if (st) return sfail(st, cl_last_error(h));
            if (per_jump) per_jump[j] = rec;
            o = rec;
            sc = sca;
            bg = cl_scalars{a, b, eta1, step1};
        } else {
            // undo the jump (back to the untouched buffer, the scalar block
            // as it was) and run the integrator instead
            h->cur = cur0;
            SHIP(hipMemcpyAsync(h->sc, &sc, sizeof(cl::Scal), hipMemcpyHostToDevice, h->stream));
            SHIP(hipStreamSynchronize(h->stream));
            st = cl_set_state(h, &bg);
            if (st) return sfail(st, cl_last_error(h));
            std::vector<cl_observables> recs(K);
            st = cl_step(h, fallback, dt, K, recs.data());
            if (st) return sfail(st, cl_last_error(h));
            ++fallbacks;
            o = recs.back();
            SHIP(hipMemcpyAsync(&sc, h->sc, sizeof(cl::Scal), hipMemcpyDeviceToHost, h->stream));
            SHIP(hipStreamSynchronize(h->stream));
            bg = cl_scalars{sc.a, sc.b, sc.eta, h->step};
            if (per_jump) per_jump[j] = o;
        }
    }
    SHIP(hipStreamSynchronize(h->stream));
    if (rep) {
        rep->jumps = n_jumps;
        rep->fallbacks = fallbacks;
        rep->max_residual = maxr;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        rep->net_seconds = 1e-3 * net_ms;
        rep->fluct_rejects = fluct_rejects;
    }
    return CL_OK;
}

}  // extern "C"
