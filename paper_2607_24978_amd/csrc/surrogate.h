// Internal declarations of the learned-surrogate kernels (surrogate.hip)
// and their host runtime (surrogate_api.cpp).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace cl {
namespace sg {

// Periodic 3x3x3 convolution, channels-last BF16 in, FP32 and/or BF16 out.
struct ConvArgs {
    const void* in;      // BF16 [site][cin]
    const void* w;       // BF16 [o][nb*16][cin]
    const float* bias;   // [>= cout] or null
    float* z_out;        // FP32 [site][z_stride] (pre-activation) or null
    void* zh_out;        // BF16 [site][zh_stride] pre-activation (kept for the backward pass) or null
    int zh_stride;
    void* a_out;         // BF16 [site][a_stride] (GELU(z) if gelu, else z) or null
    const void* gz;      // BF16 [site][gz_stride] or null: a_out = z * GELU'(gz) (input gradient
                         // through the activation of the layer below)
    int gz_stride;
    int N;
    int nsites;          // N^3, a multiple of 16
    int cout;            // output channels stored (multiple of 4)
    int z_stride, a_stride;
    int gelu;
};

struct WgradArgs {
    const void* dz;      // BF16 [site][cout_stride]
    const void* x;       // BF16 [site][cin]
    float* partials;     // [WgradShape::parts][partial_stride]
    int N, nsites;
    int cout_stride;
    int partial_stride;  // WgradShape::stride
    int L;               // x planes per workgroup (WgradShape::L)
};

// Launch shape of the weight-gradient kernel on an N^3 lattice (N a multiple
// of 32): workgroups, x planes each marches over, partial-sum slots written
// and their stride (27*coutp*cinp + coutp floats).
struct WgradShape {
    int grid, L, parts, stride;
};
WgradShape wgrad_shape(int N, int cin, int cout_stride);

struct WgradReduceArgs {
    const float* partials;
    int nparts, partial_stride;
    int coutp, cinp, cout, cin;
    float* gW;  // flat [cout][cin][27]
    float* gb;  // [cout]
};

struct PrepArgs {
    const float* theta;  // flat W[co][ci][27] of this layer
    int bias_offset;     // theta index of b[0] (relative to theta)
    int cout, cin, coutp, cinp, no_f;
    int coutp_d, cinp_d, no_d;
    uint16_t* wf;        // forward weights [no_f][coutp][cinp]
    uint16_t* wd;        // input-gradient weights [no_d][coutp_d][cinp_d] or null
    float* bias;         // [cout]
};

struct PackArgs {
    const void* state;   // row-interleaved lattice state
    int N, nf;
    double mean[4];
    double inv_scale[4];
    float extra[4];
    int nextra;
    uint16_t* x_out;     // BF16 [site][8] or null
    float* fluct_out;    // FP32 [c][site] or null
    float* fluct_sub;    // FP32 [c][site]: (fluctuation - fluct_sub_ref) or null
    const float* fluct_sub_ref;
};

struct SampleArgs {
    const float* fluct;  // [c][n3]
    const float* incr;   // [c][n3]
    float inv_in[4], inv_out[4], extra[4];
    int nextra, nfc;
    uint16_t* x;         // BF16 [site][8]
    float* target;       // [c][n3]
    size_t n3;
};

struct UnpackArgs {
    const void* state;   // the state before the jump
    void* out;           // the state after it (may not alias `state`)
    int N, nf;
    double old_mean[4], new_mean[4], out_scale[4];
    const float* y;      // FP32 [site][ystride]
    int ystride;
};

hipError_t launch_conv_fwd(const ConvArgs& a, int cin, int nb, int grid, hipStream_t s);
hipError_t launch_conv_wgrad(const WgradArgs& a, int cin, hipStream_t s);
hipError_t launch_wgrad_reduce(const WgradReduceArgs& a, hipStream_t s);
hipError_t launch_mse_grad(const float* y, int ystride, const float* t, int cout, size_t nsites, double scale,
                           void* dy, double* partial, int grid, hipStream_t s);
hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
hipError_t launch_prepare_layer(const PrepArgs& a, hipStream_t s);
hipError_t launch_pack_state(const PackArgs& a, bool fp32, hipStream_t s);
hipError_t launch_pack_sample(const SampleArgs& a, hipStream_t s);
hipError_t launch_unpack_jump(const UnpackArgs& a, bool fp32, hipStream_t s);

}  // namespace sg
}  // namespace cl
