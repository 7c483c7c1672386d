/*
 * cl_surrogate.h -- C ABI of the learned surrogate for the lattice path.
 *
 * A stack of periodic 3x3x3 convolutions (hidden width `hidden`, GELU
 * between layers, no activation after the last) that maps the fluctuations
 * of a lattice state about its volume means, plus broadcast background
 * features, to the increment of those fluctuations over `jump_steps`
 * integrator steps.  BF16 weights and activations with FP32 accumulation
 * (gfx950 MFMA); FP32 master weights trained with Adam by the library's own
 * forward and backward kernels.  The homogeneous modes and the scale factor
 * are advanced over a jump by the FP64 equations of the method (Sect. 2.1,
 * Eqs. singletEOM without gradients, Friedmann1), and the Hubble constraint
 * (Eq. Friedmann2) -- the accuracy monitor of Sect. 2.1 -- gates every jump:
 * above the threshold the jump is undone and the integrator runs instead.
 *
 * The paper itself has no learned component; this is an extension of the
 * hot path.  Conventions as in cl_lattice.h.
 *
 * Parameter layout (host FP32, cl_surrogate_get/set_params): for each layer
 * l in order, W_l[c_out][c_in][3][3][3] with W[o][i][dx+1][dy+1][dz+1]
 * multiplying input channel i at site n + (dx, dy, dz) (periodic), then
 * b_l[c_out].  Layer 0 has c_in = 2*n_fields + extra_inputs, the last layer
 * c_out = 2*n_fields.
 */
#ifndef CL_SURROGATE_H
#define CL_SURROGATE_H

#include <stdint.h>

#include "cl_lattice.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cl_surrogate cl_surrogate;

typedef struct {
    int n_fields;       /* lattice fields (2: phi, chi); channels = 2*n_fields */
    int extra_inputs;   /* broadcast inputs: 2 = (a, H), 4 = (a, H, <f_0>, <pi_0>) */
    int hidden;         /* hidden channels (32) */
    int layers;         /* convolution layers (>= 2) */
    int jump_steps;     /* integrator steps one application replaces (16) */
    uint64_t init_seed; /* weight initialisation (uniform, He bound) */
} cl_surrogate_cfg;

typedef struct {
    int epochs;         /* passes over the recorded pairs */
    double lr;          /* initial Adam step (cosine decay to lr_final) */
    double lr_final;
    uint64_t shuffle_seed;
    int holdout;        /* last `holdout` pairs are not trained on */
} cl_train_cfg;

typedef struct {
    int steps;
    double first_loss;     /* loss of the first step */
    double last_epoch_loss;/* mean training loss over the last epoch */
    double holdout_loss;   /* mean loss on the held-out pairs after training */
    double holdout_zero;   /* mean loss of the zero-increment predictor on them */
    double seconds;
} cl_train_report;

typedef struct {
    int jumps;
    int fallbacks;
    double max_residual;   /* largest Hubble residual seen after a network jump */
    double seconds;        /* wall time of the call */
    double net_seconds;    /* device time of the network evaluations (HIP events) */
    int fluct_rejects;     /* jumps the second gate (fluctuations) rejected */
    int reserved;
} cl_surrogate_report;

/* Message for the last failing cl_surrogate_* call on this thread. */
const char* cl_surrogate_last_error(void);

/* Create / destroy.  hidden must be 32, the input and output channel counts
 * at most 8; layers >= 2; jump_steps >= 1. */
cl_status cl_surrogate_create(const cl_surrogate_cfg* cfg, cl_surrogate** out);
cl_status cl_surrogate_destroy(cl_surrogate* s);

/* Number of FP32 parameters; get / set them in the layout above. */
cl_status cl_surrogate_num_params(const cl_surrogate* s, int64_t* n);
cl_status cl_surrogate_get_params(cl_surrogate* s, float* theta);
cl_status cl_surrogate_set_params(cl_surrogate* s, const float* theta);

/* One network evaluation on host data: x[c][N^3] (c_in channels, FP32,
 * rounded to BF16 on the device) -> y[c][N^3] (c_out channels, FP32).  N a
 * power of two >= 16. */
cl_status cl_surrogate_forward(cl_surrogate* s, int N, const float* x, float* y);

/* Mean-squared error of the network on (x, t) over every output element and
 * its gradient with respect to all parameters (layout above); if grad_x is
 * not NULL it receives the gradient with respect to the input x (c_in
 * channels, the layout of x).  N a power of two >= 32 (as for every
 * training call).  Backward pass: output gradient and the GELU-scaled layer
 * gradients rounded to BF16 (GELU' taken at the pre-activations as kept by
 * the forward pass, rounded to BF16), weight gradients as FP32 sums over
 * sites of their products with the BF16 layer inputs, input gradients as FP32
 * convolutions with the flipped, transposed BF16 weights.  GELU and GELU'
 * evaluate the normal distribution function through a rational-exponential
 * erfc approximation of relative error below 1.2e-7. */
cl_status cl_surrogate_loss_grad(cl_surrogate* s, int N, const float* x, const float* t, double* loss,
                                 float* grad, float* grad_x);

/* One Adam step (beta = 0.9, 0.999, eps = 1e-8, bias-corrected with the
 * handle's step count, which set_params resets) of the FP32 master weights
 * with a caller-supplied gradient (host FP32, parameter layout) and step
 * size lr, in FP32 on the device; the BF16 copies the kernels use are
 * refreshed.  With cl_surrogate_loss_grad it makes a training loop of the
 * caller's own -- for instance one that all-reduces the gradients of
 * several devices before the step. */
cl_status cl_surrogate_apply_grad(cl_surrogate* s, const float* grad, double lr);

/* Normalisation of the network's inputs and outputs: the fluctuation of
 * field channel c about its volume mean enters divided by in_scale[c], the
 * output times out_scale[c] is the increment of that fluctuation over one
 * jump; broadcast feature k enters as (value - extra_mean[k]) / extra_std[k].
 * Fixed from the training pairs by the first cl_surrogate_train, saved and
 * loaded with the parameters, or set here (scales and spreads > 0). */
typedef struct {
    double in_scale[4];
    double out_scale[4];
    double extra_mean[4];
    double extra_std[4];
} cl_surrogate_norm;

cl_status cl_surrogate_get_normalisation(const cl_surrogate* s, cl_surrogate_norm* out);
cl_status cl_surrogate_set_normalisation(cl_surrogate* s, const cl_surrogate_norm* in);

/* Training data: pairs (state, state jump_steps later) of lattices of size
 * N (a power of two >= 32), recorded on the device from lattice handles (FP32
 * or FP64 fields). */
cl_status cl_surrogate_dataset_reserve(cl_surrogate* s, int N, int max_pairs);
cl_status cl_surrogate_record_input(cl_surrogate* s, cl_lattice* h);
cl_status cl_surrogate_record_target(cl_surrogate* s, cl_lattice* h);
cl_status cl_surrogate_dataset_size(const cl_surrogate* s, int* pairs);

/* Train with Adam on the recorded pairs (one pair per step); fixes the
 * input / output normalisation from the training pairs on the first call. */
cl_status cl_surrogate_train(cl_surrogate* s, const cl_train_cfg* cfg, cl_train_report* rep);

/* Save / load parameters and normalisation (binary file). */
cl_status cl_surrogate_save(const cl_surrogate* s, const char* path);
cl_status cl_surrogate_load(cl_surrogate* s, const char* path);

/* Advance the lattice by n_jumps applications of the network, each standing
 * for jump_steps steps of size dt.  One jump: the new state is formed in the
 * lattice's second state buffer (the current one is kept as the snapshot and
 * becomes the other buffer if the jump is kept); the network predicts the
 * fluctuation increment; the homogeneous modes and (a, a') are
 * advanced over the jump by the FP64 equations of motion of a uniform
 * lattice with the integrator's sub-step pattern (predictor: force and
 * potential averaged over Gaussian fluctuations of the start variances, the
 * rest of the fluctuations' energy redshifting as radiation); the new state
 * is the predicted means plus the old fluctuations plus the increment; then
 * (a, a') are re-integrated from the start (corrector) with rho and p from the
 * a-independent volume sums <pi^2>/2, <(grad f)^2>/2, <V>, split into their
 * homogeneous part along the predictor's trajectory and the fluctuations'
 * share, which moves linearly from its start value to that of the new state.
 * The endpoint's residual of the Hubble constraint (Eq. Friedmann2, the
 * accuracy monitor of Sect. 2.1) is evaluated from those sums at the
 * corrected a.  The jump is undone and the integrator `fallback` (CL_LEAPFROG
 * or CL_VV4) runs jump_steps steps instead if any sum is non-finite, if the
 * residual exceeds `threshold`, or if the second gate (cl_surrogate_set_gate)
 * fails.  One reduction of the lattice per jump; the predictor runs on the
 * host while the device evaluates the network.  per_jump (nullable) receives
 * one record per jump. */
/* Second gate of cl_surrogate_advance (an energy residual of the
 * fluctuations, which the Hubble residual -- set by the homogeneous energy --
 * hardly sees): a jump is also undone if any field's variance, or the energy
 * of the fluctuations (lattice rho minus the homogeneous kinetic energy and
 * the Gaussian-averaged potential of the means), changes over the jump by
 * more than the relative tolerance fluct_tol against its start value
 * (the energy redshifted as radiation over the jump).  Their physical change
 * over one jump of 16 steps is a few per cent; default 0.25; <= 0 switches
 * the gate off. */
cl_status cl_surrogate_set_gate(cl_surrogate* s, double fluct_tol);

/* How cl_surrogate_advance forms a jump's new fluctuations.
 * CL_JUMP_NETWORK (default): the network's predicted increment.
 * CL_JUMP_LINEAR: no network; every lattice Fourier mode of the fluctuations
 * is advanced by the integrator's own kick-drift-kick sub-steps of the
 * equations of motion (Sect. 2.1, Eq. singletEOM in program variables)
 * linearised about the FP64 background the predictor integrates: the
 * 7-point Laplacian's eigenvalue kappa^2 = sum_i (2/dx)^2 sin^2(pi n_i / N)
 * and the mass matrix d2V/df_i df_j at the predicted homogeneous values,
 * Hartree-averaged over Gaussian fluctuations of the start variances.  The
 * fluctuations go through the library's line FFT (two real channels per
 * complex transform) in the lattice's precision -- FP64 for FP64 lattices,
 * FP32 for FP32 lattices, where its rounding relative to the fluctuations
 * stays below that of the FP32 state -- so the jump costs a few lattice
 * passes however many steps it stands for.  Exact up to rounding for free
 * fields on a static background; otherwise its error is the fluctuations'
 * self-interaction over the jump, which the gates catch as it grows.  Needs
 * no training or normalisation.  The propagation over a jump depends on a
 * mode only through kappa^2, even in each mode index and symmetric in their
 * order, so one transfer matrix per sorted triple of folded indices is built
 * per jump, in FP64, and stored and applied in the lattice's precision
 * (C(N/2+3, 3) entries; a workspace of 128 bytes each: 47 MB at N = 256);
 * N <= 1024 (CL_EUNSUPPORTED above).  The jump's result is written to the
 * lattice's second state buffer, which becomes the current one if the jump
 * is kept (as after an integrator pass). */
typedef enum { CL_JUMP_NETWORK = 0, CL_JUMP_LINEAR = 1 } cl_jump_mode;
cl_status cl_surrogate_set_jump(cl_surrogate* s, cl_jump_mode mode);

cl_status cl_surrogate_advance(cl_lattice* h, cl_surrogate* s, cl_integrator fallback, double dt, int n_jumps,
                               double threshold, cl_observables* per_jump, cl_surrogate_report* rep);

#ifdef __cplusplus
}
#endif

#endif /* CL_SURROGATE_H */
