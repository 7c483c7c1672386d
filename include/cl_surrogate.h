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
 * its gradient with respect to all parameters (layout above).  N a power of
 * two >= 32 (as for every training call). */
cl_status cl_surrogate_loss_grad(cl_surrogate* s, int N, const float* x, const float* t, double* loss,
                                 float* grad);

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
 * for jump_steps steps of size dt.  One jump: snapshot the state; the network
 * predicts the fluctuation increment; the homogeneous modes and (a, a') are
 * advanced by the FP64 equations of motion over the jump (predictor, with the
 * fluctuations' energy redshifting as radiation); then (a, a') are
 * re-integrated with the volume sums <pi^2>, <(grad f)^2>, <V> interpolated
 * linearly between the start and the predicted endpoint (corrector; the sums
 * do not depend on a, so one pass is converged).  If the Hubble-constraint
 * residual at the endpoint exceeds `threshold` (or any sum is non-finite) the
 * jump is undone and the integrator `fallback` (CL_LEAPFROG or CL_VV4) runs
 * jump_steps steps instead.  per_jump (nullable) receives one record per jump. */
cl_status cl_surrogate_advance(cl_lattice* h, cl_surrogate* s, cl_integrator fallback, double dt, int n_jumps,
                               double threshold, cl_observables* per_jump, cl_surrogate_report* rep);

#ifdef __cplusplus
}
#endif

#endif /* CL_SURROGATE_H */
