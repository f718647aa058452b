/*
 * Learned warm start of the batched XPBD substep: C ABI.
 *
 * This is an extension built on FF-SRL's solver (Dall'Alba et al., arXiv
 * 2503.18616, Sec. III-A.1, Alg. 1); the paper itself has no learned part.
 * After the prediction of a substep, a per-particle network maps 27 local
 * features of the predicted state to a correction of the predicted position,
 * so that the Gauss-Seidel sweeps start closer to the solution.  The plain
 * sweeps still decide convergence: after min_iterations the residual RMS of the
 * environment (the mean over all constraints of ((C + alpha~ lambda) / rest)^2,
 * square-rooted, as XPBD_FIELD_RESIDUAL reports it) is compared with a
 * threshold, and the sweeps continue to max_iterations when it is above
 * (unless the sweeps have stalled, see stall_ratio).
 *
 * Features f of particle i (float32; the network sees (f - in_shift) * in_scale
 * rounded to bfloat16), from the start-of-substep positions x and velocities
 * v, the predicted positions x_hat and the rest positions X:
 *   [0:3] x_hat_i - x_i, [3:6] v_i, [6:9] x_hat_i - X_i,
 *   [9 + 3k : 12 + 3k] (x_hat_n - x_hat_i) - (X_n - X_i) for the axis
 *   neighbour n of i in direction k = -x, +x, -y, +y, -z, +z (0 if none);
 *   [27:31] zero, [31] 1.0 for a free particle (w_i > 0), else 0.
 * The axis neighbour in direction +x is the particle with the same rest y and
 * z and the nearest larger rest x (smallest id among equals); likewise for
 * the other directions.
 *
 * Network (weights [out][in], float32 master copy, bfloat16 operands of the
 * matrix cores, float32 accumulation): a1 = bf16(relu(a0 W1^T + b1)),
 * a2 = bf16(relu(a1 W2^T + b2)), y = a2 W3^T + b3, correction =
 * out_shift + clamp(y, -8, 8) * out_scale (applied to free particles only;
 * the clamp keeps a network queried outside its training range from throwing
 * particles far).  Flat parameter order (float32):
 * W1 [128][27], b1 [128], W2 [128][128], b2 [128], W3 [3][128], b3 [3].
 *
 * Training: mean squared error over the free rows of a batch,
 * L = (1/2n) sum |y - t|^2, t = (x - x_hat - out_shift) / out_scale the
 * normalised correction the sweeps found; gradients from the
 * unnormalised error with bfloat16 backward operands, divided by n; one Adam
 * step (beta1 0.9, beta2 0.999, eps 1e-8) on the float32 master weights.
 *
 * Pointers named "device" must be device memory; others are host memory.
 * Errors: negative xpbd_status values with xpbd_last_error() set; no device
 * work is done after an argument error.  Calls are asynchronous on the
 * stream given at creation unless they return host data.
 */
#ifndef XPBD_LEARNED_H
#define XPBD_LEARNED_H

#include <stdint.h>

#include "xpbd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define XPBD_MLP_FEATURES 27
#define XPBD_MLP_FEATURE_STRIDE 32   /* bfloat16 values per feature row */
#define XPBD_MLP_HIDDEN 128
#define XPBD_MLP_OUTPUTS 3
#define XPBD_MLP_PARAMS 20483

typedef struct xpbd_mlp xpbd_mlp;

/* Create a network on the current device.  params: [XPBD_MLP_PARAMS] initial
 * float32 weights (NULL: all zero); in_shift, in_scale: [27] feature
 * normalisation; out_shift (m), out_scale (m per network unit): [3]; either
 * shift may be NULL (zero).  Adam state starts at zero.
 * hip_stream: the stream every later call of this network uses (NULL: null
 * stream).  The network owns its device memory until xpbd_mlp_destroy. */
xpbd_status xpbd_mlp_create(const float *params, const float *in_shift, const float *in_scale,
                            const float *out_shift, const float *out_scale, void *hip_stream,
                            xpbd_mlp **out);

/* Copy the float32 master weights to params [XPBD_MLP_PARAMS] (host);
 * synchronises the stream. */
xpbd_status xpbd_mlp_get_params(xpbd_mlp *net, float *params);

/* Replace the weights (host [XPBD_MLP_PARAMS]) and reset the Adam state. */
xpbd_status xpbd_mlp_set_params(xpbd_mlp *net, const float *params);

/* Network outputs y (device float32 [n][4]; columns 0..2 are written) of n
 * feature rows (device bfloat16 [n][XPBD_MLP_FEATURE_STRIDE]). */
xpbd_status xpbd_mlp_forward(xpbd_mlp *net, const uint16_t *features, int32_t n, float *y);

/* One training step on n samples: sample j is row rows[j] (device int32 [n];
 * the caller keeps every index inside the two tables) or, with rows NULL,
 * row j of features (device bfloat16 [.][32]; a row counts only if its free
 * flag, feature 31, is set) and targets (device float32 [.][4], normalised,
 * columns 0..2).  learning_rate 0 computes the loss and gradient without
 * updating.  loss (may be NULL) receives the mean loss: a host pointer after
 * a synchronisation of the stream, a device pointer (one float) in stream
 * order without one; grad (device float32 [XPBD_MLP_PARAMS], may be NULL)
 * the normalised gradient.  n >= 1. */
xpbd_status xpbd_mlp_train_step(xpbd_mlp *net, const uint16_t *features, const float *targets,
                                const int32_t *rows, int32_t n, float learning_rate, float *loss,
                                float *grad);

/* num_steps training steps in one call (no host work between them).  Step s
 * trains on the batch rows rows[(start_s + j) mod num_rows], j < batch: a
 * window of the device int32 row list rows [num_rows] (num_rows >= batch;
 * the caller keeps every index inside the two tables, as for
 * xpbd_mlp_train_step) that may wrap around its end, with start_s = starts[s]
 * (host int64 [num_steps], each in [0, num_rows)) or, with starts NULL,
 * (s batch) mod num_rows; its learning rate is
 * first_rate (last_rate / first_rate)^(s / (num_steps - 1)) (computed in
 * double, rounded to float); its mean loss goes to losses[s] (device float32
 * [num_steps], or NULL).  Step for step the same computation as
 * xpbd_mlp_train_step on those rows with that rate.  XPBD_E_ARG for null or
 * misplaced tables, batch < 1, num_rows < batch, num_steps < 0, a start
 * outside [0, num_rows) or rates that are not finite and positive. */
xpbd_status xpbd_mlp_train_steps(xpbd_mlp *net, const uint16_t *features, const float *targets,
                                 const int32_t *rows, int64_t num_rows, const int64_t *starts,
                                 int32_t batch, int32_t num_steps, float first_rate,
                                 float last_rate, float *losses);

/* Normalisation of the network's inputs and outputs from a recording made
 * with the identity normalisation (in_shift 0, in_scale 1): over the n rows
 * (device bfloat16 features [n][32], float32 targets [n][4]) whose free flag
 * (feature 31) is set, the mean and the population standard deviation of
 * every feature and target column, computed on the device in double
 * precision in a fixed order.  Host outputs: in_shift [27] the feature
 * means, in_scale [27] 1 / std (1 where the std is 0), out_shift [3] the
 * target means, out_scale [3] max(std, 1e-12).  Runs on hip_stream (NULL:
 * the null stream) and synchronises it; allocates and frees a device
 * workspace of about 60 KB.  XPBD_E_ARG for null or host inputs or n < 1. */
xpbd_status xpbd_mlp_normalisation(const uint16_t *features, const float *targets, int64_t n,
                                   void *hip_stream, float *in_shift, float *in_scale,
                                   float *out_shift, float *out_scale);

void xpbd_mlp_destroy(xpbd_mlp *net);

/* Axis-neighbour table of a mesh (host): out [num_vertices][6], -1 for none. */
xpbd_status xpbd_axis_neighbours(const xpbd_mesh *mesh, int32_t *out);

typedef struct {
    int32_t apply_correction;  /* 1: add the network's correction to the predicted positions */
    int32_t min_iterations;    /* sweeps before the residual check, >= 0 */
    int32_t max_iterations;    /* sweeps when the residual is above the threshold, >= min */
    float threshold;           /* residual RMS threshold */
    int32_t record_substep;    /* -1: none; else the substep (of every step) whose features and
                                  training targets are written to the two buffers below */
    uint16_t *record_features; /* device bfloat16 [total particles][32] */
    float *record_targets;     /* device float32 [total particles][4]: (x - x_hat - out_shift) /
                                  out_scale after the sweeps (zero rows for pinned particles) */
    int32_t *iterations;       /* device int32 [num_steps][substeps][N] sweeps run, or NULL */
    float stall_ratio;         /* 0: off.  In (0, 1], with min_iterations >= 1: the residual
                                  is also evaluated before the last of the min_iterations
                                  sweeps, and the sweeps continue past the minimum only if
                                  that sweep lowered it to at most stall_ratio times that
                                  value (a stalled sweep marks a state the further sweeps
                                  cannot improve, as where the tool holds particles) */
    float *residuals;          /* device float32 [num_steps][substeps][N]: the residual RMS
                                  after each substep's last sweep (the check's value when no
                                  further sweep ran, else evaluated once more), or NULL */
} xpbd_learned_params;

/* Advance every environment by num_steps steps one substep at a time: the
 * prediction and the features (with net's normalisation), the network's correction
 * when apply_correction is set, then the sweeps of xpbd_learned_params.
 * tool_pos and tool_pos_bytes as in xpbd_step.  net may be NULL only without correction and
 * without recording (plain sweeps with the residual check).  Needs sphere
 * tools and the register variant with one environment per workgroup and one
 * size class (XPBD_E_CAPACITY otherwise).  XPBD_F_RESIDUAL and XPBD_F_LAMBDA apply to the last substep.
 * With apply_correction 0, min_iterations = max_iterations = the batch's
 * iterations and no recording, the result equals xpbd_step's bit for bit. */
xpbd_status xpbd_step_learned(xpbd_batch *batch, const xpbd_mlp *net, int32_t num_steps,
                              const float *tool_pos, size_t tool_pos_bytes,
                              const xpbd_learned_params *params);

/* Bytes of the device array that holds the allocation-free step's workspace
 * (80 MiB; one copy per device the library runs on, held until the process
 * ends). */
#define XPBD_NOALLOC_SCRATCH_BYTES (80u << 20)

/* xpbd_step_learned for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same steps and results, with the workspace (predicted
 * positions 12 B, feature rows 64 B with the correction, candidate bits 1 B
 * per particle, 4 B per mesh, each part 256-byte aligned) taken from a
 * fixed device array of XPBD_NOALLOC_SCRATCH_BYTES instead of buffers the
 * batch allocates; no hipMalloc, hipFree or other allocation.  tool_pos must
 * be device memory (tool_pos_bytes as in xpbd_step).  The batch's device must be current.
 * Errors: XPBD_E_CAPACITY when the workspace exceeds the array (about 1.09 M
 * particles with the correction), XPBD_E_ARG for host tool poses or another
 * device, and every error of xpbd_step_learned; no device work is done after
 * an error.  Every call on a device shares that device's array and finds the
 * last call's contents in it (each call writes what it reads first): calls
 * that overlap on one device race, so callers serialise them (one stream, or
 * events between streams). */
xpbd_status xpbd_step_learned_noalloc(xpbd_batch *batch, const xpbd_mlp *net, int32_t num_steps,
                                      const float *tool_pos, size_t tool_pos_bytes,
                                      const xpbd_learned_params *params);


#ifdef __cplusplus
}
#endif

#endif /* XPBD_LEARNED_H */
