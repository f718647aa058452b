/*
 * RL-style step of the batched XPBD simulation: C ABI.
 *
 * FF-SRL couples its simulator to a reinforcement-learning library through a
 * thin layer that, once per simulation step, extracts every environment's
 * observations, applies the agent's actions and steps the simulation, all on
 * the GPU (Dall'Alba et al., arXiv 2503.18616, Sec. III-B).  Its grasper
 * holds tissue through a dragging constraint (Sec. III-A.2).  This library
 * runs that loop for a batch with two sphere tools, tool 0 the grasper and
 * tool 1 a probe, with the agent's policy network evaluated in the same
 * stream; training the policy and computing rewards are the RL library's
 * business and are not part of this interface.
 *
 * One step of every environment, in this order:
 *  1. Observation o (64 float32 values) of the start-of-step state; points
 *     are taken relative to obs_origin and all lengths are metres times
 *     obs_scale:
 *       o[0:3] tool 0 centre, o[3:6] tool 1 centre, o[6:9] target point,
 *       o[9] 1 while the grasper holds a particle, else 0,
 *       o[10 + 3j : 13 + 3j] x_p - X_p of particle p = tracked[j], j = 0..17
 *       (displacement from its rest position).
 *  2. Policy (64 -> 256 -> 256 -> 7, weights [out][in] held as bfloat16,
 *     float32 biases, float32 accumulation on the matrix cores):
 *       a1 = bf16(relu(W1 bf16(o) + b1)), a2 = bf16(relu(W2 a1 + b2)),
 *       a = W3 a2 + b3; bf16() rounds to nearest, ties to even.
 *  3. Tool motion: tool t moves by clamp(a[3t .. 3t+2], -1, 1) * max_speed
 *     * dt (dt of the batch's xpbd_params) and its centre is then clamped
 *     into [box_lo, box_hi].
 *  4. Grasp (Sec. III-A.2 with a sphere for the closed clamps): a[6] > 0
 *     closes the grasper.  Closed while holding nothing: the free particle
 *     closest to the dragging point (tool 0 centre + grasp_offset) strictly
 *     within grasp_radius (r_l) on the start-of-step positions is taken,
 *     ties to the lowest particle id; open: the held particle is released;
 *     closed while holding: the particle stays held.
 *  5. The simulation step of xpbd_step with both spheres at their moved
 *     centres; the held particle is moved onto the dragging point after the
 *     tool contacts of every iteration (a distance constraint of rest length
 *     0 with k_s = 1 to a kinematic point).
 *
 * Pointers named "device" must be device memory.  Errors: negative
 * xpbd_status values with xpbd_last_error() set; no device work is done
 * after an argument error.  Calls are asynchronous on the batch's stream.
 */
#ifndef XPBD_RL_H
#define XPBD_RL_H

#include <stdint.h>

#include "xpbd.h"
#include "xpbd_learned.h"

#ifdef __cplusplus
extern "C" {
#endif

#define XPBD_RL_OBS 64
#define XPBD_RL_HIDDEN 256
#define XPBD_RL_ACTIONS 7
#define XPBD_RL_TRACKED 18
/* W1 [256][64], b1 [256], W2 [256][256], b2 [256], W3 [7][256], b3 [7] */
#define XPBD_RL_POLICY_PARAMS 84231

typedef struct xpbd_policy xpbd_policy;

typedef struct {
    float grasp_radius;               /* r_l (m), > 0 */
    float grasp_offset[3];            /* dragging point relative to the tool 0 centre (m) */
    float max_speed;                  /* m/s per axis at |action| >= 1, >= 0 */
    float obs_scale;                  /* observation lengths are metres times this */
    float obs_origin[3];              /* observed points are relative to this point (m) */
    float box_lo[3], box_hi[3];       /* workspace of the tool centres, box_lo <= box_hi */
    int32_t tracked[XPBD_RL_TRACKED]; /* observed particles, ids within each environment
                                         (every environment's mesh must have them) */
} xpbd_rl_params;

/*
 * Upload a policy: params (host, float32 [XPBD_RL_POLICY_PARAMS] in the order
 * above) are rounded to bfloat16 (weights) and laid out for the matrix cores
 * on the device of the current HIP context, on hip_stream (NULL: the null
 * stream); the call returns after the upload.  *out receives the handle.
 * XPBD_E_ARG: a null pointer, a wrong count or a non-finite parameter.
 */
xpbd_status xpbd_policy_create(const float *params, int64_t num_params, void *hip_stream,
                               xpbd_policy **out);
void xpbd_policy_destroy(xpbd_policy *p);

/*
 * Run num_steps RL steps (see above) on the batch's stream.  The batch needs
 * num_tools == 2, sphere tools and the register-multiplier solver (variant
 * XPBD_VARIANT_REGISTERS, or AUTO resolving to it).
 *   tool_pos  device float [N][2][3], read and overwritten with the centres
 *             the last step ran with
 *   grasped   device int32 [N], read and overwritten: the particle each
 *             environment's grasper holds (id within the environment), -1 for
 *             none; any negative id, and an id that is not a free particle
 *             of the environment's mesh, reads as none
 *   target    device float [N][3] target points (observed only)
 *   obs       device float [num_steps][N][64] observations of every step, or NULL
 *   actions   device float [num_steps][N][7] policy outputs of every step, or NULL
 * The contact-candidate fields of xpbd_read_state describe the last step.
 * num_steps == 0 does nothing.  XPBD_E_ARG: null pointers (obs and actions
 * aside), invalid parameters, a tracked id outside some environment's mesh,
 * or a batch that does not meet the needs above.
 */
xpbd_status xpbd_rl_step(xpbd_batch *b, const xpbd_policy *policy, const xpbd_rl_params *params,
                         int32_t num_steps, float *tool_pos, int32_t *grasped,
                         const float *target, float *obs, float *actions);

/*
 * xpbd_rl_step with the learned warm start (include/xpbd_learned.h): the
 * simulation step of every RL step is one step of xpbd_step_learned with the
 * network net and the settings *learned (correction, minimum sweeps, residual
 * threshold, stall ratio, fallback sweeps), the grasper included.
 * learned->iterations (device int32, or NULL) receives
 * [num_steps][substeps][N] sweep counts; a recording (record_substep >= 0)
 * holds the last RL step's.  Needs, besides xpbd_rl_step's, what
 * xpbd_step_learned needs (one environment per workgroup, one size class).
 */
xpbd_status xpbd_rl_step_learned(xpbd_batch *b, const xpbd_policy *policy,
                                 const xpbd_rl_params *params, const xpbd_mlp *net,
                                 const xpbd_learned_params *learned, int32_t num_steps,
                                 float *tool_pos, int32_t *grasped, const float *target,
                                 float *obs, float *actions);

#ifdef __cplusplus
}
#endif

#endif /* XPBD_RL_H */
