/*
 * Captured steps of the batched XPBD simulation: C ABI.
 *
 * A step of the learned warm start is three launches per substep, an RL step
 * adds the policy's; these entry points record one step of a batch, with
 * fixed buffers, into a HIP graph once, and replay it on the batch's stream.
 * Every replay is exactly the step the corresponding call would run (same
 * kernels, same arguments; the buffers are read and written in place, so
 * a caller updates, for instance, the tool poses between replays).
 *
 * Capture records and runs nothing; it happens on a stream of its own, so
 * the batch's stream may be the null stream.  The settings in effect at
 * capture (the batch's flags, the learned and RL parameters) hold for every
 * replay.  A graph belongs to its batch: destroy it before the batch, the
 * policy and the network it names.  Errors: negative xpbd_status values with
 * xpbd_last_error() set.  A batch of several size classes (uneven meshes:
 * one launch per class on streams of its own) is captured with its fork and
 * join, so the classes run as parallel branches of the graph; the learned
 * step itself needs one size class.
 */
#ifndef XPBD_GRAPH_H
#define XPBD_GRAPH_H

#include <stdint.h>

#include "xpbd.h"
#include "xpbd_learned.h"
#include "xpbd_rl.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xpbd_graph xpbd_graph;

/*
 * One step of xpbd_step (learned == NULL) or of xpbd_step_learned (net and
 * *learned as for that call) with the tool poses read from tool_pos (device
 * float [N][num_tools][3] or [6] for capsules, at every replay;
 * tool_pos_bytes its size, one step's poses as in xpbd_step).
 * XPBD_E_ARG: null pointers, tool_pos not in device memory or of another
 * size, or what the step itself rejects.
 */
xpbd_status xpbd_step_graph_create(xpbd_batch *b, const xpbd_mlp *net,
                                   const xpbd_learned_params *learned, const float *tool_pos,
                                   size_t tool_pos_bytes, xpbd_graph **out);

/*
 * One RL step (include/xpbd_rl.h): xpbd_rl_step when learned is NULL, else
 * xpbd_rl_step_learned, with the given buffers.
 */
xpbd_status xpbd_rl_graph_create(xpbd_batch *b, const xpbd_policy *policy,
                                 const xpbd_rl_params *params, const xpbd_mlp *net,
                                 const xpbd_learned_params *learned, float *tool_pos,
                                 int32_t *grasped, const float *target, float *obs,
                                 float *actions, xpbd_graph **out);

/* Replay the captured step `times` times (>= 0) on the batch's stream. */
xpbd_status xpbd_graph_launch(xpbd_graph *g, int32_t times);

void xpbd_graph_destroy(xpbd_graph *g);

#ifdef __cplusplus
}
#endif

#endif /* XPBD_GRAPH_H */
