// The learned step's checks and launches, shared by the learned-step and the
// RL-step entry points (include/xpbd_learned.h, include/xpbd_rl.h).
#pragma once

#include "../../include/xpbd_learned.h"
#include "batch.h"

namespace xpbd {

// The learned step's workspace (allocated on first use).
xpbd_status learned_workspace(xpbd_batch *b, const xpbd_learned_params *lp);
// Batch and parameter checks of a learned step (host only).
xpbd_status check_learned(const xpbd_batch *b, const xpbd_mlp *net,
                          const xpbd_learned_params *lp);
// num_steps learned steps with the tool poses in device memory
// ([num_steps][N][tools][3]); grasp is null or names the grasp state.
xpbd_status run_learned(xpbd_batch *b, const xpbd_mlp *net, int32_t num_steps,
                        const float *tools_dev, const xpbd_learned_params *lp,
                        const GraspArgs *grasp);

}  // namespace xpbd
