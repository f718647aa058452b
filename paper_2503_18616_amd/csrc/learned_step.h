// The learned step's checks and launches, shared by the learned-step and the
// RL-step entry points (include/xpbd_learned.h, include/xpbd_rl.h).
#pragma once

#include "../../include/xpbd_learned.h"
#include "batch.h"

#include <vector>

namespace xpbd {

// Device buffers a learned step works in besides the batch's state.
struct LearnedWorkspace {
    float *xhat = nullptr;         // [3][total particles] predicted (then corrected) positions
    uint16_t *feat = nullptr;      // [total particles][32] features of the correction
    uint8_t *cand = nullptr;       // [total particles] contact-candidate bits
    int32_t *chunk0 = nullptr;     // [meshes] first 32-particle chunk with a free particle
    int32_t chunks = 0;            // chunks per environment the correction visits
    int32_t correct_workgroups = 0;
};

// The learned step's workspace (allocated on first use).
xpbd_status learned_workspace(xpbd_batch *b, const xpbd_learned_params *lp);
// The correction's chunk table of a batch: the first 32-particle chunk of every
// mesh that holds a free particle (the chunks before hold pinned particles
// only and are skipped), and the chunks per environment it visits.
void learned_chunks(const xpbd_batch *b, std::vector<int32_t> &chunk0, int32_t &chunks);
// Batch and parameter checks of a learned step (host only).
xpbd_status check_learned(const xpbd_batch *b, const xpbd_mlp *net,
                          const xpbd_learned_params *lp);
// num_steps learned steps with the tool poses in device memory
// ([num_steps][N][tools][3]); grasp is null or names the grasp state.
// ws: the workspace to use (null: the batch's own, allocated on first use).
xpbd_status run_learned(xpbd_batch *b, const xpbd_mlp *net, int32_t num_steps,
                        const float *tools_dev, const xpbd_learned_params *lp,
                        const GraspArgs *grasp, const LearnedWorkspace *ws = nullptr);

}  // namespace xpbd
