// Device-side data of the RL-style step (include/xpbd_rl.h), shared by the
// runtime and the policy kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "xpbd_device.h"

namespace xpbd {

constexpr int kRlObs = 64;
constexpr int kRlHidden = 256;
constexpr int kRlActions = 7;
constexpr int kRlTracked = 18;
constexpr int kRlEnvsPerWave = 16;   // one column block of the matrix-core tiles

// The policy as the matrix cores read it: every weight matrix cut into
// 16 x 32 (output unit x input) fragments, fragment (tile, k block) stored as
// 64 lanes x 8 bfloat16 (lane l: unit 16 tile + l % 16, inputs
// 32 kb + 8 (l / 16) .. + 7), so that a wave loads one fragment with one
// 16-byte load per lane.  W2 and W3 take their inputs in the permuted order
// of the previous layer's result fragments: slot 8 g + i of a 32-input block
// is input 4 g + i for i < 4 and 16 + 4 g + (i - 4) for i >= 4.
struct PolicyDev {
    const uint16_t *w1;   // [16 tiles][2 k blocks][64][8]
    const uint16_t *w2;   // [16][8][64][8]
    const uint16_t *w3;   // [1][8][64][8], units 7..15 zero
    const float *b1;      // [256]
    const float *b2;      // [256]
    const float *b3;      // [16], entries 7..15 zero
};

struct RlArgs {
    const MeshDev *meshes;
    const EnvDev *envs;
    const float *pos;            // [3][total particles]
    int32_t total_particles;
    int32_t num_envs;
    float *tool_pos;             // [N][2][3], read and overwritten
    int32_t *grasp;              // [N]: held id, -1 none; written -2 for a closed, empty grasper
    const float *target;         // [N][3]
    float *obs;                  // [N][64] or null
    float *actions;              // [N][7] or null
    int32_t tracked[kRlTracked];
    float obs_scale;
    float obs_origin[3];
    float max_speed;
    float dt;
    float box_lo[3];
    float box_hi[3];
};

hipError_t launch_rl_policy(const RlArgs &args, const PolicyDev &policy, hipStream_t stream);

}  // namespace xpbd
