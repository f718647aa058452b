// Host runtime of the RL-style step: the C ABI declared in include/xpbd_rl.h
// (policy objects and the observe / act / simulate loop on a batch's stream).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/xpbd_rl.h"
#include "batch.h"
#include "learned_step.h"
#include "rl_device.h"
#include "runtime_util.h"
#include "xpbd_device.h"

using xpbd::fail;
using xpbd::g_error;
using xpbd::is_device_pointer;

static_assert(XPBD_RL_OBS == xpbd::kRlObs, "observation count");
static_assert(XPBD_RL_HIDDEN == xpbd::kRlHidden, "hidden width");
static_assert(XPBD_RL_ACTIONS == xpbd::kRlActions, "action count");
static_assert(XPBD_RL_TRACKED == xpbd::kRlTracked, "tracked particles");
static_assert(XPBD_RL_POLICY_PARAMS == xpbd::kRlHidden * xpbd::kRlObs + xpbd::kRlHidden +
                                           xpbd::kRlHidden * xpbd::kRlHidden + xpbd::kRlHidden +
                                           xpbd::kRlActions * xpbd::kRlHidden + xpbd::kRlActions,
              "policy parameter count");

struct xpbd_policy {
    int device = 0;
    xpbd::PolicyDev d{};
    void *block = nullptr;   // one allocation: fragments, then biases

    ~xpbd_policy()
    {
        if (block)
            (void)hipFree(block);
    }
};

namespace {

// float32 -> bfloat16, nearest, ties to even (finite values).
uint16_t to_bf16(float v)
{
    uint32_t u;
    std::memcpy(&u, &v, sizeof u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Cut W [rows][cols] (row-major, float32) into matrix-core fragments: tiles
// of 16 units x 32 inputs, fragment (tile, k block) as 64 lanes x 8 values
// (lane l: unit 16 tile + l % 16, k slots 8 (l / 16) .. + 7).  permuted: slot
// 8 g + i of a block reads input 4 g + i (i < 4) or 16 + 4 g + i - 4.
void cut(const float *w, int rows, int cols, bool permuted, uint16_t *out)
{
    const int tiles = (rows + 15) / 16, blocks = cols / 32;
    for (int t = 0; t < tiles; ++t)
        for (int kb = 0; kb < blocks; ++kb)
            for (int lane = 0; lane < 64; ++lane)
                for (int i = 0; i < 8; ++i) {
                    const int row = 16 * t + lane % 16, g = lane / 16;
                    const int slot = permuted ? (i < 4 ? 4 * g + i : 16 + 4 * g + i - 4) : 8 * g + i;
                    const size_t at = (((size_t)t * blocks + kb) * 64 + lane) * 8 + i;
                    out[at] = row < rows ? to_bf16(w[(size_t)row * cols + 32 * kb + slot]) : 0;
                }
}

// Checks shared by the RL entry points (host only).
xpbd_status check_rl(const xpbd_batch *b, const xpbd_policy *policy, const xpbd_rl_params *params,
                     int32_t num_steps, const float *tool_pos, const int32_t *grasped,
                     const float *target, const float *obs, const float *actions)
{
    if (!b || !policy || !params)
        return fail(XPBD_E_ARG, "batch, policy and params must not be NULL");
    if (num_steps < 0)
        return fail(XPBD_E_ARG, "num_steps must be >= 0 (got %d)", num_steps);
    if (b->params.num_tools != 2 || b->params.tool_shape != XPBD_TOOL_SPHERE)
        return fail(XPBD_E_ARG, "the RL step needs a batch with two sphere tools");
    if (!b->register_variant)
        return fail(XPBD_E_ARG, "the RL step needs the register-multiplier solver variant");
    if (!tool_pos || !grasped || !target)
        return fail(XPBD_E_ARG, "tool_pos, grasped and target must not be NULL");
    const void *device_ptrs[5] = {tool_pos, grasped, target, obs, actions};
    for (const void *q : device_ptrs)
        if (q && !is_device_pointer(q))
            return fail(XPBD_E_ARG, "tool_pos, grasped, target, obs and actions must be device memory");
    const xpbd_rl_params &P = *params;
    if (!(std::isfinite(P.grasp_radius) && P.grasp_radius > 0.0f))
        return fail(XPBD_E_ARG, "grasp_radius must be finite and > 0");
    if (!(std::isfinite(P.max_speed) && P.max_speed >= 0.0f) || !std::isfinite(P.obs_scale))
        return fail(XPBD_E_ARG, "max_speed must be finite and >= 0, obs_scale finite");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(P.grasp_offset[k]) || !std::isfinite(P.obs_origin[k]) ||
            !std::isfinite(P.box_lo[k]) || !std::isfinite(P.box_hi[k]) ||
            !(P.box_lo[k] <= P.box_hi[k]))
            return fail(XPBD_E_ARG, "offsets, origin and box must be finite with box_lo <= box_hi");
    for (int j = 0; j < XPBD_RL_TRACKED; ++j)
        for (const auto &m : b->meshes)
            if (P.tracked[j] < 0 || P.tracked[j] >= m.num_vertices)
                return fail(XPBD_E_ARG, "tracked[%d] = %d is outside a mesh of %d particles", j,
                            P.tracked[j], m.num_vertices);
    return XPBD_OK;
}

xpbd::RlArgs rl_args(const xpbd_batch *b, const xpbd_rl_params &P, float *tool_pos,
                     int32_t *grasped, const float *target)
{
    xpbd::RlArgs r;
    std::memset(&r, 0, sizeof r);
    r.meshes = b->meshes_dev;
    r.envs = b->envs_dev;
    r.pos = b->pos;
    r.total_particles = b->total_particles;
    r.num_envs = b->num_envs;
    r.tool_pos = tool_pos;
    r.grasp = grasped;
    r.target = target;
    for (int j = 0; j < XPBD_RL_TRACKED; ++j)
        r.tracked[j] = P.tracked[j];
    r.obs_scale = P.obs_scale;
    r.max_speed = P.max_speed;
    r.dt = b->params.dt;
    for (int k = 0; k < 3; ++k) {
        r.obs_origin[k] = P.obs_origin[k];
        r.box_lo[k] = P.box_lo[k];
        r.box_hi[k] = P.box_hi[k];
    }
    return r;
}

xpbd::GraspArgs grasp_args(const xpbd_rl_params &P, int32_t *grasped)
{
    xpbd::GraspArgs g;
    g.state = grasped;
    g.radius = P.grasp_radius;
    for (int k = 0; k < 3; ++k)
        g.offset[k] = P.grasp_offset[k];
    return g;
}

}  // namespace

extern "C" {

xpbd_status xpbd_policy_create(const float *params, int64_t num_params, void *hip_stream,
                               xpbd_policy **out)
{
    g_error.clear();
    if (!params || !out)
        return fail(XPBD_E_ARG, "params and out must not be NULL");
    *out = nullptr;
    if (num_params != XPBD_RL_POLICY_PARAMS)
        return fail(XPBD_E_ARG, "a policy has %d parameters (got %lld)", XPBD_RL_POLICY_PARAMS,
                    (long long)num_params);
    for (int64_t i = 0; i < num_params; ++i)
        if (!std::isfinite(params[i]))
            return fail(XPBD_E_ARG, "policy parameter %lld is not finite", (long long)i);
    constexpr int H = xpbd::kRlHidden, F = xpbd::kRlObs, A = xpbd::kRlActions;
    const float *w1 = params, *b1 = w1 + H * F, *w2 = b1 + H, *b2 = w2 + H * H, *w3 = b2 + H,
                *b3 = w3 + A * H;
    constexpr size_t n1 = 16 * 2 * 64 * 8, n2 = 16 * 8 * 64 * 8, n3 = 1 * 8 * 64 * 8;
    std::vector<uint16_t> frag(n1 + n2 + n3);
    cut(w1, H, F, false, frag.data());
    cut(w2, H, H, true, frag.data() + n1);
    cut(w3, A, H, true, frag.data() + n1 + n2);
    std::vector<float> bias(2 * H + 16, 0.0f);
    std::memcpy(bias.data(), b1, sizeof(float) * H);
    std::memcpy(bias.data() + H, b2, sizeof(float) * H);
    std::memcpy(bias.data() + 2 * H, b3, sizeof(float) * A);

    xpbd_policy *p = new xpbd_policy();
    hipError_t e = hipGetDevice(&p->device);
    const size_t frag_bytes = frag.size() * sizeof(uint16_t);
    const size_t bytes = frag_bytes + bias.size() * sizeof(float);
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (e == hipSuccess)
        e = hipMalloc(&p->block, bytes);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->block, frag.data(), frag_bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(static_cast<char *>(p->block) + frag_bytes, bias.data(),
                           bias.size() * sizeof(float), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        delete p;
        return fail(XPBD_E_HIP, "uploading the policy failed: %s", hipGetErrorString(e));
    }
    const uint16_t *f = static_cast<const uint16_t *>(p->block);
    const float *bd = reinterpret_cast<const float *>(static_cast<const char *>(p->block) + frag_bytes);
    p->d.w1 = f;
    p->d.w2 = f + n1;
    p->d.w3 = f + n1 + n2;
    p->d.b1 = bd;
    p->d.b2 = bd + H;
    p->d.b3 = bd + 2 * H;
    *out = p;
    return XPBD_OK;
}

void xpbd_policy_destroy(xpbd_policy *p) { delete p; }

xpbd_status xpbd_rl_step(xpbd_batch *b, const xpbd_policy *policy, const xpbd_rl_params *params,
                         int32_t num_steps, float *tool_pos, int32_t *grasped,
                         const float *target, float *obs, float *actions)
{
    g_error.clear();
    xpbd_status st = check_rl(b, policy, params, num_steps, tool_pos, grasped, target, obs, actions);
    if (st != XPBD_OK || num_steps == 0)
        return st;
    xpbd::RlArgs r = rl_args(b, *params, tool_pos, grasped, target);
    const xpbd::GraspArgs grasp = grasp_args(*params, grasped);
    const size_t N = (size_t)b->num_envs;
    for (int32_t step = 0; step < num_steps; ++step) {
        r.obs = obs ? obs + (size_t)step * N * XPBD_RL_OBS : nullptr;
        r.actions = actions ? actions + (size_t)step * N * XPBD_RL_ACTIONS : nullptr;
        HIP_TRY(xpbd::launch_rl_policy(r, policy->d, b->stream));
        st = xpbd::run_step(b, 1, tool_pos, &grasp);
        if (st != XPBD_OK)
            return st;
    }
    return XPBD_OK;
}

xpbd_status xpbd_rl_step_learned(xpbd_batch *b, const xpbd_policy *policy,
                                 const xpbd_rl_params *params, const xpbd_mlp *net,
                                 const xpbd_learned_params *learned, int32_t num_steps,
                                 float *tool_pos, int32_t *grasped, const float *target,
                                 float *obs, float *actions)
{
    g_error.clear();
    if (!learned)
        return fail(XPBD_E_ARG, "learned params must not be NULL");
    xpbd_status st = check_rl(b, policy, params, num_steps, tool_pos, grasped, target, obs, actions);
    if (st != XPBD_OK)
        return st;
    if ((st = xpbd::check_learned(b, net, learned)) != XPBD_OK || num_steps == 0)
        return st;
    xpbd::RlArgs r = rl_args(b, *params, tool_pos, grasped, target);
    const xpbd::GraspArgs grasp = grasp_args(*params, grasped);
    const size_t N = (size_t)b->num_envs;
    xpbd_learned_params lp = *learned;
    for (int32_t step = 0; step < num_steps; ++step) {
        r.obs = obs ? obs + (size_t)step * N * XPBD_RL_OBS : nullptr;
        r.actions = actions ? actions + (size_t)step * N * XPBD_RL_ACTIONS : nullptr;
        lp.iterations = learned->iterations
                            ? learned->iterations + (size_t)step * b->params.substeps * N
                            : nullptr;
        lp.residuals = learned->residuals
                           ? learned->residuals + (size_t)step * b->params.substeps * N
                           : nullptr;
        HIP_TRY(xpbd::launch_rl_policy(r, policy->d, b->stream));
        st = xpbd::run_learned(b, net, 1, tool_pos, &lp, &grasp);
        if (st != XPBD_OK)
            return st;
    }
    return XPBD_OK;
}

}  // extern "C"
