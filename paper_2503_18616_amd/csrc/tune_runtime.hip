// Autotuner of the batch's launch configuration (include/xpbd.h,
// xpbd_autotune): each candidate is a real batch of the caller's meshes and
// environments, stepped once untimed and then timed with HIP events on the
// caller's stream; the fastest candidate's configuration is returned.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/xpbd.h"
#include "batch.h"
#include "runtime_util.h"

namespace {

struct Candidate {
    int32_t variant, block, group, packing;
};

std::vector<Candidate> candidates()
{
    std::vector<Candidate> out;
    out.push_back({XPBD_VARIANT_AUTO, 0, 0, XPBD_PACKING_AUTO});   // the library's own choice
    for (int32_t block : {0, 256, 512, 1024})
        for (int32_t group : {1, 2})
            for (int32_t packing : {XPBD_PACKING_AUTO, XPBD_PACKING_BANKS16})
                out.push_back({XPBD_VARIANT_REGISTERS, block, group, packing});
    for (int32_t block : {0, 256, 512, 1024})
        out.push_back({XPBD_VARIANT_LDS, block, 1, XPBD_PACKING_AUTO});
    return out;
}

}  // namespace

extern "C" {

xpbd_status xpbd_autotune(const xpbd_mesh *meshes, int32_t num_meshes, const int32_t *env_mesh,
                          int32_t num_envs, const float *compliance, xpbd_params *params,
                          void *hip_stream, int32_t num_steps, const float *tool_pos,
                          size_t tool_pos_bytes, float *ms_per_step)
{
    using xpbd::fail;
    xpbd::g_error.clear();
    if (!params || !ms_per_step)
        return fail(XPBD_E_ARG, "params and ms_per_step are required");
    if (num_steps < 1)
        return fail(XPBD_E_ARG, "num_steps must be >= 1 (got %d)", num_steps);
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    HIP_TRY(hipEventCreate(&t0));
    hipError_t ev = hipEventCreate(&t1);
    if (ev != hipSuccess) {
        (void)hipEventDestroy(t0);
        return fail(XPBD_E_HIP, "hipEventCreate failed: %s", hipGetErrorString(ev));
    }
    float best = -1.0f, default_ms = -1.0f;
    Candidate chosen{};
    xpbd_status status = XPBD_OK;
    for (const Candidate &c : candidates()) {
        xpbd_params p = *params;
        p.solver_variant = c.variant;
        p.block_size = c.block;
        p.envs_per_group = c.group;
        p.colour_packing = c.packing;
        p.flags = 0;
        xpbd_batch *b = nullptr;
        xpbd_status st = xpbd_create_batch(meshes, num_meshes, env_mesh, num_envs, compliance, &p,
                                           hip_stream, &b);
        if (st == XPBD_E_CAPACITY)
            continue;   // this configuration cannot hold the meshes
        if (st != XPBD_OK) {
            status = st;
            break;
        }
        float ms = 0.0f;
        // one untimed step on the first step's poses, then the timed steps
        st = xpbd_step(b, 1, tool_pos, tool_pos_bytes / (size_t)num_steps);
        hipError_t e = hipSuccess;
        if (st == XPBD_OK && (e = hipEventRecord(t0, stream)) == hipSuccess) {
            st = xpbd_step(b, num_steps, tool_pos, tool_pos_bytes);
            if (st == XPBD_OK && (e = hipEventRecord(t1, stream)) == hipSuccess &&
                (e = hipEventSynchronize(t1)) == hipSuccess)
                e = hipEventElapsedTime(&ms, t0, t1);
        }
        xpbd_destroy_batch(b);
        if (st == XPBD_OK && e != hipSuccess)
            st = fail(XPBD_E_HIP, "timing a candidate failed: %s", hipGetErrorString(e));
        if (st != XPBD_OK) {
            status = st;
            break;
        }
        ms /= (float)num_steps;
        if (default_ms < 0.0f)
            default_ms = ms;
        if (best < 0.0f || ms < best) {
            best = ms;
            chosen = c;
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (status != XPBD_OK)
        return status;
    if (best < 0.0f)
        return fail(XPBD_E_CAPACITY, "no launch configuration holds these meshes");
    params->solver_variant = chosen.variant;
    params->block_size = chosen.block;
    params->envs_per_group = chosen.group;
    params->colour_packing = chosen.packing;
    ms_per_step[0] = best;
    ms_per_step[1] = default_ms;
    xpbd::g_error.clear();
    return XPBD_OK;
}

xpbd_status xpbd_get_batch_info(const xpbd_batch *b, xpbd_batch_info *out)
{
    using xpbd::fail;
    xpbd::g_error.clear();
    if (!b || !out)
        return fail(XPBD_E_ARG, "batch and out must not be NULL");
    std::memset(out, 0, sizeof *out);
    out->solver_variant = b->register_variant ? XPBD_VARIANT_REGISTERS
                          : b->params.solver_variant == XPBD_VARIANT_JACOBI ? XPBD_VARIANT_JACOBI
                                                                           : XPBD_VARIANT_LDS;
    out->envs_per_group = b->envs_per_group;
    int block = b->block, banks = b->lambda_banks, groups = b->num_envs, group = 1;
    bool barriers = true;
    uint32_t lds = b->lds_bytes;
    if (b->register_variant) {
        out->size_classes = (int32_t)b->classes.size();
        int32_t most = -1;
        for (const RegClass &c : b->classes)
            if (c.num_groups > most) {
                most = c.num_groups;
                block = c.block;
                banks = c.lambda_banks;
                lds = c.lds_bytes;
                groups = c.num_groups;
                barriers = c.round_barriers;
                group = c.group;
            }
    } else {
        out->size_classes = 1;
        banks = 0;
    }
    int lds_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                  b->device));
    const int waves = (block + 63) / 64;
    int per_cu = 16 / (waves > 0 ? waves : 1);
    if (lds > 0 && lds_cu > 0)
        per_cu = std::min(per_cu, (int)((uint32_t)lds_cu / lds));
    if (b->register_variant) {
        // the kernel's own registers may allow fewer (capsule tools)
        xpbd::StepArgs a{};
        a.tool_shape = b->params.tool_shape;
        a.round_barriers = barriers ? 1 : 0;
        HIP_TRY(xpbd::step_reg_occupancy(a, block, banks, group, lds, &per_cu));
    }
    out->block_size = block;
    out->lambda_banks = banks;
    out->lds_bytes = (int32_t)lds;
    out->workgroups = groups;
    out->workgroups_per_cu = std::max(per_cu, 1);
    out->waves_per_cu = out->workgroups_per_cu * waves;
    return XPBD_OK;
}

}  // extern "C"
