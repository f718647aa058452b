// Host runtime of the learned warm start: the C ABI declared in
// include/xpbd_learned.h (network objects, training steps, and the
// one-substep-per-launch stepping of a batch with the network's correction).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/xpbd_learned.h"
#include "batch.h"
#include "learned_step.h"
#include "mesh_setup.h"
#include "mlp_device.h"
#include "runtime_util.h"
#include "xpbd_device.h"

using xpbd::fail;
using xpbd::g_error;
using xpbd::is_device_pointer;

static_assert(XPBD_MLP_PARAMS == xpbd::kMlpParams, "parameter count");
static_assert(XPBD_MLP_FEATURE_STRIDE == xpbd::kMlpFeatPad, "feature row width");

struct xpbd_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    xpbd::MlpDev d{};
    float *in_shift = nullptr;               // device [32]
    float *in_scale = nullptr;               // device [32]
    std::vector<xpbd::DeviceBuffer> allocations;
    float *partial = nullptr;                // [groups][params] training scratch
    float *stats = nullptr;                  // [groups][2]
    float *loss = nullptr;                   // [1]
    int partial_groups = 0;
    int adam_step = 0;

    ~xpbd_mlp()
    {
        (void)hipStreamSynchronize(stream);
        for (auto &a : allocations)
            (void)hipFree(a.ptr);
        if (partial)
            (void)hipFree(partial);
        if (stats)
            (void)hipFree(stats);
    }

    template <typename T>
    xpbd_status zeros(T **out, size_t count)
    {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, std::max<size_t>(count * sizeof(T), 16));
        if (e != hipSuccess)
            return fail(XPBD_E_HIP, "hipMalloc failed: %s", hipGetErrorString(e));
        allocations.push_back({p, count * sizeof(T)});
        HIP_TRY(hipMemset(p, 0, std::max<size_t>(count * sizeof(T), 16)));
        *out = static_cast<T *>(p);
        return XPBD_OK;
    }
};

namespace {

xpbd_status upload_params(xpbd_mlp *net, const float *params)
{
    std::vector<float> host(xpbd::kMlpParams, 0.0f);
    if (params)
        std::memcpy(host.data(), params, sizeof(float) * xpbd::kMlpParams);
    for (float v : host)
        if (!std::isfinite(v))
            return fail(XPBD_E_ARG, "network parameters must be finite");
    HIP_TRY(hipMemcpy(net->d.master, host.data(), sizeof(float) * xpbd::kMlpParams,
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(net->d.adam_m, 0, sizeof(float) * xpbd::kMlpParams));
    HIP_TRY(hipMemset(net->d.adam_v, 0, sizeof(float) * xpbd::kMlpParams));
    net->adam_step = 0;
    HIP_TRY(xpbd::launch_mlp_sync(net->d, net->stream));
    HIP_TRY(hipStreamSynchronize(net->stream));
    return XPBD_OK;
}

}  // namespace

extern "C" {

xpbd_status xpbd_mlp_create(const float *params, const float *in_shift, const float *in_scale,
                            const float *out_shift, const float *out_scale, void *hip_stream,
                            xpbd_mlp **out)
{
    g_error.clear();
    if (!out)
        return fail(XPBD_E_ARG, "out is NULL");
    *out = nullptr;
    if (!in_scale || !out_scale)
        return fail(XPBD_E_ARG, "in_scale and out_scale are required");
    for (int k = 0; k < XPBD_MLP_FEATURES; ++k)
        if (!std::isfinite(in_scale[k]) || (in_shift && !std::isfinite(in_shift[k])))
            return fail(XPBD_E_ARG, "in_shift[%d] / in_scale[%d] are not finite", k, k);
    for (int k = 0; k < XPBD_MLP_OUTPUTS; ++k)
        if (!(std::isfinite(out_scale[k]) && out_scale[k] > 0.0f) ||
            (out_shift && !std::isfinite(out_shift[k])))
            return fail(XPBD_E_ARG, "out_scale[%d] must be finite and > 0, out_shift finite", k);
    auto *net = new xpbd_mlp();
    net->stream = reinterpret_cast<hipStream_t>(hip_stream);
    auto cleanup = [&](xpbd_status st) {
        delete net;
        return st;
    };
    xpbd_status st;
    if (hipGetDevice(&net->device) != hipSuccess)
        return cleanup(fail(XPBD_E_HIP, "no HIP device"));
    xpbd::MlpDev &d = net->d;
    if ((st = net->zeros(&d.master, xpbd::kMlpParams)) || (st = net->zeros(&d.adam_m, xpbd::kMlpParams)) ||
        (st = net->zeros(&d.adam_v, xpbd::kMlpParams)) ||
        (st = net->zeros(&d.w1, (size_t)xpbd::kMlpHidden * xpbd::kMlpFeatPad)) ||
        (st = net->zeros(&d.w2, (size_t)xpbd::kMlpHidden * xpbd::kMlpHidden)) ||
        (st = net->zeros(&d.w2t, (size_t)xpbd::kMlpHidden * xpbd::kMlpHidden)) ||
        (st = net->zeros(&d.w3, (size_t)16 * xpbd::kMlpHidden)) ||
        (st = net->zeros(&d.w3t, (size_t)xpbd::kMlpHidden * 32)) ||
        (st = net->zeros(&d.b1, xpbd::kMlpHidden)) || (st = net->zeros(&d.b2, xpbd::kMlpHidden)) ||
        (st = net->zeros(&d.b3, 4)) || (st = net->zeros(&d.out_scale, 4)) ||
        (st = net->zeros(&d.out_shift, 4)) || (st = net->zeros(&net->in_shift, 32)) ||
        (st = net->zeros(&net->in_scale, 32)) || (st = net->zeros(&net->loss, 1)))
        return cleanup(st);
    float in_sh[32] = {0.0f}, in_sc[32] = {0.0f}, out_sh[4] = {0.0f}, out_sc[4] = {0.0f};
    std::memcpy(in_sc, in_scale, sizeof(float) * XPBD_MLP_FEATURES);
    std::memcpy(out_sc, out_scale, sizeof(float) * XPBD_MLP_OUTPUTS);
    if (in_shift)
        std::memcpy(in_sh, in_shift, sizeof(float) * XPBD_MLP_FEATURES);
    if (out_shift)
        std::memcpy(out_sh, out_shift, sizeof(float) * XPBD_MLP_OUTPUTS);
    if (hipMemcpy(net->in_scale, in_sc, sizeof in_sc, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net->in_shift, in_sh, sizeof in_sh, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d.out_scale, out_sc, sizeof out_sc, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d.out_shift, out_sh, sizeof out_sh, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(XPBD_E_HIP, "upload of the normalisation failed"));
    if ((st = upload_params(net, params)))
        return cleanup(st);
    *out = net;
    return XPBD_OK;
}

xpbd_status xpbd_mlp_get_params(xpbd_mlp *net, float *params)
{
    g_error.clear();
    if (!net || !params)
        return fail(XPBD_E_ARG, "net and params are required");
    HIP_TRY(hipStreamSynchronize(net->stream));
    HIP_TRY(hipMemcpy(params, net->d.master, sizeof(float) * xpbd::kMlpParams,
                      hipMemcpyDeviceToHost));
    return XPBD_OK;
}

xpbd_status xpbd_mlp_set_params(xpbd_mlp *net, const float *params)
{
    g_error.clear();
    if (!net || !params)
        return fail(XPBD_E_ARG, "net and params are required");
    HIP_TRY(hipStreamSynchronize(net->stream));
    return upload_params(net, params);
}

xpbd_status xpbd_mlp_forward(xpbd_mlp *net, const uint16_t *features, int32_t n, float *y)
{
    g_error.clear();
    if (!net || !features || !y || n < 1)
        return fail(XPBD_E_ARG, "net, features, y and n >= 1 are required");
    if (!is_device_pointer(features) || !is_device_pointer(y))
        return fail(XPBD_E_ARG, "features and y must be device memory");
    HIP_TRY(xpbd::launch_mlp_forward(net->d, features, n, y, nullptr, 0, net->stream));
    return XPBD_OK;
}

xpbd_status xpbd_mlp_train_step(xpbd_mlp *net, const uint16_t *features, const float *targets,
                                const int32_t *rows, int32_t n, float learning_rate, float *loss,
                                float *grad)
{
    g_error.clear();
    if (!net || !features || !targets || n < 1)
        return fail(XPBD_E_ARG, "net, features, targets and n >= 1 are required");
    if (!(std::isfinite(learning_rate) && learning_rate >= 0.0f))
        return fail(XPBD_E_ARG, "learning_rate must be finite and >= 0");
    if (!is_device_pointer(features) || !is_device_pointer(targets) ||
        (grad && !is_device_pointer(grad)) || (rows && !is_device_pointer(rows)))
        return fail(XPBD_E_ARG, "features, targets, rows and grad must be device memory");
    const bool loss_on_device = loss && is_device_pointer(loss);
    const int groups = (n + xpbd::kMlpTile - 1) / xpbd::kMlpTile;
    if (groups > net->partial_groups) {
        HIP_TRY(hipStreamSynchronize(net->stream));
        if (net->partial)
            HIP_TRY(hipFree(net->partial));
        if (net->stats)
            HIP_TRY(hipFree(net->stats));
        net->partial = nullptr;
        net->stats = nullptr;
        net->partial_groups = 0;
        HIP_TRY(hipMalloc(&net->partial, sizeof(float) * (size_t)groups * xpbd::kMlpParams));
        HIP_TRY(hipMalloc(&net->stats, sizeof(float) * 2 * (size_t)groups));
        net->partial_groups = groups;
    }
    int step = net->adam_step;
    if (learning_rate > 0.0f)
        step = ++net->adam_step;
    HIP_TRY(xpbd::launch_mlp_train(net->d, features, targets, rows, 0, n, n, net->partial,
                                   net->stats,
                                   learning_rate, 0.9f, 0.999f, 1e-8f, step, grad,
                                   loss_on_device ? loss : net->loss, net->stream));
    if (loss && !loss_on_device) {
        HIP_TRY(hipMemcpyAsync(loss, net->loss, sizeof(float), hipMemcpyDeviceToHost, net->stream));
        HIP_TRY(hipStreamSynchronize(net->stream));
    }
    return XPBD_OK;
}

xpbd_status xpbd_mlp_train_steps(xpbd_mlp *net, const uint16_t *features, const float *targets,
                                 const int32_t *rows, int64_t num_rows, const int64_t *starts,
                                 int32_t batch, int32_t num_steps, float first_rate,
                                 float last_rate, float *losses)
{
    g_error.clear();
    if (!net || !features || !targets || !rows || batch < 1 || num_steps < 0 ||
        num_rows < batch)
        return fail(XPBD_E_ARG, "net, features, targets, rows, batch >= 1, num_rows >= batch and "
                    "num_steps >= 0 are required");
    if (!(std::isfinite(first_rate) && first_rate > 0.0f && std::isfinite(last_rate) &&
          last_rate > 0.0f))
        return fail(XPBD_E_ARG, "the learning rates must be finite and > 0");
    if (!is_device_pointer(features) || !is_device_pointer(targets) || !is_device_pointer(rows) ||
        (losses && !is_device_pointer(losses)))
        return fail(XPBD_E_ARG, "features, targets, rows and losses must be device memory");
    if (starts && is_device_pointer(starts))
        return fail(XPBD_E_ARG, "starts must be host memory");
    for (int32_t s = 0; starts && s < num_steps; ++s)
        if (starts[s] < 0 || starts[s] >= num_rows)
            return fail(XPBD_E_ARG, "starts[%d] = %lld is outside [0, num_rows)", s,
                        (long long)starts[s]);
    if (num_steps == 0)
        return XPBD_OK;
    const int groups = (batch + xpbd::kMlpTile - 1) / xpbd::kMlpTile;
    if (groups > net->partial_groups) {
        HIP_TRY(hipStreamSynchronize(net->stream));
        if (net->partial)
            HIP_TRY(hipFree(net->partial));
        if (net->stats)
            HIP_TRY(hipFree(net->stats));
        net->partial = nullptr;
        net->stats = nullptr;
        net->partial_groups = 0;
        HIP_TRY(hipMalloc(&net->partial, sizeof(float) * (size_t)groups * xpbd::kMlpParams));
        HIP_TRY(hipMalloc(&net->stats, sizeof(float) * 2 * (size_t)groups));
        net->partial_groups = groups;
    }
    // the rate of step s: first_rate (last_rate / first_rate)^(s / (num_steps - 1)),
    // evaluated in double and rounded once
    const double ratio = (double)last_rate / (double)first_rate;
    for (int32_t s = 0; s < num_steps; ++s) {
        const double f = num_steps > 1 ? (double)s / (double)(num_steps - 1) : 0.0;
        const float rate = (float)((double)first_rate * std::pow(ratio, f));
        const int64_t start = starts ? starts[s] : (int64_t)s * batch % num_rows;
        const int step = ++net->adam_step;
        HIP_TRY(xpbd::launch_mlp_train(net->d, features, targets, rows, start, num_rows, batch,
                                       net->partial, net->stats, rate, 0.9f, 0.999f, 1e-8f, step,
                                       nullptr, losses ? losses + s : net->loss, net->stream));
    }
    return XPBD_OK;
}

xpbd_status xpbd_mlp_normalisation(const uint16_t *features, const float *targets, int64_t n,
                                   void *hip_stream, float *in_shift, float *in_scale,
                                   float *out_shift, float *out_scale)
{
    g_error.clear();
    if (!features || !targets || n < 1 || !in_shift || !in_scale || !out_shift || !out_scale)
        return fail(XPBD_E_ARG, "features, targets, n >= 1 and the four outputs are required");
    if (!is_device_pointer(features) || !is_device_pointer(targets))
        return fail(XPBD_E_ARG, "features and targets must be device memory");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t bytes = xpbd::mlp_normalisation_workspace();
    void *ws = nullptr;
    HIP_TRY(hipMalloc(&ws, bytes));
    float host[2 * xpbd::kMlpFeatures + 6];
    hipError_t e = xpbd::launch_mlp_normalisation(features, targets, n, ws, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host, static_cast<char *>(ws) + bytes - sizeof host, sizeof host,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    (void)hipFree(ws);
    if (e != hipSuccess)
        return fail(XPBD_E_HIP, "normalisation: %s", hipGetErrorString(e));
    const int F = xpbd::kMlpFeatures;
    for (int c = 0; c < F; ++c) {
        in_shift[c] = host[c];
        in_scale[c] = host[F + c];
    }
    for (int k = 0; k < 3; ++k) {
        out_shift[k] = host[2 * F + k];
        out_scale[k] = host[2 * F + 3 + k];
    }
    return XPBD_OK;
}

void xpbd_mlp_destroy(xpbd_mlp *net) { delete net; }

xpbd_status xpbd_axis_neighbours(const xpbd_mesh *mesh, int32_t *out)
{
    g_error.clear();
    if (!mesh || !out || !mesh->rest_pos || mesh->num_vertices < 1)
        return fail(XPBD_E_ARG, "mesh with rest positions and out are required");
    std::vector<int32_t> nbr;
    xpbd::axis_neighbours(mesh->num_vertices, mesh->rest_pos, nbr);
    std::memcpy(out, nbr.data(), sizeof(int32_t) * nbr.size());
    return XPBD_OK;
}

xpbd_status xpbd_step_learned(xpbd_batch *b, const xpbd_mlp *net, int32_t num_steps,
                              const float *tool_pos, size_t tool_pos_bytes,
                              const xpbd_learned_params *lp)
{
    g_error.clear();
    if (!b || !lp)
        return fail(XPBD_E_ARG, "batch and params are required");
    if (num_steps < 0)
        return fail(XPBD_E_ARG, "num_steps must be >= 0");
    xpbd_status st = xpbd::check_learned(b, net, lp);
    if (st != XPBD_OK)
        return st;
    if (num_steps == 0)
        return XPBD_OK;
    st = xpbd::check_tool_bytes(b, num_steps, tool_pos, tool_pos_bytes);
    if (st != XPBD_OK)
        return st;
    const int tools = b->params.num_tools;
    const float *tools_dev = nullptr;
    if (tools > 0) {
        const size_t bytes = tool_pos_bytes;
        if (is_device_pointer(tool_pos)) {
            tools_dev = tool_pos;
        } else {
            if (b->tool_staging_bytes < bytes) {
                if (b->tool_staging)
                    HIP_TRY(hipFree(b->tool_staging));
                b->tool_staging = nullptr;
                b->tool_staging_bytes = 0;
                HIP_TRY(hipMalloc(&b->tool_staging, bytes));
                b->tool_staging_bytes = bytes;
            }
            HIP_TRY(hipMemcpyAsync(b->tool_staging, tool_pos, bytes, hipMemcpyHostToDevice,
                                   b->stream));
            HIP_TRY(hipStreamSynchronize(b->stream));
            tools_dev = b->tool_staging;
        }
    }
    return xpbd::run_learned(b, net, num_steps, tools_dev, lp, nullptr);
}

}  // extern "C"

// Checks of a learned step's batch and parameters (before any device work).
xpbd_status xpbd::check_learned(const xpbd_batch *b, const xpbd_mlp *net,
                                const xpbd_learned_params *lp)
{
    if (!b->register_variant || b->envs_per_group != 1 || b->classes.size() != 1 ||
        b->params.tool_shape != XPBD_TOOL_SPHERE)
        return fail(XPBD_E_CAPACITY, "the learned step needs sphere tools and the register "
                    "variant with one environment per workgroup and one size class (set "
                    "block_size for meshes of different sizes)");
    if (lp->min_iterations < 0 || lp->max_iterations < lp->min_iterations)
        return fail(XPBD_E_ARG, "need 0 <= min_iterations <= max_iterations");
    if (!std::isfinite(lp->threshold) && !std::isinf(lp->threshold))
        return fail(XPBD_E_ARG, "threshold must not be NaN");
    if (!(lp->stall_ratio >= 0.0f && lp->stall_ratio <= 1.0f))
        return fail(XPBD_E_ARG, "stall_ratio must be in [0, 1] (got %g)", (double)lp->stall_ratio);
    const bool record = lp->record_substep >= 0;
    if ((lp->apply_correction || record) && !net)
        return fail(XPBD_E_ARG, "the correction and the recording need a network");
    if (record && (lp->record_substep >= b->params.substeps || !lp->record_features ||
                   !lp->record_targets || !is_device_pointer(lp->record_features) ||
                   !is_device_pointer(lp->record_targets)))
        return fail(XPBD_E_ARG, "record_substep must name a substep and both record buffers "
                    "must be device memory");
    if (lp->iterations && !is_device_pointer(lp->iterations))
        return fail(XPBD_E_ARG, "iterations must be device memory");
    if (lp->residuals && !is_device_pointer(lp->residuals))
        return fail(XPBD_E_ARG, "residuals must be device memory");
    return XPBD_OK;
}

// The learned step's device workspace, allocated on first use (before any
// launch, so that a captured step allocates nothing).
xpbd_status xpbd::learned_workspace(xpbd_batch *b, const xpbd_learned_params *lp)
{
    const int64_t NP = b->total_particles;
    xpbd_status st;
    if (!b->learned_xhat && ((st = b->alloc(reinterpret_cast<void **>(&b->learned_xhat),
                                            sizeof(float) * 3 * (size_t)NP)) ||
                             (st = b->alloc(reinterpret_cast<void **>(&b->learned_cand),
                                            (size_t)NP))))
        return st;
    if (lp->apply_correction && !b->learned_feat &&
        (st = b->alloc(reinterpret_cast<void **>(&b->learned_feat),
                       sizeof(uint16_t) * 32 * (size_t)NP)))
        return st;
    if (lp->apply_correction && !b->learned_chunk0) {
        std::vector<int32_t> c0;
        int32_t chunks = 1;
        learned_chunks(b, c0, chunks);
        if ((st = b->upload(&b->learned_chunk0, c0)))
            return st;
        b->learned_chunks = chunks;
    }
    if (lp->apply_correction && !b->correct_workgroups) {
        int device = 0, cus = 0;
        HIP_TRY(hipGetDevice(&device));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
        b->correct_workgroups = kCorrectWorkgroupsPerCu * std::max(cus, 1);
    }

    return XPBD_OK;
}

void xpbd::learned_chunks(const xpbd_batch *b, std::vector<int32_t> &c0, int32_t &chunks)
{
    c0.assign(b->meshes.size(), 0);
    chunks = 1;
    for (size_t m = 0; m < b->meshes.size(); ++m) {
        const auto &pm = b->meshes[m];
        int32_t first = 0;
        while (first < pm.num_vertices && !(pm.inv_mass[(size_t)first] > 0.0f))
            ++first;
        c0[m] = std::min(first, pm.num_vertices - 1) / kCorrectChunk;
        chunks = std::max(chunks, (pm.num_vertices + kCorrectChunk - 1) / kCorrectChunk - c0[m]);
    }
}

// num_steps learned steps with the tool poses in device memory; grasp is null
// or names the RL step's grasp state.
xpbd_status xpbd::run_learned(xpbd_batch *b, const xpbd_mlp *net, int32_t num_steps,
                              const float *tools_dev, const xpbd_learned_params *lp,
                              const GraspArgs *grasp, const LearnedWorkspace *ws)
{
    const int tools = b->params.num_tools;
    const bool record = lp->record_substep >= 0;
    LearnedWorkspace own;
    if (!ws) {
        xpbd_status st = learned_workspace(b, lp);
        if (st != XPBD_OK)
            return st;
        own.xhat = b->learned_xhat;
        own.feat = b->learned_feat;
        own.cand = b->learned_cand;
        own.chunk0 = b->learned_chunk0;
        own.chunks = b->learned_chunks;
        own.correct_workgroups = b->correct_workgroups;
        ws = &own;
    }

    xpbd::StepArgs a;
    std::memset(&a, 0, sizeof a);
    a.meshes = b->meshes_dev;
    a.envs = b->envs_dev;
    a.groups = b->groups_dev;
    a.num_groups = b->num_groups;
    a.round_barriers = b->classes.size() == 1 && b->classes[0].round_barriers ? 1 : 0;
    a.compliance = b->compliance;
    a.tool_pos = tools_dev;
    a.pos = b->pos;
    a.vel = b->vel;
    a.contacts = b->contacts;
    a.contact_counts = b->contact_counts;
    a.residual = b->residual;
    a.nonfinite = b->nonfinite;
    a.num_envs = b->num_envs;
    a.total_particles = b->total_particles;
    a.num_steps = num_steps;
    a.substeps = b->params.substeps;
    a.iterations = b->params.iterations;
    a.num_tools = tools;
    const double h = (double)b->params.dt / (double)b->params.substeps;
    a.h = (float)h;
    a.inv_h = (float)(1.0 / h);
    for (int k = 0; k < 3; ++k)
        a.gravity[k] = b->params.gravity[k];
    for (int t = 0; t < tools; ++t) {
        const float r = b->params.tool_radius[t];
        a.tool_radius[t] = r;
        a.tool_radius2[t] = r * r;
        const float reach = 2.0f * r;
        a.tool_reach2[t] = reach * reach;
    }
    if (grasp) {
        a.grasp = grasp->state;
        for (int k = 0; k < 3; ++k)
            a.grasp_offset[k] = grasp->offset[k];
        a.grasp_radius2 = grasp->radius * grasp->radius;
    }
    xpbd::LearnedArgs L;
    std::memset(&L, 0, sizeof L);
    L.xhat = ws->xhat;
    L.cand = ws->cand;
    L.in_shift = net ? net->in_shift : nullptr;
    L.in_scale = net ? net->in_scale : nullptr;
    L.out_shift = net ? net->d.out_shift : nullptr;
    L.out_scale = net ? net->d.out_scale : nullptr;
    L.threshold = lp->threshold;
    L.min_iterations = lp->min_iterations;
    L.max_iterations = lp->max_iterations;
    L.stall_ratio = lp->stall_ratio;
    L.max_vertices = b->max_vertices;
    L.chunk0 = ws->chunk0;
    L.chunks = ws->chunks;
    const bool resid = (b->params.flags & XPBD_F_RESIDUAL) != 0;
    const bool want_lambda = (b->params.flags & XPBD_F_LAMBDA) || resid;
    const int S = b->params.substeps;
    auto feature_buffer = [&](int sub) {
        return record && sub == lp->record_substep ? lp->record_features : ws->feat;
    };
    for (int step = 0; step < num_steps; ++step)
        for (int sub = 0; sub < S; ++sub) {
            const bool last = step == num_steps - 1 && sub == S - 1;
            const bool rec = record && sub == lp->record_substep;
            L.first_substep = sub == 0;
            L.step = step;
            L.features = rec ? lp->record_features : nullptr;
            L.record_targets = rec ? lp->record_targets : nullptr;
            L.iterations = lp->iterations ? lp->iterations + ((size_t)step * S + sub) * b->num_envs
                                          : nullptr;
            L.residuals = lp->residuals ? lp->residuals + ((size_t)step * S + sub) * b->num_envs
                                        : nullptr;
            a.lambda_out = last && want_lambda ? b->lambda : nullptr;
            L.next_features = nullptr;
            if (lp->apply_correction) {
                // the first substep of the call predicts in a kernel of its own; every
                // substep kernel leaves the next one's prediction and features
                L.features = feature_buffer(sub);
                if (step == 0 && sub == 0)
                    HIP_TRY(xpbd::launch_learned_predict(a, L, b->stream));
                HIP_TRY(xpbd::launch_learned_correct(a, L, net->d, ws->correct_workgroups,
                                                     b->stream));
                if (!last)
                    L.next_features = feature_buffer((sub + 1) % S);
            } else {
                HIP_TRY(xpbd::launch_learned_predict(a, L, b->stream));
            }
            HIP_TRY(xpbd::launch_substep_reg(a, L, b->block, b->lambda_banks, b->lds_bytes,
                                             last && resid, b->stream));
        }
    b->residual_valid = b->residual_valid || resid;
    return XPBD_OK;
}
