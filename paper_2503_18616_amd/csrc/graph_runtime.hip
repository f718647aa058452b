// Captured steps (include/xpbd_graph.h): a step of the public entry points
// recorded into a HIP graph on a private stream, replayed on the batch's.
#include <hip/hip_runtime.h>

#include "../../include/xpbd_graph.h"
#include "batch.h"
#include "learned_step.h"
#include "runtime_util.h"

using xpbd::fail;
using xpbd::g_error;
using xpbd::is_device_pointer;

struct xpbd_graph {
    xpbd_batch *batch = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~xpbd_graph()
    {
        if (exec)
            (void)hipGraphExecDestroy(exec);
        if (graph)
            (void)hipGraphDestroy(graph);
    }
};

namespace {

// Record body() (launches on b->stream, no allocation, no synchronisation)
// into a graph.  A batch of several size classes forks its class streams from
// the batch's stream with an event and joins them back with events; inside
// the capture those streams join it, so the classes become parallel branches
// of the graph between the fork and the join.
template <typename Body>
xpbd_status capture(xpbd_batch *b, Body &&body, xpbd_graph **out)
{
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipStream_t saved = b->stream;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return fail(XPBD_E_HIP, "hipStreamBeginCapture failed: %s", hipGetErrorString(e));
    }
    b->stream = cs;
    xpbd_status st = body();
    b->stream = saved;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (st != XPBD_OK) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess || !graph) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return fail(XPBD_E_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    }
    xpbd_graph *g = new xpbd_graph();
    g->batch = b;
    g->graph = graph;
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        g->exec = nullptr;
        delete g;
        return fail(XPBD_E_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    *out = g;
    return XPBD_OK;
}

}  // namespace

extern "C" {

xpbd_status xpbd_step_graph_create(xpbd_batch *b, const xpbd_mlp *net,
                                   const xpbd_learned_params *learned, const float *tool_pos,
                                   size_t tool_pos_bytes, xpbd_graph **out)
{
    g_error.clear();
    if (!b || !out)
        return fail(XPBD_E_ARG, "batch and out must not be NULL");
    *out = nullptr;
    xpbd_status checked = xpbd::check_tool_bytes(b, 1, tool_pos, tool_pos_bytes);
    if (checked != XPBD_OK)
        return checked;
    if (b->params.num_tools > 0 && !is_device_pointer(tool_pos))
        return fail(XPBD_E_ARG, "tool_pos must be device memory");
    if (learned) {
        xpbd_status st = xpbd::check_learned(b, net, learned);
        if (st == XPBD_OK)
            st = xpbd::learned_workspace(b, learned);
        if (st != XPBD_OK)
            return st;
        return capture(
            b, [&] { return xpbd_step_learned(b, net, 1, tool_pos, tool_pos_bytes, learned); },
            out);
    }
    return capture(b, [&] { return xpbd_step(b, 1, tool_pos, tool_pos_bytes); }, out);
}

xpbd_status xpbd_rl_graph_create(xpbd_batch *b, const xpbd_policy *policy,
                                 const xpbd_rl_params *params, const xpbd_mlp *net,
                                 const xpbd_learned_params *learned, float *tool_pos,
                                 int32_t *grasped, const float *target, float *obs,
                                 float *actions, xpbd_graph **out)
{
    g_error.clear();
    if (!b || !out)
        return fail(XPBD_E_ARG, "batch and out must not be NULL");
    *out = nullptr;
    if (learned) {
        xpbd_status st = xpbd::check_learned(b, net, learned);
        if (st == XPBD_OK)
            st = xpbd::learned_workspace(b, learned);
        if (st != XPBD_OK)
            return st;
        return capture(b, [&] {
            return xpbd_rl_step_learned(b, policy, params, net, learned, 1, tool_pos, grasped,
                                        target, obs, actions);
        }, out);
    }
    return capture(b, [&] {
        return xpbd_rl_step(b, policy, params, 1, tool_pos, grasped, target, obs, actions);
    }, out);
}

xpbd_status xpbd_graph_launch(xpbd_graph *g, int32_t times)
{
    g_error.clear();
    if (!g)
        return fail(XPBD_E_ARG, "graph is NULL");
    if (times < 0)
        return fail(XPBD_E_ARG, "times must be >= 0 (got %d)", times);
    for (int32_t k = 0; k < times; ++k)
        HIP_TRY(hipGraphLaunch(g->exec, g->batch->stream));
    return XPBD_OK;
}

void xpbd_graph_destroy(xpbd_graph *g) { delete g; }

}  // extern "C"
