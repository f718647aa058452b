// The learned step without allocation: xpbd_step_learned_noalloc
// (include/xpbd_learned.h).  Its workspace -- predicted positions, feature
// rows, contact-candidate bits and the correction's chunk table -- lives in
// one file-scope device array instead of buffers the batch allocates on its
// first learned call; everything else is the learned step's own code.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/xpbd_learned.h"
#include "batch.h"
#include "learned_step.h"
#include "mlp_device.h"
#include "runtime_util.h"
#include "xpbd_device.h"

using xpbd::fail;
using xpbd::g_error;
using xpbd::is_device_pointer;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

// The workspace of every call on a device.  In host code the name stands for
// a host-side shadow, not for device memory: host code uses the address that
// hipGetSymbolAddress returns for the current device (scratch_base) instead.
static __device__ __align__(256) unsigned char scratch[XPBD_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices];

size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// Device address of this device's scratch array, looked up once per device
// (with that device current).
xpbd_status scratch_base(int device, unsigned char **out)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(XPBD_E_ARG, "device %d is outside the %d devices the library tracks", device,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(XPBD_E_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                        hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[device]);
    return XPBD_OK;
}

// First kCorrectChunk-particle chunk of every mesh that holds a free particle (the
// correction skips the chunks before it): one thread per mesh.
__global__ void chunk_table_kernel(const xpbd::MeshDev *__restrict__ meshes, int32_t num_meshes,
                                   int32_t *__restrict__ chunk0)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= num_meshes)
        return;
    const int V = meshes[m].num_vertices;
    const float *w = meshes[m].inv_mass;
    int first = 0;
    while (first < V && !(w[first] > 0.0f))
        ++first;
    chunk0[m] = (first < V - 1 ? first : V - 1) / xpbd::kCorrectChunk;
}

}  // namespace

extern "C" {

xpbd_status xpbd_step_learned_noalloc(xpbd_batch *b, const xpbd_mlp *net, int32_t num_steps,
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
    st = xpbd::check_tool_bytes(b, num_steps, tool_pos, tool_pos_bytes);
    if (st != XPBD_OK)
        return st;
    const int tools = b->params.num_tools;
    if (tools > 0 && num_steps > 0 && !is_device_pointer(tool_pos))
        return fail(XPBD_E_ARG, "tool_pos must be device memory (host poses would need a "
                    "staging buffer)");
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    if (device != b->device)
        return fail(XPBD_E_ARG, "the batch lives on device %d but device %d is current",
                    b->device, device);

    // workspace layout: xhat [3][NP] f32, feat [NP][32] bf16 (with the
    // correction), cand [NP] u8, chunk0 [meshes] i32, each 256-byte aligned
    const size_t NP = (size_t)b->total_particles;
    const size_t num_meshes = b->meshes.size();
    const size_t xhat_bytes = align_up(3 * NP * sizeof(float));
    const size_t feat_bytes = lp->apply_correction ? align_up(NP * XPBD_MLP_FEATURE_STRIDE * 2) : 0;
    const size_t cand_bytes = align_up(NP);
    const size_t chunk_bytes = align_up(num_meshes * sizeof(int32_t));
    const size_t need = xhat_bytes + feat_bytes + cand_bytes + chunk_bytes;
    if (need > (size_t)XPBD_NOALLOC_SCRATCH_BYTES)
        return fail(XPBD_E_CAPACITY, "the batch's learned workspace needs %zu bytes; the "
                    "allocation-free step holds at most %zu (%zu particles, %zu meshes%s)",
                    need, (size_t)XPBD_NOALLOC_SCRATCH_BYTES, NP, num_meshes,
                    lp->apply_correction ? ", with the correction's feature rows" : "");
    if (num_steps == 0)
        return XPBD_OK;

    unsigned char *base = nullptr;
    if ((st = scratch_base(device, &base)) != XPBD_OK)
        return st;
    xpbd::LearnedWorkspace ws;
    ws.xhat = reinterpret_cast<float *>(base);
    ws.feat = feat_bytes ? reinterpret_cast<uint16_t *>(base + xhat_bytes) : nullptr;
    ws.cand = base + xhat_bytes + feat_bytes;
    ws.chunk0 = reinterpret_cast<int32_t *>(base + xhat_bytes + feat_bytes + cand_bytes);
    if (lp->apply_correction) {
        // chunks per environment: the most any mesh needs from its first
        // chunk with a free particle on (the same rule as the kernel above)
        int32_t chunks = 1;
        for (const auto &pm : b->meshes) {
            int32_t first = 0;
            while (first < pm.num_vertices && !(pm.inv_mass[(size_t)first] > 0.0f))
                ++first;
            const int32_t c0 = std::min(first, pm.num_vertices - 1) / xpbd::kCorrectChunk;
            const int32_t n = (pm.num_vertices + xpbd::kCorrectChunk - 1) / xpbd::kCorrectChunk;
            chunks = std::max(chunks, n - c0);
        }
        ws.chunks = chunks;
        int cus = 0;
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
        ws.correct_workgroups = xpbd::kCorrectWorkgroupsPerCu * std::max(cus, 1);   // as the allocating step
        const int block = 64;
        const int grid = (int)((num_meshes + block - 1) / block);
        hipLaunchKernelGGL(chunk_table_kernel, dim3(grid), dim3(block), 0, b->stream,
                           b->meshes_dev, (int32_t)num_meshes, ws.chunk0);
        HIP_TRY(hipGetLastError());
    }
    return xpbd::run_learned(b, net, num_steps, tool_pos, lp, nullptr, &ws);
}

}  // extern "C"
