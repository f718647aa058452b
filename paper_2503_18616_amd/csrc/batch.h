// The batch object behind the C ABI's xpbd_batch handle (host side), shared
// by the runtime sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/xpbd.h"
#include "mesh_setup.h"
#include "runtime_util.h"
#include "xpbd_device.h"

// A size class of the register variant: environments whose meshes share a
// block size, an LDS tier and a number of environments per workgroup run in
// one launch; several classes run concurrently on up to kClassLanes streams
// (the batch's own and streams forked from and joined to it).
struct RegClass {
    int block = 256;
    int group = 1;                  // environments per workgroup
    int lambda_banks = 1;
    int rounds = 0;                 // rounds per sweep of its largest mesh
    bool round_barriers = true;     // every colour of every mesh of the class is one round
    uint32_t lds_bytes = 0;
    int32_t num_groups = 0;
    int32_t *groups_dev = nullptr;
    int lane = 0;                   // 0: the batch's stream, k > 0: lanes[k - 1]
};

// Streams a multi-class step uses at most, the batch's own included: HIP maps
// a process's streams onto 4 hardware queues by default, and classes whose
// streams share a queue run one after the other.
constexpr int kClassLanes = 4;

struct xpbd_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    xpbd_params params{};
    int32_t num_envs = 0;
    int32_t total_particles = 0;
    int32_t total_lambda = 0;
    int block = 64;
    int particles_per_thread = 1;
    bool stage_topology = false;
    bool register_variant = false;
    int lambda_banks = 1;
    int envs_per_group = 1;
    int32_t num_groups = 0;
    int32_t *groups_dev = nullptr;
    uint32_t lds_bytes = 0;
    std::vector<RegClass> classes;           // register variant
    std::vector<int> class_order;            // launch order: largest estimated work first
    std::vector<hipStream_t> lanes;          // forked streams of a multi-class step
    std::vector<hipEvent_t> lane_done;
    hipEvent_t fork = nullptr;               // start of a step on the batch's stream
    std::vector<xpbd::PreparedMesh> meshes;
    std::vector<int32_t> env_mesh;
    std::vector<int32_t> env_offsets;       // [N+1]
    std::vector<int32_t> colours;           // concatenated per mesh: edges then tets
    std::vector<xpbd::DeviceBuffer> allocations;
    float *pos = nullptr, *vel = nullptr, *lambda = nullptr, *residual = nullptr;
    float *compliance = nullptr;
    int32_t *contacts = nullptr, *contact_counts = nullptr, *nonfinite = nullptr;
    xpbd::MeshDev *meshes_dev = nullptr;
    xpbd::EnvDev *envs_dev = nullptr;
    float *staging = nullptr;                // [sum V][3] for AoS <-> SoA and host tool poses
    size_t staging_bytes = 0;
    float *tool_staging = nullptr;
    size_t tool_staging_bytes = 0;
    bool residual_valid = false;   // a step has computed the residual
    // learned warm start workspace (allocated on first use)
    float *learned_xhat = nullptr;           // [3][total particles]
    uint16_t *learned_feat = nullptr;        // [total particles][32] features of the correction
    uint8_t *learned_cand = nullptr;         // [total particles]
    int32_t correct_workgroups = 0;          // persistent workgroups of the correction pass
    int32_t *learned_chunk0 = nullptr;       // [meshes] first 32-particle chunk with a free particle
    int32_t learned_chunks = 0;              // chunks per environment the correction visits
    int32_t max_vertices = 0;

    ~xpbd_batch()
    {
        (void)hipStreamSynchronize(stream);
        for (hipStream_t l : lanes) {
            (void)hipStreamSynchronize(l);
            (void)hipStreamDestroy(l);
        }
        for (hipEvent_t e : lane_done)
            (void)hipEventDestroy(e);
        if (fork)
            (void)hipEventDestroy(fork);
        for (auto &a : allocations)
            (void)hipFree(a.ptr);
        if (tool_staging)
            (void)hipFree(tool_staging);
    }

    xpbd_status alloc(void **out, size_t bytes)
    {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, bytes ? bytes : 16);
        if (e != hipSuccess)
            return xpbd::fail(XPBD_E_HIP, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        allocations.push_back({p, bytes});
        *out = p;
        return XPBD_OK;
    }

    template <typename T>
    xpbd_status upload(T **out, const std::vector<T> &host)
    {
        xpbd_status s = alloc(reinterpret_cast<void **>(out), host.size() * sizeof(T));
        if (s != XPBD_OK)
            return s;
        if (!host.empty())  // blocking: the host vectors are temporaries of creation
            HIP_TRY(hipMemcpy(*out, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice));
        return XPBD_OK;
    }
};

namespace xpbd {

// Grasp state of the RL-style step handed to the step launches.
struct GraspArgs {
    int32_t *state;      // device [N]: held id, -1 none, -2 closed and empty
    float offset[3];     // dragging point relative to tool 0's centre
    float radius;        // r_l
};

// Bytes of num_steps steps of tool poses ([num_steps][N][tools][3], or [6]
// for capsules), and the check of a caller's declared byte count against it
// (XPBD_E_ARG on a mismatch or a NULL buffer when the batch has tools).
size_t tool_bytes(const xpbd_batch *b, int32_t num_steps);
xpbd_status check_tool_bytes(const xpbd_batch *b, int32_t num_steps, const float *tool_pos,
                             size_t tool_pos_bytes);

// num_steps steps with the tool poses in device memory ([num_steps][N][tools][3]
// or [6] for capsules); grasp is null or names the grasp state (register variant).
xpbd_status run_step(xpbd_batch *b, int32_t num_steps, const float *tools_dev,
                     const GraspArgs *grasp);

}  // namespace xpbd
