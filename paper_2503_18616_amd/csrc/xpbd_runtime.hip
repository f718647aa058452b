// Host runtime of the XPBD library: the C ABI declared in include/xpbd.h.
//
// Creation prepares every distinct mesh on the host (orientation, rest
// values, edges, greedy colours), lays the constraints out in colour-major
// schedule order, plans the per-workgroup LDS footprint and uploads
// everything once.  A step is one kernel launch over all environments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <random>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <thread>
#include <atomic>

#include "../../include/xpbd.h"
#include "mesh_setup.h"
#include "batch.h"
#include "runtime_util.h"
#include "xpbd_device.h"

using xpbd::EnvDev;
using xpbd::MeshDev;
using xpbd::PreparedMesh;

using xpbd::DeviceBuffer;
using xpbd::fail;
using xpbd::g_error;
using xpbd::is_device_pointer;

namespace {

xpbd_status validate_params(const xpbd_params *p)
{
    if (!p)
        return fail(XPBD_E_ARG, "params is NULL");
    if (!(std::isfinite(p->dt) && p->dt > 0.0f))
        return fail(XPBD_E_ARG, "dt must be finite and > 0 (got %g)", (double)p->dt);
    if (p->substeps < 1)
        return fail(XPBD_E_ARG, "substeps must be >= 1 (got %d)", p->substeps);
    if (p->iterations < 0)
        return fail(XPBD_E_ARG, "iterations must be >= 0 (got %d)", p->iterations);
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(p->gravity[k]))
            return fail(XPBD_E_ARG, "gravity must be finite");
    if (p->num_tools < 0 || p->num_tools > 2)
        return fail(XPBD_E_ARG, "num_tools must be 0, 1 or 2 (got %d)", p->num_tools);
    for (int t = 0; t < p->num_tools; ++t)
        if (!(std::isfinite(p->tool_radius[t]) && p->tool_radius[t] > 0.0f))
            return fail(XPBD_E_ARG, "tool_radius[%d] must be finite and > 0", t);
    if (p->flags & ~(XPBD_F_RESIDUAL | XPBD_F_LAMBDA))
        return fail(XPBD_E_ARG, "unknown flag bits 0x%x", p->flags);
    if (p->block_size != 0 &&
        (p->block_size < 64 || p->block_size > 1024 || p->block_size % 64 != 0))
        return fail(XPBD_E_ARG, "block_size must be 0 or a multiple of 64 in [64, 1024]");
    if (p->solver_variant < XPBD_VARIANT_AUTO || p->solver_variant > XPBD_VARIANT_JACOBI)
        return fail(XPBD_E_ARG, "unknown solver_variant %d", p->solver_variant);
    if (p->colour_packing < XPBD_PACKING_AUTO || p->colour_packing > XPBD_PACKING_SEARCH)
        return fail(XPBD_E_ARG, "unknown colour_packing %d", p->colour_packing);
    if (p->colouring < XPBD_COLOURING_GREEDY || p->colouring > XPBD_COLOURING_CAPPED_FIT)
        return fail(XPBD_E_ARG, "unknown colouring %d", p->colouring);
    if (p->envs_per_group < 0 || p->envs_per_group > xpbd::kMaxEnvsPerGroup)
        return fail(XPBD_E_ARG, "envs_per_group must be 0, 1 or 2 (got %d)", p->envs_per_group);
    if (p->tool_shape != XPBD_TOOL_SPHERE && p->tool_shape != XPBD_TOOL_CAPSULE)
        return fail(XPBD_E_ARG, "unknown tool_shape %d", p->tool_shape);
    return XPBD_OK;
}

// Local-search moves per constraint of the SEARCH colour packing.
constexpr int32_t kLaneSearchEffort = 64;
// Distinct particles (summed over the batch's meshes) up to which the default
// colour packing runs the lane search.
constexpr int64_t kSearchParticles = 16384;

int next_pow2(int x)
{
    int p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

// Schedule of one constraint type: slot -> constraint id, colour-major and
// ascending inside a colour, plus the colour offsets.
void build_schedule(const std::vector<int32_t> &colour, int32_t num_colours,
                    std::vector<int32_t> &slot_id, std::vector<int32_t> &ptr)
{
    ptr.assign((size_t)num_colours + 1, 0);
    for (int32_t c : colour)
        ptr[(size_t)c + 1]++;
    for (int32_t c = 0; c < num_colours; ++c)
        ptr[(size_t)c + 1] += ptr[(size_t)c];
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    slot_id.assign(colour.size(), 0);
    for (size_t j = 0; j < colour.size(); ++j)
        slot_id[(size_t)fill[(size_t)colour[j]]++] = (int32_t)j;
}

// Rounds of the register-multiplier kernel for block size B: each colour is
// cut into ceil(size / B) rounds, the last of which carries the barrier.
void build_rounds(const std::vector<int32_t> &edge_ptr, const std::vector<int32_t> &tet_ptr, int B,
                  std::vector<int4> &rounds)
{
    rounds.clear();
    const std::vector<int32_t> *ptrs[2] = {&edge_ptr, &tet_ptr};
    for (int kind = 0; kind < 2; ++kind) {
        const std::vector<int32_t> &ptr = *ptrs[kind];
        for (size_t c = 0; c + 1 < ptr.size(); ++c) {
            const int32_t begin = ptr[c], end = ptr[c + 1];
            for (int32_t b0 = begin; b0 < end; b0 += B)
                rounds.push_back(make_int4(b0, end, kind == 0 ? xpbd::ROUND_EDGE : xpbd::ROUND_TET,
                                           b0 + B >= end ? 1 : 0));
        }
    }
}

// Rounds of a group of G copies of the mesh at block size B.
int count_rounds(const PreparedMesh &pm, int B, int G)
{
    std::vector<int32_t> n_e((size_t)pm.num_edge_colours, 0), n_t((size_t)pm.num_tet_colours, 0);
    for (int32_t c : pm.edge_colour)
        n_e[(size_t)c]++;
    for (int32_t c : pm.tet_colour)
        n_t[(size_t)c]++;
    int re = 0, rt = 0;
    for (int32_t n : n_e)
        re += (G * n + B - 1) / B;
    for (int32_t n : n_t)
        rt += (G * n + B - 1) / B;
    // as build_round_schedule pads them: the edge rounds to an even count, then
    // the total
    const int r = re + (re & 1) + rt;
    return r + (r & 1);
}

xpbd_status field_bytes(const xpbd_batch *b, int32_t field, size_t *bytes)
{
    const size_t NP = (size_t)b->total_particles, N = (size_t)b->num_envs;
    const size_t tools = (size_t)b->params.num_tools;
    switch (field) {
    case XPBD_FIELD_POS:
    case XPBD_FIELD_VEL: *bytes = NP * 3 * sizeof(float); return XPBD_OK;
    case XPBD_FIELD_LAMBDA: *bytes = (size_t)b->total_lambda * sizeof(float); return XPBD_OK;
    case XPBD_FIELD_CONTACTS: *bytes = tools * NP * sizeof(int32_t); return XPBD_OK;
    case XPBD_FIELD_CONTACT_COUNTS: *bytes = N * tools * sizeof(int32_t); return XPBD_OK;
    case XPBD_FIELD_COLOURS: *bytes = b->colours.size() * sizeof(int32_t); return XPBD_OK;
    case XPBD_FIELD_RESIDUAL: *bytes = N * 2 * sizeof(float); return XPBD_OK;
    case XPBD_FIELD_ENV_OFFSETS: *bytes = (N + 1) * sizeof(int32_t); return XPBD_OK;
    case XPBD_FIELD_NONFINITE: *bytes = N * sizeof(int32_t); return XPBD_OK;
    default: return fail(XPBD_E_STATE, "unknown field %d", field);
    }
}

// Copy bytes from host memory to dst (host or device).
xpbd_status copy_host_out(xpbd_batch *b, void *dst, const void *src, size_t bytes)
{
    if (bytes == 0)
        return XPBD_OK;
    if (is_device_pointer(dst)) {
        HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
    } else {
        std::memcpy(dst, src, bytes);
    }
    return XPBD_OK;
}

}  // namespace

extern "C" {

const char *xpbd_last_error(void) { return g_error.c_str(); }

xpbd_status xpbd_prepare_mesh(const xpbd_mesh *mesh, int32_t *counts, int32_t *edges,
                              int32_t *tets, int32_t *colours, float *rest)
{
    return xpbd_prepare_mesh_coloured(mesh, XPBD_COLOURING_GREEDY, counts, edges, tets, colours,
                                      rest);
}

xpbd_status xpbd_prepare_mesh_coloured(const xpbd_mesh *mesh, int32_t colouring, int32_t *counts,
                                       int32_t *edges, int32_t *tets, int32_t *colours,
                                       float *rest)
{
    g_error.clear();
    if (!mesh || !counts)
        return fail(XPBD_E_ARG, "mesh and counts must not be NULL");
    if (colouring < XPBD_COLOURING_GREEDY || colouring > XPBD_COLOURING_CAPPED_FIT)
        return fail(XPBD_E_ARG, "unknown colouring %d", colouring);
    PreparedMesh pm;
    std::string err;
    int rc = xpbd::prepare_mesh(mesh->num_vertices, mesh->num_tets, mesh->rest_pos,
                                mesh->inv_mass, mesh->tets, pm, err, colouring);
    if (rc != XPBD_OK)
        return fail((xpbd_status)rc, "%s", err.c_str());
    const int32_t E = pm.num_edges(), T = pm.num_tets();
    counts[0] = E;
    counts[1] = T;
    counts[2] = pm.num_edge_colours;
    counts[3] = pm.num_tet_colours;
    if (edges)
        std::copy(pm.edges.begin(), pm.edges.end(), edges);
    if (tets)
        std::copy(pm.tets.begin(), pm.tets.end(), tets);
    if (colours) {
        std::copy(pm.edge_colour.begin(), pm.edge_colour.end(), colours);
        std::copy(pm.tet_colour.begin(), pm.tet_colour.end(), colours + E);
    }
    if (rest) {
        for (int32_t e = 0; e < E; ++e)
            rest[e] = (float)pm.rest_length[(size_t)e];
        for (int32_t t = 0; t < T; ++t)
            rest[E + t] = (float)pm.rest_volume[(size_t)t];
    }
    return XPBD_OK;
}

xpbd_status xpbd_surface_faces(const xpbd_mesh *mesh, int32_t *counts, int32_t *faces,
                               int32_t *colours)
{
    g_error.clear();
    if (!mesh || !counts)
        return fail(XPBD_E_ARG, "mesh and counts must not be NULL");
    PreparedMesh pm;
    std::string err;
    int rc = xpbd::prepare_mesh(mesh->num_vertices, mesh->num_tets, mesh->rest_pos,
                                mesh->inv_mass, mesh->tets, pm, err);
    if (rc != XPBD_OK)
        return fail((xpbd_status)rc, "%s", err.c_str());
    counts[0] = pm.num_faces();
    counts[1] = pm.num_face_colours;
    if (faces)
        std::copy(pm.faces.begin(), pm.faces.end(), faces);
    if (colours)
        std::copy(pm.face_colour.begin(), pm.face_colour.end(), colours);
    return XPBD_OK;
}

xpbd_status xpbd_create_batch(const xpbd_mesh *meshes, int32_t num_meshes,
                              const int32_t *env_mesh, int32_t num_envs,
                              const float *compliance, const xpbd_params *params,
                              void *hip_stream, xpbd_batch **out)
{
    g_error.clear();
    if (!out)
        return fail(XPBD_E_ARG, "out is NULL");
    *out = nullptr;
    if (!meshes || num_meshes < 1)
        return fail(XPBD_E_ARG, "need at least one mesh");
    if (!env_mesh || num_envs < 1)
        return fail(XPBD_E_ARG, "need at least one environment");
    if (!compliance)
        return fail(XPBD_E_ARG, "compliance is NULL");
    xpbd_status s = validate_params(params);
    if (s != XPBD_OK)
        return s;
    for (int32_t e = 0; e < num_envs; ++e) {
        if (env_mesh[e] < 0 || env_mesh[e] >= num_meshes)
            return fail(XPBD_E_ARG, "env %d uses mesh %d of %d", e, env_mesh[e], num_meshes);
        for (int k = 0; k < 2; ++k)
            if (!(std::isfinite(compliance[2 * e + k]) && compliance[2 * e + k] >= 0.0f))
                return fail(XPBD_E_ARG, "compliance of env %d must be finite and >= 0", e);
    }

    std::vector<PreparedMesh> prepared((size_t)num_meshes);
    for (int32_t m = 0; m < num_meshes; ++m) {
        std::string err;
        int rc = xpbd::prepare_mesh(meshes[m].num_vertices, meshes[m].num_tets,
                                    meshes[m].rest_pos, meshes[m].inv_mass, meshes[m].tets,
                                    prepared[(size_t)m], err, params->colouring);
        if (rc != XPBD_OK)
            return fail((xpbd_status)rc, "mesh %d: %s", m, err.c_str());
    }

    // launch shape: enough threads for the largest colour, particles per thread a power of two
    int vmax = 0, largest_colour = 1;
    for (const auto &pm : prepared) {
        vmax = std::max(vmax, pm.num_vertices);
        std::vector<int32_t> n((size_t)pm.num_edge_colours, 0), q((size_t)pm.num_tet_colours, 0);
        for (int32_t c : pm.edge_colour)
            n[(size_t)c]++;
        for (int32_t c : pm.tet_colour)
            q[(size_t)c]++;
        for (int32_t x : n)
            largest_colour = std::max(largest_colour, x);
        for (int32_t x : q)
            largest_colour = std::max(largest_colour, x);
    }
    int block = params->block_size;
    if (block == 0)
        block = std::min(512, std::max(64, (largest_colour / 2 + 63) / 64 * 64));
    int ppt = next_pow2((vmax + block - 1) / block);
    while (ppt > 8 && block < 1024) {
        block = std::min(1024, block * 2);
        ppt = next_pow2((vmax + block - 1) / block);
    }
    if (ppt > 8)
        return fail(XPBD_E_CAPACITY, "mesh of %d particles needs more than 8 particles per "
                    "thread at 1024 threads", vmax);

    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    int lds_limit = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, device));

    // register-multiplier variant.  A batch of one mesh with the block size
    // left to the library takes the (B, G) of B in {128, 256, 512, 1024} and G
    // in {1, 2} (or the requested G) that the occupancy model below rates
    // fastest.  Otherwise: G as requested, else 1, then the smallest block of
    // 256, 512 or 1024 threads (or the requested one) whose round schedule for
    // G copies of every mesh fits the register banks.
    bool use_registers = false;
    int reg_block = 0, reg_rounds = 0, reg_group = 1;
    bool scored = false;
    int lds_cu = 0, num_cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                  device));
    HIP_TRY(hipDeviceGetAttribute(&num_cus, hipDeviceAttributeMultiprocessorCount, device));
    lds_cu = std::max(lds_cu, lds_limit);
    const bool pow2_block = params->block_size == 0 ||
                            (params->block_size & (params->block_size - 1)) == 0;
    const bool jacobi = params->solver_variant == XPBD_VARIANT_JACOBI;
    const bool capsules = params->tool_shape == XPBD_TOOL_CAPSULE && params->num_tools > 0;
    if (capsules && params->envs_per_group > 1)
        return fail(XPBD_E_CAPACITY, "capsule tools run one environment per workgroup");
    const bool reg_possible = params->solver_variant != XPBD_VARIANT_LDS && !jacobi && pow2_block;
    // LDS of a register-variant workgroup of G environments of a mesh (capsule
    // tools add their candidate faces: flags and a compacted list per tool)
    const int face_tools = capsules ? params->num_tools : 0;
    auto face_bytes = [&](const PreparedMesh &pm) {
        return face_tools *
               (int32_t)xpbd::capsule_face_layout(pm.num_faces(), pm.num_face_colours).total;
    };
    auto reg_lds = [&](const PreparedMesh &pm, int G) {
        return xpbd::reg_lds_layout(G * pm.num_vertices, face_bytes(pm)).total;
    };
    int32_t max_face_bytes = 0;
    for (const auto &pm : prepared)
        max_face_bytes = std::max(max_face_bytes, face_bytes(pm));
    if (reg_possible && prepared.size() == 1 && params->block_size == 0) {
        // Occupancy model: a round (a lane's constraint of one colour, then
        // the colour's barrier) costs about the same whatever B and G, and a
        // CU holds as many workgroups as its 16 resident waves of this kernel
        // (its registers allow four per SIMD) and its LDS allow.  Time of a
        // step ~ (passes of groups over the CUs) x rounds; ties go to the
        // smaller block, then to one environment per workgroup.
        const PreparedMesh &pm = prepared[0];
        double best = 0.0;
        for (int B : {128, 256, 512, 1024})
            for (int G : {1, 2}) {
                if (capsules && B > xpbd::kMaxCapsuleBlock)
                    continue;
                if ((params->envs_per_group && G != params->envs_per_group) || (capsules && G > 1))
                    continue;
                int r = count_rounds(pm, B, G);
                r += r % 2;
                const uint32_t lm = reg_lds(pm, G);
                if (r > xpbd::kMaxRounds || G * pm.num_vertices > 16 * B ||
                    G * pm.num_vertices > 16384 || lm > (uint32_t)lds_limit)
                    continue;
                const int per_cu = std::max(1, std::min(16 / (B / 64), (int)((uint32_t)lds_cu / lm)));
                const int64_t groups = ((int64_t)num_envs + G - 1) / G;
                const int64_t slots = (int64_t)per_cu * std::max(num_cus, 1);
                const double cost = (double)((groups + slots - 1) / slots) * r;
                if (!use_registers || cost < best) {
                    use_registers = scored = true;
                    best = cost;
                    reg_block = B;
                    reg_rounds = r;
                    reg_group = G;
                }
            }
    }
    if (reg_possible && !scored) {
        std::vector<int> group_tries;
        if (params->envs_per_group)
            group_tries.push_back(params->envs_per_group);
        else
            group_tries.push_back(1);
        const int tries[3] = {256, 512, 1024};
        const int n_tries = params->block_size ? 1 : capsules ? 2 : 3;
        for (int G : group_tries) {
            for (int k = 0; k < n_tries && !use_registers; ++k) {
                const int B = params->block_size ? params->block_size : tries[k];
                int worst = 0;
                for (const auto &pm : prepared)
                    worst = std::max(worst, count_rounds(pm, B, G));
                worst += worst % 2;   // padded to an even count
                const bool fits = worst <= xpbd::kMaxRounds && G * vmax <= 16 * B &&
                                  (!capsules || B <= xpbd::kMaxCapsuleBlock) &&
                                  G * vmax <= 16384 && B / 64 <= 16 &&
                                  xpbd::reg_lds_layout(G * vmax, max_face_bytes).total <=
                                      (uint32_t)lds_limit;
                if (fits) {
                    use_registers = true;
                    reg_block = B;
                    reg_rounds = worst;
                    reg_group = G;
                }
            }
            if (use_registers)
                break;
        }
    }
    if (!use_registers && params->solver_variant == XPBD_VARIANT_REGISTERS)
        return fail(XPBD_E_CAPACITY, "the register variant needs a power-of-two block, at most %d "
                    "rounds per lane and LDS for the particles of a group; use the LDS variant",
                    xpbd::kMaxRounds);
    if (!use_registers && params->envs_per_group > 1)
        return fail(XPBD_E_CAPACITY, "%d environments per workgroup need the register variant and "
                    "must fit its rounds and LDS", params->envs_per_group);
    if (use_registers) {
        block = reg_block;
        ppt = 1;
    }
    uint32_t lds_staged = 0, lds_global = 0;
    for (const auto &pm : prepared) {
        const int32_t nf = capsules ? pm.num_faces() : 0;
        lds_staged = std::max(lds_staged, xpbd::lds_layout(pm.num_vertices, pm.num_edges(),
                                                           pm.num_tets(), params->num_tools,
                                                           true, jacobi, nf).total);
        lds_global = std::max(lds_global, xpbd::lds_layout(pm.num_vertices, pm.num_edges(),
                                                           pm.num_tets(), params->num_tools,
                                                           false, jacobi, nf).total);
    }
    bool stage = lds_staged <= (uint32_t)lds_limit && !jacobi;
    uint32_t lds = stage ? lds_staged : lds_global;
    if (use_registers) {
        stage = false;
        lds = xpbd::reg_lds_layout(reg_group * vmax, max_face_bytes).total;
        // the round records hold 16-bit particle fields: LDS byte offsets with
        // one environment per workgroup (the LDS limit keeps them below 65536)
        if (reg_group == 1 && 16 * ((int64_t)vmax + 1) > 0xffff)
            return fail(XPBD_E_CAPACITY, "mesh of %d particles is too large for the register "
                        "variant", vmax);
    }
    if (lds > (uint32_t)lds_limit)
        return fail(XPBD_E_CAPACITY, "environment needs %u bytes of LDS; the device has %d",
                    lds, lds_limit);

    auto *b = new xpbd_batch();
    b->device = device;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->params = *params;
    b->params.block_size = block;
    b->num_envs = num_envs;
    b->block = block;
    b->particles_per_thread = ppt;
    b->stage_topology = stage;
    b->register_variant = use_registers;
    b->lambda_banks = reg_rounds > 32 ? 2 : 1;
    b->envs_per_group = use_registers ? reg_group : 1;
    b->lds_bytes = lds;
    b->env_mesh.assign(env_mesh, env_mesh + num_envs);
    b->max_vertices = vmax;
    b->meshes = std::move(prepared);

    // register variant: each mesh gets the smallest block whose rounds fit the
    // register banks (every mesh fits the batch-wide choice), a number of
    // environments per workgroup and an LDS tier: the most workgroups per CU
    // its LDS and the 16 resident waves of a CU allow.  Meshes of equal
    // (block, tier, environments per workgroup) form a size class, launched
    // together; a requested block size makes one class.  With several meshes
    // and the environments per workgroup left to the library, a mesh shares
    // its workgroups between two environments where the occupancy model rates
    // that faster: environments resident per CU divided by rounds per sweep
    // (the small meshes, whose colours fill a fraction of a block, run two to
    // a workgroup in about the rounds of one).
    std::vector<int> mesh_block((size_t)num_meshes, block), mesh_class((size_t)num_meshes, 0);
    std::vector<int> mesh_group((size_t)num_meshes, reg_group);
    if (use_registers) {
        std::vector<std::array<int, 3>> keys;
        for (int32_t m = 0; m < num_meshes; ++m) {
            const PreparedMesh &pm = b->meshes[(size_t)m];
            int B = block;
            if (params->block_size == 0 && !scored) {
                for (int cand : {256, 512, 1024}) {
                    if (capsules && cand > xpbd::kMaxCapsuleBlock)
                        continue;
                    int r = count_rounds(pm, cand, reg_group);
                    r += r % 2;
                    if (r <= xpbd::kMaxRounds && reg_group * pm.num_vertices <= 16 * cand) {
                        B = cand;
                        break;
                    }
                }
            }
            int G = reg_group;
            if (num_meshes > 1 && params->envs_per_group == 0 && params->block_size == 0 &&
                !capsules) {
                double best_rate = 0.0;
                for (int g : {1, 2}) {
                    int r = count_rounds(pm, B, g);
                    r += r % 2;
                    const uint32_t lm = reg_lds(pm, g);
                    if (r > xpbd::kMaxRounds || g * pm.num_vertices > 16 * B ||
                        g * pm.num_vertices > 16384 || lm > (uint32_t)lds_limit)
                        continue;
                    const int per_cu =
                        std::max(1, std::min(16 / (B / 64), (int)((uint32_t)lds_cu / lm)));
                    const double rate = (double)(per_cu * g) / (double)std::max(r, 1);
                    if (rate > best_rate * 1.0001) {
                        best_rate = rate;
                        G = g;
                    }
                }
            }
            mesh_block[(size_t)m] = B;
            mesh_group[(size_t)m] = G;
            const uint32_t lm = reg_lds(pm, G);
            const int tier = std::max(1, std::min(16 / (B / 64), (int)((uint32_t)lds_cu / lm)));
            const std::array<int, 3> key{B, tier, G};
            auto it = std::find(keys.begin(), keys.end(), key);
            if (it == keys.end()) {
                keys.push_back(key);
                it = keys.end() - 1;
            }
            mesh_class[(size_t)m] = (int)(it - keys.begin());
        }
        b->classes.resize(keys.size());
        for (size_t c = 0; c < keys.size(); ++c) {
            b->classes[c].block = keys[c][0];
            b->classes[c].group = keys[c][2];
            b->classes[c].lds_bytes = 0;
            b->classes[c].lambda_banks = 1;
        }
        for (int32_t m = 0; m < num_meshes; ++m) {
            RegClass &c = b->classes[(size_t)mesh_class[(size_t)m]];
            const PreparedMesh &pm = b->meshes[(size_t)m];
            c.lds_bytes = std::max(c.lds_bytes, reg_lds(pm, c.group));
            int r = count_rounds(pm, c.block, c.group);
            r += r % 2;
            c.rounds = std::max(c.rounds, r);
            if (r > 32)
                c.lambda_banks = 2;
        }
    }

    auto cleanup = [&](xpbd_status st) {
        delete b;
        return st;
    };

    // per-mesh tables in schedule order, built on host threads (the meshes are
    // independent), then uploaded in mesh order
    struct MeshHost {
        MeshDev d;
        std::vector<int32_t> eslot, eptr, tslot, tptr, rr_id, nbr;
        std::vector<uint32_t> pair, round_rec;
        std::vector<float> erest, trest;
        std::vector<uint2> quad;
        std::vector<uint16_t> slot16, id16;
        std::vector<float4> rest4;
        std::vector<float> inv_count;
        std::vector<uint2> faces;         // schedule order: a | b << 16, c
        std::vector<int32_t> face_ptr;
        bool one_round_colours = true;    // register variant: no colour takes two rounds
    };
    std::vector<MeshHost> host((size_t)num_meshes);
    // the lane search costs about a second per thousand particles: the default
    // uses it while the batch's distinct meshes stay small in total
    int64_t distinct_particles = 0;
    for (const auto &pm : b->meshes)
        distinct_particles += pm.num_vertices;
    auto build = [&](int32_t m) {
        MeshHost &h = host[(size_t)m];
        const PreparedMesh &pm = b->meshes[(size_t)m];
        const int block = mesh_block[(size_t)m];
        const int32_t V = pm.num_vertices, E = pm.num_edges(), T = pm.num_tets();
        int packing = params->colour_packing;
        if (packing == XPBD_PACKING_AUTO)
            packing = !use_registers                            ? XPBD_PACKING_BANKS16
                      : distinct_particles <= kSearchParticles ? XPBD_PACKING_SEARCH
                                                                : XPBD_PACKING_SCATTERED_BANKS16;
        if ((packing == XPBD_PACKING_SCATTERED_BANKS16 || packing == XPBD_PACKING_SEARCH) &&
            !use_registers)
            packing = XPBD_PACKING_BANKS16;
        const int group = packing == XPBD_PACKING_BANKS8     ? 8
                          : packing == XPBD_PACKING_ID_ORDER ? 0
                                                             : 16;

        // one environment's schedule (LDS variant and the residual kernel): mesh ids,
        // packed for the LDS variant's identity placement
        std::vector<int32_t> &eslot = h.eslot, &eptr = h.eptr, &tslot = h.tslot, &tptr = h.tptr;
        build_schedule(pm.edge_colour, pm.num_edge_colours, eslot, eptr);
        build_schedule(pm.tet_colour, pm.num_tet_colours, tslot, tptr);
        if (!use_registers) {
            xpbd::pack_colours(pm.edges.data(), 2, eptr, group, group, eslot);
            xpbd::pack_colours(pm.tets.data(), 4, tptr, group, group, tslot);
        }
        std::vector<uint32_t> &pair = h.pair;
        std::vector<float> &erest = h.erest, &trest = h.trest;
        std::vector<uint2> &quad = h.quad;
        pair.resize((size_t)E);
        erest.resize((size_t)E);
        trest.resize((size_t)T);
        quad.resize((size_t)T);
        for (int32_t j = 0; j < E; ++j) {
            const int32_t e = eslot[(size_t)j];
            pair[(size_t)j] = (uint32_t)pm.edges[2 * (size_t)e] |
                              ((uint32_t)pm.edges[2 * (size_t)e + 1] << 16);
            erest[(size_t)j] = (float)pm.rest_length[(size_t)e];
        }
        for (int32_t j = 0; j < T; ++j) {
            const int32_t t = tslot[(size_t)j];
            const int32_t *q = &pm.tets[4 * (size_t)t];
            quad[(size_t)j] = make_uint2((uint32_t)q[0] | ((uint32_t)q[1] << 16),
                                         (uint32_t)q[2] | ((uint32_t)q[3] << 16));
            trest[(size_t)j] = (float)pm.rest_volume[(size_t)t];
        }

        // register variant: a group of G copies of the mesh (group particle e V + i,
        // group constraint e E + j / e T + j), its LDS placement, lane packing and
        // round-major record tables with per-wave activity and the kind / barrier
        // masks of the round schedule
        const int G = use_registers ? mesh_group[(size_t)m] : 1;
        const int32_t GV = G * V;
        std::vector<int32_t> gedges((size_t)G * E * 2), gtets((size_t)G * T * 4);
        std::vector<int32_t> gecol((size_t)G * E), gtcol((size_t)G * T);
        for (int e = 0; e < G; ++e) {
            for (int32_t j = 0; j < E; ++j) {
                gecol[(size_t)e * E + j] = pm.edge_colour[(size_t)j];
                for (int k = 0; k < 2; ++k)
                    gedges[((size_t)e * E + j) * 2 + k] = pm.edges[2 * (size_t)j + k] + e * V;
            }
            for (int32_t j = 0; j < T; ++j) {
                gtcol[(size_t)e * T + j] = pm.tet_colour[(size_t)j];
                for (int k = 0; k < 4; ++k)
                    gtets[((size_t)e * T + j) * 4 + k] = pm.tets[4 * (size_t)j + k] + e * V;
            }
        }
        std::vector<int32_t> geslot, geptr, gtslot, gtptr;
        build_schedule(gecol, pm.num_edge_colours, geslot, geptr);
        build_schedule(gtcol, pm.num_tet_colours, gtslot, gtptr);
        std::vector<int32_t> slot_of((size_t)GV);
        std::iota(slot_of.begin(), slot_of.end(), 0);
        std::vector<uint8_t> eorder(geslot.size(), 0), torder(gtslot.size(), 0);
        if (use_registers) {
            if (packing == XPBD_PACKING_SCATTERED_BANKS16 || packing == XPBD_PACKING_SEARCH) {
                std::mt19937 gen(0x5eedu + (uint32_t)m);
                std::shuffle(slot_of.begin(), slot_of.end(), gen);
            }
            if (packing == XPBD_PACKING_SEARCH) {
                xpbd::LaneSchedule kinds[2] = {
                    {gedges.data(), 2, &geptr, &geslot, &eorder},
                    {gtets.data(), 4, &gtptr, &gtslot, &torder}};
                xpbd::pack_lds(GV, slot_of, kinds, 2, 0x9e37u + (uint32_t)m, kLaneSearchEffort);
            } else {
                std::vector<int32_t> e_lds(gedges.size()), t_lds(gtets.size());
                for (size_t q = 0; q < gedges.size(); ++q)
                    e_lds[q] = slot_of[(size_t)gedges[q]];
                for (size_t q = 0; q < gtets.size(); ++q)
                    t_lds[q] = slot_of[(size_t)gtets[q]];
                xpbd::pack_colours(e_lds.data(), 2, geptr, group, group, geslot);
                xpbd::pack_colours(t_lds.data(), 4, gtptr, group, group, gtslot);
            }
        }
        std::vector<uint16_t> &slot16 = h.slot16, &id16 = h.id16;
        slot16.resize((size_t)GV);
        id16.resize((size_t)GV);
        for (int32_t i = 0; i < GV; ++i) {
            slot16[(size_t)i] = (uint16_t)slot_of[(size_t)i];
            id16[(size_t)slot_of[(size_t)i]] = (uint16_t)i;
        }
        std::vector<int4> rounds;
        build_rounds(geptr, gtptr, block, rounds);
        // the kernel runs the edge rounds and the tetrahedron rounds in loops of
        // their own, both in pairs: pad each with an empty round to an even count
        int32_t edge_rounds = 0;
        for (const int4 &rd : rounds)
            edge_rounds += rd.z == xpbd::ROUND_EDGE ? 1 : 0;
        if (edge_rounds % 2)
            rounds.insert(rounds.begin() + edge_rounds++, make_int4(0, 0, xpbd::ROUND_EDGE, 0));
        if (rounds.size() % 2)
            rounds.push_back(make_int4(0, 0, xpbd::ROUND_TET, 0));
        const int32_t num_rounds = (int32_t)rounds.size();
        // two rows beyond the last round repeat rounds 0 and 1: the kernel
        // fetches the record of round r + 2 in round r without wrapping
        std::vector<uint32_t> &round_rec = h.round_rec;
        round_rec.assign(((size_t)std::max(num_rounds, 1) + 2) * block * 3, 0u);
        // particle fields: LDS byte offsets with one environment per workgroup,
        // slot indices (16 bytes each) with more
        // (16 (G V + 1) <= 65535: checked where the variant is chosen)
        const uint32_t unit = G == 1 ? 16u : 1u;
        const uint32_t pad = (uint32_t)GV * unit | ((uint32_t)GV * unit << 16);   // padding particle
        for (size_t q = 0; q < round_rec.size(); q += 3)
            round_rec[q] = pad;
        std::vector<int32_t> &rr_id = h.rr_id;
        rr_id.assign((size_t)std::max(num_rounds, 1) * block, -1);
        MeshDev &d = h.d;
        std::memset(&d, 0, sizeof d);
        // With fewer waves per workgroup than a CU has SIMDs, the 64-lane
        // blocks of a round go to the waves that have worked least so far (a
        // tetrahedron round counts three edge rounds): colours that fill only
        // some of the waves then spread their work over every wave of the
        // workgroup instead of always loading its first one.  Whole blocks
        // move, so the bank-conflict pattern of each wave's accesses and the
        // results stay the same.  Measured (same box, alternating runs): +4.2 %
        // on the 12x8x3 slab's 128-thread workgroups, -0.8 % on the 16x10x4
        // slab's 256-thread ones, whose four waves already cover the SIMDs.
        const int num_waves = block / 64;
        const bool rotate = num_waves < 4;
        std::vector<int64_t> wave_load((size_t)num_waves, 0);
        std::vector<int> wave_order((size_t)num_waves);
        for (int32_t r = 0; r < num_rounds && use_registers; ++r) {
            const int4 rd = rounds[(size_t)r];
            const bool is_edge = r < edge_rounds;
            const int32_t n = rd.y - rd.x;
            std::iota(wave_order.begin(), wave_order.end(), 0);
            if (rotate)
                std::stable_sort(wave_order.begin(), wave_order.end(), [&](int a, int c) {
                    return wave_load[(size_t)a] < wave_load[(size_t)c];
                });
            for (int k = 0; k < (n + 63) / 64 && k < num_waves; ++k)
                wave_load[(size_t)wave_order[(size_t)k]] += is_edge ? 1 : 3;
            auto lane_of = [&](int32_t l) { return wave_order[(size_t)(l / 64)] * 64 + l % 64; };
            for (int32_t l = 0; l < block && !is_edge; ++l)
                round_rec[((size_t)r * block + l) * 3 + 1] = pad;   // tet padding: c = d = pad
            for (int32_t l = 0; l < block && rd.x + l < rd.y; ++l) {
                const int32_t j = rd.x + l;   // slot within its kind
                const int32_t pl = lane_of(l);
                uint32_t *at = &round_rec[((size_t)r * block + pl) * 3];
                if (is_edge) {
                    const int32_t q = geslot[(size_t)j], e = q / E, id = q - e * E;
                    const uint8_t *o = xpbd::vertex_order(2, eorder[(size_t)q]);
                    const uint32_t a = unit * (uint32_t)slot_of[(size_t)gedges[2 * (size_t)q + o[0]]];
                    const uint32_t bb = unit * (uint32_t)slot_of[(size_t)gedges[2 * (size_t)q + o[1]]];
                    const float rest = (float)pm.rest_length[(size_t)id];
                    at[0] = a | (bb << 16) | ((uint32_t)e << 30);
                    std::memcpy(&at[1], &rest, 4);
                    at[2] = 0u;
                    rr_id[(size_t)r * block + pl] = (e << 24) | id;
                } else {
                    const int32_t q = gtslot[(size_t)j], e = q / T, id = q - e * T;
                    const uint8_t *o = xpbd::vertex_order(4, torder[(size_t)q]);
                    uint32_t v[4];
                    for (int k = 0; k < 4; ++k)
                        v[k] = unit * (uint32_t)slot_of[(size_t)gtets[4 * (size_t)q + o[k]]];
                    const float rest = (float)pm.rest_volume[(size_t)id];
                    at[0] = v[0] | (v[1] << 16) | ((uint32_t)e << 30);
                    at[1] = v[2] | (v[3] << 16);
                    std::memcpy(&at[2], &rest, 4);
                    rr_id[(size_t)r * block + pl] = (e << 24) | (E + id);
                }
                d.wave_active[pl / 64] |= 1ull << r;
            }
            if (!is_edge)
                d.tet_mask |= 1ull << r;
            if (rd.w)
                d.barrier_mask |= 1ull << r;
            else if (rd.y > rd.x)
                h.one_round_colours = false;   // a colour continues in the next round
        }
        if (num_rounds >= 2)
            std::copy(round_rec.begin(), round_rec.begin() + (size_t)2 * block * 3,
                      round_rec.begin() + (size_t)num_rounds * block * 3);
        d.num_rounds = use_registers ? num_rounds : 0;
        d.num_edge_rounds = edge_rounds;
        d.num_vertices = V;
        d.num_edges = E;
        d.num_tets = T;
        d.num_edge_colours = pm.num_edge_colours;
        d.num_tet_colours = pm.num_tet_colours;
        {
            std::vector<int32_t> fslot;
            build_schedule(pm.face_colour, pm.num_face_colours, fslot, h.face_ptr);
            h.faces.resize(fslot.size());
            for (size_t j = 0; j < fslot.size(); ++j) {
                const int32_t *f = &pm.faces[3 * (size_t)fslot[j]];
                h.faces[j] = make_uint2((uint32_t)f[0] | ((uint32_t)f[1] << 16), (uint32_t)f[2]);
            }
        }
        h.inv_count.assign((size_t)V, 0.0f);
        {
            std::vector<int32_t> n((size_t)V, 0);
            for (int32_t q = 0; q < 2 * E; ++q)
                n[(size_t)pm.edges[(size_t)q]]++;
            for (int32_t q = 0; q < 4 * T; ++q)
                n[(size_t)pm.tets[(size_t)q]]++;
            for (int32_t i = 0; i < V; ++i)
                h.inv_count[(size_t)i] = n[(size_t)i] > 0 ? 1.0f / (float)n[(size_t)i] : 0.0f;
        }
        xpbd::axis_neighbours(V, pm.rest_pos.data(), h.nbr);
        h.rest4.resize((size_t)V);
        for (int i = 0; i < V; ++i)
            h.rest4[(size_t)i] = make_float4(pm.rest_pos[3 * (size_t)i], pm.rest_pos[3 * (size_t)i + 1],
                                             pm.rest_pos[3 * (size_t)i + 2], pm.inv_mass[(size_t)i]);
    };
    {
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        const int workers = (int)std::min<unsigned>(hw, (unsigned)num_meshes);
        std::atomic<int> next{0};
        std::atomic<bool> failed{false};
        auto work = [&]() {
            for (int m; (m = next.fetch_add(1)) < num_meshes;) {
                try {
                    build(m);
                } catch (...) {
                    failed = true;
                }
            }
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < workers; ++t)
            pool.emplace_back(work);
        work();
        for (auto &t : pool)
            t.join();
        if (failed)
            return cleanup(fail(XPBD_E_ARG, "out of host memory while building the mesh tables"));
    }
    std::vector<MeshDev> mdev((size_t)num_meshes);
    for (int32_t m = 0; m < num_meshes; ++m) {
        const PreparedMesh &pm = b->meshes[(size_t)m];
        MeshHost &h = host[(size_t)m];
        MeshDev &d = mdev[(size_t)m];
        d = h.d;
        uint32_t *p_pair;
        float *p_erest, *p_trest, *p_w;
        uint2 *p_quad;
        int32_t *p_eptr, *p_tptr, *p_eid, *p_tid;
        xpbd_status st;
        float *p_rest;
        int32_t *p_nbr;
        float4 *p_rest4;
        float *p_inv_count;
        if ((st = b->upload(&p_rest, pm.rest_pos)) || (st = b->upload(&p_nbr, h.nbr)) ||
            (st = b->upload(&p_rest4, h.rest4)) || (st = b->upload(&p_inv_count, h.inv_count)))
            return cleanup(st);
        d.inv_count = p_inv_count;
        uint2 *p_faces;
        int32_t *p_face_ptr;
        if ((st = b->upload(&p_faces, h.faces)) || (st = b->upload(&p_face_ptr, h.face_ptr)))
            return cleanup(st);
        d.faces = p_faces;
        d.face_ptr = p_face_ptr;
        d.num_faces = pm.num_faces();
        d.num_face_colours = pm.num_face_colours;
        d.rest_pos = p_rest;
        d.nbr = p_nbr;
        d.rest4 = p_rest4;
        if ((st = b->upload(&p_pair, h.pair)) || (st = b->upload(&p_erest, h.erest)) ||
            (st = b->upload(&p_quad, h.quad)) || (st = b->upload(&p_trest, h.trest)) ||
            (st = b->upload(&p_eptr, h.eptr)) || (st = b->upload(&p_tptr, h.tptr)) ||
            (st = b->upload(&p_eid, h.eslot)) || (st = b->upload(&p_tid, h.tslot)) ||
            (st = b->upload(&p_w, pm.inv_mass)))
            return cleanup(st);
        uint32_t *p_rr;
        int32_t *p_rrid;
        uint16_t *p_slot, *p_id;
        if ((st = b->upload(&p_rr, h.round_rec)) || (st = b->upload(&p_rrid, h.rr_id)) ||
            (st = b->upload(&p_slot, h.slot16)) || (st = b->upload(&p_id, h.id16)))
            return cleanup(st);
        if (use_registers && !h.one_round_colours)
            b->classes[(size_t)mesh_class[(size_t)m]].round_barriers = false;
        d.round_rec = p_rr;
        d.rr_id = p_rrid;
        d.slot_of = p_slot;
        d.id_of = p_id;
        d.edge_pair = p_pair;
        d.edge_rest = p_erest;
        d.tet_quad = p_quad;
        d.tet_rest = p_trest;
        d.edge_ptr = p_eptr;
        d.tet_ptr = p_tptr;
        d.edge_id = p_eid;
        d.tet_id = p_tid;
        d.inv_mass = p_w;
        b->colours.insert(b->colours.end(), pm.edge_colour.begin(), pm.edge_colour.end());
        b->colours.insert(b->colours.end(), pm.tet_colour.begin(), pm.tet_colour.end());
        host[(size_t)m] = MeshHost();   // release the host tables
    }

    // workgroups of the register variant, per size class: environments of one
    // mesh, G at a time; meshes with more constraints first, so the longest
    // workgroups start first; a group left short repeats its last environment
    // as filler (~env)
    if (use_registers) {
        std::vector<int32_t> order((size_t)num_meshes);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
            const PreparedMesh &px = b->meshes[(size_t)x], &py = b->meshes[(size_t)y];
            return px.num_edges() + px.num_tets() > py.num_edges() + py.num_tets();
        });
        std::vector<std::vector<int32_t>> mine((size_t)num_meshes);
        for (int32_t e = 0; e < num_envs; ++e)
            mine[(size_t)env_mesh[e]].push_back(e);
        for (size_t c = 0; c < b->classes.size(); ++c) {
            const int G = b->classes[c].group;
            std::vector<int32_t> groups;
            for (int32_t m : order) {
                if (mesh_class[(size_t)m] != (int)c)
                    continue;
                const std::vector<int32_t> &v = mine[(size_t)m];
                for (size_t k = 0; k < v.size(); k += (size_t)G)
                    for (int f = 0; f < G; ++f)
                        groups.push_back(k + (size_t)f < v.size() ? v[k + (size_t)f] : ~v.back());
            }
            RegClass &rc = b->classes[c];
            rc.num_groups = (int32_t)(groups.size() / (size_t)G);
            xpbd_status st = b->upload(&rc.groups_dev, groups);
            if (st != XPBD_OK)
                return cleanup(st);
        }
        // streams of a multi-class step: the classes, largest estimated work
        // first (passes of their workgroups over the CUs at their occupancy,
        // times rounds per sweep), each to the stream with the least work so
        // far, the batch's own stream first
        const int ncls = (int)b->classes.size();
        b->class_order.resize((size_t)ncls);
        std::iota(b->class_order.begin(), b->class_order.end(), 0);
        if (ncls > 1) {
            const int cus = num_cus;
            std::vector<double> est((size_t)ncls, 0.0);
            for (int c = 0; c < ncls; ++c) {
                const RegClass &rc = b->classes[(size_t)c];
                const int waves = rc.block / 64;
                const int per_cu = std::max(1, std::min(16 / std::max(waves, 1),
                                                        (int)((uint32_t)lds_cu /
                                                              std::max(rc.lds_bytes, 1u))));
                const int64_t slots = (int64_t)per_cu * std::max(cus, 1);
                const int64_t passes = (rc.num_groups + slots - 1) / slots;
                est[(size_t)c] = (double)passes * (double)rc.rounds;
            }
            std::stable_sort(b->class_order.begin(), b->class_order.end(),
                             [&](int x, int y) { return est[(size_t)x] > est[(size_t)y]; });
            const int nl = std::min(ncls, kClassLanes);
            std::vector<double> load((size_t)nl, 0.0);
            for (int c : b->class_order) {
                if (b->classes[(size_t)c].num_groups == 0)
                    continue;
                int best = 0;
                for (int l = 1; l < nl; ++l)
                    if (load[(size_t)l] < load[(size_t)best])
                        best = l;
                load[(size_t)best] += est[(size_t)c];
                b->classes[(size_t)c].lane = best;
            }
            hipError_t he = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
            for (int l = 1; l < nl && he == hipSuccess; ++l) {
                hipStream_t ls = nullptr;
                hipEvent_t ev = nullptr;
                he = hipStreamCreateWithFlags(&ls, hipStreamNonBlocking);
                if (he == hipSuccess)
                    b->lanes.push_back(ls);   // the batch destroys what it holds
                if (he == hipSuccess)
                    he = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
                if (he == hipSuccess)
                    b->lane_done.push_back(ev);
            }
            if (he != hipSuccess)
                return cleanup(fail(XPBD_E_HIP, "creating the class streams failed: %s",
                                    hipGetErrorString(he)));
        }
        // the single-class fields of the batch (the learned step needs one class)
        b->groups_dev = b->classes[0].groups_dev;
        b->num_groups = b->classes[0].num_groups;
        b->block = b->classes[0].block;
        b->lds_bytes = b->classes[0].lds_bytes;
        b->lambda_banks = b->classes[0].lambda_banks;
        b->envs_per_group = b->classes[0].group;
        for (const RegClass &c : b->classes)
            b->envs_per_group = std::max(b->envs_per_group, c.group);
    }

    // environments
    std::vector<EnvDev> edev((size_t)num_envs);
    b->env_offsets.assign((size_t)num_envs + 1, 0);
    int64_t np = 0, nl = 0;
    for (int32_t e = 0; e < num_envs; ++e) {
        const PreparedMesh &pm = b->meshes[(size_t)env_mesh[e]];
        edev[(size_t)e] = EnvDev{env_mesh[e], (int32_t)np, (int32_t)nl, 0};
        b->env_offsets[(size_t)e] = (int32_t)np;
        np += pm.num_vertices;
        nl += pm.num_edges() + pm.num_tets();
        if (np > INT32_MAX / 3 || nl > INT32_MAX)
            return cleanup(fail(XPBD_E_CAPACITY, "batch too large: %lld particles", (long long)np));
    }
    b->env_offsets[(size_t)num_envs] = (int32_t)np;
    b->total_particles = (int32_t)np;
    b->total_lambda = (int32_t)nl;

    // initial state: rest positions, zero velocity (structure of arrays)
    std::vector<float> pos_soa((size_t)(3 * np));
    for (int32_t e = 0; e < num_envs; ++e) {
        const PreparedMesh &pm = b->meshes[(size_t)env_mesh[e]];
        const size_t off = (size_t)b->env_offsets[(size_t)e];
        for (int32_t i = 0; i < pm.num_vertices; ++i)
            for (int k = 0; k < 3; ++k)
                pos_soa[(size_t)k * (size_t)np + off + (size_t)i] = pm.rest_pos[3 * (size_t)i + k];
    }
    std::vector<float> zeros_f((size_t)(3 * np), 0.0f);
    std::vector<float> comp(compliance, compliance + 2 * (size_t)num_envs);
    std::vector<int32_t> zeros_env((size_t)num_envs, 0);
    const size_t tools = (size_t)params->num_tools;
    std::vector<int32_t> no_contacts(tools * (size_t)np, -1), no_counts(tools * (size_t)num_envs, 0);
    std::vector<float> resid((size_t)num_envs * 2, 0.0f);
    std::vector<float> lam_init((size_t)nl, 0.0f);
    xpbd_status st;
    if ((st = b->upload(&b->meshes_dev, mdev)) || (st = b->upload(&b->envs_dev, edev)) ||
        (st = b->upload(&b->pos, pos_soa)) || (st = b->upload(&b->vel, zeros_f)) ||
        (st = b->upload(&b->compliance, comp)) || (st = b->upload(&b->nonfinite, zeros_env)) ||
        (st = b->upload(&b->contacts, no_contacts)) ||
        (st = b->upload(&b->contact_counts, no_counts)) ||
        (st = b->upload(&b->residual, resid)) ||
        (st = b->alloc(reinterpret_cast<void **>(&b->staging), 3 * (size_t)np * sizeof(float))))
        return cleanup(st);
    b->staging_bytes = 3 * (size_t)np * sizeof(float);
    // the register variant hands its multipliers to the residual kernel through this buffer
    if ((params->flags & XPBD_F_LAMBDA) ||
        (use_registers && (params->flags & XPBD_F_RESIDUAL)))
        if ((st = b->upload(&b->lambda, lam_init)))
            return cleanup(st);
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess)
        return cleanup(fail(XPBD_E_HIP, "hipStreamSynchronize failed: %s", hipGetErrorString(e)));
    *out = b;
    return XPBD_OK;
}

xpbd_status xpbd_step(xpbd_batch *b, int32_t num_steps, const float *tool_pos,
                      size_t tool_pos_bytes)
{
    g_error.clear();
    if (!b)
        return fail(XPBD_E_ARG, "batch is NULL");
    if (num_steps < 0)
        return fail(XPBD_E_ARG, "num_steps must be >= 0");
    if (num_steps == 0)
        return XPBD_OK;
    const xpbd_status checked = xpbd::check_tool_bytes(b, num_steps, tool_pos, tool_pos_bytes);
    if (checked != XPBD_OK)
        return checked;
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
    return xpbd::run_step(b, num_steps, tools_dev, nullptr);
}

}  // extern "C"

size_t xpbd::tool_bytes(const xpbd_batch *b, int32_t num_steps)
{
    const size_t per_tool = b->params.tool_shape == XPBD_TOOL_CAPSULE ? 6 : 3;
    const size_t tools = b->params.num_tools > 0 ? (size_t)b->params.num_tools : 0;
    return (size_t)(num_steps > 0 ? num_steps : 0) * (size_t)b->num_envs * tools * per_tool *
           sizeof(float);
}

xpbd_status xpbd::check_tool_bytes(const xpbd_batch *b, int32_t num_steps, const float *tool_pos,
                                   size_t tool_pos_bytes)
{
    const int tools = b->params.num_tools;
    if (tools <= 0 || num_steps <= 0)
        return XPBD_OK;
    if (!tool_pos)
        return fail(XPBD_E_ARG, "tool_pos is NULL but the batch has %d tools", tools);
    const size_t want = tool_bytes(b, num_steps);
    if (tool_pos_bytes != want)
        return fail(XPBD_E_ARG, "tool_pos holds %zu bytes; %d steps of %d environments with %d "
                    "tools read %zu", tool_pos_bytes, num_steps, b->num_envs, tools, want);
    return XPBD_OK;
}

// The launches of num_steps steps with the tool poses in device memory; the
// RL-style step passes its grasp state (register variant only).
xpbd_status xpbd::run_step(xpbd_batch *b, int32_t num_steps, const float *tools_dev,
                           const GraspArgs *grasp)
{
    const int tools = b->params.num_tools;
    xpbd::StepArgs a;
    std::memset(&a, 0, sizeof a);
    a.meshes = b->meshes_dev;
    a.envs = b->envs_dev;
    a.groups = b->groups_dev;
    a.num_groups = b->num_groups;
    a.compliance = b->compliance;
    a.tool_pos = tools_dev;
    a.pos = b->pos;
    a.vel = b->vel;
    const bool resid_now = (b->params.flags & XPBD_F_RESIDUAL) != 0;
    a.lambda_out = ((b->params.flags & XPBD_F_LAMBDA) || (b->register_variant && resid_now))
                       ? b->lambda : nullptr;
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
    a.tool_shape = b->params.tool_shape;
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
    const bool resid = (b->params.flags & XPBD_F_RESIDUAL) != 0;
    b->residual_valid = b->residual_valid || resid;
    if (b->register_variant && b->classes.size() == 1) {
        const RegClass &c = b->classes[0];
        a.groups = c.groups_dev;
        a.num_groups = c.num_groups;
        a.round_barriers = c.round_barriers ? 1 : 0;
        HIP_TRY(xpbd::launch_step_reg(a, c.block, c.lambda_banks, c.group, c.lds_bytes,
                                      resid, b->stream));
    } else if (b->register_variant) {
        // one launch per size class, largest first, on the batch's stream and
        // the lanes forked from it, joined before the residual
        HIP_TRY(hipEventRecord(b->fork, b->stream));
        for (hipStream_t l : b->lanes)
            HIP_TRY(hipStreamWaitEvent(l, b->fork, 0));
        for (int ci : b->class_order) {
            const RegClass &c = b->classes[(size_t)ci];
            if (c.num_groups == 0)
                continue;
            a.groups = c.groups_dev;
            a.num_groups = c.num_groups;
            a.round_barriers = c.round_barriers ? 1 : 0;
            HIP_TRY(xpbd::launch_step_reg(a, c.block, c.lambda_banks, c.group, c.lds_bytes,
                                          false,
                                          c.lane == 0 ? b->stream : b->lanes[(size_t)c.lane - 1]));
        }
        for (size_t l = 0; l < b->lanes.size(); ++l) {
            HIP_TRY(hipEventRecord(b->lane_done[l], b->lanes[l]));
            HIP_TRY(hipStreamWaitEvent(b->stream, b->lane_done[l], 0));
        }
        if (resid)
            HIP_TRY(xpbd::launch_residual(a, b->stream));
    } else
        HIP_TRY(xpbd::launch_step(a, b->block, b->particles_per_thread,
                                  b->params.solver_variant == XPBD_VARIANT_JACOBI, b->stage_topology,
                                  b->lds_bytes, resid, b->stream));
    return XPBD_OK;
}

extern "C" {

xpbd_status xpbd_set_flags(xpbd_batch *b, uint32_t flags)
{
    g_error.clear();
    if (!b)
        return fail(XPBD_E_ARG, "batch is NULL");
    if (flags & ~(XPBD_F_RESIDUAL | XPBD_F_LAMBDA))
        return fail(XPBD_E_ARG, "unknown flag bits 0x%x", flags);
    const bool need_lambda = (flags & XPBD_F_LAMBDA) ||
                             (b->register_variant && (flags & XPBD_F_RESIDUAL));
    if (need_lambda && !b->lambda) {
        HIP_TRY(hipStreamSynchronize(b->stream));
        std::vector<float> zeros((size_t)b->total_lambda, 0.0f);
        xpbd_status s = b->upload(&b->lambda, zeros);
        if (s != XPBD_OK)
            return s;
    }
    b->params.flags = flags;
    return XPBD_OK;
}

xpbd_status xpbd_field_bytes(const xpbd_batch *b, int32_t field, size_t *bytes)
{
    g_error.clear();
    if (!b || !bytes)
        return fail(XPBD_E_ARG, "batch and bytes must not be NULL");
    return field_bytes(b, field, bytes);
}

xpbd_status xpbd_read_state(xpbd_batch *b, int32_t field, void *dst, size_t dst_bytes)
{
    g_error.clear();
    if (!b || !dst)
        return fail(XPBD_E_ARG, "batch and dst must not be NULL");
    size_t need = 0;
    xpbd_status s = field_bytes(b, field, &need);
    if (s != XPBD_OK)
        return s;
    if (dst_bytes != need)
        return fail(XPBD_E_STATE, "field %d needs %zu bytes, got %zu", field, need, dst_bytes);
    if (field == XPBD_FIELD_LAMBDA && !(b->params.flags & XPBD_F_LAMBDA))
        return fail(XPBD_E_STATE, "multipliers are stored only with XPBD_F_LAMBDA");
    if (field == XPBD_FIELD_RESIDUAL && !b->residual_valid)
        return fail(XPBD_E_STATE, "no xpbd_step with XPBD_F_RESIDUAL has run on this batch");
    switch (field) {
    case XPBD_FIELD_COLOURS:
        s = copy_host_out(b, dst, b->colours.data(), need);
        if (s != XPBD_OK)
            return s;
        break;
    case XPBD_FIELD_ENV_OFFSETS:
        s = copy_host_out(b, dst, b->env_offsets.data(), need);
        if (s != XPBD_OK)
            return s;
        break;
    case XPBD_FIELD_POS:
    case XPBD_FIELD_VEL:
        HIP_TRY(xpbd::launch_soa_to_aos(field == XPBD_FIELD_POS ? b->pos : b->vel, b->staging,
                                        b->total_particles, b->stream));
        HIP_TRY(hipMemcpyAsync(dst, b->staging, need, hipMemcpyDefault, b->stream));
        break;
    default: {
        const void *src = field == XPBD_FIELD_LAMBDA           ? (const void *)b->lambda
                          : field == XPBD_FIELD_CONTACTS       ? (const void *)b->contacts
                          : field == XPBD_FIELD_CONTACT_COUNTS ? (const void *)b->contact_counts
                          : field == XPBD_FIELD_RESIDUAL       ? (const void *)b->residual
                                                               : (const void *)b->nonfinite;
        if (need)
            HIP_TRY(hipMemcpyAsync(dst, src, need, hipMemcpyDefault, b->stream));
    }
    }
    std::vector<int32_t> flags((size_t)b->num_envs);
    HIP_TRY(hipMemcpyAsync(flags.data(), b->nonfinite, flags.size() * sizeof(int32_t),
                           hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (size_t e = 0; e < flags.size(); ++e)
        if (flags[e])
            return fail(XPBD_E_NONFINITE, "environment %zu has a non-finite state", e);
    return XPBD_OK;
}

xpbd_status xpbd_write_state(xpbd_batch *b, int32_t field, const void *src, size_t src_bytes)
{
    g_error.clear();
    if (!b || !src)
        return fail(XPBD_E_ARG, "batch and src must not be NULL");
    if (field != XPBD_FIELD_POS && field != XPBD_FIELD_VEL)
        return fail(XPBD_E_STATE, "only positions and velocities can be written");
    size_t need = 0;
    xpbd_status s = field_bytes(b, field, &need);
    if (s != XPBD_OK)
        return s;
    if (src_bytes != need)
        return fail(XPBD_E_STATE, "field %d needs %zu bytes, got %zu", field, need, src_bytes);
    HIP_TRY(hipMemcpyAsync(b->staging, src, need, hipMemcpyDefault, b->stream));
    HIP_TRY(xpbd::launch_aos_to_soa(b->staging, field == XPBD_FIELD_POS ? b->pos : b->vel,
                                    b->total_particles, b->stream));
    HIP_TRY(hipMemsetAsync(b->nonfinite, 0, (size_t)b->num_envs * sizeof(int32_t), b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return XPBD_OK;
}

void xpbd_destroy_batch(xpbd_batch *b) { delete b; }

}  // extern "C"
