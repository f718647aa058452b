// Device-side data layout of the XPBD library, shared by the runtime (host)
// and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace xpbd {

// One distinct mesh, in the order the kernel consumes it.  Constraint arrays
// are in schedule order: colour-major, constraint id ascending inside a colour.
struct MeshDev {
    int32_t num_vertices;
    int32_t num_edges;
    int32_t num_tets;
    int32_t num_edge_colours;
    int32_t num_tet_colours;
    int32_t pad[3];
    const uint32_t *edge_pair;   // [E]  a | b << 16 (local particle ids)
    const float *edge_rest;      // [E]  rest length
    const uint2 *tet_quad;       // [T]  (a | b << 16, c | d << 16), oriented
    const float *tet_rest;       // [T]  rest volume
    const int32_t *edge_ptr;     // [edge colours + 1] schedule offsets
    const int32_t *tet_ptr;      // [tet colours + 1]
    const int32_t *edge_id;      // [E]  constraint id of each schedule slot
    const int32_t *tet_id;       // [T]
    const float *inv_mass;       // [V]
    const float *rest_pos;       // [V][3] (learned warm start's features)
    const int32_t *nbr;          // [V][6] axis neighbours -x, +x, -y, +y, -z, +z, -1 for none
    const float4 *rest4;         // [V] (rest position, inverse mass)
    const float *inv_count;      // [V] 1 / (kept constraints that include the particle), 0 if none
    const uint2 *faces;          // [F] surface triangles in schedule order (a | b << 16, c)
    const int32_t *face_ptr;     // [face colours + 1]
    int32_t num_faces;
    int32_t num_face_colours;
    // particle placement of the register-multiplier kernel for a group of G
    // environments: particle i of the group's e-th environment (group id
    // e V + i) lives in LDS slot slot_of[e V + i]; records name slots
    const uint16_t *slot_of;     // [G V]
    const uint16_t *id_of;       // [G V]  inverse of slot_of
    // round-major records of the register-multiplier kernel: the record of
    // lane l in round r sits at [r][l]; particles as LDS byte offsets with one
    // environment per workgroup, as slot indices with more; edge (pair, rest
    // length bits, 0),
    // tet (ab, cd, rest volume bits); the top two bits of the first word hold
    // the environment index within the group; lanes without a constraint hold
    // a padding record whose slots all name slot G V (an LDS particle at the
    // origin with zero inverse mass, so its projections change nothing), rest 0
    const uint32_t *round_rec;   // [padded rounds + 2][block][3], the last two rows = rows 0, 1
    const int32_t *rr_id;        // [padded rounds][block] e << 24 | constraint id (tets: E + id), -1
    uint64_t wave_active[16];    // bit r: wave w has a constraint in round r
    uint64_t tet_mask;           // bit r: round r projects tetrahedra
    uint64_t barrier_mask;       // bit r: a workgroup barrier follows round r
    int32_t num_rounds;          // padded to an even count (<= kMaxRounds)
    int32_t num_edge_rounds;     // rounds 0 .. num_edge_rounds - 1 project edges (an even count)
    int32_t pad2[2];
};


// Rounds of the register-multiplier kernel: a colour is cut into rounds of at
// most blockDim constraints (lane l takes the l-th); a workgroup barrier
// follows the last round of a colour.  Each lane keeps the multiplier of its
// constraint of round r in register r.
enum { ROUND_EDGE = 0, ROUND_TET = 1 };
constexpr int kMaxRounds = 64;

struct EnvDev {
    int32_t mesh;
    int32_t particle_offset;     // into the concatenated particle arrays
    int32_t lambda_offset;       // into the concatenated multiplier array
    int32_t pad;
};

struct StepArgs {
    const MeshDev *meshes;
    const EnvDev *envs;
    const int32_t *groups;       // register variant: [num_groups][G] env ids, ~env = filler
    int32_t num_groups;
    const float *compliance;     // [N][2] (edge, tet)
    const float *tool_pos;       // [num_steps][N][num_tools][3]
    float *pos;                  // [3][total_particles]  SoA
    float *vel;                  // [3][total_particles]  SoA
    float *lambda_out;           // [sum (E+T)] or null
    int32_t *contacts;           // [num_tools][total_particles]
    int32_t *contact_counts;     // [N][num_tools]
    float *residual;             // [N][2] or null
    int32_t *nonfinite;          // [N]
    int32_t num_envs;
    int32_t total_particles;
    int32_t num_steps;
    int32_t substeps;
    int32_t iterations;
    int32_t num_tools;
    int32_t tool_shape;          // XPBD_TOOL_SPHERE or XPBD_TOOL_CAPSULE (p0, p1 per tool)
    float h;                     // dt / substeps
    float inv_h;
    float gravity[3];
    float tool_radius[2];
    float tool_radius2[2];       // r^2
    float tool_reach2[2];        // (2r)^2, rounded to float
    // grasping (register variant; null: no grasper): per environment the
    // particle tool 0 holds (id within the environment), -1 for none, -2 for
    // a closed grasper that holds nothing yet (the kernel then takes the free
    // particle closest to tool 0's centre + grasp_offset strictly within
    // sqrt(grasp_radius2) and writes its id, or -1)
    int32_t *grasp;
    float grasp_offset[3];
    float grasp_radius2;
    // register variant: 1 when every colour of every mesh of the launch is one
    // round, so that a barrier closes every round (no test of barrier_mask)
    int32_t round_barriers;
};

// Arguments of the learned warm start's per-substep kernels (one substep per
// launch; see include/xpbd_learned.h).
struct LearnedArgs {
    float *xhat;                 // [3][total particles] predicted (then corrected) positions
    uint16_t *features;          // [total particles][32] bfloat16 scaled features, [31] = free flag
    uint16_t *next_features;     // the substep kernel writes the next substep's prediction to
                                 // xhat and its features here when set
    uint8_t *cand;               // [total particles] bit t: candidate of tool t in this step
    const float *in_shift;       // [32] features are (f - in_shift) * in_scale
    const float *in_scale;       // [32]
    const float *out_shift;      // [4]
    const float *out_scale;      // [4]
    float *record_targets;       // [total particles][4] (x - x_hat - out_shift) / out_scale, or null
    int32_t *iterations;         // [N] sweeps run in this substep, or null
    float *residuals;            // [N] residual RMS after this substep's last sweep, or null
    float threshold;             // residual RMS above which the sweeps continue
    float stall_ratio;           // > 0: no further sweeps when the last minimum sweep stalled
    int32_t min_iterations;
    int32_t max_iterations;
    int32_t first_substep;       // 1: find the contact candidates on the start-of-step positions
    int32_t step;                // row of tool_pos used by this substep
    int32_t max_vertices;
    // network pass: per mesh the first 32-particle chunk that holds a free
    // particle (the chunks before it hold pinned particles only, which the
    // correction leaves alone), and the chunks per environment it visits
    const int32_t *chunk0;       // [meshes]
    int32_t chunks;
};

// Per-workgroup LDS layout for an environment of a given mesh.
struct LdsLayout {
    uint32_t xw;        // float4 [V]
    uint32_t lambda;    // float [E + T]
    uint32_t contacts;  // uint16 [tools][V]
    uint32_t edge_pair; // uint32 [E]  (staged topology only)
    uint32_t edge_rest; // float [E]
    uint32_t tet_quad;  // uint2 [T]
    uint32_t tet_rest;  // float [T]
    uint32_t scratch;   // 64 x uint32 for reductions and counts
    uint32_t dx;        // float [3][V] summed corrections (Jacobi only)
    uint32_t inv_count; // float [V] 1 / constraints per particle (Jacobi only)
    uint32_t face_flag; // uint8 [tools][F] candidate faces of capsule tools
    uint32_t total;
};

__host__ __device__ inline uint32_t align_up(uint32_t x, uint32_t a) { return (x + a - 1) / a * a; }

__host__ __device__ inline LdsLayout lds_layout(int32_t V, int32_t E, int32_t T, int32_t tools,
                                                bool stage_topology, bool jacobi = false,
                                                int32_t capsule_faces = 0)
{
    LdsLayout l;
    uint32_t o = 0;
    l.xw = o;
    o += 16u * (uint32_t)V;
    l.lambda = o;
    o = align_up(o + 4u * (uint32_t)(E + T), 16);
    l.contacts = o;
    o = align_up(o + 2u * (uint32_t)(tools > 0 ? tools : 0) * (uint32_t)V, 16);
    if (stage_topology) {
        l.edge_pair = o;
        o += 4u * (uint32_t)E;
        l.edge_rest = o;
        o = align_up(o + 4u * (uint32_t)E, 16);
        l.tet_quad = o;
        o += 8u * (uint32_t)T;
        l.tet_rest = o;
        o = align_up(o + 4u * (uint32_t)T, 16);
    } else {
        l.edge_pair = l.edge_rest = l.tet_quad = l.tet_rest = 0;
    }
    l.scratch = o;
    o += 64u * 4u;
    l.dx = l.inv_count = 0;
    if (jacobi) {
        l.dx = o;
        o = align_up(o + 12u * (uint32_t)V, 16);
        l.inv_count = o;
        o = align_up(o + 4u * (uint32_t)V, 16);
    }
    l.face_flag = o;
    if (capsule_faces > 0)
        o = align_up(o + (uint32_t)(tools > 0 ? tools : 0) * (uint32_t)capsule_faces, 16);
    l.total = o;
    return l;
}

// Launchers (xpbd_kernels.hip).
// LDS-multiplier kernel; jacobi selects the paper's Jacobi iteration instead
// of the coloured Gauss-Seidel sweep.
hipError_t launch_step(const StepArgs &args, int block, int particles_per_thread, bool jacobi,
                       bool stage_topology, uint32_t lds_bytes, bool want_residual,
                       hipStream_t stream);
// LDS layout of the register-multiplier kernel for a group holding V particles
// in all.  Scratch: words 0..15 per-wave counts, 32..95 flags of the
// workgroup-wide OR (16 per environment), bytes kRegScratchTools.. the sphere
// centres of the group's environments (float4 [G][2]), bytes
// kRegScratchGrasp.. the grasp state (int32 [G] held slots, int32 [G] search
// flags, uint64 [16 waves][G] partial minima of the grasp search).
struct RegLdsLayout {
    uint32_t xw;       // float4 [V + 1]  position + inverse mass; slot V: padding particle
    uint32_t vel;      // float [3][V]
    uint32_t prev;     // float [3][V]  positions at the start of the substep
    uint32_t scratch;  // kRegScratchBytes
    uint32_t faces;    // capsule tools: [tools] x capsule_face_bytes (below)
    uint32_t total;
};

// LDS of one capsule tool in the register variant, for a mesh of F surface
// faces in C colours: the candidate flags as 64-bit words [ceil(F / 64)]; the
// candidates compacted colour by colour, as the LDS slots of their corners
// (uint32 a | b << 16 [F], uint16 c [F]); the list's colour bounds uint16 [C + 1].
struct CapsuleFaceLayout {
    uint32_t flags, ab, c, bounds, total;
};

__host__ __device__ inline CapsuleFaceLayout capsule_face_layout(int32_t F, int32_t C)
{
    CapsuleFaceLayout l;
    l.flags = 0;
    l.ab = align_up(8u * (((uint32_t)F + 63u) / 64u), 16);
    l.c = l.ab + align_up(4u * (uint32_t)F, 16);
    l.bounds = l.c + align_up(2u * (uint32_t)F, 16);
    l.total = l.bounds + align_up(2u * ((uint32_t)C + 1u), 16);
    return l;
}

constexpr uint32_t kRegScratchTools = 384;
constexpr uint32_t kRegScratchGrasp = 512;
constexpr uint32_t kRegScratchBytes = 1024;
constexpr int kMaxEnvsPerGroup = 2;
constexpr int kMaxCapsuleBlock = 512;   // register variant with capsule tools

// face_bytes: tools x capsule_face_layout(F, C).total for capsule tools, else 0
__host__ __device__ inline RegLdsLayout reg_lds_layout(int32_t V, int32_t face_bytes = 0)
{
    RegLdsLayout l;
    l.xw = 0;
    l.vel = 16u * ((uint32_t)V + 1u);
    l.prev = l.vel + 12u * (uint32_t)V;
    l.scratch = align_up(l.prev + 12u * (uint32_t)V, 16);
    l.faces = l.scratch + kRegScratchBytes;
    l.total = l.faces + align_up((uint32_t)face_bytes, 16);
    return l;
}

// Register-multiplier kernel; lambda_banks = ceil(rounds / 32) in {1, 2},
// envs_per_group in {1, 2}; one workgroup per group.
hipError_t launch_step_reg(const StepArgs &args, int block, int lambda_banks, int envs_per_group,
                           uint32_t lds_bytes, bool want_residual, hipStream_t stream);
// Workgroups of the register kernel that a launch with these arguments runs
// (tool shape, grasp, round barriers) a CU holds at once, as the HIP
// runtime's occupancy calculator gives it from the kernel's registers, the
// block and the LDS.
hipError_t step_reg_occupancy(const StepArgs &args, int block, int lambda_banks,
                              int envs_per_group, uint32_t lds_bytes, int *per_cu);
// Residual RMS and max of every environment from the multipliers of the last
// launch (register variant).
hipError_t launch_residual(const StepArgs &args, hipStream_t stream);
// Learned warm start: prediction + features of one substep (every particle of
// every environment), then one substep of the register-multiplier solver
// starting from the predicted (and corrected) positions.
hipError_t launch_learned_predict(const StepArgs &args, const LearnedArgs &largs, hipStream_t stream);
// The network's correction of the predicted positions in largs.xhat (in
// place, free particles only) from the feature rows in largs.features:
// num_workgroups persistent workgroups.
struct MlpDev;
hipError_t launch_learned_correct(const StepArgs &args, const LearnedArgs &largs,
                                  const MlpDev &net, int num_workgroups, hipStream_t stream);
hipError_t launch_substep_reg(const StepArgs &args, const LearnedArgs &largs, int block,
                              int lambda_banks, uint32_t lds_bytes, bool want_residual,
                              hipStream_t stream);
hipError_t launch_soa_to_aos(const float *soa, float *aos, int32_t n, hipStream_t stream);
hipError_t launch_aos_to_soa(const float *aos, float *soa, int32_t n, hipStream_t stream);

}  // namespace xpbd
