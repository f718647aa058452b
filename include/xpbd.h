/*
 * xpbd.h -- C ABI of the MI355X batched XPBD substep library (libxpbd.so).
 *
 * The library advances many independent soft-tissue environments with the
 * simulation loop of FF-SRL (Dall'Alba et al., arXiv 2503.18616, Sec. III-A,
 * Algorithm 1): per step the tool pose is read; per substep velocities and
 * positions are predicted under gravity, edge-distance (Eq. 1) and
 * tetrahedral-volume (Eqs. 2-3) constraints are projected in compliance form
 * with one Lagrange multiplier per constraint, the particles are pushed out of
 * the tool (Sec. III-A.3), and velocities are recomputed from the position
 * change.  All environments' arrays are concatenated, one array per variable
 * (Sec. III-B).
 *
 * Conventions shared by every call:
 *   - Units are SI.  Positions are float32 [V][3] (x, y, z per particle).
 *   - Environment e owns particles [env_offset[e], env_offset[e+1]) of the
 *     concatenated particle arrays, in the order of its mesh's vertex ids.
 *   - No call throws; every failure returns a negative xpbd_status and leaves
 *     a message for xpbd_last_error() on the calling thread.
 *   - Pointers documented "host or device" may point to host memory or to
 *     device memory of the batch's GPU; the library tells them apart.
 *   - A batch is bound to the HIP device that was current at creation and to
 *     the stream given then.  Calls on one batch must not overlap.
 */
#ifndef XPBD_H
#define XPBD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xpbd_batch xpbd_batch; /* opaque; freed by xpbd_destroy_batch */

typedef enum {
    XPBD_OK = 0,
    XPBD_E_ARG = -1,       /* null pointer, bad count, bad size or non-finite parameter */
    XPBD_E_MESH = -2,      /* index out of range, repeated vertex, zero-volume tetrahedron,
                              more than 65535 particles, non-finite rest position or mass */
    XPBD_E_CAPACITY = -3,  /* a mesh does not fit the per-workgroup LDS plan */
    XPBD_E_HIP = -4,       /* a HIP runtime call failed (message names it) */
    XPBD_E_NONFINITE = -5, /* some environment's state became NaN or infinite */
    XPBD_E_STATE = -6      /* buffer size does not match the field, or unknown field */
} xpbd_status;

/* Fields for xpbd_read_state / xpbd_write_state / xpbd_field_bytes. */
enum {
    XPBD_FIELD_POS = 0,            /* float [sum V][3]  positions (read, write) */
    XPBD_FIELD_VEL = 1,            /* float [sum V][3]  velocities (read, write) */
    XPBD_FIELD_LAMBDA = 2,         /* float [sum over envs of (E_m + T_m)] multipliers after the
                                      last iteration of the last substep, per env: edges in
                                      constraint order, then tetrahedra.  Needs XPBD_F_LAMBDA. */
    XPBD_FIELD_CONTACTS = 3,       /* int32 [num_tools][sum V]: for tool t and env e, the
                                      contact candidates of the last step as ascending local
                                      particle ids at [t][env_offset[e] ...], padded with -1 */
    XPBD_FIELD_CONTACT_COUNTS = 4, /* int32 [N][num_tools] number of candidates of the last step */
    XPBD_FIELD_COLOURS = 5,        /* int32 [sum over meshes of (E_m + T_m)] colour of every kept
                                      constraint of every mesh, mesh order, edges then tetrahedra */
    XPBD_FIELD_RESIDUAL = 6,       /* float [N][2] (RMS, max |r|) of the constraint residual
                                      (C + alpha~ lambda)/rest, at the last substep of the last
                                      xpbd_step call made with XPBD_F_RESIDUAL. */
    XPBD_FIELD_ENV_OFFSETS = 7,    /* int32 [N+1] particle offsets of the environments */
    XPBD_FIELD_NONFINITE = 8,      /* int32 [N] 1 where the env's state went non-finite */
    XPBD_FIELD_COUNT = 9
};

/* Flags for xpbd_params.flags. */
#define XPBD_F_RESIDUAL 0x1u /* compute the residual at the end of every xpbd_step call */
#define XPBD_F_LAMBDA 0x2u   /* store the multipliers at the end of every xpbd_step call */

/*
 * One tetrahedral mesh (Sec. III-A.1: V particles with masses, a tetrahedral
 * mesh, edges between adjacent particles).  Host memory, read during
 * xpbd_create_batch only.
 *   rest_pos  [V][3]  rest positions; also the initial positions
 *   inv_mass  [V]     inverse masses w = 1/m; 0 pins a particle
 *   tets      [T][4]  particle ids.  The library swaps the last two ids of a
 *                     tetrahedron whose rest volume is negative.
 * Edges are the unique particle pairs of the tetrahedra; constraints whose
 * particles are all pinned are dropped.  Rest lengths and volumes are taken
 * from rest_pos in double precision and rounded to float.
 */
typedef struct {
    int32_t num_vertices; /* V, 1 .. 65535 */
    int32_t num_tets;     /* T, >= 1 */
    const float *rest_pos;
    const float *inv_mass;
    const int32_t *tets;
} xpbd_mesh;

/*
 * Solver settings (Algorithm 1: dt, simSubSteps; the iteration count of the
 * Gauss-Seidel colour sweeps per substep; Sec. III-A.2/3: the tool).
 */
typedef struct {
    float dt;            /* step length, > 0 */
    int32_t substeps;    /* substeps per step, >= 1; h = dt / substeps */
    int32_t iterations;  /* colour sweeps per substep, >= 0 */
    float gravity[3];    /* m/s^2 */
    int32_t num_tools;   /* kinematic spheres, 0 .. 2 */
    float tool_radius[2];/* m, > 0 for each used tool */
    uint32_t flags;      /* XPBD_F_* */
    int32_t block_size;  /* threads per workgroup: 0 = chosen by the library (register
                            variant, one mesh: the block of 128 .. 1024 and, unless
                            envs_per_group fixes it, the environments per workgroup
                            whose rounds, times the passes of workgroups over the CUs
                            at the occupancy their waves and LDS allow, are fewest; several
                            meshes: per mesh, the smallest of 256, 512, 1024 whose rounds
                            fit; meshes of equal block and LDS tier form a size class,
                            and the classes run concurrently), else a multiple of 64 in
                            [64, 1024] for every mesh */
    int32_t solver_variant; /* XPBD_VARIANT_*: where the multipliers live */
    int32_t colour_packing; /* XPBD_PACKING_*: order of the constraints inside a colour */
    int32_t envs_per_group; /* register variant: environments that share one workgroup,
                               its LDS and its rounds (lanes of a round may belong to
                               different environments): 0 = chosen by the library (see
                               block_size; 1 for several meshes),
                               else 1 or 2.  Environments are grouped per mesh in index
                               order; the LDS variant always uses 1. */
    int32_t tool_shape;     /* XPBD_TOOL_*: spheres against particles, or capsules against
                               the surface triangles */
    int32_t colouring;      /* XPBD_COLOURING_*: how the edge and tetrahedron constraints
                               are split into colours (0 = greedy) */
} xpbd_params;

/* Values of xpbd_params.tool_shape.
 *   SPHERE   a tool is a sphere of radius tool_radius[t] around a centre;
 *            tool_pos holds 3 floats per tool; particles within 2r of the
 *            centre at the start of a step are pushed out to the surface
 *            after the deformation constraints of every iteration.
 *   CAPSULE  the grasper capsules of Sec. III-A.2/3: a tool is a segment
 *            (p0, p1) with radius tool_radius[t]; tool_pos holds 6 floats
 *            per tool (p0 then p1).  It acts on the mesh's surface triangles
 *            (faces of exactly one kept tetrahedron): a face with a free
 *            particle closer than 2r to the segment at the start of a step
 *            is a candidate; after the deformation constraints of every
 *            iteration each candidate, face colour by face colour, is pushed
 *            out with k_c = 1 as the constraint d - r >= 0 on its point
 *            closest to the segment (d that distance; the correction of
 *            corner i is proportional to w_i and its barycentric weight).
 *            Runs on every variant with one environment per workgroup
 *            (AUTO picks the register variant where the rounds fit);
 *            the contact fields then hold the number of candidate faces per
 *            tool and no particle lists (all -1). */
enum { XPBD_TOOL_SPHERE = 0, XPBD_TOOL_CAPSULE = 1 };

/* Values of xpbd_params.colouring.  The colours of a mesh are the sets of
 * constraints projected in parallel (no two share a particle); the sweeps of
 * Alg. 1 visit the distance colours, then the volume colours, in ascending
 * order.  A different colouring is a different Gauss-Seidel order: an equally
 * valid solve, not the same numbers.
 *   GREEDY         constraints in index order, each taking the smallest colour
 *                  no constraint sharing a particle holds (the default)
 *   LARGEST_FIRST  recursive largest first: each colour in turn is grown into
 *                  a maximal set from the uncoloured constraints, starting from
 *                  the one with the most uncoloured conflicts and adding the
 *                  candidate with the most conflicts among those already ruled
 *                  out (then the fewest among the candidates, then the lowest
 *                  index); fewer and larger colours
 *   WAVES          LARGEST_FIRST, but a colour that would end with 65 to 100
 *                  members keeps its first 64 (the others stay uncoloured),
 *                  so that it fills one 64-lane wave instead of most of two
 *   CAPPED         LARGEST_FIRST, but a colour keeps at most its first 256
 *                  members (the others stay uncoloured), so that every colour
 *                  is one round of a 256-thread workgroup
 *   CAPPED_128     the same with at most 128 members: one round of a
 *                  128-thread workgroup
 *   CAPPED_FIT     chosen per mesh: CAPPED where its colours, the distance
 *                  colours and the volume colours each counted up to an even
 *                  number, add up to at most 64 (every colour one round of a
 *                  256-thread workgroup, within the register variant's 64
 *                  rounds), else LARGEST_FIRST */
enum { XPBD_COLOURING_GREEDY = 0, XPBD_COLOURING_LARGEST_FIRST = 1, XPBD_COLOURING_WAVES = 2,
       XPBD_COLOURING_CAPPED = 3, XPBD_COLOURING_CAPPED_128 = 4, XPBD_COLOURING_CAPPED_FIT = 5 };

/* Values of xpbd_params.colour_packing.  Constraints of one colour share no
 * particle, so their order changes no result; it only decides which lanes
 * the LDS serves together.
 *   ID_ORDER ascending constraint id
 *   BANKS8   every aligned run of 8 lanes reads particles in distinct
 *            16-byte LDS bank groups modulo 8, as far as a greedy fill allows
 *   BANKS16  the same for runs of 16 lanes modulo 16
 *   SCATTERED_BANKS16  BANKS16 after placing the particles in LDS in a fixed
 *            pseudo-random order (register variant only; the placement is
 *            internal and changes no result either)
 *   SEARCH   the scattered placement, then a seeded local search over the
 *            lane order and the vertex order of every constraint so that
 *            each aligned run of 16 lanes reads, and each run of 8 lanes
 *            writes, distinct LDS bank groups (register variant only).  An
 *            edge may list its particles in either order and a tetrahedron
 *            in any even permutation (the projection is the same function
 *            of the particles), so results change only in rounding.
 * AUTO picks SEARCH for the register variant while the batch's distinct
 * meshes hold at most 16384 particles in total (the search costs about a
 * second of host time per thousand particles at creation),
 * SCATTERED_BANKS16 for larger register-variant batches, and BANKS16 for the
 * LDS variant. */
enum { XPBD_PACKING_AUTO = 0, XPBD_PACKING_ID_ORDER = 1, XPBD_PACKING_BANKS8 = 2,
       XPBD_PACKING_BANKS16 = 3, XPBD_PACKING_SCATTERED_BANKS16 = 4, XPBD_PACKING_SEARCH = 5 };

/* Values of xpbd_params.solver_variant.  Both variants compute the same
 * projections in the same colour order; they differ only in data placement.
 *   AUTO      registers when every mesh's round schedule fits, else LDS
 *   REGISTERS each lane keeps the multipliers of its constraints in registers
 *             (one per round of <= block_size constraints of one colour, at
 *             most 64 rounds); only particle state occupies LDS
 *   LDS       multipliers in LDS next to the particles; constraint lists in
 *             LDS when they fit
 * JACOBI is a different solver, the paper's own parallel one (Sec. III-A.1,
 * Alg. 1), for comparison: in every iteration all constraints are projected
 * from the same positions (multipliers as above), each particle's corrections
 * are summed and the particle moves by the sum divided by the number of kept
 * constraints that include it; tool contact follows as in the other
 * variants.  The sums run colour by colour (no atomics, a fixed order), so
 * results are reproducible.  Multipliers and particles in LDS. */
enum { XPBD_VARIANT_AUTO = 0, XPBD_VARIANT_REGISTERS = 1, XPBD_VARIANT_LDS = 2,
       XPBD_VARIANT_JACOBI = 3 };

/*
 * Create a batch of num_envs environments; environment e uses mesh
 * env_mesh[e] and compliances compliance[2e] (edges) and compliance[2e+1]
 * (tetrahedra), both >= 0 and finite (alpha~ = alpha / h^2).  All inputs are
 * host memory and are copied.  Every environment starts at its mesh's rest
 * positions with zero velocity.  hip_stream (a hipStream_t, NULL for the
 * default stream) orders every later device operation of the batch.
 * On failure *out is set to NULL.
 */
xpbd_status xpbd_create_batch(const xpbd_mesh *meshes, int32_t num_meshes,
                              const int32_t *env_mesh, int32_t num_envs,
                              const float *compliance, const xpbd_params *params,
                              void *hip_stream, xpbd_batch **out);

/*
 * Advance every environment by num_steps steps in one kernel launch.
 * tool_pos: float [num_steps][N][num_tools][3] sphere centres (capsules: [6],
 * the two axis ends), host or device, ignored when num_tools == 0;
 * tool_pos_bytes: its size in bytes, which must equal what the steps read
 * (num_steps * N * num_tools * 3 or 6 * 4), else XPBD_E_ARG and no work.
 * Asynchronous on the batch's stream (a host tool_pos is copied before the
 * call returns).  num_steps == 0 does nothing.
 */
xpbd_status xpbd_step(xpbd_batch *b, int32_t num_steps, const float *tool_pos,
                      size_t tool_pos_bytes);

/*
 * Copy a field (XPBD_FIELD_*) into dst (host or device), dst_bytes must equal
 * xpbd_field_bytes.  Ordered after all earlier work on the batch's stream;
 * returns after the copy has completed.  Returns XPBD_E_NONFINITE (after
 * copying) when any environment's state is non-finite.
 */
xpbd_status xpbd_read_state(xpbd_batch *b, int32_t field, void *dst, size_t dst_bytes);

/*
 * Overwrite XPBD_FIELD_POS or XPBD_FIELD_VEL from src (host or device,
 * [sum V][3] float).  Pinned particles take the given values too.  Clears
 * the non-finite flags.  Used to resume from a saved state: a state saved
 * between xpbd_step calls is exactly (positions, velocities).
 */
xpbd_status xpbd_write_state(xpbd_batch *b, int32_t field, const void *src, size_t src_bytes);

/*
 * Replace the batch's flags (XPBD_F_*) for later xpbd_step calls, e.g. to
 * compute the residual only on the last step of an episode.  Setting
 * XPBD_F_LAMBDA or XPBD_F_RESIDUAL on a batch created without them allocates
 * the multiplier buffer (synchronously, on the batch's stream).  Returns
 * XPBD_E_ARG for unknown bits.
 */
xpbd_status xpbd_set_flags(xpbd_batch *b, uint32_t flags);

/* Byte size of a field of this batch. */
xpbd_status xpbd_field_bytes(const xpbd_batch *b, int32_t field, size_t *bytes);

/*
 * Autotuner of the launch configuration (not a method of the paper: a tool
 * for picking the fastest data placement).  Candidates vary four fields of
 * *params: solver_variant (registers, LDS), block_size (0, 256, 512, 1024),
 * envs_per_group (1, 2; registers only) and colour_packing (AUTO, BANKS16);
 * the first candidate is the library's default (all four 0).  Each candidate
 * is a batch created from the given meshes, environments and compliances
 * (the other fields of *params are kept, flags cleared) on hip_stream,
 * stepped once untimed (on the first step's poses) and then num_steps times
 * with tool_pos (tool_pos_bytes as in xpbd_step for num_steps steps; from the
 * rest state) between two events, and destroyed;
 * candidates the library rejects with XPBD_E_CAPACITY are skipped.  On
 * success the four fields of *params hold the fastest candidate,
 * ms_per_step[0] its time per step and ms_per_step[1] the default's (host
 * float [2]).  The candidates compute the same projections in the same
 * colour order; they differ only in rounding where colour_packing says so.
 * Blocks the calling thread until every candidate has run.
 */
xpbd_status xpbd_autotune(const xpbd_mesh *meshes, int32_t num_meshes, const int32_t *env_mesh,
                          int32_t num_envs, const float *compliance, xpbd_params *params,
                          void *hip_stream, int32_t num_steps, const float *tool_pos,
                          size_t tool_pos_bytes, float *ms_per_step);

/*
 * The launch configuration a batch runs with (what the library chose for
 * the zero, "library's choice", entries of xpbd_params), for inspection.
 * For the register variant the figures are those of the largest size class;
 * workgroups_per_cu is how many of its workgroups a CU holds at once (for
 * the register variant as the HIP runtime's occupancy calculator gives it,
 * on the current device, for the kernel a step without a grasp runs: its
 * registers, block and LDS; for the others by 16 resident waves and the
 * CU's LDS), waves_per_cu the waves that makes.  Host only.  XPBD_E_ARG for
 * NULL pointers, XPBD_E_HIP if the occupancy query fails.
 */
typedef struct {
    int32_t solver_variant;    /* XPBD_VARIANT_REGISTERS, _LDS or _JACOBI */
    int32_t block_size;        /* threads per workgroup */
    int32_t envs_per_group;    /* environments per workgroup */
    int32_t size_classes;      /* concurrent launches per step (register variant) */
    int32_t lambda_banks;      /* 32-round multiplier banks (register variant) */
    int32_t lds_bytes;         /* LDS per workgroup */
    int32_t workgroups;        /* workgroups of the largest class */
    int32_t workgroups_per_cu;
    int32_t waves_per_cu;
} xpbd_batch_info;

xpbd_status xpbd_get_batch_info(const xpbd_batch *b, xpbd_batch_info *out);

/* Free the batch and its device memory (waits for its stream).  NULL is ignored. */
void xpbd_destroy_batch(xpbd_batch *b);

/* Message of the last failure on the calling thread ("" if none). */
const char *xpbd_last_error(void);

/*
 * Host-only mesh set-up, the same the batch performs at creation, for
 * inspection without a GPU.  counts[0..3] receive (E, T, edge colours,
 * tetrahedron colours) of the kept constraints.  Each output pointer may be
 * NULL; otherwise it must hold:
 *   edges       int32 [E][2]  ascending (smaller id, larger id)
 *   tets        int32 [T][4]  kept tetrahedra in input order, oriented
 *   colours     int32 [E+T]   greedy colour of each constraint
 *   rest        float [E+T]   rest lengths, then rest volumes
 * Call once with NULL outputs to size them.
 */
xpbd_status xpbd_prepare_mesh(const xpbd_mesh *mesh, int32_t *counts, int32_t *edges,
                              int32_t *tets, int32_t *colours, float *rest);

/* xpbd_prepare_mesh with the colouring of the edge and tetrahedron
 * constraints named (XPBD_COLOURING_*; XPBD_E_ARG for another value). */
xpbd_status xpbd_prepare_mesh_coloured(const xpbd_mesh *mesh, int32_t colouring, int32_t *counts,
                                       int32_t *edges, int32_t *tets, int32_t *colours,
                                       float *rest);

/*
 * Host-only: the surface triangles the capsule tools act on (the same set-up
 * the batch performs).  counts[0..1] receive (F, face colours).  faces int32
 * [F][3]: the faces of exactly one kept tetrahedron, each ordered so that
 * (x1 - x0) x (x2 - x0) points away from its tetrahedron, sorted by their
 * ascending vertex triple; colours int32 [F]: greedy colours in that order
 * (faces sharing a particle differ).  Either output may be NULL; call once
 * with NULL outputs to size them.
 */
xpbd_status xpbd_surface_faces(const xpbd_mesh *mesh, int32_t *counts, int32_t *faces,
                               int32_t *colours);

#ifdef __cplusplus
}
#endif

#endif /* XPBD_H */
