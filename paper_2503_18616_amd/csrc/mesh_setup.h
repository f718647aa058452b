// Host-side mesh set-up of the XPBD library: orientation, rest values, edge
// extraction and greedy graph colouring of the constraints (FF-SRL Sec. III-A.1:
// rest length and rest volume are computed before the simulation loop).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace xpbd {

struct PreparedMesh {
    int32_t num_vertices = 0;
    std::vector<float> rest_pos;        // [V][3] as given
    std::vector<float> inv_mass;        // [V]
    std::vector<int32_t> edges;         // [E][2] ascending pairs, at least one free particle
    std::vector<int32_t> tets;          // [T][4] kept, oriented
    std::vector<double> rest_length;    // [E]
    std::vector<double> rest_volume;    // [T]
    std::vector<int32_t> edge_colour;   // [E]
    std::vector<int32_t> tet_colour;    // [T]
    int32_t num_edge_colours = 0;
    int32_t num_tet_colours = 0;

    std::vector<int32_t> faces;         // [F][3] outward surface triangles, sorted by vertex set
    std::vector<int32_t> face_colour;   // [F]
    int32_t num_face_colours = 0;
    int32_t num_edges() const { return (int32_t)rest_length.size(); }
    int32_t num_tets() const { return (int32_t)rest_volume.size(); }
    int32_t num_faces() const { return (int32_t)(faces.size() / 3); }
};

// Returns 0 on success; on failure a negative xpbd_status and a message.
// colouring: XPBD_COLOURING_* of the edge and tetrahedron constraints (the
// surface faces always take the greedy colouring).
int prepare_mesh(int32_t num_vertices, int32_t num_tets, const float *rest_pos,
                 const float *inv_mass, const int32_t *tets, PreparedMesh &out,
                 std::string &error, int32_t colouring = 0);

// Greedy colouring: constraints are visited in index order and each takes the
// smallest colour not held by an already coloured constraint that shares a
// particle.  ids: [n][k].  Returns the number of colours.
int32_t greedy_colouring(int32_t num_vertices, int32_t n, int32_t k, const int32_t *ids,
                         std::vector<int32_t> &colour);

// Recursive largest-first colouring (Leighton 1979): colours are built one at
// a time, each as a maximal set of constraints that share no particle, drawn
// from the constraints not yet coloured.  A colour starts with the constraint
// that conflicts with the most uncoloured ones; every further pick is a
// candidate (one sharing no particle with the colour so far) with the most
// conflicts among the constraints already excluded from the colour, then the
// fewest among the remaining candidates, then the lowest index.  With
// cut_above > 64, a colour that ends with more than 64 and at most cut_above
// members keeps only its first 64 picks (the rest return to the uncoloured
// pool), so that it fills one 64-wide wave instead of most of a second one.
// With cap > 0 a colour keeps at most its first cap picks (the rest return
// to the pool), so that it fits one round of a cap-thread workgroup.
// ids: [n][k].  Returns the number of colours.
int32_t largest_first_colouring(int32_t num_vertices, int32_t n, int32_t k, const int32_t *ids,
                                int32_t cut_above, int32_t cap, std::vector<int32_t> &colour);

// Order of the constraints inside each colour (the "packing"; it does not
// change results because constraints of one colour share no particle).
// slot_id lists constraint ids colour by colour, ptr holds the colour offsets.
// With group > 0 each aligned run of `group` slots of a colour (the lanes that
// the LDS serves together) is filled greedily with constraints whose particle
// ids at every vertex position are distinct modulo `modulus` (the LDS bank
// group of a 16-byte particle record); group == 0 keeps ascending id order.
void pack_colours(const int32_t *ids, int32_t k, const std::vector<int32_t> &ptr, int32_t group,
                  int32_t modulus, std::vector<int32_t> &slot_id);

// Axis neighbours of every particle, for the learned warm start's features:
// in direction d = -x, +x, -y, +y, -z, +z the particle whose rest coordinates
// on the other two axes equal particle i's and whose rest coordinate along
// the axis is the nearest one beyond X_i on that side (the smallest id among
// equals), or -1.  out: [V][6].
void axis_neighbours(int32_t num_vertices, const float *rest_pos, std::vector<int32_t> &out);

// Even permutations of the vertices of a constraint: the edge update is
// symmetric in its two particles and the volume update is invariant under the
// even permutations of its four (they keep the orientation), so a record may
// list its particles in any of these orders.  Tables: [count][k].
int32_t num_vertex_orders(int32_t k);
const uint8_t *vertex_order(int32_t k, int32_t index);

// Lane order and vertex order of the constraints of every colour, searched so
// that the register kernel's LDS accesses avoid bank conflicts.  gfx950's LDS
// has 64 four-byte banks: a ds_read_b128 serves 16 lanes per clock and is
// conflict-free when the 16-byte records read by each aligned group of 16
// lanes are distinct modulo 16; a ds_write_b96 serves 8 lanes per clock and is
// conflict-free when the records written by each aligned group of 8 lanes are
// distinct modulo 8.  slots: [n][k] LDS slots of constraint ids 0..n-1.
// slot_id: in, colour-major constraint ids (colour offsets ptr); out, the same
// sets in lane order.  order: out, [n] vertex_order index per constraint id.
// Deterministic for a given seed; effort scales the local-search moves per
// lane (0: greedy pass only).
void pack_lanes(const int32_t *slots, int32_t k, const std::vector<int32_t> &ptr, uint32_t seed,
                int32_t effort, std::vector<int32_t> &slot_id, std::vector<uint8_t> &order);

// One constraint type for pack_lds: particle ids [n][k] (mesh order), colour
// offsets, and the two outputs of pack_lanes.
struct LaneSchedule {
    const int32_t *ids;
    int32_t k;
    const std::vector<int32_t> *ptr;
    std::vector<int32_t> *slot_id;   // in: colour-major ids; out: lane order
    std::vector<uint8_t> *order;     // out: [n] vertex_order index
};

// pack_lanes for several constraint types at once, with the LDS placement of
// the particles searched as well: slot_of (in: a starting bijection particle
// -> slot, out: the searched one) decides the bank group (slot modulo 16) of
// each particle in every constraint that uses it.  Moves swap two particles'
// slots, swap two lanes of a colour, or change a vertex order.
void pack_lds(int32_t num_particles, std::vector<int32_t> &slot_of, LaneSchedule *kinds,
              int32_t num_kinds, uint32_t seed, int32_t effort);

// Bank-conflict cost of a lane order in LDS clocks beyond the conflict-free
// count, summed over the colours (reads: extra passes of each 16-lane group;
// writes: extra passes of each 8-lane group), as pack_lanes models it.
int64_t lane_conflicts(const int32_t *slots, int32_t k, const std::vector<int32_t> &ptr,
                       const std::vector<int32_t> &slot_id, const std::vector<uint8_t> &order);

}  // namespace xpbd
