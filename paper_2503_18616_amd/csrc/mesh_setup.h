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

    int32_t num_edges() const { return (int32_t)rest_length.size(); }
    int32_t num_tets() const { return (int32_t)rest_volume.size(); }
};

// Returns 0 on success; on failure a negative xpbd_status and a message.
int prepare_mesh(int32_t num_vertices, int32_t num_tets, const float *rest_pos,
                 const float *inv_mass, const int32_t *tets, PreparedMesh &out,
                 std::string &error);

// Greedy colouring: constraints are visited in index order and each takes the
// smallest colour not held by an already coloured constraint that shares a
// particle.  ids: [n][k].  Returns the number of colours.
int32_t greedy_colouring(int32_t num_vertices, int32_t n, int32_t k, const int32_t *ids,
                         std::vector<int32_t> &colour);

// Order of the constraints inside each colour (the "packing"; it does not
// change results because constraints of one colour share no particle).
// slot_id lists constraint ids colour by colour, ptr holds the colour offsets.
// With group > 0 each aligned run of `group` slots of a colour (the lanes that
// the LDS serves together) is filled greedily with constraints whose particle
// ids at every vertex position are distinct modulo `modulus` (the LDS bank
// group of a 16-byte particle record); group == 0 keeps ascending id order.
void pack_colours(const int32_t *ids, int32_t k, const std::vector<int32_t> &ptr, int32_t group,
                  int32_t modulus, std::vector<int32_t> &slot_id);

}  // namespace xpbd
