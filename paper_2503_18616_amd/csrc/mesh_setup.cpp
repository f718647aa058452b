// Host-side mesh set-up; see mesh_setup.h.
#include "mesh_setup.h"

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "../../include/xpbd.h"

namespace xpbd {
namespace {

// Six times the signed volume of (a, b, c, d): the determinant of the edge
// vectors b - a, c - a, d - a, expanded along its first row.
double six_volume(const float *p, int32_t a, int32_t b, int32_t c, int32_t d)
{
    double e[3][3];
    const int32_t q[3] = {b, c, d};
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            e[r][k] = (double)p[3 * q[r] + k] - (double)p[3 * a + k];
    return e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
           e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
           e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
}

}  // namespace

int32_t greedy_colouring(int32_t num_vertices, int32_t n, int32_t k, const int32_t *ids,
                         std::vector<int32_t> &colour)
{
    colour.assign((size_t)n, -1);
    // colours already taken at each particle, appended as constraints are coloured
    std::vector<std::vector<int32_t>> taken((size_t)num_vertices);
    std::vector<int32_t> stamp;  // stamp[c] == j: colour c is forbidden for constraint j
    int32_t count = 0;
    for (int32_t j = 0; j < n; ++j) {
        const int32_t *q = ids + (size_t)j * k;
        for (int32_t i = 0; i < k; ++i)
            for (int32_t c : taken[(size_t)q[i]])
                stamp[(size_t)c] = j;
        int32_t c = 0;
        while (c < count && stamp[(size_t)c] == j)
            ++c;
        if (c == count) {
            ++count;
            stamp.push_back(-1);
        }
        colour[(size_t)j] = c;
        for (int32_t i = 0; i < k; ++i)
            taken[(size_t)q[i]].push_back(c);
    }
    return count;
}

void pack_colours(const int32_t *ids, int32_t k, const std::vector<int32_t> &ptr, int32_t group,
                  int32_t modulus, std::vector<int32_t> &slot_id)
{
    if (group <= 0 || modulus <= 0)
        return;
    std::vector<int32_t> pool, packed;
    std::vector<uint8_t> used((size_t)k * (size_t)modulus);
    for (size_t c = 0; c + 1 < ptr.size(); ++c) {
        pool.assign(slot_id.begin() + ptr[c], slot_id.begin() + ptr[c + 1]);
        packed.clear();
        while (!pool.empty()) {
            std::fill(used.begin(), used.end(), 0);
            for (int32_t pos = 0; pos < group && !pool.empty(); ++pos) {
                // first constraint without a bank collision, else the one with fewest
                size_t best = 0;
                int best_hits = k + 1;
                for (size_t q = 0; q < pool.size() && best_hits > 0; ++q) {
                    const int32_t *v = ids + (size_t)pool[q] * (size_t)k;
                    int hits = 0;
                    for (int32_t j = 0; j < k; ++j)
                        hits += used[(size_t)j * (size_t)modulus + (size_t)(v[j] % modulus)];
                    if (hits < best_hits) {
                        best_hits = hits;
                        best = q;
                    }
                }
                const int32_t *v = ids + (size_t)pool[best] * (size_t)k;
                for (int32_t j = 0; j < k; ++j)
                    used[(size_t)j * (size_t)modulus + (size_t)(v[j] % modulus)] = 1;
                packed.push_back(pool[best]);
                pool.erase(pool.begin() + (std::ptrdiff_t)best);
            }
        }
        std::copy(packed.begin(), packed.end(), slot_id.begin() + ptr[c]);
    }
}

int prepare_mesh(int32_t num_vertices, int32_t num_tets, const float *rest_pos,
                 const float *inv_mass, const int32_t *tets, PreparedMesh &out,
                 std::string &error)
{
    char msg[256];
    if (num_vertices < 1 || num_vertices > 65535) {
        snprintf(msg, sizeof msg, "mesh has %d particles; 1..65535 supported", num_vertices);
        error = msg;
        return XPBD_E_MESH;
    }
    if (num_tets < 1 || !rest_pos || !inv_mass || !tets) {
        error = "mesh needs at least one tetrahedron and non-null arrays";
        return XPBD_E_ARG;
    }
    const size_t V = (size_t)num_vertices;
    for (size_t i = 0; i < V; ++i) {
        if (!std::isfinite(inv_mass[i]) || inv_mass[i] < 0.0f ||
            !std::isfinite(rest_pos[3 * i]) || !std::isfinite(rest_pos[3 * i + 1]) ||
            !std::isfinite(rest_pos[3 * i + 2])) {
            snprintf(msg, sizeof msg, "particle %zu has a non-finite position or a negative or "
                     "non-finite inverse mass", i);
            error = msg;
            return XPBD_E_MESH;
        }
    }
    out = PreparedMesh();
    out.num_vertices = num_vertices;
    out.rest_pos.assign(rest_pos, rest_pos + 3 * V);
    out.inv_mass.assign(inv_mass, inv_mass + V);

    // tetrahedra: validate, drop all-pinned, orient, rest volume
    for (int32_t t = 0; t < num_tets; ++t) {
        int32_t q[4];
        for (int i = 0; i < 4; ++i) {
            q[i] = tets[4 * (size_t)t + i];
            if (q[i] < 0 || q[i] >= num_vertices) {
                snprintf(msg, sizeof msg, "tetrahedron %d refers to particle %d of %d", t, q[i],
                         num_vertices);
                error = msg;
                return XPBD_E_MESH;
            }
        }
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < i; ++j)
                if (q[i] == q[j]) {
                    snprintf(msg, sizeof msg, "tetrahedron %d repeats particle %d", t, q[i]);
                    error = msg;
                    return XPBD_E_MESH;
                }
        if (inv_mass[q[0]] == 0.0f && inv_mass[q[1]] == 0.0f && inv_mass[q[2]] == 0.0f &&
            inv_mass[q[3]] == 0.0f)
            continue;
        double v6 = six_volume(rest_pos, q[0], q[1], q[2], q[3]);
        if (v6 == 0.0) {
            snprintf(msg, sizeof msg, "tetrahedron %d has zero rest volume", t);
            error = msg;
            return XPBD_E_MESH;
        }
        if (v6 < 0.0) {
            std::swap(q[2], q[3]);
            v6 = six_volume(rest_pos, q[0], q[1], q[2], q[3]);
        }
        out.tets.insert(out.tets.end(), q, q + 4);
        out.rest_volume.push_back(v6 / 6.0);
    }
    const size_t T = out.rest_volume.size();

    // edges: unique pairs of the kept tetrahedra, sorted, both-pinned dropped
    std::vector<uint64_t> keys;
    keys.reserve(6 * T);
    for (size_t t = 0; t < T; ++t)
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j) {
                uint32_t a = (uint32_t)out.tets[4 * t + i], b = (uint32_t)out.tets[4 * t + j];
                if (a > b)
                    std::swap(a, b);
                keys.push_back(((uint64_t)a << 32) | b);
            }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    for (uint64_t key : keys) {
        const int32_t a = (int32_t)(key >> 32), b = (int32_t)(key & 0xffffffffu);
        if (inv_mass[a] == 0.0f && inv_mass[b] == 0.0f)
            continue;
        out.edges.push_back(a);
        out.edges.push_back(b);
        double s = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double d = (double)rest_pos[3 * a + k] - (double)rest_pos[3 * b + k];
            s += d * d;
        }
        out.rest_length.push_back(std::sqrt(s));
    }

    out.num_edge_colours = greedy_colouring(num_vertices, out.num_edges(), 2, out.edges.data(),
                                            out.edge_colour);
    out.num_tet_colours = greedy_colouring(num_vertices, out.num_tets(), 4, out.tets.data(),
                                           out.tet_colour);
    return XPBD_OK;
}

}  // namespace xpbd
