// Host-side mesh set-up; see mesh_setup.h.
#include "mesh_setup.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <random>

#include "../../include/xpbd.h"

namespace xpbd {
namespace {

// WAVES colouring: a colour of 65 .. kWaveCutAbove members is cut to 64.
constexpr int32_t kWaveCutAbove = 100;
// CAPPED and CAPPED_128 colourings: a colour keeps at most this many members.
constexpr int32_t kColourCap = 256;
constexpr int32_t kColourCap128 = 128;
// CAPPED_FIT: the most colours (each kind's count rounded up to even) for
// which a mesh keeps the cap; the register variant holds 64 rounds.
constexpr int32_t kFitRounds = 64;

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

int32_t largest_first_colouring(int32_t num_vertices, int32_t n, int32_t k, const int32_t *ids,
                                int32_t cut_above, int32_t cap, std::vector<int32_t> &colour)
{
    colour.assign((size_t)n, -1);
    // conflict lists: constraints sharing a particle, without repeats
    std::vector<std::vector<int32_t>> at((size_t)num_vertices);
    for (int32_t j = 0; j < n; ++j)
        for (int32_t i = 0; i < k; ++i)
            at[(size_t)ids[(size_t)j * k + i]].push_back(j);
    std::vector<std::vector<int32_t>> adj((size_t)n);
    std::vector<int32_t> seen((size_t)n, -1);
    for (int32_t j = 0; j < n; ++j) {
        seen[(size_t)j] = j;
        for (int32_t i = 0; i < k; ++i)
            for (int32_t o : at[(size_t)ids[(size_t)j * k + i]])
                if (seen[(size_t)o] != j) {
                    seen[(size_t)o] = j;
                    adj[(size_t)j].push_back(o);
                }
    }
    // state of a constraint while one colour is built
    enum : uint8_t { DONE = 0, CANDIDATE = 1, EXCLUDED = 2 };
    std::vector<uint8_t> state((size_t)n, CANDIDATE);
    std::vector<int32_t> in_u((size_t)n), in_x((size_t)n);   // conflicts among candidates / excluded
    std::vector<int32_t> picked;
    int32_t left = n, count = 0;
    while (left > 0) {
        int32_t best = -1;
        for (int32_t j = 0; j < n; ++j) {
            if (state[(size_t)j] == DONE)
                continue;
            in_x[(size_t)j] = 0;
            int32_t u = 0;
            for (int32_t o : adj[(size_t)j])
                u += state[(size_t)o] != DONE;
            in_u[(size_t)j] = u;
            if (best < 0 || u > in_u[(size_t)best])
                best = j;
        }
        picked.clear();
        while (best >= 0) {
            picked.push_back(best);
            state[(size_t)best] = EXCLUDED;   // taken: leaves the candidates
            for (int32_t o : adj[(size_t)best])
                if (state[(size_t)o] != DONE)
                    --in_u[(size_t)o];
            for (int32_t o : adj[(size_t)best])
                if (state[(size_t)o] == CANDIDATE) {
                    state[(size_t)o] = EXCLUDED;
                    for (int32_t p : adj[(size_t)o])
                        if (state[(size_t)p] != DONE) {
                            --in_u[(size_t)p];
                            ++in_x[(size_t)p];
                        }
                }
            best = -1;
            for (int32_t j = 0; j < n; ++j)
                if (state[(size_t)j] == CANDIDATE &&
                    (best < 0 || in_x[(size_t)j] > in_x[(size_t)best] ||
                     (in_x[(size_t)j] == in_x[(size_t)best] && in_u[(size_t)j] < in_u[(size_t)best])))
                    best = j;
        }
        size_t keep = picked.size();
        if (cut_above > 64 && keep > 64 && keep <= (size_t)cut_above)
            keep = 64;
        if (cap > 0 && keep > (size_t)cap)
            keep = (size_t)cap;
        for (size_t q = 0; q < keep; ++q)
            colour[(size_t)picked[q]] = count;
        left -= (int32_t)keep;
        for (int32_t j = 0; j < n; ++j)
            state[(size_t)j] = colour[(size_t)j] >= 0 ? DONE : CANDIDATE;
        ++count;
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

namespace {

struct VertexOrders {
    uint8_t p[24][4];
    int32_t n = 0;
    explicit VertexOrders(int32_t k)
    {
        uint8_t a[4] = {0, 1, 2, 3};
        do {
            int inversions = 0;
            for (int i = 0; i < k; ++i)
                for (int j = i + 1; j < k; ++j)
                    inversions += a[i] > a[j];
            if (k == 2 || inversions % 2 == 0) {
                std::copy(a, a + 4, p[n]);
                ++n;
            }
        } while (std::next_permutation(a, a + k));
    }
};

const VertexOrders &orders_of(int32_t k)
{
    static const VertexOrders two(2), four(4);
    return k == 2 ? two : four;
}

// Conflict counters of the lanes of one colour: per aligned 16-lane group,
// vertex position and residue modulo 16 (reads), per aligned 8-lane group,
// position and residue modulo 8 (writes).
struct LaneCounts {
    int32_t k;
    std::vector<uint8_t> rd, wr;
    LaneCounts(int32_t n, int32_t k_)
        : k(k_), rd((size_t)((n + 15) / 16) * k_ * 16), wr((size_t)((n + 7) / 8) * k_ * 8) {}
    // pair cost of placing residues res[0..k) at lane l, against the lanes present
    int32_t cost(int32_t l, const uint8_t *res) const
    {
        const uint8_t *r = &rd[(size_t)(l / 16) * k * 16];
        const uint8_t *w = &wr[(size_t)(l / 8) * k * 8];
        int32_t c = 0;
        for (int32_t j = 0; j < k; ++j)
            c += 2 * r[j * 16 + res[j]] + 3 * w[j * 8 + (res[j] & 7)];
        return c;
    }
    void add(int32_t l, const uint8_t *res, int delta)
    {
        uint8_t *r = &rd[(size_t)(l / 16) * k * 16];
        uint8_t *w = &wr[(size_t)(l / 8) * k * 8];
        for (int32_t j = 0; j < k; ++j) {
            r[j * 16 + res[j]] = (uint8_t)(r[j * 16 + res[j]] + delta);
            w[j * 8 + (res[j] & 7)] = (uint8_t)(w[j * 8 + (res[j] & 7)] + delta);
        }
    }
};

}  // namespace

int32_t num_vertex_orders(int32_t k) { return orders_of(k).n; }

const uint8_t *vertex_order(int32_t k, int32_t index) { return orders_of(k).p[index]; }

void pack_lanes(const int32_t *slots, int32_t k, const std::vector<int32_t> &ptr, uint32_t seed,
                int32_t effort, std::vector<int32_t> &slot_id, std::vector<uint8_t> &order)
{
    const VertexOrders &O = orders_of(k);
    const int32_t P = O.n;
    order.assign(slot_id.size(), 0);
    std::mt19937 gen(seed);
    std::vector<uint8_t> res;
    std::vector<int32_t> items, pool, lane_q, lane_o;
    for (size_t c = 0; c + 1 < ptr.size(); ++c) {
        const int32_t b = ptr[c], n = ptr[c + 1] - ptr[c];
        if (n <= 0)
            continue;
        items.assign(slot_id.begin() + b, slot_id.begin() + b + n);
        // residues modulo 16 of every item under every vertex order
        res.assign((size_t)n * P * k, 0);
        for (int32_t q = 0; q < n; ++q)
            for (int32_t o = 0; o < P; ++o)
                for (int32_t j = 0; j < k; ++j)
                    res[((size_t)q * P + o) * k + j] =
                        (uint8_t)(slots[(size_t)items[(size_t)q] * k + O.p[o][j]] & 15);
        auto R = [&](int32_t q, int32_t o) { return &res[((size_t)q * P + o) * k]; };
        LaneCounts cnt(n, k);
        lane_q.assign((size_t)n, 0);
        lane_o.assign((size_t)n, 0);

        // greedy: each lane takes the cheapest (item, order) among a sample of the pool
        pool.resize((size_t)n);
        for (int32_t q = 0; q < n; ++q)
            pool[(size_t)q] = q;
        for (int32_t l = 0; l < n; ++l) {
            const int32_t m = (int32_t)pool.size();
            const int32_t tries = std::min(m, 96);
            int32_t best_p = 0, best_o = 0, best_c = INT32_MAX;
            for (int32_t t = 0; t < tries && best_c > 0; ++t) {
                const int32_t pi = tries == m ? t : (int32_t)(gen() % (uint32_t)m);
                for (int32_t o = 0; o < P && best_c > 0; ++o) {
                    const int32_t cst = cnt.cost(l, R(pool[(size_t)pi], o));
                    if (cst < best_c) {
                        best_c = cst;
                        best_p = pi;
                        best_o = o;
                    }
                }
            }
            lane_q[(size_t)l] = pool[(size_t)best_p];
            lane_o[(size_t)l] = best_o;
            cnt.add(l, R(lane_q[(size_t)l], best_o), 1);
            pool[(size_t)best_p] = pool.back();
            pool.pop_back();
        }

        // local search: swap two lanes (each item then takes its best order at
        // its new lane) or re-order one lane; keep moves that do not add cost
        auto best_order = [&](int32_t l, int32_t q, int32_t &o_out) {
            int32_t bc = INT32_MAX;
            for (int32_t o = 0; o < P; ++o) {
                const int32_t cst = cnt.cost(l, R(q, o));
                if (cst < bc) {
                    bc = cst;
                    o_out = o;
                }
            }
            return bc;
        };
        const int64_t moves = n > 1 ? (int64_t)effort * n : 0;
        for (int64_t mv = 0; mv < moves; ++mv) {
            const int32_t l1 = (int32_t)(gen() % (uint32_t)n);
            const int32_t q1 = lane_q[(size_t)l1], o1 = lane_o[(size_t)l1];
            cnt.add(l1, R(q1, o1), -1);
            const int32_t c1 = cnt.cost(l1, R(q1, o1));
            if (c1 == 0) {   // conflict-free lane: leave it
                cnt.add(l1, R(q1, o1), 1);
                continue;
            }
            if (gen() % 4 == 0) {
                int32_t o = o1;
                const int32_t bc = best_order(l1, q1, o);
                lane_o[(size_t)l1] = bc < c1 ? o : o1;
                cnt.add(l1, R(q1, lane_o[(size_t)l1]), 1);
                continue;
            }
            const int32_t l2 = (int32_t)(gen() % (uint32_t)n);
            if (l2 / 8 == l1 / 8) {
                cnt.add(l1, R(q1, o1), 1);
                continue;
            }
            const int32_t q2 = lane_q[(size_t)l2], o2 = lane_o[(size_t)l2];
            cnt.add(l2, R(q2, o2), -1);
            const int32_t before = c1 + cnt.cost(l2, R(q2, o2));
            int32_t n1 = 0, n2 = 0;
            int32_t after = best_order(l1, q2, n1);
            cnt.add(l1, R(q2, n1), 1);
            after += best_order(l2, q1, n2);
            if (after <= before) {
                cnt.add(l2, R(q1, n2), 1);
                lane_q[(size_t)l1] = q2;
                lane_o[(size_t)l1] = n1;
                lane_q[(size_t)l2] = q1;
                lane_o[(size_t)l2] = n2;
            } else {
                cnt.add(l1, R(q2, n1), -1);
                cnt.add(l1, R(q1, o1), 1);
                cnt.add(l2, R(q2, o2), 1);
            }
        }
        for (int32_t l = 0; l < n; ++l) {
            const int32_t id = items[(size_t)lane_q[(size_t)l]];
            slot_id[(size_t)(b + l)] = id;
            order[(size_t)id] = (uint8_t)lane_o[(size_t)l];
        }
    }
}

namespace {

// State of the joint search: every kind's lanes with their group counters,
// and for every particle the constraints that use it.
struct PackState {
    struct Kind {
        const int32_t *ids;
        int32_t k, n;
        const VertexOrders *O;
        std::vector<int32_t> lane_of, item, colour_begin, colour_end;   // per lane / item
        std::vector<uint8_t> ord;                                        // per item
        std::vector<int32_t> g16, g8;                                    // per lane
        std::vector<uint8_t> rd, wr;                                     // counters
    };
    std::vector<Kind> kinds;
    std::vector<int32_t> &slot_of;
    std::vector<std::vector<std::pair<int32_t, int32_t>>> uses;   // particle -> (kind, item)

    explicit PackState(std::vector<int32_t> &s) : slot_of(s) {}

    void residues(const Kind &K, int32_t q, int32_t o, uint8_t *res) const
    {
        for (int32_t j = 0; j < K.k; ++j)
            res[j] = (uint8_t)(slot_of[(size_t)K.ids[(size_t)q * K.k + K.O->p[o][j]]] & 15);
    }
    int32_t cost(const Kind &K, int32_t lane, const uint8_t *res) const
    {
        const uint8_t *r = &K.rd[(size_t)K.g16[(size_t)lane] * K.k * 16];
        const uint8_t *w = &K.wr[(size_t)K.g8[(size_t)lane] * K.k * 8];
        int32_t c = 0;
        for (int32_t j = 0; j < K.k; ++j)
            c += 2 * r[j * 16 + res[j]] + 3 * w[j * 8 + (res[j] & 7)];
        return c;
    }
    void count(Kind &K, int32_t lane, const uint8_t *res, int delta)
    {
        uint8_t *r = &K.rd[(size_t)K.g16[(size_t)lane] * K.k * 16];
        uint8_t *w = &K.wr[(size_t)K.g8[(size_t)lane] * K.k * 8];
        for (int32_t j = 0; j < K.k; ++j) {
            r[j * 16 + res[j]] = (uint8_t)(r[j * 16 + res[j]] + delta);
            w[j * 8 + (res[j] & 7)] = (uint8_t)(w[j * 8 + (res[j] & 7)] + delta);
        }
    }
    // remove item q's lane from the counters; returns its cost against the rest
    int32_t take(Kind &K, int32_t q)
    {
        uint8_t res[4];
        residues(K, q, K.ord[(size_t)q], res);
        count(K, K.lane_of[(size_t)q], res, -1);
        return cost(K, K.lane_of[(size_t)q], res);
    }
    int32_t put(Kind &K, int32_t q)
    {
        uint8_t res[4];
        residues(K, q, K.ord[(size_t)q], res);
        const int32_t c = cost(K, K.lane_of[(size_t)q], res);
        count(K, K.lane_of[(size_t)q], res, 1);
        return c;
    }
    // best vertex order of item q at its lane (counters without q); returns the cost
    int32_t best_order(Kind &K, int32_t q)
    {
        uint8_t res[4];
        int32_t bc = INT32_MAX, bo = K.ord[(size_t)q];
        for (int32_t o = 0; o < K.O->n; ++o) {
            residues(K, q, o, res);
            const int32_t c = cost(K, K.lane_of[(size_t)q], res);
            if (c < bc || (c == bc && o == K.ord[(size_t)q])) {
                bc = c;
                bo = o;
            }
        }
        K.ord[(size_t)q] = (uint8_t)bo;
        return bc;
    }
};

}  // namespace

namespace {

// Placement pre-pass: swap particles' slots so that, in every colour of every
// kind, the particles used are spread evenly over the 16 bank groups (a colour
// whose particles crowd one bank group cannot be packed conflict-free).
// Objective: sum over (kind, colour, bank group) of the squared count.
void balance_placement(int32_t num_particles, std::vector<int32_t> &slot_of,
                       const LaneSchedule *kinds, int32_t num_kinds, std::mt19937 &gen,
                       int64_t moves)
{
    // colour rows of every (kind, colour), and each particle's rows (with multiplicity)
    std::vector<std::vector<int32_t>> rows_of((size_t)num_particles);
    int32_t rows = 0;
    for (int32_t t = 0; t < num_kinds; ++t) {
        const LaneSchedule &L = kinds[t];
        const std::vector<int32_t> &ptr = *L.ptr;
        for (size_t c = 0; c + 1 < ptr.size(); ++c, ++rows)
            for (int32_t l = ptr[c]; l < ptr[c + 1]; ++l) {
                const int32_t q = (*L.slot_id)[(size_t)l];
                for (int32_t j = 0; j < L.k; ++j)
                    rows_of[(size_t)L.ids[(size_t)q * L.k + j]].push_back(rows);
            }
    }
    std::vector<int32_t> cnt((size_t)rows * 16, 0);
    for (int32_t p = 0; p < num_particles; ++p)
        for (int32_t r : rows_of[(size_t)p])
            cnt[(size_t)r * 16 + (slot_of[(size_t)p] & 15)]++;
    for (int64_t mv = 0; mv < moves && num_particles > 1; ++mv) {
        const int32_t p1 = (int32_t)(gen() % (uint32_t)num_particles);
        const int32_t p2 = (int32_t)(gen() % (uint32_t)num_particles);
        const int32_t g1 = slot_of[(size_t)p1] & 15, g2 = slot_of[(size_t)p2] & 15;
        if (g1 == g2)
            continue;
        // change of sum(cnt^2) when p1 moves g1 -> g2 and p2 moves g2 -> g1
        int64_t delta = 0;
        for (int32_t r : rows_of[(size_t)p1]) {
            int32_t &a = cnt[(size_t)r * 16 + g1], &b = cnt[(size_t)r * 16 + g2];
            delta += 2 * (b - a) + 2;
            --a;
            ++b;
        }
        for (int32_t r : rows_of[(size_t)p2]) {
            int32_t &a = cnt[(size_t)r * 16 + g2], &b = cnt[(size_t)r * 16 + g1];
            delta += 2 * (b - a) + 2;
            --a;
            ++b;
        }
        if (delta <= 0) {
            std::swap(slot_of[(size_t)p1], slot_of[(size_t)p2]);
        } else {
            for (int32_t r : rows_of[(size_t)p2]) {
                cnt[(size_t)r * 16 + g2]++;
                cnt[(size_t)r * 16 + g1]--;
            }
            for (int32_t r : rows_of[(size_t)p1]) {
                cnt[(size_t)r * 16 + g1]++;
                cnt[(size_t)r * 16 + g2]--;
            }
        }
    }
}

}  // namespace

void pack_lds(int32_t num_particles, std::vector<int32_t> &slot_of, LaneSchedule *kinds,
              int32_t num_kinds, uint32_t seed, int32_t effort)
{
    std::mt19937 gen(seed);
    balance_placement(num_particles, slot_of, kinds, num_kinds, gen, 200 * (int64_t)num_particles);
    // greedy start per kind, on the starting placement
    std::vector<int32_t> slots;
    for (int32_t t = 0; t < num_kinds; ++t) {
        const LaneSchedule &L = kinds[t];
        const size_t n = L.slot_id->size();
        slots.resize(n * (size_t)L.k);
        for (size_t i = 0; i < slots.size(); ++i)
            slots[i] = slot_of[(size_t)L.ids[i]];
        pack_lanes(slots.data(), L.k, *L.ptr, (uint32_t)gen(), 0, *L.slot_id, *L.order);
    }
    PackState S(slot_of);
    S.uses.assign((size_t)num_particles, {});
    S.kinds.resize((size_t)num_kinds);
    int64_t total_lanes = 0;
    for (int32_t t = 0; t < num_kinds; ++t) {
        const LaneSchedule &L = kinds[t];
        PackState::Kind &K = S.kinds[(size_t)t];
        K.ids = L.ids;
        K.k = L.k;
        K.n = (int32_t)L.slot_id->size();
        K.O = &orders_of(L.k);
        K.item = *L.slot_id;
        K.ord = *L.order;
        K.lane_of.assign((size_t)K.n, 0);
        K.colour_begin.assign((size_t)K.n, 0);
        K.colour_end.assign((size_t)K.n, 0);
        K.g16.assign((size_t)K.n, 0);
        K.g8.assign((size_t)K.n, 0);
        int32_t n16 = 0, n8 = 0;
        const std::vector<int32_t> &ptr = *L.ptr;
        for (size_t c = 0; c + 1 < ptr.size(); ++c) {
            for (int32_t l = ptr[c]; l < ptr[c + 1]; ++l) {
                K.colour_begin[(size_t)l] = ptr[c];
                K.colour_end[(size_t)l] = ptr[c + 1];
                K.g16[(size_t)l] = n16 + (l - ptr[c]) / 16;
                K.g8[(size_t)l] = n8 + (l - ptr[c]) / 8;
            }
            n16 += (ptr[c + 1] - ptr[c] + 15) / 16;
            n8 += (ptr[c + 1] - ptr[c] + 7) / 8;
        }
        K.rd.assign((size_t)n16 * K.k * 16, 0);
        K.wr.assign((size_t)n8 * K.k * 8, 0);
        for (int32_t l = 0; l < K.n; ++l)
            K.lane_of[(size_t)K.item[(size_t)l]] = l;
        for (int32_t q = 0; q < K.n; ++q) {
            S.put(K, q);
            for (int32_t j = 0; j < K.k; ++j)
                S.uses[(size_t)K.ids[(size_t)q * K.k + j]].push_back({t, q});
        }
        total_lanes += K.n;
    }

    std::vector<std::pair<int32_t, int32_t>> touched;
    std::vector<uint8_t> old_ord;
    std::vector<std::vector<int32_t>> seen((size_t)num_kinds);
    int32_t epoch = 0;
    for (int32_t t = 0; t < num_kinds; ++t)
        seen[(size_t)t].assign((size_t)S.kinds[(size_t)t].n, -1);
    const int64_t moves = (int64_t)effort * total_lanes;
    for (int64_t mv = 0; mv < moves; ++mv) {
        const uint32_t kind_of_move = gen() % 8;
        if (kind_of_move < 3 && num_particles > 1) {
            // swap the slots of two particles in different bank groups
            const int32_t p1 = (int32_t)(gen() % (uint32_t)num_particles);
            const int32_t p2 = (int32_t)(gen() % (uint32_t)num_particles);
            if (((slot_of[(size_t)p1] ^ slot_of[(size_t)p2]) & 15) == 0)
                continue;
            touched.clear();
            old_ord.clear();
            ++epoch;
            for (int32_t p : {p1, p2})
                for (const auto &u : S.uses[(size_t)p])
                    if (seen[(size_t)u.first][(size_t)u.second] != epoch) {
                        seen[(size_t)u.first][(size_t)u.second] = epoch;
                        touched.push_back(u);
                    }
            int32_t before = 0, after = 0;
            for (const auto &u : touched) {
                old_ord.push_back(S.kinds[(size_t)u.first].ord[(size_t)u.second]);
                before += S.take(S.kinds[(size_t)u.first], u.second);
            }
            std::swap(slot_of[(size_t)p1], slot_of[(size_t)p2]);
            for (const auto &u : touched) {
                PackState::Kind &K = S.kinds[(size_t)u.first];
                after += S.best_order(K, u.second);
                S.put(K, u.second);
            }
            if (after > before) {
                for (const auto &u : touched)
                    S.take(S.kinds[(size_t)u.first], u.second);
                std::swap(slot_of[(size_t)p1], slot_of[(size_t)p2]);
                for (size_t i = 0; i < touched.size(); ++i) {
                    PackState::Kind &K = S.kinds[(size_t)touched[i].first];
                    K.ord[(size_t)touched[i].second] = old_ord[i];
                    S.put(K, touched[i].second);
                }
            }
            continue;
        }
        // lane moves inside one colour of one kind (kinds chosen by size)
        int64_t pick = (int64_t)(gen() % (uint64_t)total_lanes);
        int32_t t = 0;
        while (pick >= S.kinds[(size_t)t].n) {
            pick -= S.kinds[(size_t)t].n;
            ++t;
        }
        PackState::Kind &K = S.kinds[(size_t)t];
        const int32_t l1 = (int32_t)pick;
        const int32_t q1 = K.item[(size_t)l1];
        const uint8_t o1 = K.ord[(size_t)q1];
        const int32_t c1 = S.take(K, q1);
        if (c1 == 0) {
            S.put(K, q1);
            continue;
        }
        if (kind_of_move == 3) {
            S.best_order(K, q1);
            S.put(K, q1);
            continue;
        }
        const int32_t b = K.colour_begin[(size_t)l1], e = K.colour_end[(size_t)l1];
        const int32_t l2 = b + (int32_t)(gen() % (uint32_t)(e - b));
        if (K.g8[(size_t)l2] == K.g8[(size_t)l1]) {
            S.put(K, q1);
            continue;
        }
        const int32_t q2 = K.item[(size_t)l2];
        const uint8_t o2 = K.ord[(size_t)q2];
        const int32_t before = c1 + S.take(K, q2);
        K.lane_of[(size_t)q1] = l2;
        K.lane_of[(size_t)q2] = l1;
        K.item[(size_t)l1] = q2;
        K.item[(size_t)l2] = q1;
        int32_t after = S.best_order(K, q2);
        S.put(K, q2);
        after += S.best_order(K, q1);
        if (after <= before) {
            S.put(K, q1);
        } else {
            S.take(K, q2);
            K.lane_of[(size_t)q1] = l1;
            K.lane_of[(size_t)q2] = l2;
            K.item[(size_t)l1] = q1;
            K.item[(size_t)l2] = q2;
            K.ord[(size_t)q1] = o1;
            K.ord[(size_t)q2] = o2;
            S.put(K, q1);
            S.put(K, q2);
        }
    }
    for (int32_t t = 0; t < num_kinds; ++t) {
        *kinds[t].slot_id = S.kinds[(size_t)t].item;
        *kinds[t].order = S.kinds[(size_t)t].ord;
    }
}

int64_t lane_conflicts(const int32_t *slots, int32_t k, const std::vector<int32_t> &ptr,
                       const std::vector<int32_t> &slot_id, const std::vector<uint8_t> &order)
{
    const VertexOrders &O = orders_of(k);
    int64_t extra = 0;
    for (size_t c = 0; c + 1 < ptr.size(); ++c)
        for (int32_t j = 0; j < k; ++j)
            for (int32_t width = 16; width >= 8; width -= 8)
                for (int32_t g = ptr[c]; g < ptr[c + 1]; g += width) {
                    int32_t m[16] = {0}, top = 0;
                    for (int32_t l = g; l < std::min(g + width, ptr[c + 1]); ++l) {
                        const int32_t id = slot_id[(size_t)l];
                        const int32_t s = slots[(size_t)id * k + O.p[order[(size_t)id]][j]];
                        top = std::max(top, ++m[s % width]);
                    }
                    extra += top - 1;
                }
    return extra;
}

void axis_neighbours(int32_t num_vertices, const float *rest_pos, std::vector<int32_t> &out)
{
    const size_t V = (size_t)std::max(num_vertices, 0);
    out.assign(V * 6, -1);
    std::vector<int32_t> ids(V);
    for (int axis = 0; axis < 3; ++axis) {
        const int o1 = (axis + 1) % 3, o2 = (axis + 2) % 3;
        auto c = [&](int32_t i, int k) { return rest_pos[3 * (size_t)i + k]; };
        std::iota(ids.begin(), ids.end(), 0);
        std::sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) {
            if (c(a, o1) != c(b, o1))
                return c(a, o1) < c(b, o1);
            if (c(a, o2) != c(b, o2))
                return c(a, o2) < c(b, o2);
            if (c(a, axis) != c(b, axis))
                return c(a, axis) < c(b, axis);
            return a < b;
        });
        // runs of equal (o1, o2); inside a run, blocks of equal coordinate along the axis
        size_t r = 0;
        while (r < V) {
            size_t e = r;
            while (e < V && c(ids[e], o1) == c(ids[r], o1) && c(ids[e], o2) == c(ids[r], o2))
                ++e;
            size_t prev_block = V;   // first index of the previous block
            size_t b = r;
            while (b < e) {
                size_t nb = b;
                while (nb < e && c(ids[nb], axis) == c(ids[b], axis))
                    ++nb;
                for (size_t k = b; k < nb; ++k) {
                    if (prev_block != V)
                        out[(size_t)ids[k] * 6 + 2 * axis] = ids[prev_block];
                    if (nb < e)
                        out[(size_t)ids[k] * 6 + 2 * axis + 1] = ids[nb];
                }
                prev_block = b;
                b = nb;
            }
            r = e;
        }
    }
}

int prepare_mesh(int32_t num_vertices, int32_t num_tets, const float *rest_pos,
                 const float *inv_mass, const int32_t *tets, PreparedMesh &out,
                 std::string &error, int32_t colouring)
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

    if (colouring == XPBD_COLOURING_GREEDY) {
        out.num_edge_colours = greedy_colouring(num_vertices, out.num_edges(), 2,
                                                out.edges.data(), out.edge_colour);
        out.num_tet_colours = greedy_colouring(num_vertices, out.num_tets(), 4, out.tets.data(),
                                               out.tet_colour);
    } else {
        const int32_t cut = colouring == XPBD_COLOURING_WAVES ? kWaveCutAbove : 0;
        const int32_t cap = colouring == XPBD_COLOURING_CAPPED || colouring == XPBD_COLOURING_CAPPED_FIT
                                ? kColourCap
                            : colouring == XPBD_COLOURING_CAPPED_128 ? kColourCap128
                                                                      : 0;
        out.num_edge_colours = largest_first_colouring(num_vertices, out.num_edges(), 2,
                                                       out.edges.data(), cut, cap, out.edge_colour);
        out.num_tet_colours = largest_first_colouring(num_vertices, out.num_tets(), 4,
                                                      out.tets.data(), cut, cap, out.tet_colour);
        // CAPPED_FIT: keep the cap only while one round per colour stays within
        // the register variant's rounds (each kind's count rounded up to even)
        const auto even = [](int32_t n) { return n + (n & 1); };
        if (colouring == XPBD_COLOURING_CAPPED_FIT &&
            even(out.num_edge_colours) + even(out.num_tet_colours) > kFitRounds) {
            out.num_edge_colours = largest_first_colouring(num_vertices, out.num_edges(), 2,
                                                           out.edges.data(), 0, 0, out.edge_colour);
            out.num_tet_colours = largest_first_colouring(num_vertices, out.num_tets(), 4,
                                                          out.tets.data(), 0, 0, out.tet_colour);
        }
    }

    // surface triangles (capsule tools): faces of exactly one kept tetrahedron,
    // ordered outward (away from the tetrahedron's fourth vertex), sorted by
    // their ascending vertex triple
    struct FaceKey {
        int32_t v[3];      // ascending
        int32_t tri[3];    // as taken from the tetrahedron
        int32_t opposite;
    };
    std::vector<FaceKey> fk;
    fk.reserve(4 * T);
    for (size_t t = 0; t < T; ++t)
        for (int skip = 0; skip < 4; ++skip) {
            FaceKey f;
            int n = 0;
            for (int k = 0; k < 4; ++k)
                if (k != skip)
                    f.tri[n++] = out.tets[4 * t + k];
            f.opposite = out.tets[4 * t + skip];
            std::copy(f.tri, f.tri + 3, f.v);
            std::sort(f.v, f.v + 3);
            fk.push_back(f);
        }
    std::sort(fk.begin(), fk.end(), [](const FaceKey &x, const FaceKey &y) {
        return std::lexicographical_compare(x.v, x.v + 3, y.v, y.v + 3);
    });
    for (size_t k = 0; k < fk.size();) {
        size_t e = k + 1;
        while (e < fk.size() && std::equal(fk[e].v, fk[e].v + 3, fk[k].v))
            ++e;
        if (e - k == 1) {
            int32_t i = fk[k].tri[0], j = fk[k].tri[1], m = fk[k].tri[2];
            double u[3], w[3], o[3];
            for (int c = 0; c < 3; ++c) {
                u[c] = (double)rest_pos[3 * j + c] - (double)rest_pos[3 * i + c];
                w[c] = (double)rest_pos[3 * m + c] - (double)rest_pos[3 * i + c];
                o[c] = (double)rest_pos[3 * fk[k].opposite + c] - (double)rest_pos[3 * i + c];
            }
            const double nx = u[1] * w[2] - u[2] * w[1], ny = u[2] * w[0] - u[0] * w[2],
                         nz = u[0] * w[1] - u[1] * w[0];
            if (nx * o[0] + ny * o[1] + nz * o[2] > 0.0)
                std::swap(j, m);
            out.faces.push_back(i);
            out.faces.push_back(j);
            out.faces.push_back(m);
        }
        k = e;
    }
    out.num_face_colours = greedy_colouring(num_vertices, out.num_faces(), 3, out.faces.data(),
                                            out.face_colour);
    return XPBD_OK;
}

}  // namespace xpbd
