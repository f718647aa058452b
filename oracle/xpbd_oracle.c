/*
 * FP64 oracle for the batched XPBD substep of FF-SRL
 * (Dall'Alba, Naskret, Kaminska, Korzeniowski: "FF-SRL: High Performance
 * GPU-Based Surgical Simulation For Robot Learning", arXiv 2503.18616).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct
 * CPU implementation of what the GPU library computes.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may build, load or
 * call it.  It shares no code, header, table or helper with the GPU library,
 * and the library never calls it.
 *
 * What it follows, by passage of the paper:
 *   Sec. III-A.1      particles with inverse masses w, positions x, velocities v;
 *                     edges and tetrahedra; rest length and rest volume
 *                     computed once before the simulation loop.
 *   Sec. III-A.1 Eq.1 distance constraint C = |x_a - x_b| - d_ab.
 *   Sec. III-A.1 Eq.2-3 volume constraint C = (1/6)(x_ba x x_ca).x_da - V0.
 *   Sec. III-A.1 Alg.1 step loop around a substep loop with h = dt/substeps,
 *                     velocity prediction v + h g, position prediction x + h v,
 *                     constraint projection, v = (x_new - x_old)/h.
 *   Sec. III-A.3      tool contact: after the deformation constraints, a
 *                     penetrating point is pushed out along the penetration
 *                     direction with stiffness k_c = 1.
 *   Sec. III-A        the solver is XPBD (the paper's cited method): every
 *                     constraint j carries a multiplier lambda_j and a compliance
 *                     alpha_j, alpha~ = alpha / h^2, and one projection is
 *                       dlambda = (-C - alpha~ lambda) / (sum_i w_i |grad_i C|^2 + alpha~)
 *                       x_i    += w_i * dlambda * grad_i C
 *                     With alpha = 0 and lambda = 0 this is exactly the paper's
 *                     stiffness form (Eq. 1 and corrected Eqs. 2-3) with k = 1.
 *
 * Readings taken where the paper is silent, garbled or at odds with the
 * configurations this oracle serves:
 *   R1  Gauss-Seidel over graph colours replaces the paper's Jacobi average
 *       (Sec. III-A.1): all edge colours ascending, then all tetrahedron
 *       colours ascending, then contact, repeated `iterations` times per substep.
 *   R2  Eq. 2 as printed permutes the gradient terms and flips one sign; the
 *       analytic gradients of the printed C are used:
 *       g_b = x_ca x x_da / 6, g_c = x_da x x_ba / 6, g_d = x_ba x x_ca / 6,
 *       g_a = -(g_b + g_c + g_d).
 *   R3  Eq. 3 omits inverse masses; the XPBD denominator sum_i w_i |g_i|^2 is
 *       used, identical to the paper for uniform free masses.
 *   R4  lambda is reset to zero at every substep and accumulates over the
 *       iterations of that substep.
 *   R5  Pinned particles (w = 0) are not predicted and never move; constraints
 *       whose particles are all pinned are dropped before colouring.
 *   R6  The tool pose is constant within a step.  Contact candidates
 *       K = { i : w_i > 0, |x_i - c|^2 < (2r)^2 } are found once per step on
 *       the start-of-step positions; the push-out runs after the deformation
 *       constraints of every iteration: if |x_i - c|^2 < r^2 the particle
 *       moves to c + r (x_i - c)/|x_i - c|, or to c + (0,0,r) when x_i = c.
 *   R7  A distance constraint with |x_a - x_b| < 1e-9 m, and any constraint
 *       whose denominator is <= 1e-30, is skipped.
 *   R8  Residual of constraint j: (C_j + alpha~_j lambda_j) / s_j with
 *       s_j = rest length (edges) or rest volume (tetrahedra), evaluated after
 *       the last iteration of a substep, before the velocity update; reported
 *       as the RMS and the maximum absolute value over all kept constraints.
 *   R9  Tetrahedra with negative rest volume have their last two vertices
 *       swapped; a zero rest volume is an error.
 *   R10 Edges are the unique vertex pairs of the kept tetrahedra, ordered by
 *       (smaller id, larger id).  Greedy colouring visits constraints in index
 *       order and gives each the smallest colour not used by an earlier
 *       constraint sharing any particle; edges and tetrahedra are coloured
 *       separately.
 *       R13 below is an alternative colouring the same way (largest first).
 *   R11 Capsule tools (the paper's grasper capsules, Sec. III-A.2/3) act on
 *       the surface triangles (faces of exactly one kept tetrahedron, ordered
 *       outward), not on particles: a capsule is a segment p0 p1 and a radius
 *       r, its SDF is the distance to the segment minus r.  The deepest point
 *       of a face is its exact closest point to the segment (the local
 *       optimisation of the cited contact scheme reaches it: the distance is
 *       convex over the triangle).  Candidates: faces with a free particle
 *       closer than 2r to the segment on the start-of-step positions, found
 *       once per step; after the deformation constraints of every iteration
 *       each candidate (face colour ascending, face id ascending) is pushed
 *       out with k_c = 1 as a constraint C = d - r on its closest point
 *       q = sum_i b_i x_i (gradient b_i n, n from the axis to q, the face
 *       normal when d ~ 0).
 *   R12 Grasping (Sec. III-A.2) with a sphere standing in for the closed
 *       clamps: the dragging point is the grasping tool's centre plus a fixed
 *       offset.  Closing the grasper (a policy output above 0, the analogue of
 *       a clamp angle below 3 degrees) while nothing is held takes the free
 *       particle closest to the dragging point strictly within r_l, on the
 *       start-of-step positions after the tool has moved; opening releases
 *       it; a held particle stays held while the grasper stays closed.  One
 *       particle per grasper is held (the per-particle drag flag is true for
 *       at most that one).  The drag constraint (k_s = 1, rest length 0)
 *       runs after the tool contacts of every iteration, so the held
 *       particle ends every iteration on the dragging point.
 *
 *   R13 Largest-first colouring, selectable instead of R10 for the edges and
 *       the tetrahedra (recursive largest first, Leighton 1979): colours are
 *       built one at a time as maximal sets of disjoint uncoloured
 *       constraints (rules at oracle_largest_first_colour); optionally a
 *       colour of 65 .. cut_above members is cut to its first 64, so that it
 *       fills one 64-wide group of parallel lanes, or every colour is capped
 *       at its first cap members, so that it fits one pass of cap parallel
 *       lanes; a per-mesh choice keeps the 256 cap only while the mesh's
 *       edge and tetrahedron colour counts, each rounded up to even, sum to
 *       at most 64, and else takes the uncapped colouring (oracle/__init__.py,
 *       mesh_colours).  A colouring only fixes the Gauss-Seidel order (R1);
 *       both sides take it from the same rules.
 *
 * Every function below is pinned by the not-gpu tests (closed forms,
 * invariants and brute force on tiny meshes).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fused multiply-add, so
 * that every product and sum is rounded as written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_E_ARG (-1)
#define ORACLE_E_MESH (-2)
#define ORACLE_E_NOMEM (-3)

#define MIN_EDGE_LENGTH 1e-9
#define MIN_DENOMINATOR 1e-30

/* ------------------------------------------------------------------ */
/* 3-vector helpers                                                    */
/* ------------------------------------------------------------------ */
static void sub3(const double *a, const double *b, double *o)
{
    o[0] = a[0] - b[0];
    o[1] = a[1] - b[1];
    o[2] = a[2] - b[2];
}

static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------------ */
/* Constraint functions (Sec. III-A.1)                                 */
/* ------------------------------------------------------------------ */

/* Signed volume of tetrahedron (a, b, c, d) (Sec. III-A.1, volume constraint):
 * (1/6)(x_ba x x_ca) . x_da with x_ba = x_b - x_a, evaluated as the equal
 * triple product x_ba . (x_ca x x_da / 6), the same expression the constraint
 * uses, so that a mesh at its rest positions has C = 0 exactly. */
double oracle_tet_volume(const double *xa, const double *xb, const double *xc,
                         const double *xd)
{
    double xba[3], xca[3], xda[3], gb[3];
    sub3(xb, xa, xba);
    sub3(xc, xa, xca);
    sub3(xd, xa, xda);
    cross3(xca, xda, gb);
    for (int k = 0; k < 3; ++k)
        gb[k] /= 6.0;
    return dot3(xba, gb);
}

/* Gradients of the volume constraint (Eqs. 2-3 with reading R2).
 * x: [4][3] positions of a, b, c, d; g: [4][3] output.  Returns the volume. */
double oracle_tet_gradients(const double *x, double *g)
{
    const double *xa = x, *xb = x + 3, *xc = x + 6, *xd = x + 9;
    double xba[3], xca[3], xda[3];
    sub3(xb, xa, xba);
    sub3(xc, xa, xca);
    sub3(xd, xa, xda);
    double *ga = g, *gb = g + 3, *gc = g + 6, *gd = g + 9;
    cross3(xca, xda, gb);
    cross3(xda, xba, gc);
    cross3(xba, xca, gd);
    for (int k = 0; k < 3; ++k) {
        gb[k] /= 6.0;
        gc[k] /= 6.0;
        gd[k] /= 6.0;
        ga[k] = -(gb[k] + gc[k] + gd[k]);
    }
    return dot3(xba, gb);
}

/* One XPBD projection of the distance constraint of edge (a, b)
 * (Eq. 1 in compliance form).  Updates x and *lambda. */
void oracle_project_distance(double *x, const double *w, int a, int b,
                             double rest_length, double alpha_tilde, double *lambda)
{
    double xab[3];
    sub3(x + 3 * a, x + 3 * b, xab);
    double length = sqrt(dot3(xab, xab));
    if (length < MIN_EDGE_LENGTH)
        return;
    double C = length - rest_length;
    double denominator = w[a] + w[b] + alpha_tilde;
    if (denominator <= MIN_DENOMINATOR)
        return;
    double dlambda = (-C - alpha_tilde * (*lambda)) / denominator;
    *lambda += dlambda;
    for (int k = 0; k < 3; ++k) {
        double n = xab[k] / length;            /* grad_a C = n, grad_b C = -n */
        x[3 * a + k] += w[a] * dlambda * n;
        x[3 * b + k] -= w[b] * dlambda * n;
    }
}

/* One XPBD projection of the volume constraint of tetrahedron q[4]
 * (Eqs. 2-3 with readings R2, R3).  Updates x and *lambda. */
void oracle_project_volume(double *x, const double *w, const int32_t *q,
                           double rest_volume, double alpha_tilde, double *lambda)
{
    double p[12], g[12];
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 3; ++k)
            p[3 * i + k] = x[3 * q[i] + k];
    double volume = oracle_tet_gradients(p, g);
    double C = volume - rest_volume;
    double denominator = alpha_tilde;
    for (int i = 0; i < 4; ++i)
        denominator += w[q[i]] * dot3(g + 3 * i, g + 3 * i);
    if (denominator <= MIN_DENOMINATOR)
        return;
    double dlambda = (-C - alpha_tilde * (*lambda)) / denominator;
    *lambda += dlambda;
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 3; ++k)
            x[3 * q[i] + k] += w[q[i]] * dlambda * g[3 * i + k];
}

/* Push a particle out of a sphere tool (Sec. III-A.3, reading R6). */
void oracle_project_contact(double *xi, const double *centre, double radius)
{
    double d[3];
    sub3(xi, centre, d);
    double d2 = dot3(d, d);
    if (!(d2 < radius * radius))
        return;
    double dist = sqrt(d2);
    if (dist > 0.0) {
        for (int k = 0; k < 3; ++k)
            xi[k] = centre[k] + d[k] * (radius / dist);
    } else {
        xi[0] = centre[0];
        xi[1] = centre[1];
        xi[2] = centre[2] + radius;
    }
}

/* ------------------------------------------------------------------ */
/* Set-up (Sec. III-A.1: rest values computed before the loop)         */
/* ------------------------------------------------------------------ */

/* Keep the tetrahedra that have at least one free particle, orient them
 * (R9) and compute their rest volumes.  tets_out/rest_volume_out hold up to
 * T entries; *kept receives the count.  rest: [V][3]. */
int oracle_setup_tets(int V, const double *rest, const double *w, int T,
                      const int32_t *tets_in, int32_t *tets_out,
                      double *rest_volume_out, int *kept)
{
    if (V <= 0 || T < 0 || !rest || !w || (T > 0 && (!tets_in || !tets_out || !rest_volume_out)) || !kept)
        return ORACLE_E_ARG;
    int n = 0;
    for (int t = 0; t < T; ++t) {
        int32_t q[4];
        for (int i = 0; i < 4; ++i) {
            q[i] = tets_in[4 * t + i];
            if (q[i] < 0 || q[i] >= V)
                return ORACLE_E_ARG;
        }
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j)
                if (q[i] == q[j])
                    return ORACLE_E_MESH;
        if (w[q[0]] == 0.0 && w[q[1]] == 0.0 && w[q[2]] == 0.0 && w[q[3]] == 0.0)
            continue;
        double vol = oracle_tet_volume(rest + 3 * q[0], rest + 3 * q[1], rest + 3 * q[2],
                                       rest + 3 * q[3]);
        if (vol == 0.0)
            return ORACLE_E_MESH;
        if (vol < 0.0) {
            int32_t s = q[2];
            q[2] = q[3];
            q[3] = s;
            vol = oracle_tet_volume(rest + 3 * q[0], rest + 3 * q[1], rest + 3 * q[2],
                                    rest + 3 * q[3]);
        }
        memcpy(tets_out + 4 * n, q, sizeof q);
        rest_volume_out[n] = vol;
        ++n;
    }
    *kept = n;
    return ORACLE_OK;
}

static int compare_pairs(const void *pa, const void *pb)
{
    const int32_t *a = (const int32_t *)pa, *b = (const int32_t *)pb;
    if (a[0] != b[0])
        return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1])
        return a[1] < b[1] ? -1 : 1;
    return 0;
}

/* Unique edges of the tetrahedra (R10), both-pinned edges dropped (R5), rest
 * lengths in FP64.  edges_out must hold 6*T pairs; *E receives the count. */
int oracle_setup_edges(int V, const double *rest, const double *w, int T,
                       const int32_t *tets, int32_t *edges_out, double *rest_length_out,
                       int *E)
{
    if (V <= 0 || T < 0 || !rest || !w || !E)
        return ORACLE_E_ARG;
    if (T == 0) {
        *E = 0;
        return ORACLE_OK;
    }
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * 12 * (size_t)T);
    if (!pairs)
        return ORACLE_E_NOMEM;
    int n = 0;
    for (int t = 0; t < T; ++t)
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j) {
                int32_t a = tets[4 * t + i], b = tets[4 * t + j];
                pairs[2 * n] = a < b ? a : b;
                pairs[2 * n + 1] = a < b ? b : a;
                ++n;
            }
    qsort(pairs, (size_t)n, 2 * sizeof(int32_t), compare_pairs);
    int m = 0;
    for (int i = 0; i < n; ++i) {
        int32_t a = pairs[2 * i], b = pairs[2 * i + 1];
        if (i > 0 && a == pairs[2 * i - 2] && b == pairs[2 * i - 1])
            continue;
        if (w[a] == 0.0 && w[b] == 0.0)
            continue;
        edges_out[2 * m] = a;
        edges_out[2 * m + 1] = b;
        double d[3];
        sub3(rest + 3 * a, rest + 3 * b, d);
        rest_length_out[m] = sqrt(dot3(d, d));
        ++m;
    }
    free(pairs);
    *E = m;
    return ORACLE_OK;
}

/* Greedy colouring (R10).  verts: [n][k] particle ids of n constraints with
 * k particles each.  colour_out: [n].  Returns the number of colours, or a
 * negative error code. */
int oracle_greedy_colour(int V, int n, int k, const int32_t *verts, int32_t *colour_out)
{
    if (V <= 0 || n < 0 || k <= 0 || (n > 0 && (!verts || !colour_out)))
        return ORACLE_E_ARG;
    /* incidence lists: constraints touching each particle */
    int *count = (int *)calloc((size_t)V + 1, sizeof(int));
    int *incident = (int *)malloc(sizeof(int) * ((size_t)n * k + 1));
    int *used = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    if (!count || !incident || !used) {
        free(count);
        free(incident);
        free(used);
        return ORACLE_E_NOMEM;
    }
    for (int i = 0; i < n * k; ++i)
        count[verts[i] + 1]++;
    for (int v = 0; v < V; ++v)
        count[v + 1] += count[v];
    int *fill = (int *)malloc(sizeof(int) * (size_t)(V + 1));
    if (!fill) {
        free(count);
        free(incident);
        free(used);
        return ORACLE_E_NOMEM;
    }
    memcpy(fill, count, sizeof(int) * (size_t)(V + 1));
    for (int c = 0; c < n; ++c)
        for (int j = 0; j < k; ++j)
            incident[fill[verts[c * k + j]]++] = c;
    free(fill);

    int num_colours = 0;
    for (int c = 0; c < n; ++c) {
        /* mark the colours of earlier constraints that share a particle */
        for (int i = 0; i <= num_colours; ++i)
            used[i] = 0;
        for (int j = 0; j < k; ++j) {
            int v = verts[c * k + j];
            for (int p = count[v]; p < count[v + 1]; ++p) {
                int other = incident[p];
                if (other < c)
                    used[colour_out[other]] = 1;
            }
        }
        int colour = 0;
        while (used[colour])
            ++colour;
        colour_out[c] = colour;
        if (colour + 1 > num_colours)
            num_colours = colour + 1;
    }
    free(count);
    free(incident);
    free(used);
    return num_colours;
}

/* Recursive largest-first colouring (R13), an alternative to R10 with fewer
 * and larger colours.  Colours are built one after the other; colour c is a
 * maximal set of mutually disjoint constraints (no shared particle) taken
 * from those without a colour yet:
 *   - it starts with the uncoloured constraint that conflicts with the most
 *     other uncoloured constraints (ties: the lowest index);
 *   - then, while some uncoloured constraint conflicts with no member
 *     ("candidate"), it adds the candidate that conflicts with the most
 *     "excluded" constraints (uncoloured ones that conflict with a member),
 *     ties broken by the fewest conflicts with other candidates, then by the
 *     lowest index.
 * With cut_above > 64, a colour that ends with 65 .. cut_above members keeps
 * only its first 64 (in the order they were added); with cap > 0, a colour
 * keeps at most its first cap members.  The members a colour does not keep
 * stay uncoloured for the following colours.  Counts are recomputed from
 * scratch for every choice.  Returns the number of colours or a negative
 * error. */
int oracle_largest_first_colour(int V, int n, int k, const int32_t *verts, int cut_above, int cap,
                                int32_t *colour_out)
{
    if (V <= 0 || n < 0 || k <= 0 || (n > 0 && (!verts || !colour_out)))
        return ORACLE_E_ARG;
    /* neighbours of every constraint (sharing a particle), without repeats */
    int *start = (int *)calloc((size_t)V + 1, sizeof(int));
    int *touch = (int *)malloc(sizeof(int) * ((size_t)n * k + 1));
    int *nb_start = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int *mark = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int *state = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int *order = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    if (!start || !touch || !nb_start || !mark || !state || !order) {
        free(start); free(touch); free(nb_start); free(mark); free(state); free(order);
        return ORACLE_E_NOMEM;
    }
    for (int i = 0; i < n * k; ++i)
        start[verts[i] + 1]++;
    for (int v = 0; v < V; ++v)
        start[v + 1] += start[v];
    {
        int *pos = (int *)malloc(sizeof(int) * ((size_t)V + 1));
        if (!pos) {
            free(start); free(touch); free(nb_start); free(mark); free(state); free(order);
            return ORACLE_E_NOMEM;
        }
        memcpy(pos, start, sizeof(int) * (size_t)(V + 1));
        for (int c = 0; c < n; ++c)
            for (int j = 0; j < k; ++j)
                touch[pos[verts[c * k + j]]++] = c;
        free(pos);
    }
    size_t total = 0;
    for (int c = 0; c < n; ++c)
        mark[c] = -1;
    for (int c = 0; c < n; ++c) {
        nb_start[c] = (int)total;
        for (int j = 0; j < k; ++j) {
            int v = verts[c * k + j];
            for (int p = start[v]; p < start[v + 1]; ++p)
                if (touch[p] != c && mark[touch[p]] != c) {
                    mark[touch[p]] = c;
                    ++total;
                }
        }
    }
    nb_start[n] = (int)total;
    int *nb = (int *)malloc(sizeof(int) * (total + 1));
    if (!nb) {
        free(start); free(touch); free(nb_start); free(mark); free(state); free(order);
        return ORACLE_E_NOMEM;
    }
    for (int c = 0; c < n; ++c)
        mark[c] = -1;
    for (int c = 0; c < n; ++c) {
        int q = nb_start[c];
        for (int j = 0; j < k; ++j) {
            int v = verts[c * k + j];
            for (int p = start[v]; p < start[v + 1]; ++p)
                if (touch[p] != c && mark[touch[p]] != c) {
                    mark[touch[p]] = c;
                    nb[q++] = touch[p];
                }
        }
    }
    free(start);
    free(touch);

    enum { COLOURED = 0, CANDIDATE = 1, EXCLUDED = 2, MEMBER = 3 };
    for (int c = 0; c < n; ++c)
        colour_out[c] = -1;
    int left = n, num_colours = 0;
    while (left > 0) {
        for (int c = 0; c < n; ++c)
            state[c] = colour_out[c] >= 0 ? COLOURED : CANDIDATE;
        /* first member: most conflicts among the uncoloured */
        int best = -1, best_count = -1;
        for (int c = 0; c < n; ++c) {
            if (state[c] != CANDIDATE)
                continue;
            int cnt = 0;
            for (int p = nb_start[c]; p < nb_start[c + 1]; ++p)
                cnt += state[nb[p]] != COLOURED;
            if (cnt > best_count) {
                best = c;
                best_count = cnt;
            }
        }
        int members = 0;
        while (best >= 0) {
            state[best] = MEMBER;
            order[members++] = best;
            for (int p = nb_start[best]; p < nb_start[best + 1]; ++p)
                if (state[nb[p]] == CANDIDATE)
                    state[nb[p]] = EXCLUDED;
            /* next member: most conflicts with the excluded, then fewest with candidates */
            best = -1;
            int best_x = -1, best_u = 0;
            for (int c = 0; c < n; ++c) {
                if (state[c] != CANDIDATE)
                    continue;
                int x = 0, u = 0;
                for (int p = nb_start[c]; p < nb_start[c + 1]; ++p) {
                    x += state[nb[p]] == EXCLUDED;
                    u += state[nb[p]] == CANDIDATE;
                }
                if (x > best_x || (x == best_x && u < best_u)) {
                    best = c;
                    best_x = x;
                    best_u = u;
                }
            }
        }
        int keep = members;
        if (cut_above > 64 && members > 64 && members <= cut_above)
            keep = 64;
        if (cap > 0 && keep > cap)
            keep = cap;
        for (int q = 0; q < keep; ++q)
            colour_out[order[q]] = num_colours;
        left -= keep;
        ++num_colours;
    }
    free(nb);
    free(nb_start);
    free(mark);
    free(state);
    free(order);
    return num_colours;
}

/* ------------------------------------------------------------------ */
/* Simulation (Algorithm 1 with readings R1-R8)                        */
/* ------------------------------------------------------------------ */

/* Residual of all kept constraints (R8).  out[0] = RMS, out[1] = max |r|. */
void oracle_residual(const double *x, int E, const int32_t *edges, const double *rest_length,
                     int T, const int32_t *tets, const double *rest_volume,
                     double alpha_tilde_d, double alpha_tilde_v, const double *lambda,
                     double *out)
{
    double sum = 0.0, largest = 0.0;
    for (int e = 0; e < E; ++e) {
        double d[3];
        sub3(x + 3 * edges[2 * e], x + 3 * edges[2 * e + 1], d);
        double C = sqrt(dot3(d, d)) - rest_length[e];
        double r = (C + alpha_tilde_d * lambda[e]) / rest_length[e];
        sum += r * r;
        if (fabs(r) > largest)
            largest = fabs(r);
    }
    for (int t = 0; t < T; ++t) {
        const int32_t *q = tets + 4 * t;
        double C = oracle_tet_volume(x + 3 * q[0], x + 3 * q[1], x + 3 * q[2], x + 3 * q[3])
                   - rest_volume[t];
        double r = (C + alpha_tilde_v * lambda[E + t]) / rest_volume[t];
        sum += r * r;
        if (fabs(r) > largest)
            largest = fabs(r);
    }
    out[0] = (E + T) > 0 ? sqrt(sum / (double)(E + T)) : 0.0;
    out[1] = largest;
}

/*
 * Contact candidates of one sphere (R6): ascending ids i with w_i > 0 and
 * |x_i - c|^2 < (2r)^2 on the positions x; returns their number.
 */
int oracle_candidates(int V, const double *w, const double *x, const double *centre,
                      double radius, int32_t *out)
{
    double reach = 2.0 * radius;
    int n = 0;
    for (int i = 0; i < V; ++i) {
        double d[3];
        sub3(x + 3 * i, centre, d);
        if (w[i] > 0.0 && dot3(d, d) < reach * reach)
            out[n++] = i;
    }
    return n;
}

/*
 * Prediction of one substep (Alg. 1): x_prev = x; for free particles
 * v += h g and x += h v; pinned particles stay (R5).
 */
void oracle_predict(int V, const double *w, double h, const double *gravity, double *x,
                    double *v, double *x_prev)
{
    for (int i = 0; i < V; ++i) {
        for (int k = 0; k < 3; ++k)
            x_prev[3 * i + k] = x[3 * i + k];
        if (w[i] > 0.0)
            for (int k = 0; k < 3; ++k) {
                v[3 * i + k] += h * gravity[k];
                x[3 * i + k] += h * v[3 * i + k];
            }
    }
}

/*
 * One Gauss-Seidel iteration (R1): every edge colour in ascending order, every
 * tetrahedron colour in ascending order, then the push-out of every tool's
 * candidates (Sec. III-A.3).  candidates: [num_tools][V] ids, counts [num_tools].
 */
void oracle_iterate(double *x, const double *w,
                    int E, const int32_t *edges, const double *rest_length,
                    const double *rest_volume, const int32_t *tets,
                    int num_edge_colours, const int32_t *edge_colour_ptr, const int32_t *edge_order,
                    int num_tet_colours, const int32_t *tet_colour_ptr, const int32_t *tet_order,
                    double alpha_tilde_d, double alpha_tilde_v, double *lambda,
                    int V, int num_tools, const double *centres, const double *tool_radius,
                    const int32_t *candidates, const int *num_candidates)
{
    /* distance constraints, colour by colour (Eq. 1, R1) */
    for (int c = 0; c < num_edge_colours; ++c)
        for (int p = edge_colour_ptr[c]; p < edge_colour_ptr[c + 1]; ++p) {
            int e = edge_order[p];
            oracle_project_distance(x, w, edges[2 * e], edges[2 * e + 1], rest_length[e],
                                    alpha_tilde_d, &lambda[e]);
        }
    /* volume constraints, colour by colour (Eqs. 2-3, R1-R3) */
    for (int c = 0; c < num_tet_colours; ++c)
        for (int p = tet_colour_ptr[c]; p < tet_colour_ptr[c + 1]; ++p) {
            int t = tet_order[p];
            oracle_project_volume(x, w, tets + 4 * t, rest_volume[t], alpha_tilde_v,
                                  &lambda[E + t]);
        }
    /* tool contact after the deformation constraints (Sec. III-A.3) */
    for (int t = 0; t < num_tools; ++t)
        for (int n = 0; n < num_candidates[t]; ++n) {
            int i = candidates[(size_t)t * V + n];
            oracle_project_contact(x + 3 * i, centres + 3 * t, tool_radius[t]);
        }
}

/*
 * One iteration of the paper's own parallel solver (Sec. III-A.1, Alg. 1):
 * every constraint is projected from the same positions x (Jacobi), its
 * correction w_i dlambda grad_i C is summed per particle, and each particle
 * then moves by its sum divided by n_i, the number of kept constraints that
 * include it (count[i]; particles without one do not move).  The multipliers
 * accumulate as in oracle_iterate; with one iteration, zero compliance and
 * uniform free masses this is the printed update with k = 1 averaged by n.
 * dx: [V][3] scratch.  Tool contact follows, as in oracle_iterate.
 */
void oracle_iterate_jacobi(double *x, const double *w,
                           int E, const int32_t *edges, const double *rest_length,
                           int T, const int32_t *tets, const double *rest_volume,
                           double alpha_tilde_d, double alpha_tilde_v, double *lambda,
                           const int32_t *count, double *dx,
                           int V, int num_tools, const double *centres, const double *tool_radius,
                           const int32_t *candidates, const int *num_candidates)
{
    for (int i = 0; i < 3 * V; ++i)
        dx[i] = 0.0;
    for (int e = 0; e < E; ++e) {
        const int a = edges[2 * e], b = edges[2 * e + 1];
        double xab[3];
        sub3(x + 3 * a, x + 3 * b, xab);
        const double length = sqrt(dot3(xab, xab));
        if (length < MIN_EDGE_LENGTH)
            continue;
        const double C = length - rest_length[e];
        const double denominator = w[a] + w[b] + alpha_tilde_d;
        if (denominator <= MIN_DENOMINATOR)
            continue;
        const double dlambda = (-C - alpha_tilde_d * lambda[e]) / denominator;
        lambda[e] += dlambda;
        for (int k = 0; k < 3; ++k) {
            const double n = xab[k] / length;
            dx[3 * a + k] += w[a] * dlambda * n;
            dx[3 * b + k] -= w[b] * dlambda * n;
        }
    }
    for (int t = 0; t < T; ++t) {
        const int32_t *q = tets + 4 * t;
        double p[12], g[12];
        for (int i = 0; i < 4; ++i)
            for (int k = 0; k < 3; ++k)
                p[3 * i + k] = x[3 * q[i] + k];
        const double C = oracle_tet_gradients(p, g) - rest_volume[t];
        double denominator = alpha_tilde_v;
        for (int i = 0; i < 4; ++i)
            denominator += w[q[i]] * dot3(g + 3 * i, g + 3 * i);
        if (denominator <= MIN_DENOMINATOR)
            continue;
        const double dlambda = (-C - alpha_tilde_v * lambda[E + t]) / denominator;
        lambda[E + t] += dlambda;
        for (int i = 0; i < 4; ++i)
            for (int k = 0; k < 3; ++k)
                dx[3 * q[i] + k] += w[q[i]] * dlambda * g[3 * i + k];
    }
    for (int i = 0; i < V; ++i)
        if (count[i] > 0)
            for (int k = 0; k < 3; ++k)
                x[3 * i + k] += dx[3 * i + k] / (double)count[i];
    for (int t = 0; t < num_tools; ++t)
        for (int n = 0; n < num_candidates[t]; ++n) {
            int i = candidates[(size_t)t * V + n];
            oracle_project_contact(x + 3 * i, centres + 3 * t, tool_radius[t]);
        }
}

/* ------------------------------------------------------------------ */
/* Capsule tools against surface faces (Sec. III-A.3: each capsule of   */
/* the grasper is an SDF tested against the mesh faces; a penetrating  */
/* face is pushed out along the penetration direction with k_c = 1).   */
/* ------------------------------------------------------------------ */

/* Closest point on triangle (a, b, c) to p, by the region of p's projection:
 * vertex, edge or interior.  Writes the point and its barycentrics.  The
 * region tests are the published method of C. Ericson, Real-Time Collision
 * Detection (Morgan Kaufmann 2005), Sec. 5.1.5. */
static void closest_on_triangle(const double *p, const double *a, const double *b,
                                const double *c, double *q, double *bary)
{
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    sub3(b, a, ab);
    sub3(c, a, ac);
    sub3(p, a, ap);
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) {                       /* vertex a */
        bary[0] = 1.0, bary[1] = 0.0, bary[2] = 0.0;
    } else {
        sub3(p, b, bp);
        double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
        sub3(p, c, cp);
        double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
        double vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
        if (d3 >= 0.0 && d4 <= d3) {                    /* vertex b */
            bary[0] = 0.0, bary[1] = 1.0, bary[2] = 0.0;
        } else if (d6 >= 0.0 && d5 <= d6) {             /* vertex c */
            bary[0] = 0.0, bary[1] = 0.0, bary[2] = 1.0;
        } else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {   /* edge ab */
            double t = d1 / (d1 - d3);
            bary[0] = 1.0 - t, bary[1] = t, bary[2] = 0.0;
        } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {   /* edge ac */
            double t = d2 / (d2 - d6);
            bary[0] = 1.0 - t, bary[1] = 0.0, bary[2] = t;
        } else if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {   /* edge bc */
            double t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
            bary[0] = 0.0, bary[1] = 1.0 - t, bary[2] = t;
        } else {                                        /* interior */
            double den = 1.0 / (va + vb + vc);
            bary[1] = vb * den, bary[2] = vc * den, bary[0] = 1.0 - bary[1] - bary[2];
        }
    }
    for (int k = 0; k < 3; ++k)
        q[k] = bary[0] * a[k] + bary[1] * b[k] + bary[2] * c[k];
}

/* Closest points of segments p0 p1 and q0 q1: parameters s, t in [0, 1]
 * (the clamped solution of C. Ericson, Real-Time Collision Detection, 2005,
 * Sec. 5.1.9). */
static void closest_segments(const double *p0, const double *p1, const double *q0,
                             const double *q1, double *s_out, double *t_out)
{
    double d1[3], d2[3], r[3];
    sub3(p1, p0, d1);
    sub3(q1, q0, d2);
    sub3(p0, q0, r);
    double a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r);
    double s = 0.0, t = 0.0;
    if (a <= 1e-30 && e <= 1e-30) {
        s = t = 0.0;
    } else if (a <= 1e-30) {
        t = fmin(fmax(f / e, 0.0), 1.0);
    } else {
        double c = dot3(d1, r);
        if (e <= 1e-30) {
            s = fmin(fmax(-c / a, 0.0), 1.0);
        } else {
            double b = dot3(d1, d2), den = a * e - b * b;
            s = den > 0.0 ? fmin(fmax((b * f - c * e) / den, 0.0), 1.0) : 0.0;
            t = (b * s + f) / e;
            if (t < 0.0) {
                t = 0.0;
                s = fmin(fmax(-c / a, 0.0), 1.0);
            } else if (t > 1.0) {
                t = 1.0;
                s = fmin(fmax((b - c) / a, 0.0), 1.0);
            }
        }
    }
    *s_out = s;
    *t_out = t;
}

/*
 * Closest points between segment p0 p1 and triangle (a, b, c): the minimum
 * of |S(t) - T(u, v)| over the segment and the triangle is attained at a
 * segment end against the triangle, at a triangle edge against the segment,
 * or where the segment crosses the triangle (distance 0).  Writes the
 * triangle point q with barycentrics bary and the segment point s; returns
 * the squared distance.
 */
double oracle_segment_triangle(const double *p0, const double *p1, const double *a,
                               const double *b, const double *c, double *q, double *s,
                               double *bary)
{
    double best = INFINITY, qq[3], bb[3], d[3];
    /* segment ends against the triangle */
    for (int e = 0; e < 2; ++e) {
        const double *p = e == 0 ? p0 : p1;
        closest_on_triangle(p, a, b, c, qq, bb);
        sub3(qq, p, d);
        double d2 = dot3(d, d);
        if (d2 < best) {
            best = d2;
            memcpy(q, qq, sizeof qq);
            memcpy(bary, bb, sizeof bb);
            memcpy(s, p, 3 * sizeof(double));
        }
    }
    /* triangle edges against the segment */
    const double *v[3] = {a, b, c};
    for (int e = 0; e < 3; ++e) {
        const double *e0 = v[e], *e1 = v[(e + 1) % 3];
        double ts, te;
        closest_segments(p0, p1, e0, e1, &ts, &te);
        double ps[3], pe[3];
        for (int k = 0; k < 3; ++k) {
            ps[k] = p0[k] + ts * (p1[k] - p0[k]);
            pe[k] = e0[k] + te * (e1[k] - e0[k]);
        }
        sub3(pe, ps, d);
        double d2 = dot3(d, d);
        if (d2 < best) {
            best = d2;
            memcpy(q, pe, sizeof pe);
            memcpy(s, ps, sizeof ps);
            bary[0] = bary[1] = bary[2] = 0.0;
            bary[e] = 1.0 - te;
            bary[(e + 1) % 3] = te;
        }
    }
    /* the segment crossing the triangle */
    double ab[3], ac[3], n[3], dir[3], w0[3];
    sub3(b, a, ab);
    sub3(c, a, ac);
    cross3(ab, ac, n);
    sub3(p1, p0, dir);
    double den = dot3(n, dir);
    if (fabs(den) > 1e-30) {
        sub3(a, p0, w0);
        double t = dot3(n, w0) / den;
        if (t >= 0.0 && t <= 1.0) {
            double x[3];
            for (int k = 0; k < 3; ++k)
                x[k] = p0[k] + t * dir[k];
            double bc[3];
            closest_on_triangle(x, a, b, c, qq, bc);
            sub3(qq, x, d);
            if (dot3(d, d) <= 1e-24 * (1.0 + dot3(ab, ab))) {   /* inside the triangle */
                best = 0.0;
                memcpy(q, qq, sizeof qq);
                memcpy(bary, bc, sizeof bc);
                memcpy(s, x, sizeof x);
            }
        }
    }
    return best;
}

/*
 * Push face f = (a, b, c) (outward oriented) out of the capsule p0 p1 of
 * radius r, k_c = 1: with q = sum_i b_i x_i its closest point to the axis
 * point s at distance d < r, the constraint C = d - r has gradient b_i n
 * (n = (q - s)/d, or the face normal when d ~ 0) and one projection moves
 * x_i by -w_i b_i C n / sum_j w_j b_j^2.
 */
void oracle_project_capsule_face(double *x, const double *w, const int32_t *f, const double *p0,
                                 const double *p1, double radius)
{
    const double *a = x + 3 * f[0], *b = x + 3 * f[1], *c = x + 3 * f[2];
    double q[3], s[3], bary[3], n[3];
    double d2 = oracle_segment_triangle(p0, p1, a, b, c, q, s, bary);
    if (d2 >= radius * radius)
        return;
    double d = sqrt(d2);
    if (d > 1e-12) {
        for (int k = 0; k < 3; ++k)
            n[k] = (q[k] - s[k]) / d;
    } else {
        double ab[3], ac[3];
        sub3(b, a, ab);
        sub3(c, a, ac);
        cross3(ab, ac, n);
        double l = sqrt(dot3(n, n));
        if (l <= 0.0)
            return;
        for (int k = 0; k < 3; ++k)
            n[k] /= l;
    }
    double den = 0.0;
    for (int i = 0; i < 3; ++i)
        den += w[f[i]] * bary[i] * bary[i];
    if (den <= MIN_DENOMINATOR)
        return;
    double C = d - radius;
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
            x[3 * f[i] + k] += -w[f[i]] * bary[i] * C / den * n[k];
}

/* Face candidates of a capsule for a step: faces with a free vertex whose
 * closest distance to the axis is below 2r on the start-of-step positions,
 * in the given processing order.  Returns the count. */
int oracle_face_candidates(const double *x, const double *w, int F, const int32_t *faces,
                           const int32_t *order, const double *p0, const double *p1,
                           double radius, int32_t *out)
{
    int n = 0;
    for (int p = 0; p < F; ++p) {
        const int32_t *f = faces + 3 * order[p];
        if (!(w[f[0]] > 0.0 || w[f[1]] > 0.0 || w[f[2]] > 0.0))
            continue;
        double q[3], s[3], bary[3];
        double d2 = oracle_segment_triangle(p0, p1, x + 3 * f[0], x + 3 * f[1], x + 3 * f[2], q,
                                            s, bary);
        if (d2 < 4.0 * radius * radius)
            out[n++] = order[p];
    }
    return n;
}

/* The push-out of a list of faces in the given order (one capsule). */
void oracle_project_capsule_faces(double *x, const double *w, const int32_t *faces,
                                  const int32_t *list, int n, const double *p0, const double *p1,
                                  double radius)
{
    for (int k = 0; k < n; ++k)
        oracle_project_capsule_face(x, w, faces + 3 * list[k], p0, p1, radius);
}

/*
 * Grasp selection (Sec. III-A.2, reading R12): the free particle closest to
 * the dragging point among those strictly within r_l of it, on the positions
 * x; the lowest id wins a tie.  Returns its id, or -1 when none is within
 * reach.  dist2_out (optional) receives the squared distance of the chosen
 * particle (unchanged when none is chosen).
 */
int oracle_grasp_select(int V, const double *w, const double *x, const double *point,
                        double radius, double *dist2_out)
{
    int best = -1;
    double best_d2 = 0.0;
    for (int i = 0; i < V; ++i) {
        if (!(w[i] > 0.0))
            continue;
        double d[3];
        sub3(x + 3 * i, point, d);
        double d2 = dot3(d, d);
        if (d2 < radius * radius && (best < 0 || d2 < best_d2)) {
            best = i;
            best_d2 = d2;
        }
    }
    if (best >= 0 && dist2_out)
        *dist2_out = best_d2;
    return best;
}

/*
 * The dragging constraint (Sec. III-A.2, reading R12): a distance constraint
 * of rest length 0 and stiffness k_s = 1 between the dragging point p
 * (kinematic: inverse mass 0) and particle i.  C = |x_i - p|, grad_i C =
 * (x_i - p) / |x_i - p|, dlambda = -C / w_i, x_i += w_i dlambda grad_i C:
 * the particle lands on p.  Skipped for a pinned particle and when the
 * particle already sits on p (|x_i - p| below the edge threshold of R7).
 */
void oracle_project_drag(double *x, const double *w, int i, const double *point)
{
    double d[3];
    sub3(x + 3 * i, point, d);
    double C = sqrt(dot3(d, d));
    if (!(w[i] > 0.0) || C < MIN_EDGE_LENGTH)
        return;
    double dlambda = -C / w[i];
    for (int k = 0; k < 3; ++k)
        x[3 * i + k] += w[i] * dlambda * (d[k] / C);
}

/* Velocity update of one substep (Alg. 1): v = (x - x_prev) / h. */
void oracle_velocity(int V, double h, const double *x, const double *x_prev, double *v)
{
    for (int i = 0; i < 3 * V; ++i)
        v[i] = (x[i] - x_prev[i]) / h;
}

/*
 * Advance one environment by num_steps steps.
 *
 * Mesh: V particles with inverse masses w; E edges [E][2] with rest lengths;
 * T tetrahedra [T][4] (oriented) with rest volumes.  Schedule: colour c of the
 * edges is edge_order[edge_colour_ptr[c] .. edge_colour_ptr[c+1]) (constraint
 * ids in processing order), likewise for tetrahedra.
 * Tools: num_tools spheres with radii tool_radius[t]; tool_pos is
 * [num_steps][num_tools][3].
 * State: x, v are [V][3], read and overwritten.
 * Optional outputs (NULL to skip):
 *   lambda         [E+T]  multipliers after the final iteration of the final substep
 *   contacts       [num_steps][num_tools][V]  candidate ids ascending, -1 padded
 *   contact_count  [num_steps][num_tools]
 *   residual       [num_steps][substeps][2]   (RMS, max) per substep (R8)
 */
int oracle_run(int V, const double *w,
               int E, const int32_t *edges, const double *rest_length,
               int T, const int32_t *tets, const double *rest_volume,
               int num_edge_colours, const int32_t *edge_colour_ptr, const int32_t *edge_order,
               int num_tet_colours, const int32_t *tet_colour_ptr, const int32_t *tet_order,
               double dt, int substeps, int iterations, const double *gravity,
               double alpha_d, double alpha_v,
               int num_tools, const double *tool_radius,
               int num_steps, const double *tool_pos,
               double *x, double *v,
               double *lambda_out, int32_t *contacts, int32_t *contact_count,
               double *residual, int jacobi)
{
    if (V <= 0 || E < 0 || T < 0 || substeps <= 0 || iterations < 0 || num_steps < 0 ||
        num_tools < 0 || !(dt > 0.0) || !w || !x || !v || !gravity)
        return ORACLE_E_ARG;
    if (num_tools > 0 && (!tool_radius || !tool_pos))
        return ORACLE_E_ARG;

    double *x_prev = (double *)malloc(sizeof(double) * 3 * (size_t)V);
    double *lambda = (double *)calloc((size_t)(E + T) + 1, sizeof(double));
    int32_t *candidates = (int32_t *)malloc(sizeof(int32_t) * (size_t)V * (num_tools > 0 ? num_tools : 1));
    int *num_candidates = (int *)calloc((size_t)(num_tools > 0 ? num_tools : 1), sizeof(int));
    int32_t *count = (int32_t *)calloc((size_t)V, sizeof(int32_t));
    double *dx = (double *)malloc(sizeof(double) * 3 * (size_t)V);
    if (!x_prev || !lambda || !candidates || !num_candidates || !count || !dx) {
        free(x_prev);
        free(lambda);
        free(candidates);
        free(num_candidates);
        free(count);
        free(dx);
        return ORACLE_E_NOMEM;
    }
    /* Jacobi: constraints per particle (n of Sec. III-A.1) */
    for (int e = 0; e < E; ++e) {
        count[edges[2 * e]]++;
        count[edges[2 * e + 1]]++;
    }
    for (int t = 0; t < T; ++t)
        for (int i = 0; i < 4; ++i)
            count[tets[4 * t + i]]++;

    const double h = dt / (double)substeps;                 /* Alg. 1: h = dt / simSubSteps */
    const double alpha_tilde_d = alpha_d / (h * h);
    const double alpha_tilde_v = alpha_v / (h * h);

    for (int step = 0; step < num_steps; ++step) {
        /* evaluate instrument state and the contact candidates (R6) */
        const double *centres = tool_pos + (size_t)step * num_tools * 3;
        for (int t = 0; t < num_tools; ++t) {
            int n = oracle_candidates(V, w, x, centres + 3 * t, tool_radius[t],
                                      candidates + (size_t)t * V);
            num_candidates[t] = n;
            if (contacts) {
                int32_t *row = contacts + ((size_t)step * num_tools + t) * V;
                for (int i = 0; i < V; ++i)
                    row[i] = i < n ? candidates[(size_t)t * V + i] : -1;
            }
            if (contact_count)
                contact_count[(size_t)step * num_tools + t] = n;
        }

        for (int sub = 0; sub < substeps; ++sub) {
            oracle_predict(V, w, h, gravity, x, v, x_prev);   /* Alg. 1, R5 */
            for (int j = 0; j < E + T; ++j)                  /* R4 */
                lambda[j] = 0.0;
            for (int it = 0; it < iterations; ++it) {
                if (jacobi)
                    oracle_iterate_jacobi(x, w, E, edges, rest_length, T, tets, rest_volume,
                                          alpha_tilde_d, alpha_tilde_v, lambda, count, dx,
                                          V, num_tools, centres, tool_radius, candidates,
                                          num_candidates);
                else
                    oracle_iterate(x, w, E, edges, rest_length, rest_volume, tets,
                                   num_edge_colours, edge_colour_ptr, edge_order,
                                   num_tet_colours, tet_colour_ptr, tet_order,
                                   alpha_tilde_d, alpha_tilde_v, lambda,
                                   V, num_tools, centres, tool_radius, candidates, num_candidates);
            }
            if (residual)
                oracle_residual(x, E, edges, rest_length, T, tets, rest_volume,
                                alpha_tilde_d, alpha_tilde_v, lambda,
                                residual + 2 * ((size_t)step * substeps + sub));
            oracle_velocity(V, h, x, x_prev, v);              /* Alg. 1 */
        }
    }
    if (lambda_out)
        memcpy(lambda_out, lambda, sizeof(double) * (size_t)(E + T));
    free(x_prev);
    free(lambda);
    free(candidates);
    free(num_candidates);
    free(count);
    free(dx);
    return ORACLE_OK;
}
