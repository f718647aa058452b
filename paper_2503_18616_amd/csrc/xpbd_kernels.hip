// HIP kernels of the batched XPBD substep for gfx950 (CDNA4).
//
// One workgroup advances one environment through num_steps steps of
// Algorithm 1 of FF-SRL (Sec. III-A.1): per step the tool pose is read and
// the contact candidates are collected; per substep the particles are
// predicted, the multipliers reset, and `iterations` Gauss-Seidel sweeps
// project the edge-distance (Eq. 1) and tetrahedral-volume (Eqs. 2-3)
// constraints in compliance form, colour by colour, followed by the tool
// push-out (Sec. III-A.3); velocities are then recomputed from the position
// change.
//
// Data placement: the environment's particles live in LDS as float4
// (x, y, z, inverse mass) for the whole launch, the multipliers in LDS, the
// constraint lists either staged in LDS or read from global memory (they are
// shared by every environment of a mesh and stay cache-resident).  Each
// thread keeps the velocity and start-of-substep position of its particles
// (i = k * blockDim + tid) in registers.  Inside a colour no two constraints
// share a particle, so the lanes of the workgroup project one colour's
// constraints concurrently without atomics; a workgroup barrier separates the
// colours.  Global state is read and written once per launch in
// structure-of-arrays layout, coalesced across lanes.
#include <hip/hip_runtime.h>

#include "xpbd_device.h"

namespace xpbd {
namespace {

constexpr float kMinEdgeLength2 = 1e-18f;   // skip distance constraints shorter than 1e-9 m
constexpr float kMinDenominator = 1e-30f;
constexpr float kSixth = 1.0f / 6.0f;
constexpr float kThirtySixth = 1.0f / 36.0f;

__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Particle f of the LDS array xw, f counting kUnit bytes (16: a slot index,
// 1: a byte offset).
template <int kUnit>
__device__ __forceinline__ float4 &lds_particle(float4 *xw, uint32_t f)
{
    return *reinterpret_cast<float4 *>(reinterpret_cast<unsigned char *>(xw) + f * kUnit);
}
// Store the position of p into particle r (its inverse mass is unchanged).
__device__ __forceinline__ void store_position(float4 &r, const float4 &p)
{
    r.x = p.x;
    r.y = p.y;
    r.z = p.z;
}

template <int kUnit>
__device__ __forceinline__ const float4 &lds_particle(const float4 *xw, uint32_t f)
{
    return *reinterpret_cast<const float4 *>(reinterpret_cast<const unsigned char *>(xw) + f * kUnit);
}

// Distance constraint C = |x_a - x_b| - d (Eq. 1), one XPBD projection of
// edge (a, b) with rest length `rest`; `lam` is the edge's multiplier.  An
// edge shorter than the minimum length or with a vanishing denominator is
// left as it is (its correction is selected to zero, so no branch is taken).
template <int kUnit = 16>
__device__ __forceinline__ void edge_update(float4 *xw, uint32_t a, uint32_t b, float rest,
                                            float alpha_tilde, float &lam)
{
    float4 &ra = lds_particle<kUnit>(xw, a);
    float4 &rb = lds_particle<kUnit>(xw, b);
    float4 pa = ra;
    float4 pb = rb;
    const float dx = pa.x - pb.x, dy = pa.y - pb.y, dz = pa.z - pb.z;
    const float l2 = dx * dx + dy * dy + dz * dz;
    const float inv_len = fast_rsq(l2);
    const float C = l2 * inv_len - rest;
    const float denom = pa.w + pb.w + alpha_tilde;
    const bool ok = l2 >= kMinEdgeLength2 && denom > kMinDenominator;
    const float dl = ok ? (-C - alpha_tilde * lam) * fast_rcp(denom) : 0.0f;
    lam = ok ? lam + dl : lam;
    const float s = ok ? dl * inv_len : 0.0f;   // dlambda times the unit direction's scale
    const float sa = pa.w * s, sb = pb.w * s;
    pa.x += sa * dx;
    pa.y += sa * dy;
    pa.z += sa * dz;
    pb.x -= sb * dx;
    pb.y -= sb * dy;
    pb.z -= sb * dz;
    store_position(ra, pa);
    store_position(rb, pb);
}

// Volume constraint C = (1/6)(x_ba x x_ca).x_da - V0 (Eqs. 2-3 with the
// analytic gradients), one XPBD projection of tetrahedron (a | b << 16,
// c | d << 16) with rest volume `rest`.  G_i are six times the gradients.
template <int kUnit = 16>
__device__ __forceinline__ void tet_update(float4 *xw, uint32_t ab, uint32_t cd, float rest,
                                           float alpha_tilde, float &lam)
{
    float4 &ra = lds_particle<kUnit>(xw, ab & 0xffffu);
    float4 &rb = lds_particle<kUnit>(xw, ab >> 16);
    float4 &rc = lds_particle<kUnit>(xw, cd & 0xffffu);
    float4 &rd = lds_particle<kUnit>(xw, cd >> 16);
    float4 pa = ra;
    float4 pb = rb;
    float4 pc = rc;
    float4 pd = rd;
    const float bax = pb.x - pa.x, bay = pb.y - pa.y, baz = pb.z - pa.z;
    const float cax = pc.x - pa.x, cay = pc.y - pa.y, caz = pc.z - pa.z;
    const float dax = pd.x - pa.x, day = pd.y - pa.y, daz = pd.z - pa.z;
    // G_b = x_ca x x_da, G_c = x_da x x_ba, G_d = x_ba x x_ca, G_a = -(G_b + G_c + G_d)
    const float gbx = cay * daz - caz * day, gby = caz * dax - cax * daz, gbz = cax * day - cay * dax;
    const float gcx = day * baz - daz * bay, gcy = daz * bax - dax * baz, gcz = dax * bay - day * bax;
    const float gdx = bay * caz - baz * cay, gdy = baz * cax - bax * caz, gdz = bax * cay - bay * cax;
    const float gax = -(gbx + gcx + gdx), gay = -(gby + gcy + gdy), gaz = -(gbz + gcz + gdz);
    const float C = (bax * gbx + bay * gby + baz * gbz) * kSixth - rest;
    const float wg = pa.w * (gax * gax + gay * gay + gaz * gaz) +
                     pb.w * (gbx * gbx + gby * gby + gbz * gbz) +
                     pc.w * (gcx * gcx + gcy * gcy + gcz * gcz) +
                     pd.w * (gdx * gdx + gdy * gdy + gdz * gdz);
    const float denom = wg * kThirtySixth + alpha_tilde;
    const bool ok = denom > kMinDenominator;   // else no correction (selected, no branch)
    const float dl = ok ? (-C - alpha_tilde * lam) * fast_rcp(denom) : 0.0f;
    lam = ok ? lam + dl : lam;
    const float s = dl * kSixth;
    const float sa = pa.w * s, sb = pb.w * s, sc = pc.w * s, sd = pd.w * s;
    pa.x += sa * gax;
    pa.y += sa * gay;
    pa.z += sa * gaz;
    pb.x += sb * gbx;
    pb.y += sb * gby;
    pb.z += sb * gbz;
    pc.x += sc * gcx;
    pc.y += sc * gcy;
    pc.z += sc * gcz;
    pd.x += sd * gdx;
    pd.y += sd * gdy;
    pd.z += sd * gdz;
    store_position(ra, pa);
    store_position(rb, pb);
    store_position(rc, pc);
    store_position(rd, pd);
}

// Jacobi forms of the two projections (Sec. III-A.1): the correction of every
// particle of the constraint is added to dx (structure of arrays [3][V])
// instead of being applied; the multiplier accumulates as in Gauss-Seidel.
// Callers run one colour at a time, so no two lanes add to the same particle
// and plain adds suffice (a fixed summation order: results are reproducible).
__device__ __forceinline__ void edge_delta(const float4 *xw, float *dx, int V, int a, int b,
                                           float rest, float alpha_tilde, float &lam)
{
    const float4 pa = xw[a], pb = xw[b];
    const float ex = pa.x - pb.x, ey = pa.y - pb.y, ez = pa.z - pb.z;
    const float l2 = ex * ex + ey * ey + ez * ez;
    if (!(l2 >= kMinEdgeLength2))
        return;
    const float inv_len = fast_rsq(l2);
    const float C = l2 * inv_len - rest;
    const float denom = pa.w + pb.w + alpha_tilde;
    if (!(denom > kMinDenominator))
        return;
    const float dl = (-C - alpha_tilde * lam) * fast_rcp(denom);
    lam += dl;
    const float s = dl * inv_len;
    const float sa = pa.w * s, sb = pb.w * s;
    dx[a] += sa * ex;
    dx[V + a] += sa * ey;
    dx[2 * V + a] += sa * ez;
    dx[b] -= sb * ex;
    dx[V + b] -= sb * ey;
    dx[2 * V + b] -= sb * ez;
}

__device__ __forceinline__ void tet_delta(const float4 *xw, float *dx, int V, uint32_t ab,
                                          uint32_t cd, float rest, float alpha_tilde, float &lam)
{
    const int q[4] = {(int)(ab & 0xffffu), (int)(ab >> 16), (int)(cd & 0xffffu), (int)(cd >> 16)};
    const float4 pa = xw[q[0]], pb = xw[q[1]], pc = xw[q[2]], pd = xw[q[3]];
    const float bax = pb.x - pa.x, bay = pb.y - pa.y, baz = pb.z - pa.z;
    const float cax = pc.x - pa.x, cay = pc.y - pa.y, caz = pc.z - pa.z;
    const float dax = pd.x - pa.x, day = pd.y - pa.y, daz = pd.z - pa.z;
    float g[4][3];
    g[1][0] = cay * daz - caz * day;
    g[1][1] = caz * dax - cax * daz;
    g[1][2] = cax * day - cay * dax;
    g[2][0] = day * baz - daz * bay;
    g[2][1] = daz * bax - dax * baz;
    g[2][2] = dax * bay - day * bax;
    g[3][0] = bay * caz - baz * cay;
    g[3][1] = baz * cax - bax * caz;
    g[3][2] = bax * cay - bay * cax;
    for (int k = 0; k < 3; ++k)
        g[0][k] = -(g[1][k] + g[2][k] + g[3][k]);
    const float C = (bax * g[1][0] + bay * g[1][1] + baz * g[1][2]) * kSixth - rest;
    const float w[4] = {pa.w, pb.w, pc.w, pd.w};
    float wg = 0.0f;
    for (int i = 0; i < 4; ++i)
        wg += w[i] * (g[i][0] * g[i][0] + g[i][1] * g[i][1] + g[i][2] * g[i][2]);
    const float denom = wg * kThirtySixth + alpha_tilde;
    if (!(denom > kMinDenominator))
        return;
    const float dl = (-C - alpha_tilde * lam) * fast_rcp(denom);
    lam += dl;
    const float s = dl * kSixth;
    for (int i = 0; i < 4; ++i) {
        const float si = w[i] * s;
        dx[q[i]] += si * g[i][0];
        dx[V + q[i]] += si * g[i][1];
        dx[2 * V + q[i]] += si * g[i][2];
    }
}

// ---------------------------------------------------------------------------
// Capsule tools against surface triangles (Sec. III-A.2/3).  A capsule is the
// segment p0 p1 with radius r; a face's deepest point is its closest point to
// the segment, found exactly: a segment end against the triangle, a triangle
// edge against the segment, or the segment crossing the triangle.

struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float4 p) { return {p.x, p.y, p.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Barycentrics of the point of triangle (a, b, c) closest to p (vertex, edge
// or interior region of p's projection; the region tests of C. Ericson,
// Real-Time Collision Detection, 2005, Sec. 5.1.5).
__device__ V3 triangle_closest(V3 p, V3 a, V3 b, V3 c)
{
    const V3 ab = b - a, ac = c - a, ap = p - a;
    const float d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0.f && d2 <= 0.f)
        return {1.f, 0.f, 0.f};
    const V3 bp = p - b;
    const float d3 = dot(ab, bp), d4 = dot(ac, bp);
    if (d3 >= 0.f && d4 <= d3)
        return {0.f, 1.f, 0.f};
    const V3 cp = p - c;
    const float d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0.f && d5 <= d6)
        return {0.f, 0.f, 1.f};
    const float vc = d1 * d4 - d3 * d2;
    if (vc <= 0.f && d1 >= 0.f && d3 <= 0.f) {
        const float t = d1 / (d1 - d3);
        return {1.f - t, t, 0.f};
    }
    const float vb = d5 * d2 - d1 * d6;
    if (vb <= 0.f && d2 >= 0.f && d6 <= 0.f) {
        const float t = d2 / (d2 - d6);
        return {1.f - t, 0.f, t};
    }
    const float va = d3 * d6 - d5 * d4;
    if (va <= 0.f && (d4 - d3) >= 0.f && (d5 - d6) >= 0.f) {
        const float t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        return {0.f, 1.f - t, t};
    }
    const float den = 1.f / (va + vb + vc);
    const float v = vb * den, w = vc * den;
    return {1.f - v - w, v, w};
}

// Parameters (s on p0 p1, t on q0 q1) of the closest points of two segments
// (the clamped solution of Ericson 2005, Sec. 5.1.9), returned as (s, t).
// Values, not references: a store through a reference chosen per branch
// would put the caller's variables in scratch memory.
__device__ float2 segments_closest(V3 p0, V3 p1, V3 q0, V3 q1)
{
    const V3 d1 = p1 - p0, d2 = q1 - q0, r = p0 - q0;
    const float a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
    if (a <= 1e-30f && e <= 1e-30f)
        return make_float2(0.f, 0.f);
    if (a <= 1e-30f)
        return make_float2(0.f, fminf(fmaxf(f / e, 0.f), 1.f));
    const float c = dot(d1, r);
    if (e <= 1e-30f)
        return make_float2(fminf(fmaxf(-c / a, 0.f), 1.f), 0.f);
    const float b = dot(d1, d2), den = a * e - b * b;
    float s = den > 0.f ? fminf(fmaxf((b * f - c * e) / den, 0.f), 1.f) : 0.f;
    float t = (b * s + f) / e;
    if (t < 0.f) {
        t = 0.f;
        s = fminf(fmaxf(-c / a, 0.f), 1.f);
    } else if (t > 1.f) {
        t = 1.f;
        s = fminf(fmaxf((b - c) / a, 0.f), 1.f);
    }
    return make_float2(s, t);
}

// Squared distance of segment p0 p1 and triangle (a, b, c); bary and s_pt
// receive the triangle point's barycentrics and the segment point.
__device__ float segment_triangle(V3 p0, V3 p1, V3 a, V3 b, V3 c, V3 &bary, V3 &s_pt)
{
    float best = 3.0e38f;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const V3 p = e == 0 ? p0 : p1;
        const V3 w = triangle_closest(p, a, b, c);
        const V3 q = w.x * a + w.y * b + w.z * c;
        const float d2 = dot(q - p, q - p);
        if (d2 < best) {
            best = d2;
            bary = w;
            s_pt = p;
        }
    }
    // the three edges a b, b c, c a; the weights are written out per edge, as
    // an indexed array here would live in scratch memory
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const V3 e0 = e == 0 ? a : e == 1 ? b : c, e1 = e == 0 ? b : e == 1 ? c : a;
        const float2 st = segments_closest(p0, p1, e0, e1);
        const float ts = st.x, te = st.y;
        const V3 ps = p0 + ts * (p1 - p0), pe = e0 + te * (e1 - e0);
        const float d2 = dot(pe - ps, pe - ps);
        if (d2 < best) {
            best = d2;
            bary = e == 0 ? V3{1.f - te, te, 0.f} : e == 1 ? V3{0.f, 1.f - te, te}
                                                          : V3{te, 0.f, 1.f - te};
            s_pt = ps;
        }
    }
    const V3 ab = b - a, ac = c - a, n = cross(ab, ac), dir = p1 - p0;
    const float den = dot(n, dir);
    if (fabsf(den) > 1e-30f) {
        const float t = dot(n, a - p0) / den;
        if (t >= 0.f && t <= 1.f) {
            const V3 x = p0 + t * dir;
            const V3 w = triangle_closest(x, a, b, c);
            const V3 q = w.x * a + w.y * b + w.z * c;
            if (dot(q - x, q - x) <= 1e-12f * (1.f + dot(ab, ab))) {
                best = 0.f;
                bary = w;
                s_pt = x;
            }
        }
    }
    return best;
}

// True when triangle (a, b, c) certainly lies farther than reach from segment
// p0 p1, so that the exact closest-point test can be skipped: the sphere about
// the centroid through the farthest corner stays beyond reach of the segment,
// or both end points lie on one side of the triangle's plane, beyond reach of
// it.  Both bounds keep a margin of 0.1 % of reach, far above the error of the
// hardware reciprocal and square root they use.
__device__ __forceinline__ bool face_beyond(V3 p0, V3 p1, V3 a, V3 b, V3 c, float reach)
{
    const V3 g = (1.f / 3.f) * (a + b + c);
    const float r2 = fmaxf(fmaxf(dot(a - g, a - g), dot(b - g, b - g)), dot(c - g, c - g));
    const V3 d = p1 - p0;
    const float dd = dot(d, d);
    const float s = dd > 0.f ? fminf(fmaxf(dot(g - p0, d) * __builtin_amdgcn_rcpf(dd), 0.f), 1.f)
                             : 0.f;
    const V3 q = p0 + s * d - g;
    const float lim = __builtin_amdgcn_sqrtf(r2) + 1.001f * reach;
    if (dot(q, q) > lim * lim)
        return true;
    const V3 n = cross(b - a, c - a);
    const float h0 = dot(p0 - a, n), h1 = dot(p1 - a, n);
    const float m2 = (1.001f * reach) * (1.001f * reach) * dot(n, n);
    return h0 * h1 > 0.f && h0 * h0 > m2 && h1 * h1 > m2;
}

// Push face (a | b << 16, c) out of capsule p0 p1 of radius r with k_c = 1:
// C = d - r on the closest point q = sum b_i x_i, gradient b_i n.
__device__ void capsule_push(float4 *xw, uint2 f, V3 p0, V3 p1, float r)
{
    const int ia = (int)(f.x & 0xffffu), ib = (int)(f.x >> 16), ic = (int)f.y;
    float4 pa = xw[ia], pb = xw[ib], pc = xw[ic];
    if (face_beyond(p0, p1, v3(pa), v3(pb), v3(pc), r))
        return;
    V3 bary, s;
    const float d2 = segment_triangle(p0, p1, v3(pa), v3(pb), v3(pc), bary, s);
    if (!(d2 < r * r))
        return;
    const float d = sqrtf(d2);
    V3 n;
    if (d > 1e-12f) {
        const V3 q = bary.x * v3(pa) + bary.y * v3(pb) + bary.z * v3(pc);
        n = (1.f / d) * (q - s);
    } else {
        n = cross(v3(pb) - v3(pa), v3(pc) - v3(pa));
        const float l = sqrtf(dot(n, n));
        if (!(l > 0.f))
            return;
        n = (1.f / l) * n;
    }
    const float den = pa.w * bary.x * bary.x + pb.w * bary.y * bary.y + pc.w * bary.z * bary.z;
    if (!(den > kMinDenominator))
        return;
    const float k = -(d - r) / den;
    const float sa = pa.w * bary.x * k, sb = pb.w * bary.y * k, sc = pc.w * bary.z * k;
    pa.x += sa * n.x;
    pa.y += sa * n.y;
    pa.z += sa * n.z;
    pb.x += sb * n.x;
    pb.y += sb * n.y;
    pb.z += sb * n.z;
    pc.x += sc * n.x;
    pc.y += sc * n.y;
    pc.z += sc * n.z;
    xw[ia] = pa;
    xw[ib] = pb;
    xw[ic] = pc;
}

// The push-out of capsule_push by the 4 lanes of a group (q = lane & 3, all 4
// lanes active, one face per group), with hardware reciprocals.  Every closest
// pair of a segment and a triangle is one of: an end point and its projection
// into the plane when that falls inside the triangle; the segment and an
// edge; a crossing of the triangle (distance 0); and where several pairs are
// closest (a segment parallel to the plane), one of these is among them.
// Lane q < 3 takes the segment against edge q (a b, b c, c a) and a point
// candidate: end point p0 (q = 0), p1 (q = 1), or the crossing of the plane
// (q = 2).  The group's minimum, in segment_triangle's order (end points,
// edges, with a crossing inside the triangle winning outright) and first on
// ties, gives the closest pair; lane 0 moves the face.
__device__ void capsule_push_lanes(float4 *xw, uint2 f, V3 p0, V3 p1, float r, int q)
{
    const int ia = (int)(f.x & 0xffffu), ib = (int)(f.x >> 16), ic = (int)f.y;
    float4 pa = xw[ia], pb = xw[ib], pc = xw[ic];
    const V3 a = v3(pa), b = v3(pb), c = v3(pc);
    const V3 ab = b - a, ac = c - a, dir = p1 - p0;
    // segment against edge q (Ericson 2005, Sec. 5.1.9, clamped, as selects)
    const V3 e0 = q == 0 ? a : q == 1 ? b : c, e1 = q == 0 ? b : q == 1 ? c : a;
    const V3 d2v = e1 - e0, rv = p0 - e0;
    const float sa = dot(dir, dir), se = dot(d2v, d2v), sf = dot(d2v, rv), sc = dot(dir, rv),
                sb = dot(dir, d2v);
    const float ia_ = __builtin_amdgcn_rcpf(sa), ie_ = __builtin_amdgcn_rcpf(se);
    const float den = sa * se - sb * sb;
    float ss = den > 0.f ? fminf(fmaxf((sb * sf - sc * se) * __builtin_amdgcn_rcpf(den), 0.f), 1.f)
                         : 0.f;
    float tt = (sb * ss + sf) * ie_;
    const float s_lo = fminf(fmaxf(-sc * ia_, 0.f), 1.f), s_hi = fminf(fmaxf((sb - sc) * ia_, 0.f), 1.f);
    ss = tt < 0.f ? s_lo : tt > 1.f ? s_hi : ss;
    tt = fminf(fmaxf(tt, 0.f), 1.f);
    const bool pa_deg = sa <= 1e-30f, pe_deg = se <= 1e-30f;
    ss = pa_deg ? 0.f : pe_deg ? s_lo : ss;
    tt = pa_deg ? (pe_deg ? 0.f : fminf(fmaxf(sf * ie_, 0.f), 1.f)) : pe_deg ? 0.f : tt;
    const V3 ps = p0 + ss * dir, pe = e0 + tt * d2v;
    const float d2_edge = dot(pe - ps, pe - ps);
    const V3 bary_edge = q == 0 ? V3{1.f - tt, tt, 0.f} : q == 1 ? V3{0.f, 1.f - tt, tt}
                                                              : V3{tt, 0.f, 1.f - tt};
    // point candidate: the projection of x into the plane, inside the triangle
    const V3 n = cross(ab, ac);
    const float nn = dot(n, n), inv_nn = __builtin_amdgcn_rcpf(nn);
    const float h0 = dot(p0 - a, n), h1 = dot(p1 - a, n);
    const bool crosses = h0 != h1 && ((h0 <= 0.f) != (h1 <= 0.f) || h0 == 0.f);
    const float tc = h0 != h1 ? h0 * __builtin_amdgcn_rcpf(h0 - h1) : 0.f;
    const V3 x = q == 0 ? p0 : q == 1 ? p1 : p0 + tc * dir;
    const V3 ax = x - a;
    const float d00 = dot(ab, ab), d01 = dot(ab, ac), d11 = dot(ac, ac);
    const float d20 = dot(ax, ab), d21 = dot(ax, ac), ib_ = __builtin_amdgcn_rcpf(d00 * d11 - d01 * d01);
    const float v = (d11 * d20 - d01 * d21) * ib_, w = (d00 * d21 - d01 * d20) * ib_;
    const float u = 1.f - v - w;
    const bool inside = nn > 0.f && u >= 0.f && v >= 0.f && w >= 0.f;
    const float h = dot(ax, n);
    const float d2_point = q == 2 ? (crosses && inside ? -1.f : 3.0e38f)
                                  : (inside ? h * h * inv_nn : 3.0e38f);
    // this lane's best in order (point candidates 0, 1 come before the edges,
    // the crossing after them), then the group's
    const int k_point = q == 2 ? 5 : q, k_edge = 2 + q;
    const bool point_first = q == 2 ? d2_point < 0.f : true;
    const bool take_point = point_first ? !(d2_edge < d2_point) : d2_point < d2_edge;
    float best = take_point ? d2_point : d2_edge;
    int best_k = take_point ? k_point : k_edge;
    if (q == 3) {
        best = 3.0e38f;
        best_k = 7;
    }
#pragma unroll
    for (int m = 1; m < 4; m <<= 1) {
        const float ob = __shfl_xor(best, m, 4);
        const int ok = __shfl_xor(best_k, m, 4);
        if (ob < best || (ob == best && ok < best_k)) {   // a crossing's -1 is below all
            best = ob;
            best_k = ok;
        }
    }
    // the winner's lane and candidate
    const int src = (int)(__lane_id() & ~3u) |
                    (best_k < 2 ? best_k : best_k <= 4 ? best_k - 2 : best_k == 5 ? 2 : 3);
    const bool point_won = best_k < 2 || best_k == 5;
    const V3 my_bary = point_won ? V3{u, v, w} : bary_edge, my_s = point_won ? x : ps;
    const V3 bw = {__shfl(my_bary.x, src), __shfl(my_bary.y, src), __shfl(my_bary.z, src)};
    const V3 sw = {__shfl(my_s.x, src), __shfl(my_s.y, src), __shfl(my_s.z, src)};
    const float d2 = best_k == 5 ? 0.f : best;
    if (q != 0 || !(d2 < r * r))
        return;
    const float d = __builtin_amdgcn_sqrtf(d2);
    V3 nrm;
    if (d > 1e-12f) {
        const V3 y = bw.x * a + bw.y * b + bw.z * c;
        nrm = __builtin_amdgcn_rcpf(d) * (y - sw);
    } else {
        if (!(nn > 0.f))
            return;
        nrm = __builtin_amdgcn_rsqf(nn) * n;
    }
    const float dn = pa.w * bw.x * bw.x + pb.w * bw.y * bw.y + pc.w * bw.z * bw.z;
    if (!(dn > kMinDenominator))
        return;
    const float k = -(d - r) * __builtin_amdgcn_rcpf(dn);
    const float ka = pa.w * bw.x * k, kb = pb.w * bw.y * k, kc = pc.w * bw.z * k;
    pa.x += ka * nrm.x;
    pa.y += ka * nrm.y;
    pa.z += ka * nrm.z;
    pb.x += kb * nrm.x;
    pb.y += kb * nrm.y;
    pb.z += kb * nrm.z;
    pc.x += kc * nrm.x;
    pc.y += kc * nrm.y;
    pc.z += kc * nrm.z;
    xw[ia] = pa;
    xw[ib] = pb;
    xw[ic] = pc;
}

// Contact-candidate test in float32 with every product and sum rounded
// separately (no fused multiply-add), so the host can repeat it bit for bit.
__device__ __forceinline__ bool within_reach(float4 p, float cx, float cy, float cz, float reach2)
{
#pragma clang fp contract(off)
    const float dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
    const float d2 = (dx * dx + dy * dy) + dz * dz;
    return p.w > 0.0f && d2 < reach2;
}

// Push a particle out of a sphere (Sec. III-A.3, k_c = 1).
__device__ __forceinline__ void project_contact(float4 *xw, int i, float cx, float cy, float cz,
                                                float r, float r2)
{
    float4 p = xw[i];
    const float dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
    const float d2 = dx * dx + dy * dy + dz * dz;
    if (!(d2 < r2))
        return;
    if (d2 > 0.0f) {
        const float s = r * fast_rsq(d2);
        p.x = cx + dx * s;
        p.y = cy + dy * s;
        p.z = cz + dz * s;
    } else {
        p.x = cx;
        p.y = cy;
        p.z = cz + r;
    }
    xw[i] = p;
}

__device__ __forceinline__ float wave_sum(float v)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

template <int PPT, bool STAGE, bool RESIDUAL, bool JACOBI>
__global__ void __launch_bounds__(1024) xpbd_step_lds_kernel(StepArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int env = blockIdx.x;
    const int tid = threadIdx.x;
    const int B = blockDim.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int num_waves = B >> 6;

    const EnvDev ed = A.envs[env];
    const MeshDev md = A.meshes[ed.mesh];
    const int V = md.num_vertices, E = md.num_edges, T = md.num_tets;
    const int tools = A.num_tools;
    const bool capsule = A.tool_shape == 1;   // XPBD_TOOL_CAPSULE: faces against segments
    const int F = capsule ? md.num_faces : 0;
    const LdsLayout L = lds_layout(V, E, T, tools, STAGE, JACOBI, F);
    uint8_t *fflag = reinterpret_cast<uint8_t *>(smem + L.face_flag);
    float4 *xw = reinterpret_cast<float4 *>(smem + L.xw);
    float *dxs = reinterpret_cast<float *>(smem + L.dx);            // Jacobi only
    float *inv_n = reinterpret_cast<float *>(smem + L.inv_count);   // Jacobi only
    if constexpr (JACOBI)
        for (int i = tid; i < V; i += B) {
            dxs[i] = dxs[V + i] = dxs[2 * V + i] = 0.0f;
            inv_n[i] = md.inv_count[i];
        }
    float *lam = reinterpret_cast<float *>(smem + L.lambda);
    uint16_t *clist = reinterpret_cast<uint16_t *>(smem + L.contacts);
    uint32_t *scratch = reinterpret_cast<uint32_t *>(smem + L.scratch);
    const uint32_t *e_pair = md.edge_pair;
    const float *e_rest = md.edge_rest;
    const uint2 *t_quad = md.tet_quad;
    const float *t_rest = md.tet_rest;
    if constexpr (STAGE) {
        uint32_t *sp = reinterpret_cast<uint32_t *>(smem + L.edge_pair);
        float *sr = reinterpret_cast<float *>(smem + L.edge_rest);
        uint2 *sq = reinterpret_cast<uint2 *>(smem + L.tet_quad);
        float *st = reinterpret_cast<float *>(smem + L.tet_rest);
        for (int j = tid; j < E; j += B) {
            sp[j] = md.edge_pair[j];
            sr[j] = md.edge_rest[j];
        }
        for (int j = tid; j < T; j += B) {
            sq[j] = md.tet_quad[j];
            st[j] = md.tet_rest[j];
        }
        e_pair = sp;
        e_rest = sr;
        t_quad = sq;
        t_rest = st;
    }

    const float h = A.h, inv_h = A.inv_h;
    const float gx = A.gravity[0], gy = A.gravity[1], gz = A.gravity[2];
    const float alpha_d = A.compliance[2 * env] * inv_h * inv_h;   // alpha~ = alpha / h^2
    const float alpha_v = A.compliance[2 * env + 1] * inv_h * inv_h;
    const int NP = A.total_particles;
    const int off = ed.particle_offset;

    // state: positions (+ inverse mass) to LDS, velocities to registers
    float vx[PPT], vy[PPT], vz[PPT], kx[PPT], ky[PPT], kz[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = k * B + tid;
        vx[k] = vy[k] = vz[k] = kx[k] = ky[k] = kz[k] = 0.0f;
        if (i < V) {
            xw[i] = make_float4(A.pos[off + i], A.pos[NP + off + i], A.pos[2 * NP + off + i],
                                md.inv_mass[i]);
            vx[k] = A.vel[off + i];
            vy[k] = A.vel[NP + off + i];
            vz[k] = A.vel[2 * NP + off + i];
        }
    }
    __syncthreads();

    int count[2] = {0, 0};
    float cx[2] = {0.f, 0.f}, cy[2] = {0.f, 0.f}, cz[2] = {0.f, 0.f};
    V3 cap0[2] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}}, cap1[2] = {cap0[0], cap0[1]};
    const int last_step = A.num_steps - 1;
    for (int step = 0; step < A.num_steps; ++step) {
        // capsules: candidate faces (a free corner, closer than 2r to the axis)
        // on the start-of-step positions
        for (int t = 0; t < tools && capsule; ++t) {
            const float *c = A.tool_pos + (((size_t)step * A.num_envs + env) * tools + t) * 6;
            cap0[t] = {c[0], c[1], c[2]};
            cap1[t] = {c[3], c[4], c[5]};
            const float r = A.tool_radius[t];
            int mine = 0;
            for (int j = tid; j < F; j += B) {
                const uint2 f = md.faces[j];
                const float4 pa = xw[f.x & 0xffffu], pb = xw[f.x >> 16], pc = xw[f.y];
                V3 bary, sp;
                const bool flag = (pa.w > 0.f || pb.w > 0.f || pc.w > 0.f) &&
                                  segment_triangle(cap0[t], cap1[t], v3(pa), v3(pb), v3(pc), bary,
                                                   sp) < 4.f * r * r;
                fflag[t * F + j] = flag ? 1 : 0;
                mine += flag ? 1 : 0;
            }
            const float total = wave_sum((float)mine);
            if (lane == 0)
                scratch[wave] = (uint32_t)total;
            __syncthreads();
            int n = 0;
            for (int w = 0; w < num_waves; ++w)
                n += (int)scratch[w];
            count[t] = n;
            __syncthreads();
        }
        // spheres: instrument state and contact candidates on the start-of-step positions
        for (int t = 0; t < tools && !capsule; ++t) {
            const float *c = A.tool_pos + (((size_t)step * A.num_envs + env) * tools + t) * 3;
            cx[t] = c[0];
            cy[t] = c[1];
            cz[t] = c[2];
            const float reach2 = A.tool_reach2[t];
            uint16_t *list = clist + t * V;
            int base = 0;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int i = k * B + tid;
                const bool flag = i < V && within_reach(xw[i], cx[t], cy[t], cz[t], reach2);
                const uint64_t mask = __ballot(flag);
                if (lane == 0)
                    scratch[wave] = (uint32_t)__popcll(mask);
                __syncthreads();
                int before = 0, total = 0;
                for (int w = 0; w < num_waves; ++w) {
                    const int n = (int)scratch[w];
                    before += w < wave ? n : 0;
                    total += n;
                }
                if (flag)
                    list[base + before + __popcll(mask & __lanemask_lt())] = (uint16_t)i;
                base += total;
                __syncthreads();
            }
            count[t] = base;
        }

        for (int sub = 0; sub < A.substeps; ++sub) {
            // predict velocity and position (Alg. 1); pinned particles stay put
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int i = k * B + tid;
                if (i < V) {
                    float4 p = xw[i];
                    kx[k] = p.x;
                    ky[k] = p.y;
                    kz[k] = p.z;
                    if (p.w > 0.0f) {
                        vx[k] += h * gx;
                        vy[k] += h * gy;
                        vz[k] += h * gz;
                        p.x += h * vx[k];
                        p.y += h * vy[k];
                        p.z += h * vz[k];
                        xw[i] = p;
                    }
                }
            }
            for (int j = tid; j < E + T; j += B)
                lam[j] = 0.0f;
            __syncthreads();

            for (int it = 0; it < A.iterations; ++it) {
                if constexpr (JACOBI) {
                    // the paper's iteration: every constraint from the same
                    // positions (summed colour by colour: no two lanes of a colour
                    // share a particle), then each particle moves by its mean correction
                    for (int c = 0; c < md.num_edge_colours; ++c) {
                        const int end = md.edge_ptr[c + 1];
                        for (int j = md.edge_ptr[c] + tid; j < end; j += B) {
                            const uint32_t pr = e_pair[j];
                            float l = lam[j];
                            edge_delta(xw, dxs, V, (int)(pr & 0xffffu), (int)(pr >> 16),
                                       e_rest[j], alpha_d, l);
                            lam[j] = l;
                        }
                        __syncthreads();
                    }
                    for (int c = 0; c < md.num_tet_colours; ++c) {
                        const int end = md.tet_ptr[c + 1];
                        for (int j = md.tet_ptr[c] + tid; j < end; j += B) {
                            const uint2 q = t_quad[j];
                            float l = lam[E + j];
                            tet_delta(xw, dxs, V, q.x, q.y, t_rest[j], alpha_v, l);
                            lam[E + j] = l;
                        }
                        __syncthreads();
                    }
                    for (int i = tid; i < V; i += B) {
                        float4 p = xw[i];
                        const float s = inv_n[i];
                        p.x += dxs[i] * s;
                        p.y += dxs[V + i] * s;
                        p.z += dxs[2 * V + i] * s;
                        xw[i] = p;
                        dxs[i] = dxs[V + i] = dxs[2 * V + i] = 0.0f;
                    }
                    __syncthreads();
                } else {
                for (int c = 0; c < md.num_edge_colours; ++c) {
                    const int end = md.edge_ptr[c + 1];
                    for (int j = md.edge_ptr[c] + tid; j < end; j += B) {
                        const uint32_t pr = e_pair[j];
                        float l = lam[j];
                        edge_update(xw, (int)(pr & 0xffffu), (int)(pr >> 16), e_rest[j], alpha_d, l);
                        lam[j] = l;
                    }
                    __syncthreads();
                }
                for (int c = 0; c < md.num_tet_colours; ++c) {
                    const int end = md.tet_ptr[c + 1];
                    for (int j = md.tet_ptr[c] + tid; j < end; j += B) {
                        const uint2 q = t_quad[j];
                        float l = lam[E + j];
                        tet_update(xw, q.x, q.y, t_rest[j], alpha_v, l);
                        lam[E + j] = l;
                    }
                    __syncthreads();
                }
                }
                for (int t = 0; t < tools && !capsule; ++t) {
                    if (count[t] == 0)
                        continue;
                    const uint16_t *list = clist + t * V;
                    for (int n = tid; n < count[t]; n += B)
                        project_contact(xw, list[n], cx[t], cy[t], cz[t], A.tool_radius[t],
                                        A.tool_radius2[t]);
                    __syncthreads();
                }
                for (int t = 0; t < tools && capsule; ++t) {
                    if (count[t] == 0)
                        continue;
                    for (int c = 0; c < md.num_face_colours; ++c) {
                        const int end = md.face_ptr[c + 1];
                        for (int j = md.face_ptr[c] + tid; j < end; j += B)
                            if (fflag[t * F + j])
                                capsule_push(xw, md.faces[j], cap0[t], cap1[t], A.tool_radius[t]);
                        __syncthreads();
                    }
                }
            }

            if constexpr (RESIDUAL) {
                if (step == last_step && sub == A.substeps - 1) {
                    float sum = 0.0f, big = 0.0f;
                    for (int j = tid; j < E; j += B) {
                        const uint32_t pr = e_pair[j];
                        const float4 pa = xw[pr & 0xffffu], pb = xw[pr >> 16];
                        const float dx = pa.x - pb.x, dy = pa.y - pb.y, dz = pa.z - pb.z;
                        const float len = sqrtf(dx * dx + dy * dy + dz * dz);
                        const float r = (len - e_rest[j] + alpha_d * lam[j]) / e_rest[j];
                        sum += r * r;
                        big = fmaxf(big, fabsf(r));
                    }
                    for (int j = tid; j < T; j += B) {
                        const uint2 q = t_quad[j];
                        const float4 pa = xw[q.x & 0xffffu], pb = xw[q.x >> 16];
                        const float4 pc = xw[q.y & 0xffffu], pd = xw[q.y >> 16];
                        const float bax = pb.x - pa.x, bay = pb.y - pa.y, baz = pb.z - pa.z;
                        const float cax = pc.x - pa.x, cay = pc.y - pa.y, caz = pc.z - pa.z;
                        const float dax = pd.x - pa.x, day = pd.y - pa.y, daz = pd.z - pa.z;
                        const float vol = (bax * (cay * daz - caz * day) + bay * (caz * dax - cax * daz) +
                                           baz * (cax * day - cay * dax)) * kSixth;
                        const float r = (vol - t_rest[j] + alpha_v * lam[E + j]) / t_rest[j];
                        sum += r * r;
                        big = fmaxf(big, fabsf(r));
                    }
                    sum = wave_sum(sum);
                    big = wave_max(big);
                    float *fs = reinterpret_cast<float *>(scratch);
                    if (lane == 0) {
                        fs[wave] = sum;
                        fs[32 + wave] = big;
                    }
                    __syncthreads();
                    if (tid == 0) {
                        float s = 0.0f, m = 0.0f;
                        for (int w = 0; w < num_waves; ++w) {
                            s += fs[w];
                            m = fmaxf(m, fs[32 + w]);
                        }
                        A.residual[2 * env] = E + T > 0 ? sqrtf(s / (float)(E + T)) : 0.0f;
                        A.residual[2 * env + 1] = m;
                    }
                    __syncthreads();
                }
            }

            // velocity update v = (x - x_prev) / h (Alg. 1)
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int i = k * B + tid;
                if (i < V) {
                    const float4 p = xw[i];
                    vx[k] = (p.x - kx[k]) * inv_h;
                    vy[k] = (p.y - ky[k]) * inv_h;
                    vz[k] = (p.z - kz[k]) * inv_h;
                }
            }
        }
    }

    // write back (structure of arrays, coalesced)
    int bad = 0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = k * B + tid;
        if (i < V) {
            const float4 p = xw[i];
            A.pos[off + i] = p.x;
            A.pos[NP + off + i] = p.y;
            A.pos[2 * NP + off + i] = p.z;
            A.vel[off + i] = vx[k];
            A.vel[NP + off + i] = vy[k];
            A.vel[2 * NP + off + i] = vz[k];
            bad |= !(isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(vx[k]) &&
                     isfinite(vy[k]) && isfinite(vz[k]));
        }
    }
    bad = __syncthreads_or(bad);
    if (tid == 0 && bad)
        A.nonfinite[env] = 1;
    for (int t = 0; t < tools; ++t) {
        const uint16_t *list = clist + t * V;
        for (int n = tid; n < V; n += B)
            A.contacts[(size_t)t * NP + off + n] = !capsule && n < count[t] ? (int32_t)list[n] : -1;
        if (tid == 0)
            A.contact_counts[env * tools + t] = count[t];   // capsules: candidate faces
    }
    if (A.lambda_out) {
        float *out = A.lambda_out + ed.lambda_offset;
        for (int j = tid; j < E; j += B)
            out[md.edge_id[j]] = lam[j];
        for (int j = tid; j < T; j += B)
            out[E + md.tet_id[j]] = lam[E + j];
    }
}

// Pointers into global memory seen through the global address space, so that
// loads become global_load (vector memory counter only) instead of flat loads.
#define XPBD_GLOBAL __attribute__((address_space(1)))
// Read-only kernel inputs indexed by workgroup-uniform values go through the
// constant address space, so they load into scalar registers.
#define XPBD_CONST __attribute__((address_space(4)))

// x unchanged, but opaque to the optimiser: per-lane values derived from it
// are recomputed where they are used instead of being hoisted and kept live
// (or spilled) across the solver loop.
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Workgroup-wide OR of a per-thread flag: one ballot per wave into words[],
// one barrier.  Callers separate two uses of the same words by a barrier.
__device__ __forceinline__ bool block_any(bool v, uint32_t *words, int wave, int lane,
                                          int num_waves)
{
    const uint64_t m = __ballot(v);
    if (lane == 0)
        words[wave] = m != 0u ? 1u : 0u;
    __syncthreads();
    uint32_t any = 0u;
    for (int w = 0; w < num_waves; ++w)
        any |= words[w];
    return any != 0u;
}

// Native vector types (the HIP vector classes cannot be loaded through an
// address-space-qualified pointer).
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// Multipliers of a lane's constraints: one register per round, in banks of 32
// registers held as a vector and indexed with the (workgroup-uniform) round
// counter, which the compiler lowers to relative register addressing.
typedef float lambda_bank __attribute__((ext_vector_type(32)));

// Round-major record table of one mesh seen through the global address space:
// the record of lane l in round r is rr[r][l], three words for both kinds
// (edge: pair, rest length bits, 0; tet: ab, cd, rest volume bits).
struct Record {
    uint32_t w0, w1, w2;
};

struct RoundTables {
    __amdgpu_buffer_rsrc_t rsrc;      // the mesh's record table as a buffer
    uint32_t lane_bytes;              // byte offset of this lane's record in a row
    uint32_t row_bytes;               // bytes of one row (blockDim records)
    uint32_t pad;                     // padding particle in the records' units
};

// The record table [rounds + 2][B] of a mesh (12-byte records) as a buffer:
// a row's offset is a scalar, the lane's offset a fixed register, so a fetch
// needs no per-round address arithmetic in the vector unit; reads beyond the
// table return zeros.
__device__ __forceinline__ RoundTables round_tables(const MeshDev &md, int B, int tid,
                                                    uint32_t pad)
{
    RoundTables t;
    const uint32_t row = 12u * (uint32_t)B;
    t.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(md.round_rec), (short)0,
                                               (int)(row * (uint32_t)(md.num_rounds + 2)),
                                               0x00020000);
    t.lane_bytes = 12u * (uint32_t)tid;
    t.row_bytes = row;
    t.pad = pad;
    return t;
}

// Every wave fetches exactly one record per round (also a wave without a
// constraint in round r: the table is L2-resident), so the loads retire in
// order and each round waits only for the fetch issued two rounds before it.
// The address depends only on (round, lane), so the fetch can run rounds
// ahead; rows R and R + 1 of the table repeat rows 0 and 1, so round r
// fetches row r + 2 with no wrap.
__device__ __forceinline__ Record fetch_record(const RoundTables &t, int r)
{
    typedef unsigned int v3u __attribute__((ext_vector_type(3)));
    const v3u v = __builtin_amdgcn_raw_buffer_load_b96(t.rsrc, (int)t.lane_bytes,
                                                       (int)((uint32_t)r * t.row_bytes), 0);
    Record rec;
    rec.w0 = v.x;
    rec.w1 = v.y;
    rec.w2 = v.z;
    return rec;
}

// Multiplier scale of environment e of the workgroup's group (uniform values).
template <int EG>
__device__ __forceinline__ float pick(const float (&v)[EG], uint32_t e)
{
    float x = v[0];
    if constexpr (EG > 1)
        x = e == 1u ? v[1] : x;
    if constexpr (EG > 2) {
        x = e == 2u ? v[2] : x;
        x = e == 3u ? v[3] : x;
    }
    return x;
}

// Round r of an iteration, projecting tetrahedra (TET) or edges.  `slot`
// holds this lane's record of round r (fetched two rounds earlier) and
// receives the record of round r + 2.  Waves without a constraint in a round
// skip it (uniform branch on the wave's activity mask); a barrier closes
// every colour.  With several environments per workgroup the top two bits of
// the first word name the lane's environment (whose compliance applies).
template <int EG, bool TET, bool BAR>
__device__ __forceinline__ void run_round(float4 *xw, const RoundTables &t, int r, Record &slot,
                                          uint64_t active, uint64_t barriers, lambda_bank &bank,
                                          const float (&alpha_d)[EG], const float (&alpha_v)[EG])
{
    const uint32_t w0 = slot.w0, w1 = slot.w1, w2 = slot.w2;
    if ((active >> r) & 1u) {   // padding lanes project the padding particle: no effect
        uint32_t e = 0u, ab = w0;
        if constexpr (EG > 1) {
            e = w0 >> 30;
            ab = w0 & 0x3fffffffu;
        }
        // one environment per workgroup: the records hold LDS byte offsets
        constexpr int kUnit = EG == 1 ? 1 : 16;
        float l = bank[r & 31];
        if constexpr (TET)
            tet_update<kUnit>(xw, ab, w1, __uint_as_float(w2), pick<EG>(alpha_v, e), l);
        else
            edge_update<kUnit>(xw, ab & 0xffffu, ab >> 16, __uint_as_float(w1),
                               pick<EG>(alpha_d, e), l);
        bank[r & 31] = l;
    }
    // the record of round r + 2 is fetched once this round's record is used, into
    // the same registers (no copy): it has the next round to arrive
    slot = fetch_record(t, r + 2);
    if (BAR || ((barriers >> r) & 1u))
        __syncthreads();
}

// One sweep of Alg. 1's constraint loops: the edge rounds [0, Re), then the
// tetrahedron rounds [Re, R), each kind in loops of its own (no round tests
// its kind; Re and R are even), in pairs so that the two prefetch slots never
// move.  Rounds 0..31 keep their multipliers in bank0, rounds 32..63 in bank1.
// BAR: every colour is one round, so a barrier closes every round (the
// padding rounds too) without a test of the barrier mask.
template <int EG, int NB, bool BAR>
__device__ __forceinline__ void sweep_rounds(float4 *xw, const RoundTables &t, int Re, int R,
                                             Record &slot_a, Record &slot_b, uint64_t active,
                                             uint64_t barriers, lambda_bank &bank0,
                                             lambda_bank &bank1, const float (&alpha_d)[EG],
                                             const float (&alpha_v)[EG])
{
    const int E0 = Re < 32 ? Re : 32, R0 = R < 32 ? R : 32;
    int r = 0;
    for (; r < E0; r += 2) {
        run_round<EG, false, BAR>(xw, t, r, slot_a, active, barriers, bank0, alpha_d, alpha_v);
        run_round<EG, false, BAR>(xw, t, r + 1, slot_b, active, barriers, bank0, alpha_d, alpha_v);
    }
    for (; r < R0; r += 2) {
        run_round<EG, true, BAR>(xw, t, r, slot_a, active, barriers, bank0, alpha_d, alpha_v);
        run_round<EG, true, BAR>(xw, t, r + 1, slot_b, active, barriers, bank0, alpha_d, alpha_v);
    }
    if constexpr (NB > 1) {
        int q = 32;
        for (; q < Re; q += 2) {
            run_round<EG, false, BAR>(xw, t, q, slot_a, active, barriers, bank1, alpha_d, alpha_v);
            run_round<EG, false, BAR>(xw, t, q + 1, slot_b, active, barriers, bank1, alpha_d, alpha_v);
        }
        for (; q < R; q += 2) {
            run_round<EG, true, BAR>(xw, t, q, slot_a, active, barriers, bank1, alpha_d, alpha_v);
            run_round<EG, true, BAR>(xw, t, q + 1, slot_b, active, barriers, bank1, alpha_d, alpha_v);
        }
    }
}

// Tool modes of the register kernel: spheres against particles, spheres with
// the grasper's dragging constraint (RL-style step), capsules against the
// surface faces (one environment per workgroup).
enum { kRegSpheres = 0, kRegGrasp = 1, kRegCapsules = 2 };

// One workgroup per group of EG environments of one mesh: group g holds
// environments A.groups[EG g .. EG g + EG); an entry ~e (negative) repeats
// environment e as filler and writes nothing.  The group's particles share
// the LDS (slot_of maps particle i of the group's e-th environment, e V + i,
// to its slot) and every round's lanes may mix the environments.  LDS:
// particles as float4 (x, y, z, w), velocities and start-of-substep positions
// (structure of arrays), then scratch.  Multipliers live in registers (NB
// banks of 32 rounds).
template <int NB, int EG, int MODE, bool BAR>
__device__ __forceinline__ void step_reg_body(StepArgs A)
{
    constexpr bool GRASP = MODE == kRegGrasp;
    constexpr bool CAPSULE = MODE == kRegCapsules;
    static_assert(!CAPSULE || EG == 1, "capsule tools run one environment per workgroup");
    extern __shared__ __align__(16) unsigned char smem[];
    const int group = blockIdx.x;
    const int tid = threadIdx.x;
    const int B = blockDim.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int num_waves = B >> 6;

    const XPBD_CONST int32_t *groups = (const XPBD_CONST int32_t *)(uintptr_t)A.groups;
    const XPBD_CONST float *compliance = (const XPBD_CONST float *)(uintptr_t)A.compliance;
    const float h = A.h, inv_h = A.inv_h;
    int env[EG], off[EG], lam_off[EG];
    bool writes[EG];
    float alpha_d[EG], alpha_v[EG];   // alpha~ = alpha / h^2
#pragma unroll
    for (int e = 0; e < EG; ++e) {
        const int g = groups[group * EG + e];
        env[e] = g >= 0 ? g : ~g;
        writes[e] = g >= 0;
        off[e] = A.envs[env[e]].particle_offset;
        lam_off[e] = A.envs[env[e]].lambda_offset;
        alpha_d[e] = compliance[2 * env[e]] * inv_h * inv_h;
        alpha_v[e] = compliance[2 * env[e] + 1] * inv_h * inv_h;
    }
    const MeshDev md = A.meshes[A.envs[env[0]].mesh];
    const int V = md.num_vertices;     // per environment
    const int VS = EG * V;             // LDS slots of the group
    const int R = md.num_rounds;
    const int R0 = R < 32 ? R : 32;
    const int tools = A.num_tools;
    const int F = CAPSULE ? md.num_faces : 0;
    const int FC = CAPSULE ? md.num_face_colours : 0;
    const CapsuleFaceLayout FL = capsule_face_layout(F, FC);
    const RegLdsLayout L = reg_lds_layout(VS, CAPSULE ? tools * (int)FL.total : 0);
    uint8_t *faces_lds = smem + L.faces;   // capsules: [tools] candidate faces
    float4 *xw = reinterpret_cast<float4 *>(smem + L.xw);
    float *vel = reinterpret_cast<float *>(smem + L.vel);      // [3][VS]
    float *prev = reinterpret_cast<float *>(smem + L.prev);    // [3][VS]
    uint32_t *scratch = reinterpret_cast<uint32_t *>(smem + L.scratch);
    float4 *tool_c = reinterpret_cast<float4 *>(smem + L.scratch + kRegScratchTools);  // [EG][2]

    const float hgx = h * A.gravity[0], hgy = h * A.gravity[1], hgz = h * A.gravity[2];
    const int NP = A.total_particles;

#pragma unroll
    for (int e = 0; e < EG; ++e)
        for (int i = tid; i < V; i += B) {
            const int sl = md.slot_of[e * V + i];
            xw[sl] = make_float4(A.pos[off[e] + i], A.pos[NP + off[e] + i],
                                 A.pos[2 * NP + off[e] + i], md.inv_mass[i]);
            vel[sl] = A.vel[off[e] + i];
            vel[VS + sl] = A.vel[NP + off[e] + i];
            vel[2 * VS + sl] = A.vel[2 * NP + off[e] + i];
        }
    if (tid == 0)
        xw[VS] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);   // padding particle
    // environment of each of this thread's slots k * B + tid: bits 2k, 2k + 1
    uint32_t slot_env = 0u;
    if constexpr (EG > 1)
        for (int k = 0, sl = tid; sl < VS; ++k, sl += B) {
            int q = md.id_of[sl], e = 0;
            while (q >= V) {
                q -= V;
                ++e;
            }
            slot_env |= (uint32_t)e << (2 * k);
        }
    lambda_bank bank0 = 0.0f, bank1 = 0.0f;
    __syncthreads();

    // round tables and this wave's masks (uniform); prime the two-round prefetch
    // (padding particle in the records' units)
    const RoundTables tab =
        round_tables(md, B, tid, EG == 1 ? 16u * (uint32_t)VS : (uint32_t)VS);
    const uint64_t active = A.meshes[A.envs[env[0]].mesh].wave_active[__builtin_amdgcn_readfirstlane(wave)];
    const uint64_t barriers = md.barrier_mask;
    // (issued in this order, as in every round: the loop then waits for the
    // older fetch only, instead of for both)
    Record slot_a = fetch_record(tab, 0);   // records of the next two rounds (even, odd)
    __builtin_amdgcn_sched_barrier(0);
    Record slot_b = fetch_record(tab, 1);

    uint32_t cand = 0u;  // bit 16 t + k: the particle in slot k * B + tid is a candidate of tool t
    for (int step = 0; step < A.num_steps; ++step) {
        // instrument state (sphere centres of every environment of the group;
        // capsules: the two axis end points of every tool, tool_c[2 t + k])
        if constexpr (CAPSULE) {
            if (tid < 2 * tools) {
                const float *c = A.tool_pos +
                                 (((size_t)step * A.num_envs + env[0]) * tools + (tid >> 1)) * 6 +
                                 3 * (tid & 1);
                tool_c[tid] = make_float4(c[0], c[1], c[2], 0.0f);
            }
        } else if (tid < 2 * EG) {
            const int e = tid >> 1, t = tid & 1;
            if (t < tools) {
                int g = A.groups[group * EG + e];
                g = g >= 0 ? g : ~g;
                const float *c = A.tool_pos + (((size_t)step * A.num_envs + g) * tools + t) * 3;
                tool_c[tid] = make_float4(c[0], c[1], c[2], 0.0f);
            }
        }
        __syncthreads();
        // grasping (Sec. III-A.2): the LDS slot each environment's grasper
        // holds (uniform; -1 for none) and the thread that owns that slot
        int held[EG], owner[EG];
#pragma unroll
        for (int e = 0; e < EG; ++e)
            held[e] = owner[e] = -1;
        bool grasping = false;
        if constexpr (GRASP) {
            int32_t *gs = reinterpret_cast<int32_t *>(smem + L.scratch + kRegScratchGrasp);
            uint64_t *part = reinterpret_cast<uint64_t *>(smem + L.scratch + kRegScratchGrasp + 16);
#pragma unroll
            for (int e = 0; e < EG; ++e)
                if (tid == e) {
                    const int h = A.grasp[env[e]];
                    const bool ok = h >= 0 && h < V && md.inv_mass[h] > 0.0f;
                    gs[e] = ok ? (int)md.slot_of[e * V + h] : -1;
                    gs[EG + e] = h == -2 ? 1 : 0;
                }
            __syncthreads();
            bool search = false;
#pragma unroll
            for (int e = 0; e < EG; ++e)
                search |= gs[EG + e] != 0;
            if (search) {
                // a closed grasper holding nothing: the free particle closest
                // to the dragging point strictly within reach, on the
                // start-of-step positions; key (squared distance bits, id)
                // so that the lowest id wins a tie
                uint64_t best[EG];
#pragma unroll
                for (int e = 0; e < EG; ++e)
                    best[e] = ~0ull;
                for (int k = 0, i = opaque(tid); i < VS; ++k, i += B) {
                    const int e = EG > 1 ? (int)((slot_env >> (2 * k)) & 3u) : 0;
                    const float4 ct = tool_c[2 * e];
                    const float4 p = xw[i];
                    const float dx = p.x - (ct.x + A.grasp_offset[0]);
                    const float dy = p.y - (ct.y + A.grasp_offset[1]);
                    const float dz = p.z - (ct.z + A.grasp_offset[2]);
                    const float d2 = dx * dx + dy * dy + dz * dz;
                    if (p.w > 0.0f && d2 < A.grasp_radius2) {
                        const uint64_t key = (uint64_t)__float_as_uint(d2) << 32 |
                                             (uint32_t)((int)md.id_of[i] - e * V);
#pragma unroll
                        for (int f = 0; f < EG; ++f)
                            best[f] = f == e && key < best[f] ? key : best[f];
                    }
                }
#pragma unroll
                for (int e = 0; e < EG; ++e) {
                    best[e] = wave_min_u64(best[e]);
                    if (lane == 0)
                        part[wave * EG + e] = best[e];
                }
                __syncthreads();
#pragma unroll
                for (int e = 0; e < EG; ++e)
                    if (tid == e && gs[EG + e]) {
                        uint64_t m = ~0ull;
                        for (int w = 0; w < num_waves; ++w)
                            m = part[w * EG + e] < m ? part[w * EG + e] : m;
                        const int id = m == ~0ull ? -1 : (int)(uint32_t)m;
                        gs[e] = id >= 0 ? (int)md.slot_of[e * V + id] : -1;
                        if (writes[e])
                            A.grasp[env[e]] = id;
                    }
                __syncthreads();
            }
#pragma unroll
            for (int e = 0; e < EG; ++e) {
                held[e] = __builtin_amdgcn_readfirstlane(gs[e]);
                owner[e] = held[e] >= 0 ? held[e] % B : -1;
                grasping |= held[e] >= 0;
            }
        }
        // contact candidates on the start-of-step positions
        cand = 0u;
        if constexpr (CAPSULE) {
            // faces with a free corner closer than 2r to the axis (Sec. III-A.3),
            // as 64-bit flag words (a wave's 64 consecutive faces per word);
            // bit t of cand: this thread flagged a face of tool t
            for (int t = 0; t < tools; ++t) {
                const V3 c0 = v3(tool_c[2 * t]), c1 = v3(tool_c[2 * t + 1]);
                const float r = t == 0 ? A.tool_radius[0] : A.tool_radius[1];
                uint64_t *flags = reinterpret_cast<uint64_t *>(faces_lds + t * FL.total + FL.flags);
                for (int j = tid; j < F; j += B) {
                    const uint2 f = md.faces[j];
                    const float4 pa = xw[md.slot_of[f.x & 0xffffu]], pb = xw[md.slot_of[f.x >> 16]],
                                 pc = xw[md.slot_of[f.y]];
                    bool flag = (pa.w > 0.f || pb.w > 0.f || pc.w > 0.f) &&
                                !face_beyond(c0, c1, v3(pa), v3(pb), v3(pc), 2.f * r);
                    if (flag) {
                        V3 bary, sp;
                        flag = segment_triangle(c0, c1, v3(pa), v3(pb), v3(pc), bary, sp) <
                               4.f * r * r;
                    }
                    const uint64_t word = __ballot(flag);
                    if (lane == 0)
                        flags[(j - lane) >> 6] = word;
                    cand |= flag ? 1u << t : 0u;
                }
            }
        } else {
            for (int t = 0; t < tools; ++t) {
                const float reach2 = t == 0 ? A.tool_reach2[0] : A.tool_reach2[1];
                for (int k = 0, i = opaque(tid); i < VS; ++k, i += B) {
                    const float4 ct = tool_c[2 * (int)((slot_env >> (2 * k)) & 3u) + t];
                    if (within_reach(xw[i], ct.x, ct.y, ct.z, reach2))
                        cand |= 1u << (16 * t + k);
                }
            }
        }
        const bool any_contact = block_any(cand != 0u, scratch + 32, wave, lane, num_waves);
        if constexpr (CAPSULE) {
            // one wave per tool lists the flagged faces colour by colour, as
            // the LDS slots of their corners, with the colour bounds
            for (int t = 0; t < tools; ++t)
                if (wave == (t & (num_waves - 1))) {
                    uint8_t *base = faces_lds + t * FL.total;
                    const uint64_t *flags = reinterpret_cast<const uint64_t *>(base + FL.flags);
                    uint32_t *list_ab = reinterpret_cast<uint32_t *>(base + FL.ab);
                    uint16_t *list_c = reinterpret_cast<uint16_t *>(base + FL.c);
                    uint16_t *bounds = reinterpret_cast<uint16_t *>(base + FL.bounds);
                    int n = 0;
                    for (int c = 0; c < FC; ++c) {
                        if (lane == 0)
                            bounds[c] = (uint16_t)n;
                        const int hi = md.face_ptr[c + 1];
                        for (int j0 = any_contact ? md.face_ptr[c] : hi; j0 < hi; j0 += 64) {
                            const int j = j0 + lane;
                            const bool f = j < hi && ((flags[j >> 6] >> (j & 63)) & 1u);
                            const uint64_t m = __ballot(f);
                            if (f) {
                                const int at = n + __popcll(m & __lanemask_lt());
                                const uint2 fc = md.faces[j];
                                list_ab[at] = (uint32_t)md.slot_of[fc.x & 0xffffu] |
                                              (uint32_t)md.slot_of[fc.x >> 16] << 16;
                                list_c[at] = (uint16_t)md.slot_of[fc.y];
                            }
                            n += __popcll(m);
                        }
                    }
                    if (lane == 0)
                        bounds[FC] = (uint16_t)n;
                }
            __syncthreads();
        }

        for (int sub = 0; sub < A.substeps; ++sub) {
            // predict velocity and position (Alg. 1); pinned particles stay put
            for (int i = opaque(tid); i < VS; i += B) {
                float4 p = xw[i];
                prev[i] = p.x;
                prev[VS + i] = p.y;
                prev[2 * VS + i] = p.z;
                if (p.w > 0.0f) {
                    const float vx = vel[i] + hgx, vy = vel[VS + i] + hgy, vz = vel[2 * VS + i] + hgz;
                    vel[i] = vx;
                    vel[VS + i] = vy;
                    vel[2 * VS + i] = vz;
                    p.x += h * vx;
                    p.y += h * vy;
                    p.z += h * vz;
                    xw[i] = p;
                }
            }
            bank0 = 0.0f;
            if constexpr (NB > 1)
                bank1 = 0.0f;
            __syncthreads();

            for (int it = 0; it < A.iterations; ++it) {
                sweep_rounds<EG, NB, BAR>(xw, tab, md.num_edge_rounds, R, slot_a, slot_b, active,
                                          barriers, bank0, bank1, alpha_d, alpha_v);
                if (CAPSULE && any_contact) {
                    // flagged faces pushed out of every capsule, face colour by
                    // face colour (faces of one colour share no particle); a
                    // colour without flagged faces costs no barrier, and the
                    // colours rotate over the waves
                    for (int t = 0; t < tools; ++t) {
                        const V3 c0 = v3(tool_c[2 * t]), c1 = v3(tool_c[2 * t + 1]);
                        const float rt = t == 0 ? A.tool_radius[0] : A.tool_radius[1];
                        const uint8_t *base = faces_lds + t * FL.total;
                        const uint32_t *list_ab = reinterpret_cast<const uint32_t *>(base + FL.ab);
                        const uint16_t *list_c = reinterpret_cast<const uint16_t *>(base + FL.c);
                        const uint16_t *bounds = reinterpret_cast<const uint16_t *>(base + FL.bounds);
                        for (int c = 0; c < FC; ++c) {
                            const int lo = __builtin_amdgcn_readfirstlane(bounds[c]);
                            const int hi = __builtin_amdgcn_readfirstlane(bounds[c + 1]);
                            if (lo == hi)
                                continue;
                            // face k of the colour: wave (k + c) mod waves, the
                            // 4-lane group k / waves of that wave
                            const int first = (lane >> 2) * num_waves + ((wave - c) & (num_waves - 1));
                            for (int j = lo + first; j < hi; j += 16 * num_waves)
                                capsule_push_lanes(xw, make_uint2(list_ab[j], list_c[j]), c0, c1, rt,
                                                   lane & 3);
                            __syncthreads();
                        }
                    }
                } else if (any_contact || (GRASP && grasping)) {
                    for (int t = 0; t < tools; ++t) {
                        const float rt = t == 0 ? A.tool_radius[0] : A.tool_radius[1];
                        const float rt2 = t == 0 ? A.tool_radius2[0] : A.tool_radius2[1];
                        for (int k = 0, i = opaque(tid); i < VS; ++k, i += B)
                            if ((cand >> (16 * t + k)) & 1u) {
                                const float4 ct = tool_c[2 * (int)((slot_env >> (2 * k)) & 3u) + t];
                                project_contact(xw, i, ct.x, ct.y, ct.z, rt, rt2);
                            }
                    }
                    // the dragging constraint (k_s = 1, rest length 0) moves the
                    // held particle onto the dragging point; its slot's owner
                    // runs it after its own contacts
#pragma unroll
                    for (int e = 0; e < EG; ++e)
                        if (GRASP && tid == owner[e]) {
                            const float4 ct = tool_c[2 * e];
                            float4 p = xw[held[e]];
                            p.x = ct.x + A.grasp_offset[0];
                            p.y = ct.y + A.grasp_offset[1];
                            p.z = ct.z + A.grasp_offset[2];
                            xw[held[e]] = p;
                        }
                    __syncthreads();
                }
            }

            // velocity update v = (x - x_prev) / h (Alg. 1)
            for (int i = opaque(tid); i < VS; i += B) {
                const float4 p = xw[i];
                vel[i] = (p.x - prev[i]) * inv_h;
                vel[VS + i] = (p.y - prev[VS + i]) * inv_h;
                vel[2 * VS + i] = (p.z - prev[2 * VS + i]) * inv_h;
            }
        }
    }

    // write back (structure of arrays, coalesced); slot_of[i] belongs to another
    // thread's velocity update, hence the barrier
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EG; ++e) {
        int bad = 0;
        if (writes[e])
            for (int i = tid; i < V; i += B) {
                const int sl = md.slot_of[e * V + i];
                const float4 p = xw[sl];
                const float vx = vel[sl], vy = vel[VS + sl], vz = vel[2 * VS + sl];
                A.pos[off[e] + i] = p.x;
                A.pos[NP + off[e] + i] = p.y;
                A.pos[2 * NP + off[e] + i] = p.z;
                A.vel[off[e] + i] = vx;
                A.vel[NP + off[e] + i] = vy;
                A.vel[2 * NP + off[e] + i] = vz;
                bad |= !(isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(vx) &&
                         isfinite(vy) && isfinite(vz));
            }
        // one word block per environment: no barrier needed between the calls
        bad = block_any(bad != 0, scratch + 32 + 16 * e, wave, lane, num_waves);
        if (tid == 0 && bad && writes[e])
            A.nonfinite[env[e]] = 1;
    }

    // contact candidates of the last step as ascending mesh ids, per
    // environment: flag them by mesh id in a byte map (the start-of-substep
    // positions are no longer needed), then compact in mesh order; capsules:
    // the number of candidate faces per tool of the last step (its list's
    // length) and no particle list
    uint8_t *flag_of = reinterpret_cast<uint8_t *>(prev);
    const int kmax = (V + B - 1) / B;
    if constexpr (CAPSULE) {
        for (int t = 0; t < tools; ++t) {
            const uint16_t *bounds =
                reinterpret_cast<const uint16_t *>(faces_lds + t * FL.total + FL.bounds);
            for (int i = tid; i < V; i += B)
                A.contacts[(size_t)t * NP + off[0] + i] = -1;
            if (tid == 0 && writes[0])
                A.contact_counts[env[0] * tools + t] = A.num_steps > 0 ? (int)bounds[FC] : 0;
        }
    }
#pragma unroll
    for (int e = 0; e < EG; ++e) {
        if (CAPSULE || !writes[e])
            continue;
        for (int t = 0; t < tools; ++t) {
            for (int i = tid; i < V; i += B)
                flag_of[i] = 0;
            __syncthreads();
            for (int k = 0, sl = tid; sl < VS; ++k, sl += B)
                if (((cand >> (16 * t + k)) & 1u) && (int)((slot_env >> (2 * k)) & 3u) == e)
                    flag_of[md.id_of[sl] - e * V] = 1;
            __syncthreads();
            int32_t *list = A.contacts + (size_t)t * NP + off[e];
            int base = 0;
            for (int k = 0; k < kmax; ++k) {
                const int i = k * B + tid;
                const bool flag = i < V && flag_of[i];
                const uint64_t mask = __ballot(flag);
                if (lane == 0)
                    scratch[wave] = (uint32_t)__popcll(mask);
                __syncthreads();
                int before = 0, total = 0;
                for (int w = 0; w < num_waves; ++w) {
                    const int n = (int)scratch[w];
                    before += w < wave ? n : 0;
                    total += n;
                }
                if (flag)
                    list[base + before + __popcll(mask & __lanemask_lt())] = i;
                base += total;
                __syncthreads();
            }
            for (int n = base + tid; n < V; n += B)
                list[n] = -1;
            if (tid == 0)
                A.contact_counts[env[e] * tools + t] = base;
        }
    }
    if (A.lambda_out) {
        // rr_id[r][tid]: environment index (bits 24..25) and constraint id of
        // this lane in round r, -1 for none
        auto store = [&](int r, float l) {
            const int v = md.rr_id[r * B + tid];
            if (v < 0)
                return;
            const int e = v >> 24, id = v & 0xffffff;
            int o = lam_off[0];
            bool w = writes[0];
#pragma unroll
            for (int f = 1; f < EG; ++f) {
                o = e == f ? lam_off[f] : o;
                w = e == f ? writes[f] : w;
            }
            if (w)
                A.lambda_out[o + id] = l;
        };
        for (int r = 0; r < R0; ++r)
            store(r, bank0[r & 31]);
        if constexpr (NB > 1)
            for (int r = 32; r < R; ++r)
                store(r, bank1[r & 31]);
    }
}

template <int NB, int EG, int MODE, bool BAR>
__global__ void __launch_bounds__(1024) xpbd_step_reg_kernel(StepArgs A)
{
    step_reg_body<NB, EG, MODE, BAR>(A);
}

// Capsule tools: the face push-out's closest-point search needs more
// registers than 1024-thread workgroups leave a lane, so this instantiation
// is bounded to 512 threads (two waves per SIMD and workgroup); with one
// multiplier bank it is held to the 128 registers that keep four 256-thread
// workgroups on a CU.
template <int NB>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(NB == 1 ? 4 : 2)))
xpbd_step_reg_kernel_capsules(StepArgs A)
{
    step_reg_body<NB, 1, kRegCapsules, false>(A);
}

// ---------------------------------------------------------------------------
// Learned warm start (an extension of the substep; the network itself runs in
// the matrix-core kernels).  One substep per launch: learned_predict_kernel
// predicts every particle and writes the network's features, the network adds
// its correction to the predicted positions, xpbd_substep_reg_kernel runs the
// sweeps from there with the residual check and updates the velocities.

// Prediction of one substep (Alg. 1) into L.xhat and, when L.features is
// set, the features of every particle: predicted displacement,
// start-of-substep velocity, displacement from rest, and the six
// axis-neighbour offsets minus their rest offsets, normalised
// ((f - in_shift) * in_scale) and rounded to bfloat16 (nearest, ties to
// even); feature 31 flags a free particle.  Loads are branch-free: a pinned
// particle moves by 0 * (v + h g), a missing neighbour reads the particle
// itself and its offset is then zero.
// Grid: (ceil(max V / 256), environments).
__global__ void __launch_bounds__(256) learned_predict_kernel(StepArgs A, LearnedArgs L)
{
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    const int env = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const EnvDev ed = A.envs[env];
    const MeshDev &md = A.meshes[ed.mesh];
    if (i >= md.num_vertices)
        return;
    const int NP = A.total_particles, off = ed.particle_offset;
    const XPBD_GLOBAL float *pos = (const XPBD_GLOBAL float *)(uintptr_t)A.pos;
    const XPBD_GLOBAL float *vel = (const XPBD_GLOBAL float *)(uintptr_t)A.vel;
    const XPBD_GLOBAL f32x4 *rest4 = (const XPBD_GLOBAL f32x4 *)(uintptr_t)md.rest4;
    const float h = A.h;
    const float hg[3] = {h * A.gravity[0], h * A.gravity[1], h * A.gravity[2]};
    const f32x4 Ri = rest4[i];   // rest position, inverse mass
    float x[3], v[3], xh[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        x[k] = pos[k * NP + off + i];
        v[k] = vel[k * NP + off + i];
        xh[k] = x[k] + (Ri.w > 0.0f ? h : 0.0f) * (v[k] + hg[k]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        L.xhat[k * NP + off + i] = xh[k];
    if (!L.features)
        return;
    const XPBD_GLOBAL int32_t *nbr = (const XPBD_GLOBAL int32_t *)(uintptr_t)md.nbr;
    const float rest[3] = {Ri.x, Ri.y, Ri.z};
    float f[32];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        f[k] = xh[k] - x[k];
        f[3 + k] = v[k];
        f[6 + k] = xh[k] - rest[k];
    }
    int nb[6];
#pragma unroll
    for (int d = 0; d < 6; ++d)
        nb[d] = nbr[6 * i + d];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const int j = nb[d] >= 0 ? nb[d] : i;
        const f32x4 Rj = rest4[j];
        const float rj[3] = {Rj.x, Rj.y, Rj.z};
        const float hj = Rj.w > 0.0f ? h : 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float pj = pos[k * NP + off + j] + hj * (vel[k * NP + off + j] + hg[k]);
            f[9 + 3 * d + k] = nb[d] >= 0 ? (pj - xh[k]) - (rj[k] - rest[k]) : 0.0f;
        }
    }
    uint32_t packed[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int c0 = 2 * c, c1 = 2 * c + 1;
        const float lo = c0 < 27 ? (f[c0] - L.in_shift[c0]) * L.in_scale[c0] : 0.0f;
        float hi = c1 < 27 ? (f[c1] - L.in_shift[c1]) * L.in_scale[c1] : 0.0f;
        if (c1 == 31)
            hi = Ri.w > 0.0f ? 1.0f : 0.0f;   // flags a free particle
        const f32x2 pair = {lo, hi};
        const bf16x2 b = __builtin_convertvector(pair, bf16x2);
        __builtin_memcpy(&packed[c], &b, sizeof(uint32_t));
    }
    uint4 *dst = reinterpret_cast<uint4 *>(L.features + (size_t)(off + i) * 32);
#pragma unroll
    for (int q = 0; q < 4; ++q)
        dst[q] = make_uint4(packed[4 * q], packed[4 * q + 1], packed[4 * q + 2], packed[4 * q + 3]);
}

// Residual term of this lane's constraint in round r: ((C + alpha~ lambda) / rest)^2,
// with the same prefetch pipeline as run_round (no writes, no barrier).
__device__ __forceinline__ void eval_round(const float4 *xw, const RoundTables &t, int r,
                                           Record &slot, uint64_t active, uint64_t tets,
                                           const lambda_bank &bank, float alpha_d, float alpha_v,
                                           float &acc)
{
    const uint32_t w0 = slot.w0, w1 = slot.w1, w2 = slot.w2;
    if (((active >> r) & 1u) && (w0 & 0xffffu) != t.pad) {
        const float l = bank[r & 31];
        float q;
        if ((tets >> r) & 1u) {
            const float4 pa = lds_particle<1>(xw, w0 & 0xffffu), pb = lds_particle<1>(xw, w0 >> 16);
            const float4 pc = lds_particle<1>(xw, w1 & 0xffffu), pd = lds_particle<1>(xw, w1 >> 16);
            const float bax = pb.x - pa.x, bay = pb.y - pa.y, baz = pb.z - pa.z;
            const float cax = pc.x - pa.x, cay = pc.y - pa.y, caz = pc.z - pa.z;
            const float dax = pd.x - pa.x, day = pd.y - pa.y, daz = pd.z - pa.z;
            const float vol = (bax * (cay * daz - caz * day) + bay * (caz * dax - cax * daz) +
                               baz * (cax * day - cay * dax)) * kSixth;
            const float rest = __uint_as_float(w2);
            q = (vol - rest + alpha_v * l) / rest;
        } else {
            const float4 pa = lds_particle<1>(xw, w0 & 0xffffu), pb = lds_particle<1>(xw, w0 >> 16);
            const float dx = pa.x - pb.x, dy = pa.y - pb.y, dz = pa.z - pb.z;
            const float rest = __uint_as_float(w1);
            q = (sqrtf(dx * dx + dy * dy + dz * dz) - rest + alpha_d * l) / rest;
        }
        acc += q * q;
    }
    slot = fetch_record(t, r + 2);
}

// One substep of one environment from the predicted positions in L.xhat
// (start-of-substep positions in A.pos): min_iterations sweeps, the residual
// RMS, and the remaining sweeps up to max_iterations when it exceeds the
// threshold; then v = (x - x_prev) / h and the write-back.  GRASP: tool 0
// drags the particle A.grasp names (taken at the first substep of a step, as
// in xpbd_step_reg_kernel) after the contacts of every sweep.  BAR as in
// sweep_rounds.
template <int NB, bool GRASP, bool BAR>
__global__ void __launch_bounds__(1024) xpbd_substep_reg_kernel(StepArgs A, LearnedArgs L)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int env = blockIdx.x;
    const int tid = threadIdx.x;
    const int B = blockDim.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int num_waves = B >> 6;

    const EnvDev ed = A.envs[env];
    const MeshDev md = A.meshes[ed.mesh];
    const int V = md.num_vertices;
    const int R = md.num_rounds;
    const int R0 = R < 32 ? R : 32;
    const int tools = A.num_tools;
    const RegLdsLayout Lay = reg_lds_layout(V);
    float4 *xw = reinterpret_cast<float4 *>(smem + Lay.xw);
    float *vel = reinterpret_cast<float *>(smem + Lay.vel);      // [3][V] (byte flags at the end)
    float *prev = reinterpret_cast<float *>(smem + Lay.prev);    // [3][V]
    uint32_t *scratch = reinterpret_cast<uint32_t *>(smem + Lay.scratch);
    const XPBD_CONST float *compliance = (const XPBD_CONST float *)(uintptr_t)A.compliance;
    const float inv_h = A.inv_h;
    const float alpha_d = compliance[2 * env] * inv_h * inv_h;
    const float alpha_v = compliance[2 * env + 1] * inv_h * inv_h;
    const int NP = A.total_particles;
    const int off = ed.particle_offset;

    for (int i = tid; i < V; i += B) {
        const int sl = md.slot_of[i];
        xw[sl] = make_float4(L.xhat[off + i], L.xhat[NP + off + i], L.xhat[2 * NP + off + i],
                             md.inv_mass[i]);
        prev[sl] = A.pos[off + i];
        prev[V + sl] = A.pos[NP + off + i];
        prev[2 * V + sl] = A.pos[2 * NP + off + i];
    }
    if (tid == 0)
        xw[V] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);   // padding particle
    lambda_bank bank0 = 0.0f, bank1 = 0.0f;

    // sphere centres of this step and the contact candidates (bit 16 t + k: slot k B + tid)
    float3 tool0 = make_float3(0.f, 0.f, 0.f), tool1 = tool0;
    for (int t = 0; t < tools; ++t) {
        const XPBD_CONST float *c = (const XPBD_CONST float *)(uintptr_t)A.tool_pos +
                                    (((size_t)L.step * A.num_envs + env) * tools + t) * 3;
        const float3 ct = make_float3(c[0], c[1], c[2]);
        if (t == 0)
            tool0 = ct;
        else
            tool1 = ct;
    }
    __syncthreads();
    uint32_t cand = 0u;
    for (int k = 0, sl = tid; sl < V; ++k, sl += B) {
        const int i = md.id_of[sl];
        uint32_t bits = 0u;
        if (L.first_substep) {
            // start-of-step positions: the prediction has not moved them yet
            const float4 p0 = make_float4(prev[sl], prev[V + sl], prev[2 * V + sl], xw[sl].w);
            for (int t = 0; t < tools; ++t) {
                const float3 ct = t == 0 ? tool0 : tool1;
                const float reach2 = t == 0 ? A.tool_reach2[0] : A.tool_reach2[1];
                if (within_reach(p0, ct.x, ct.y, ct.z, reach2))
                    bits |= 1u << t;
            }
            L.cand[off + i] = (uint8_t)bits;
        } else {
            bits = L.cand[off + i];
        }
        for (int t = 0; t < tools; ++t)
            if ((bits >> t) & 1u)
                cand |= 1u << (16 * t + k);
    }
    const bool any_contact = block_any(cand != 0u, scratch + 32, wave, lane, num_waves);

    // grasping (Sec. III-A.2): the held particle's slot (uniform; -1 for none);
    // a closed grasper holding nothing takes, at the first substep of the
    // step, the free particle closest to the dragging point strictly within
    // reach on the start-of-step positions (key: squared distance bits, id)
    int held = -1, owner = -1;
    float3 drag = make_float3(0.f, 0.f, 0.f);
    if constexpr (GRASP) {
        int32_t *gs = reinterpret_cast<int32_t *>(smem + Lay.scratch + kRegScratchGrasp);
        uint64_t *part = reinterpret_cast<uint64_t *>(smem + Lay.scratch + kRegScratchGrasp + 16);
        drag = make_float3(tool0.x + A.grasp_offset[0], tool0.y + A.grasp_offset[1],
                           tool0.z + A.grasp_offset[2]);
        if (tid == 0) {
            const int h = A.grasp[env];
            const bool ok = h >= 0 && h < V && md.inv_mass[h] > 0.0f;
            gs[0] = ok ? (int)md.slot_of[h] : -1;
            gs[1] = h == -2 && L.first_substep ? 1 : 0;
        }
        __syncthreads();
        if (gs[1]) {
            uint64_t best = ~0ull;
            for (int i = tid; i < V; i += B) {
                const float4 p = make_float4(prev[i], prev[V + i], prev[2 * V + i], xw[i].w);
                const float dx = p.x - drag.x, dy = p.y - drag.y, dz = p.z - drag.z;
                const float d2 = dx * dx + dy * dy + dz * dz;
                if (p.w > 0.0f && d2 < A.grasp_radius2) {
                    const uint64_t key = (uint64_t)__float_as_uint(d2) << 32 | (uint32_t)md.id_of[i];
                    best = key < best ? key : best;
                }
            }
            best = wave_min_u64(best);
            if (lane == 0)
                part[wave] = best;
            __syncthreads();
            if (tid == 0) {
                uint64_t m = ~0ull;
                for (int w = 0; w < num_waves; ++w)
                    m = part[w] < m ? part[w] : m;
                const int id = m == ~0ull ? -1 : (int)(uint32_t)m;
                gs[0] = id >= 0 ? (int)md.slot_of[id] : -1;
                A.grasp[env] = id;
            }
            __syncthreads();
        }
        held = __builtin_amdgcn_readfirstlane(gs[0]);
        owner = held >= 0 ? held % B : -1;
    }

    // (padding particle as a byte offset: one environment per workgroup)
    const RoundTables tab = round_tables(md, B, tid, 16u * (uint32_t)V);
    const uint64_t active = A.meshes[ed.mesh].wave_active[__builtin_amdgcn_readfirstlane(wave)];
    const uint64_t tets = md.tet_mask, barriers = md.barrier_mask;
    Record slot_a = fetch_record(tab, 0);   // in this order (see xpbd_step_reg_kernel)
    __builtin_amdgcn_sched_barrier(0);
    Record slot_b = fetch_record(tab, 1);
    const float alpha_d1[1] = {alpha_d}, alpha_v1[1] = {alpha_v};

    auto sweep = [&]() {
        sweep_rounds<1, NB, BAR>(xw, tab, md.num_edge_rounds, R, slot_a, slot_b, active,
                                 barriers, bank0, bank1, alpha_d1, alpha_v1);
        if (any_contact || (GRASP && held >= 0)) {
            for (int t = 0; t < tools; ++t) {
                const float3 ct = t == 0 ? tool0 : tool1;
                const float rt = t == 0 ? A.tool_radius[0] : A.tool_radius[1];
                const float rt2 = t == 0 ? A.tool_radius2[0] : A.tool_radius2[1];
                for (int k = 0, i = tid; i < V; ++k, i += B)
                    if ((cand >> (16 * t + k)) & 1u)
                        project_contact(xw, i, ct.x, ct.y, ct.z, rt, rt2);
            }
            // the dragging constraint (k_s = 1): the held particle onto the
            // dragging point, by its slot's owner after its own contacts
            if (GRASP && tid == owner) {
                float4 p = xw[held];
                p.x = drag.x;
                p.y = drag.y;
                p.z = drag.z;
                xw[held] = p;
            }
            __syncthreads();
        }
    };

    int n_it = 0;
    // residual RMS of the environment (every thread gets it; the sweeps between
    // two evaluations hold barriers, and one follows the read)
    auto residual_rms = [&]() {
        float acc = 0.0f;
        for (int r = 0; r < R0; r += 2) {
            eval_round(xw, tab, r, slot_a, active, tets, bank0, alpha_d, alpha_v, acc);
            eval_round(xw, tab, r + 1, slot_b, active, tets, bank0, alpha_d, alpha_v, acc);
        }
        if constexpr (NB > 1)
            for (int r = 32; r < R; r += 2) {
                eval_round(xw, tab, r, slot_a, active, tets, bank1, alpha_d, alpha_v, acc);
                eval_round(xw, tab, r + 1, slot_b, active, tets, bank1, alpha_d, alpha_v, acc);
            }
        acc = wave_sum(acc);
        if (lane == 0)
            scratch[64 + wave] = __float_as_uint(acc);
        __syncthreads();
        float total = 0.0f;
        for (int w = 0; w < num_waves; ++w)
            total += __uint_as_float(scratch[64 + w]);
        __syncthreads();
        const int n_con = md.num_edges + md.num_tets;
        return n_con > 0 ? sqrtf(total / (float)n_con) : 0.0f;
    };
    // min_iterations sweeps; with a stall ratio the residual is taken before the
    // last of them too, and the further sweeps run only if that sweep lowered
    // it to at most stall_ratio times that value
    const bool check = L.max_iterations > L.min_iterations;
    const bool stall_check = check && L.stall_ratio > 0.0f && L.min_iterations >= 1;
    float before = 0.0f;
    for (; n_it < L.min_iterations; ++n_it) {
        if (stall_check && n_it == L.min_iterations - 1)
            before = residual_rms();
        sweep();
    }
    float final_rms = 0.0f;
    bool measured = false;   // final_rms holds the residual after the last sweep
    if (check) {
        const float rms = residual_rms();
        final_rms = rms;
        measured = true;
        bool go_on = rms > L.threshold;
        if (go_on && stall_check)
            go_on = rms <= L.stall_ratio * before;
        if (go_on) {
            for (; n_it < L.max_iterations; ++n_it)
                sweep();
            measured = false;
        }
    }
    if (L.residuals && !measured)
        final_rms = residual_rms();

    // velocity update and write-back (structure of arrays); slot_of[i] belongs
    // to other threads' sweeps, hence the barrier
    __syncthreads();
    int bad = 0;
    for (int i = tid; i < V; i += B) {
        const int sl = md.slot_of[i];
        const float4 p = xw[sl];
        const float vx = (p.x - prev[sl]) * inv_h, vy = (p.y - prev[V + sl]) * inv_h,
                    vz = (p.z - prev[2 * V + sl]) * inv_h;
        if (L.record_targets) {
            const bool free_p = p.w > 0.0f;
            float *t = L.record_targets + (size_t)(off + i) * 4;
            t[0] = free_p ? ((p.x - L.xhat[off + i]) - L.out_shift[0]) / L.out_scale[0] : 0.0f;
            t[1] = free_p ? ((p.y - L.xhat[NP + off + i]) - L.out_shift[1]) / L.out_scale[1] : 0.0f;
            t[2] = free_p ? ((p.z - L.xhat[2 * NP + off + i]) - L.out_shift[2]) / L.out_scale[2]
                          : 0.0f;
            t[3] = 0.0f;
        }
        A.pos[off + i] = p.x;
        A.pos[NP + off + i] = p.y;
        A.pos[2 * NP + off + i] = p.z;
        A.vel[off + i] = vx;
        A.vel[NP + off + i] = vy;
        A.vel[2 * NP + off + i] = vz;
        bad |= !(isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(vx) &&
                 isfinite(vy) && isfinite(vz));
    }
    bad = block_any(bad != 0, scratch + 48, wave, lane, num_waves);
    if (tid == 0) {
        if (bad)
            A.nonfinite[env] = 1;
        if (L.iterations)
            L.iterations[env] = n_it;
        if (L.residuals)
            L.residuals[env] = final_rms;
    }

    // the prediction and features of the next substep from the state just
    // written (the same arithmetic as learned_predict_kernel): x_hat into the
    // start-of-substep slots first, then every particle reads its neighbours'
    if (L.next_features) {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        typedef float f32x4 __attribute__((ext_vector_type(4)));
        const XPBD_GLOBAL f32x4 *rest4 = (const XPBD_GLOBAL f32x4 *)(uintptr_t)md.rest4;
        const XPBD_GLOBAL int32_t *nbr = (const XPBD_GLOBAL int32_t *)(uintptr_t)md.nbr;
        const float h = A.h;
        const float hg[3] = {h * A.gravity[0], h * A.gravity[1], h * A.gravity[2]};
        for (int i = tid; i < V; i += B) {
            const int sl = md.slot_of[i];
            const float4 p = xw[sl];
            const float x[3] = {p.x, p.y, p.z};
            const float hs = p.w > 0.0f ? h : 0.0f;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float v = (x[k] - prev[k * V + sl]) * inv_h;
                prev[k * V + sl] = x[k] + hs * (v + hg[k]);
            }
        }
        __syncthreads();
        for (int i = tid; i < V; i += B) {
            const int sl = md.slot_of[i];
            const float4 p = xw[sl];
            const f32x4 Ri = rest4[i];
            const float x[3] = {p.x, p.y, p.z}, rest[3] = {Ri.x, Ri.y, Ri.z};
            float xh[3], f[32];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                xh[k] = prev[k * V + sl];
                L.xhat[k * NP + off + i] = xh[k];
                f[k] = xh[k] - x[k];
                f[3 + k] = A.vel[k * NP + off + i];
                f[6 + k] = xh[k] - rest[k];
            }
            int nb[6];
#pragma unroll
            for (int d = 0; d < 6; ++d)
                nb[d] = nbr[6 * i + d];
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const int j = nb[d] >= 0 ? nb[d] : i;
                const int sj = md.slot_of[j];
                const f32x4 Rj = rest4[j];
                const float rj[3] = {Rj.x, Rj.y, Rj.z};
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    f[9 + 3 * d + k] =
                        nb[d] >= 0 ? (prev[k * V + sj] - xh[k]) - (rj[k] - rest[k]) : 0.0f;
            }
            uint32_t packed[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int c0 = 2 * c, c1 = 2 * c + 1;
                const float lo = c0 < 27 ? (f[c0] - L.in_shift[c0]) * L.in_scale[c0] : 0.0f;
                float hi = c1 < 27 ? (f[c1] - L.in_shift[c1]) * L.in_scale[c1] : 0.0f;
                if (c1 == 31)
                    hi = Ri.w > 0.0f ? 1.0f : 0.0f;
                const f32x2 pair = {lo, hi};
                const bf16x2 b = __builtin_convertvector(pair, bf16x2);
                __builtin_memcpy(&packed[c], &b, sizeof(uint32_t));
            }
            uint4 *dst = reinterpret_cast<uint4 *>(L.next_features + (size_t)(off + i) * 32);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                dst[q] = make_uint4(packed[4 * q], packed[4 * q + 1], packed[4 * q + 2],
                                    packed[4 * q + 3]);
        }
    }

    // contact candidates of the step as ascending mesh ids (first substep only)
    if (L.first_substep) {
        uint8_t *flag_of = reinterpret_cast<uint8_t *>(vel);
        const int kmax = (V + B - 1) / B;
        for (int t = 0; t < tools; ++t) {
            for (int i = tid; i < V; i += B)
                flag_of[i] = 0;
            __syncthreads();
            for (int k = 0, sl = tid; sl < V; ++k, sl += B)
                if ((cand >> (16 * t + k)) & 1u)
                    flag_of[md.id_of[sl]] = 1;
            __syncthreads();
            int32_t *list = A.contacts + (size_t)t * NP + off;
            int base = 0;
            for (int k = 0; k < kmax; ++k) {
                const int i = k * B + tid;
                const bool flag = i < V && flag_of[i];
                const uint64_t mask = __ballot(flag);
                if (lane == 0)
                    scratch[wave] = (uint32_t)__popcll(mask);
                __syncthreads();
                int before = 0, total = 0;
                for (int w = 0; w < num_waves; ++w) {
                    const int n = (int)scratch[w];
                    before += w < wave ? n : 0;
                    total += n;
                }
                if (flag)
                    list[base + before + __popcll(mask & __lanemask_lt())] = i;
                base += total;
                __syncthreads();
            }
            for (int n = base + tid; n < V; n += B)
                list[n] = -1;
            if (tid == 0)
                A.contact_counts[env * tools + t] = base;
        }
    }
    if (A.lambda_out) {
        float *out = A.lambda_out + ed.lambda_offset;
        for (int r = 0; r < R0; ++r) {
            const int id = md.rr_id[r * B + tid];
            if (id >= 0)
                out[id & 0xffffff] = bank0[r & 31];
        }
        if constexpr (NB > 1)
            for (int r = 32; r < R; ++r) {
                const int id = md.rr_id[r * B + tid];
                if (id >= 0)
                    out[id & 0xffffff] = bank1[r & 31];
            }
    }
}

// Constraint residual (C + alpha~ lambda) / rest of every kept constraint of an
// environment, from its written-back positions and stored multipliers
// (constraint order), reduced to (RMS, max |r|).  One workgroup per environment.
__global__ void __launch_bounds__(256) residual_kernel(StepArgs A)
{
    __shared__ float part[2][4];
    const int env = blockIdx.x;
    const int tid = threadIdx.x;
    const EnvDev ed = A.envs[env];
    const MeshDev md = A.meshes[ed.mesh];
    const int E = md.num_edges, T = md.num_tets;
    const int NP = A.total_particles;
    const int off = ed.particle_offset;
    const float *px = A.pos + off, *py = A.pos + NP + off, *pz = A.pos + 2 * NP + off;
    const float *lam = A.lambda_out + ed.lambda_offset;
    const float inv_h2 = A.inv_h * A.inv_h;
    const float alpha_d = A.compliance[2 * env] * inv_h2, alpha_v = A.compliance[2 * env + 1] * inv_h2;
    float sum = 0.0f, big = 0.0f;
    for (int j = tid; j < E; j += blockDim.x) {
        const uint32_t e = md.edge_pair[j];
        const int a = (int)(e & 0xffffu), b = (int)(e >> 16);
        const float dx = px[a] - px[b], dy = py[a] - py[b], dz = pz[a] - pz[b];
        const float rest = md.edge_rest[j];
        const float r = (sqrtf(dx * dx + dy * dy + dz * dz) - rest + alpha_d * lam[md.edge_id[j]]) / rest;
        sum += r * r;
        big = fmaxf(big, fabsf(r));
    }
    for (int j = tid; j < T; j += blockDim.x) {
        const uint2 q = md.tet_quad[j];
        const int a = (int)(q.x & 0xffffu), b = (int)(q.x >> 16);
        const int c = (int)(q.y & 0xffffu), d = (int)(q.y >> 16);
        const float bax = px[b] - px[a], bay = py[b] - py[a], baz = pz[b] - pz[a];
        const float cax = px[c] - px[a], cay = py[c] - py[a], caz = pz[c] - pz[a];
        const float dax = px[d] - px[a], day = py[d] - py[a], daz = pz[d] - pz[a];
        const float vol = (bax * (cay * daz - caz * day) + bay * (caz * dax - cax * daz) +
                           baz * (cax * day - cay * dax)) * kSixth;
        const float rest = md.tet_rest[j];
        const float r = (vol - rest + alpha_v * lam[E + md.tet_id[j]]) / rest;
        sum += r * r;
        big = fmaxf(big, fabsf(r));
    }
    sum = wave_sum(sum);
    big = wave_max(big);
    if ((tid & 63) == 0) {
        part[0][tid >> 6] = sum;
        part[1][tid >> 6] = big;
    }
    __syncthreads();
    if (tid == 0) {
        float s = 0.0f, m = 0.0f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            s += part[0][w];
            m = fmaxf(m, part[1][w]);
        }
        A.residual[2 * env] = E + T > 0 ? sqrtf(s / (float)(E + T)) : 0.0f;
        A.residual[2 * env + 1] = m;
    }
}

__global__ void soa_to_aos_kernel(const float *__restrict__ soa, float *__restrict__ aos, int32_t n)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) {
        aos[3 * (size_t)i] = soa[i];
        aos[3 * (size_t)i + 1] = soa[(size_t)n + i];
        aos[3 * (size_t)i + 2] = soa[2 * (size_t)n + i];
    }
}

__global__ void aos_to_soa_kernel(const float *__restrict__ aos, float *__restrict__ soa, int32_t n)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) {
        soa[i] = aos[3 * (size_t)i];
        soa[(size_t)n + i] = aos[3 * (size_t)i + 1];
        soa[2 * (size_t)n + i] = aos[3 * (size_t)i + 2];
    }
}

template <int PPT, bool STAGE, bool RESIDUAL, bool JACOBI = false>
hipError_t launch_variant(const StepArgs &args, int block, uint32_t lds_bytes, hipStream_t stream)
{
    auto kernel = xpbd_step_lds_kernel<PPT, STAGE, RESIDUAL, JACOBI>;
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds_bytes);
    if (err != hipSuccess)
        return err;
    hipLaunchKernelGGL(kernel, dim3((unsigned)args.num_envs), dim3((unsigned)block), lds_bytes,
                       stream, args);
    return hipGetLastError();
}

template <int PPT>
hipError_t launch_ppt(const StepArgs &args, int block, bool jacobi, bool stage, uint32_t lds,
                      bool resid, hipStream_t s)
{
    if (jacobi)   // topology read from global memory
        return resid ? launch_variant<PPT, false, true, true>(args, block, lds, s)
                     : launch_variant<PPT, false, false, true>(args, block, lds, s);
    if (stage)
        return resid ? launch_variant<PPT, true, true>(args, block, lds, s)
                     : launch_variant<PPT, true, false>(args, block, lds, s);
    return resid ? launch_variant<PPT, false, true>(args, block, lds, s)
                 : launch_variant<PPT, false, false>(args, block, lds, s);
}

using RegKernel = void (*)(StepArgs);

// The register kernel a launch with these arguments runs: the grasping and
// capsule code only in the launches that use them (they cost registers).
// nullptr: capsule tools with several environments per workgroup.
template <int NB, int EG>
RegKernel reg_kernel(const StepArgs &args)
{
    if (args.tool_shape == 1) {   // XPBD_TOOL_CAPSULE
        if constexpr (EG == 1)
            return xpbd_step_reg_kernel_capsules<NB>;
        else
            return nullptr;
    }
    return args.round_barriers
               ? (args.grasp ? xpbd_step_reg_kernel<NB, EG, kRegGrasp, true>
                             : xpbd_step_reg_kernel<NB, EG, kRegSpheres, true>)
               : (args.grasp ? xpbd_step_reg_kernel<NB, EG, kRegGrasp, false>
                             : xpbd_step_reg_kernel<NB, EG, kRegSpheres, false>);
}

template <int EG>
RegKernel reg_kernel_banks(const StepArgs &args, int lambda_banks)
{
    return lambda_banks == 1 ? reg_kernel<1, EG>(args)
           : lambda_banks == 2 ? reg_kernel<2, EG>(args)
                               : nullptr;
}

RegKernel reg_kernel_for(const StepArgs &args, int lambda_banks, int envs_per_group)
{
    return envs_per_group == 1   ? reg_kernel_banks<1>(args, lambda_banks)
           : envs_per_group == 2 ? reg_kernel_banks<2>(args, lambda_banks)
                                 : nullptr;
}

template <int NB, int EG>
hipError_t launch_reg_variant(const StepArgs &args, int block, uint32_t lds_bytes, hipStream_t stream)
{
    const RegKernel kernel = reg_kernel<NB, EG>(args);
    if (!kernel || (args.tool_shape == 1 && block > kMaxCapsuleBlock))
        return hipErrorInvalidValue;
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds_bytes);
    if (err != hipSuccess)
        return err;
    hipLaunchKernelGGL(kernel, dim3((unsigned)args.num_groups), dim3((unsigned)block), lds_bytes,
                       stream, args);
    return hipGetLastError();
}

template <int EG>
hipError_t launch_reg_groups(const StepArgs &args, int block, int lambda_banks, uint32_t lds_bytes,
                             hipStream_t stream)
{
    return lambda_banks == 1   ? launch_reg_variant<1, EG>(args, block, lds_bytes, stream)
           : lambda_banks == 2 ? launch_reg_variant<2, EG>(args, block, lds_bytes, stream)
                               : hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_step(const StepArgs &args, int block, int particles_per_thread, bool jacobi,
                       bool stage_topology, uint32_t lds_bytes, bool want_residual,
                       hipStream_t stream)
{
    const bool st = stage_topology && !jacobi;
    switch (particles_per_thread) {
    case 1: return launch_ppt<1>(args, block, jacobi, st, lds_bytes, want_residual, stream);
    case 2: return launch_ppt<2>(args, block, jacobi, st, lds_bytes, want_residual, stream);
    case 4: return launch_ppt<4>(args, block, jacobi, st, lds_bytes, want_residual, stream);
    case 8: return launch_ppt<8>(args, block, jacobi, st, lds_bytes, want_residual, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_reg(const StepArgs &args, int block, int lambda_banks, int envs_per_group,
                           uint32_t lds_bytes, bool want_residual, hipStream_t stream)
{
    hipError_t err =
        envs_per_group == 1   ? launch_reg_groups<1>(args, block, lambda_banks, lds_bytes, stream)
        : envs_per_group == 2 ? launch_reg_groups<2>(args, block, lambda_banks, lds_bytes, stream)
                              : hipErrorInvalidValue;
    if (err != hipSuccess || !want_residual)
        return err;
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)args.num_envs), dim3(256), 0, stream, args);
    return hipGetLastError();
}

hipError_t step_reg_occupancy(const StepArgs &args, int block, int lambda_banks,
                              int envs_per_group, uint32_t lds_bytes, int *per_cu)
{
    const RegKernel kernel = reg_kernel_for(args, lambda_banks, envs_per_group);
    if (!kernel || !per_cu)
        return hipErrorInvalidValue;
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds_bytes);
    if (err != hipSuccess)
        return err;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        per_cu, reinterpret_cast<const void *>(kernel), block, (size_t)lds_bytes);
}

hipError_t launch_residual(const StepArgs &args, hipStream_t stream)
{
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)args.num_envs), dim3(256), 0, stream, args);
    return hipGetLastError();
}

hipError_t launch_learned_predict(const StepArgs &args, const LearnedArgs &largs, hipStream_t stream)
{
    hipLaunchKernelGGL(learned_predict_kernel,
                       dim3((unsigned)((largs.max_vertices + 255) / 256), (unsigned)args.num_envs),
                       dim3(256), 0, stream, args, largs);
    return hipGetLastError();
}

template <int NB>
hipError_t launch_substep_variant(const StepArgs &args, const LearnedArgs &largs, int block,
                                  uint32_t lds_bytes, hipStream_t stream)
{
    auto kernel = args.round_barriers
                      ? (args.grasp ? xpbd_substep_reg_kernel<NB, true, true>
                                    : xpbd_substep_reg_kernel<NB, false, true>)
                      : (args.grasp ? xpbd_substep_reg_kernel<NB, true, false>
                                    : xpbd_substep_reg_kernel<NB, false, false>);
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds_bytes);
    if (err != hipSuccess)
        return err;
    hipLaunchKernelGGL(kernel, dim3((unsigned)args.num_envs), dim3((unsigned)block), lds_bytes,
                       stream, args, largs);
    return hipGetLastError();
}

hipError_t launch_substep_reg(const StepArgs &args, const LearnedArgs &largs, int block,
                              int lambda_banks, uint32_t lds_bytes, bool want_residual,
                              hipStream_t stream)
{
    hipError_t err = lambda_banks == 1 ? launch_substep_variant<1>(args, largs, block, lds_bytes, stream)
                     : lambda_banks == 2 ? launch_substep_variant<2>(args, largs, block, lds_bytes, stream)
                                         : hipErrorInvalidValue;
    if (err != hipSuccess || !want_residual)
        return err;
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)args.num_envs), dim3(256), 0, stream, args);
    return hipGetLastError();
}

hipError_t launch_soa_to_aos(const float *soa, float *aos, int32_t n, hipStream_t stream)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(soa_to_aos_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       soa, aos, n);
    return hipGetLastError();
}

hipError_t launch_aos_to_soa(const float *aos, float *soa, int32_t n, hipStream_t stream)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(aos_to_soa_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       aos, soa, n);
    return hipGetLastError();
}

}  // namespace xpbd
