// The RL-style step's observation, policy and tool-motion pass (gfx950): one
// wave per 32 environments (two 16-environment tiles that share every weight
// fragment the wave loads).  The wave first writes the environments'
// observations (one observation per lane and environment, coalesced) to LDS
// and to the caller's buffer, then runs the 64 -> 256 -> 256 -> 7 policy on
// the matrix cores (v_mfma_f32_16x16x32_bf16, bfloat16 operands, float32
// accumulation), and finally moves the tools and sets the grasp command.
//
// The products are computed transposed (units x environments): the weights
// are the A operand, read as pre-cut fragments straight from memory (168 KB
// in all, shared by every wave through the caches), the activations the B
// operand, kept in registers.  A layer's result fragment (lane l: environment
// l % 16, units 4 (l / 16) .. + 3 of each 16-unit tile) is the next layer's B
// fragment once two unit tiles are packed together, because the next layer's
// weights were cut with their inputs in that order.
#include <hip/hip_runtime.h>

#include "rl_device.h"

namespace xpbd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

#define GLOBAL __attribute__((address_space(1)))

constexpr int kPitch = 68;   // floats per LDS observation row (16-byte reads of 16 rows hit distinct banks)

// Two floats rounded to bfloat16 (nearest, ties to even), the first in the low half.
__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi)
{
    const f32x2 v = {lo, hi};
    const bf16x2 b = __builtin_convertvector(v, bf16x2);
    uint32_t u;
    __builtin_memcpy(&u, &b, sizeof u);
    return u;
}

// relu of a bfloat16 pair (a negative value is a negative int16; rounding
// keeps the sign, so relu and rounding commute).
__device__ __forceinline__ uint32_t relu_bf16_pair(uint32_t u)
{
    typedef short s16x2 __attribute__((ext_vector_type(2)));
    s16x2 v;
    __builtin_memcpy(&v, &u, sizeof v);
    const s16x2 z = {0, 0};
    v = __builtin_elementwise_max(v, z);
    __builtin_memcpy(&u, &v, sizeof u);
    return u;
}

// bfloat16 relu of the result fragments of unit tiles 2 kb and 2 kb + 1: the
// B fragment of k block kb of the next layer.
__device__ __forceinline__ bf16x8 relu_pack(f32x4 lo, f32x4 hi)
{
    uint32_t w[4];
    w[0] = relu_bf16_pair(bf16_pair(lo[0], lo[1]));
    w[1] = relu_bf16_pair(bf16_pair(lo[2], lo[3]));
    w[2] = relu_bf16_pair(bf16_pair(hi[0], hi[1]));
    w[3] = relu_bf16_pair(bf16_pair(hi[2], hi[3]));
    bf16x8 r;
    __builtin_memcpy(&r, w, sizeof r);
    return r;
}

// Eight floats from LDS rounded to bfloat16: a B fragment of the inputs.
__device__ __forceinline__ bf16x8 pack_inputs(const float *p)
{
    const f32x4 a = *reinterpret_cast<const f32x4 *>(p);
    const f32x4 b = *reinterpret_cast<const f32x4 *>(p + 4);
    uint32_t w[4] = {bf16_pair(a[0], a[1]), bf16_pair(a[2], a[3]), bf16_pair(b[0], b[1]),
                     bf16_pair(b[2], b[3])};
    bf16x8 r;
    __builtin_memcpy(&r, w, sizeof r);
    return r;
}

__device__ __forceinline__ bf16x8 fragment(const uint16_t *base, int index)
{
    const u32x4 v = reinterpret_cast<const GLOBAL u32x4 *>((uintptr_t)base)[index];
    bf16x8 r;
    __builtin_memcpy(&r, &v, sizeof r);
    return r;
}

// Bias fragment of a unit tile from the LDS copy: lane group g holds units
// 4 g .. 4 g + 3 of the tile.
__device__ __forceinline__ f32x4 bias(const float *b, int tile, int g)
{
    return *reinterpret_cast<const f32x4 *>(b + 16 * tile + 4 * g);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr int kTiles = 2;                            // 16-environment tiles per wave
constexpr int kWaveEnvs = kRlEnvsPerWave * kTiles;   // environments per wave

// One observation of one environment, for lane l (observation l): the value
// and the grasp word (lane 9) are loaded first for all of the wave's
// environments, then combined, so that the gathers are in flight together.
struct ObsLoad {
    float v;        // loaded value (tool, target or particle coordinate), or grasp bits
    float rest;     // the tracked particle's rest coordinate (lanes >= 10)
};

// Grid: ceil(N / 32) workgroups of one wave; workgroup w takes environments
// 32 w .. 32 w + 31 as two tiles of 16.
__global__ void __launch_bounds__(64) rl_policy_kernel(RlArgs R, PolicyDev P)
{
    __shared__ __align__(16) float obs[kWaveEnvs * kPitch];
    __shared__ float act[kWaveEnvs * 8];
    __shared__ int held[kWaveEnvs];
    // the biases (b1, b2, b3 with zero padding: 528 floats) in LDS, so that
    // reading them never waits on the weight-fragment loads in flight
    __shared__ __align__(16) float bs[2 * kRlHidden + 16];
    const int l = threadIdx.x;
    {
        const GLOBAL f32x4 *src1 = reinterpret_cast<const GLOBAL f32x4 *>((uintptr_t)P.b1);
        const GLOBAL f32x4 *src2 = reinterpret_cast<const GLOBAL f32x4 *>((uintptr_t)P.b2);
        const GLOBAL f32x4 *src3 = reinterpret_cast<const GLOBAL f32x4 *>((uintptr_t)P.b3);
        const f32x4 v1 = src1[l], v2 = src2[l];
        const f32x4 v3 = l < 4 ? src3[l] : f32x4{0.f, 0.f, 0.f, 0.f};
        *reinterpret_cast<f32x4 *>(&bs[4 * l]) = v1;
        *reinterpret_cast<f32x4 *>(&bs[kRlHidden + 4 * l]) = v2;
        if (l < 4)
            *reinterpret_cast<f32x4 *>(&bs[2 * kRlHidden + 4 * l]) = v3;
    }
    const int base = blockIdx.x * kWaveEnvs;
    const int N = R.num_envs;
    const int NP = R.total_particles;
    const float s = R.obs_scale;

    // lane l computes observation l of every environment of the wave
    const int c = l < 10 ? l % 3 : (l - 10) % 3;         // axis
    const int j = l < 10 ? -1 : (l - 10) / 3;            // tracked particle
    int tp = 0;
#pragma unroll
    for (int q = 0; q < kRlTracked; ++q)
        tp = j == q ? R.tracked[q] : tp;
    const float origin = c == 0 ? R.obs_origin[0] : (c == 1 ? R.obs_origin[1] : R.obs_origin[2]);
    // the environments' particle offsets and mesh tables: one lane per
    // environment (out-of-range environments repeat the last one and are
    // not written), shared through LDS
    __shared__ int env_off[kWaveEnvs], env_nv[kWaveEnvs];
    __shared__ const float *env_rest[kWaveEnvs];
    __shared__ const float *env_w[kWaveEnvs];
    if (l < kWaveEnvs) {
        const EnvDev ed = R.envs[min(base + l, N - 1)];
        const MeshDev &md = R.meshes[ed.mesh];
        env_off[l] = ed.particle_offset;
        env_nv[l] = md.num_vertices;
        env_rest[l] = md.rest_pos;
        env_w[l] = md.inv_mass;
    }
    __syncthreads();
    // every gather of the wave's environments first, then the arithmetic
    ObsLoad ld[kWaveEnvs];
#pragma unroll
    for (int r = 0; r < kWaveEnvs; ++r) {
        const int e = min(base + r, N - 1);
        const float *src = l < 6    ? R.tool_pos + (size_t)e * 6 + l
                           : l < 9  ? R.target + (size_t)e * 3 + c
                           : l == 9 ? reinterpret_cast<const float *>(R.grasp + e)
                                    : R.pos + (size_t)c * NP + env_off[r] + tp;
        ld[r].v = *reinterpret_cast<const GLOBAL float *>((uintptr_t)src);
        ld[r].rest = l >= 10 ? reinterpret_cast<const GLOBAL float *>(
                                   (uintptr_t)env_rest[r])[3 * tp + c]
                             : origin;
    }
    // the grasp flag's inverse masses (lane 9), all gathered before any store
    // (branch-free: every lane loads, other lanes and ids out of range read
    // particle 0, so the 32 loads are in flight together)
    float wh[kWaveEnvs];
#pragma unroll
    for (int r = 0; r < kWaveEnvs; ++r) {
        const int h = __float_as_int(ld[r].v);
        const bool in = l == 9 && h >= 0 && h < env_nv[r];
        const float w = reinterpret_cast<const GLOBAL float *>((uintptr_t)env_w[r])[in ? h : 0];
        wh[r] = in ? w : 0.0f;
    }
    // the observations in registers, then every store
    float vv[kWaveEnvs];
#pragma unroll
    for (int r = 0; r < kWaveEnvs; ++r) {
        const int e = base + r;
        float v = (ld[r].v - ld[r].rest) * s;
        if (l == 9) {
            const int h = __float_as_int(ld[r].v);
            const bool ok = wh[r] > 0.0f;
            v = ok ? 1.0f : 0.0f;
            held[r] = ok && e < N ? h : -1;
        }
        vv[r] = e < N ? v : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < kWaveEnvs; ++r) {
        const int e = base + r;
        if (e < N && R.obs)
            R.obs[(size_t)e * kRlObs + l] = vv[r];
        obs[r * kPitch + l] = vv[r];
    }
    __syncthreads();

    const int n = l & 15, g = l >> 4;
    bf16x8 x0[kTiles], x1[kTiles];
#pragma unroll
    for (int t = 0; t < kTiles; ++t) {
        x0[t] = pack_inputs(&obs[(16 * t + n) * kPitch + 8 * g]);
        x1[t] = pack_inputs(&obs[(16 * t + n) * kPitch + 32 + 8 * g]);
    }
    // The three layers as one stream of 168 weight fragments (W1: 16 unit
    // tiles x 2 k blocks, W2: 16 x 8, W3: 8), each serving both environment
    // tiles.  Fragment f + kDepth is loaded while fragment f is used, from a
    // ring of kDepth registers, so that kDepth loads are in flight: with one
    // or two waves per CU nothing else hides their latency.
    constexpr int kF1 = 32, kF2 = 128, kF3 = 8, kF = kF1 + kF2 + kF3, kDepth = 16;
    auto load = [&](int f) -> bf16x8 {
        return f < kF1 ? fragment(P.w1, f * 64 + l)
               : f < kF1 + kF2 ? fragment(P.w2, (f - kF1) * 64 + l)
                               : fragment(P.w3, (f - kF1 - kF2) * 64 + l);
    };
    bf16x8 ring[kDepth];
#pragma unroll
    for (int f = 0; f < kDepth; ++f)
        ring[f] = load(f);
    bf16x8 h1[kTiles][8], h2[kTiles][8];
    f32x4 acc[kTiles][2], y[kTiles];
#pragma clang loop unroll(full)
    for (int f = 0; f < kF; ++f) {
        const bf16x8 a = ring[f % kDepth];
        if (f + kDepth < kF)
            ring[f % kDepth] = load(f + kDepth);
        if (f < kF1) {
            // layer 1: unit tile u = f / 2, k block f % 2 (the two halves of the input)
            const int u = f / 2, kb = f % 2;
            if (kb == 0) {
                const f32x4 b = bias(bs, u, g);
#pragma unroll
                for (int t = 0; t < kTiles; ++t)
                    acc[t][u % 2] = mfma(a, x0[t], b);
            } else {
#pragma unroll
                for (int t = 0; t < kTiles; ++t)
                    acc[t][u % 2] = mfma(a, x1[t], acc[t][u % 2]);
                if (u % 2 == 1) {
#pragma unroll
                    for (int t = 0; t < kTiles; ++t)
                        h1[t][u / 2] = relu_pack(acc[t][0], acc[t][1]);
                }
            }
        } else if (f < kF1 + kF2) {
            // layer 2: unit tile u, k block kb
            const int u = (f - kF1) / 8, kb = (f - kF1) % 8;
            if (kb == 0) {
                const f32x4 b = bias(bs + kRlHidden, u, g);
#pragma unroll
                for (int t = 0; t < kTiles; ++t)
                    acc[t][u % 2] = b;
            }
#pragma unroll
            for (int t = 0; t < kTiles; ++t)
                acc[t][u % 2] = mfma(a, h1[t][kb], acc[t][u % 2]);
            if (kb == 7 && u % 2 == 1) {
#pragma unroll
                for (int t = 0; t < kTiles; ++t)
                    h2[t][u / 2] = relu_pack(acc[t][0], acc[t][1]);
            }
        } else {
            // layer 3: one unit tile (actions 0..6, units 7..15 zero), k block kb
            const int kb = f - kF1 - kF2;
            if (kb == 0) {
                const f32x4 b = bias(bs + 2 * kRlHidden, 0, g);
#pragma unroll
                for (int t = 0; t < kTiles; ++t)
                    y[t] = b;
            }
#pragma unroll
            for (int t = 0; t < kTiles; ++t)
                y[t] = mfma(a, h2[t][kb], y[t]);
        }
    }
    // lane (n, g) holds actions 4 g .. 4 g + 3 of environment 16 t + n of the wave
    if (g < 2) {
#pragma unroll
        for (int t = 0; t < kTiles; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                act[(16 * t + n) * 8 + 4 * g + q] = y[t][q];
    }
    __syncthreads();

    if (l < kWaveEnvs && base + l < N) {
        const int e = base + l;
        float a[kRlActions];
#pragma unroll
        for (int o = 0; o < kRlActions; ++o)
            a[o] = act[l * 8 + o];
        if (R.actions) {
#pragma unroll
            for (int o = 0; o < kRlActions; ++o)
                R.actions[(size_t)e * kRlActions + o] = a[o];
        }
        // tool motion: clamped velocity times the step, then the workspace box
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float vel = fminf(fmaxf(a[3 * t + k], -1.0f), 1.0f) * R.max_speed;
                float p = R.tool_pos[(size_t)e * 6 + 3 * t + k] + vel * R.dt;
                p = fminf(fmaxf(p, R.box_lo[k]), R.box_hi[k]);
                R.tool_pos[(size_t)e * 6 + 3 * t + k] = p;
            }
        // grasp command: open releases, closed keeps a held particle or asks
        // the step to take one (-2)
        const int h = held[l];
        R.grasp[e] = !(a[6] > 0.0f) ? -1 : (h >= 0 ? h : -2);
    }
}

}  // namespace

hipError_t launch_rl_policy(const RlArgs &args, const PolicyDev &policy, hipStream_t stream)
{
    if (args.num_envs <= 0)
        return hipSuccess;
    const int grid = (args.num_envs + kWaveEnvs - 1) / kWaveEnvs;
    hipLaunchKernelGGL(rl_policy_kernel, dim3((unsigned)grid), dim3(64), 0, stream, args, policy);
    return hipGetLastError();
}

}  // namespace xpbd
