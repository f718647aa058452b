// The RL-style step's observation, policy and tool-motion pass (gfx950): one
// wave per 16 environments.  The wave first writes the environments'
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

__device__ __forceinline__ f32x4 bias(const float *b, int tile, int g)
{
    return reinterpret_cast<const GLOBAL f32x4 *>((uintptr_t)b)[4 * tile + g];
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Grid: ceil(N / 16) workgroups of one wave; workgroup w takes environments
// 16 w .. 16 w + 15.
__global__ void __launch_bounds__(64) rl_policy_kernel(RlArgs R, PolicyDev P)
{
    __shared__ __align__(16) float obs[kRlEnvsPerWave * kPitch];
    __shared__ float act[kRlEnvsPerWave * 8];
    __shared__ int held[kRlEnvsPerWave];
    const int l = threadIdx.x;
    const int base = blockIdx.x * kRlEnvsPerWave;
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
    for (int r = 0; r < kRlEnvsPerWave; ++r) {
        const int e = base + r;
        float v = 0.0f;
        if (e < R.num_envs) {
            const EnvDev ed = R.envs[e];
            const MeshDev &md = R.meshes[ed.mesh];
            if (l < 6) {
                v = (R.tool_pos[(size_t)e * 6 + l] - origin) * s;
            } else if (l < 9) {
                v = (R.target[(size_t)e * 3 + c] - origin) * s;
            } else if (l == 9) {
                const int h = R.grasp[e];
                const bool ok = h >= 0 && h < md.num_vertices && md.inv_mass[h] > 0.0f;
                v = ok ? 1.0f : 0.0f;
                held[r] = ok ? h : -1;
            } else {
                v = (R.pos[(size_t)c * NP + ed.particle_offset + tp] - md.rest_pos[3 * tp + c]) * s;
            }
            if (R.obs)
                R.obs[(size_t)e * kRlObs + l] = v;
        } else if (l == 9) {
            held[r] = -1;
        }
        obs[r * kPitch + l] = v;
    }
    __syncthreads();

    const int n = l & 15, g = l >> 4;
    const bf16x8 x0 = pack_inputs(&obs[n * kPitch + 8 * g]);
    const bf16x8 x1 = pack_inputs(&obs[n * kPitch + 32 + 8 * g]);
    // layer 1: 16 unit tiles, two k blocks
    bf16x8 h1[8];
#pragma unroll
    for (int t = 0; t < 16; t += 2) {
        f32x4 lo = bias(P.b1, t, g), hi = bias(P.b1, t + 1, g);
        lo = mfma(fragment(P.w1, (2 * t + 0) * 64 + l), x0, lo);
        hi = mfma(fragment(P.w1, (2 * t + 2) * 64 + l), x0, hi);
        lo = mfma(fragment(P.w1, (2 * t + 1) * 64 + l), x1, lo);
        hi = mfma(fragment(P.w1, (2 * t + 3) * 64 + l), x1, hi);
        h1[t / 2] = relu_pack(lo, hi);
    }
    // layer 2: 16 unit tiles, eight k blocks
    bf16x8 h2[8];
#pragma unroll
    for (int t = 0; t < 16; t += 2) {
        f32x4 lo = bias(P.b2, t, g), hi = bias(P.b2, t + 1, g);
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
            lo = mfma(fragment(P.w2, (8 * t + kb) * 64 + l), h1[kb], lo);
            hi = mfma(fragment(P.w2, (8 * t + 8 + kb) * 64 + l), h1[kb], hi);
        }
        h2[t / 2] = relu_pack(lo, hi);
    }
    // layer 3: one unit tile (actions 0..6, units 7..15 zero)
    f32x4 y = bias(P.b3, 0, g);
#pragma unroll
    for (int kb = 0; kb < 8; ++kb)
        y = mfma(fragment(P.w3, kb * 64 + l), h2[kb], y);
    // lane (n, g) holds actions 4 g .. 4 g + 3 of environment base + n
    if (g < 2) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            act[n * 8 + 4 * g + q] = y[q];
    }
    __syncthreads();

    if (l < kRlEnvsPerWave && base + l < R.num_envs) {
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
    const int grid = (args.num_envs + kRlEnvsPerWave - 1) / kRlEnvsPerWave;
    hipLaunchKernelGGL(rl_policy_kernel, dim3((unsigned)grid), dim3(64), 0, stream, args, policy);
    return hipGetLastError();
}

}  // namespace xpbd
