// The learned warm start's correction of a substep's predicted positions
// (gfx950): the network (v_mfma_f32_16x16x32_bf16, bfloat16 operands, float32
// accumulation) on the feature rows the prediction kernel wrote, with the
// activations kept in registers, and the clamped, scaled output added to the
// predicted positions of the free particles.
//
// Every wave works on its own: it takes 32 particles of one environment at a
// time (two 16-particle tiles) and needs no barrier after the weights are
// staged.  The products are computed transposed (units x particles): the
// weights are the A operand, the activations the B operand.  Lane l supplies
// particle l % 16 and k values 8 (l / 16) .. + 7 of a B fragment: 16 bytes of
// the particle's feature row.  A layer's result fragment (lane l: particle
// l % 16, units 4 (l / 16) .. + 3 of each 16-unit tile) is already the next
// layer's B fragment once two unit tiles are packed together, provided the
// next layer's k order is permuted the same way; the permutation is applied to
// W2 and W3 when they are staged in LDS.  A contraction does not depend on the
// order of its k terms, so this is the same network up to the order of
// float32 rounding.
#include <hip/hip_runtime.h>


#include "mlp_device.h"
#include "xpbd_device.h"

namespace xpbd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

#define GLOBAL __attribute__((address_space(1)))

constexpr int kThreads = 256;   // threads per workgroup (four independent waves)
constexpr int kTiles = kCorrectChunk / 16;   // 16-particle tiles per work item
constexpr int PF = 40;          // pitch (bfloat16) of W1 rows
constexpr int PW = 136;         // pitch (bfloat16) of W2 and W3 rows
constexpr int H = kMlpHidden;

// LDS of one workgroup (50.4 KB: three workgroups per CU).  The pitches keep
// every 16-lane group of a 16-byte fragment read on distinct 16-byte bank
// groups.
struct CorrectLds {
    uint16_t w1[H * PF];        // W1 [unit][feature]
    uint16_t w2[H * PW];        // W2 [unit][k slot]
    uint16_t w3[16 * PW];       // W3 [output][k slot], rows 3.. zero
    float b1[H];
    float b2[H];
    float b3[16];               // entries 3.. zero
};

// Two floats rounded to bfloat16 (nearest, ties to even: v_cvt_pk_bf16_f32),
// the first in the low half.
__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi)
{
    const f32x2 v = {lo, hi};
    const bf16x2 b = __builtin_convertvector(v, bf16x2);
    uint32_t u;
    __builtin_memcpy(&u, &b, sizeof u);
    return u;
}

// relu of a bfloat16 pair: a negative value (sign bit set) is a negative
// int16, so the packed integer maximum with zero clears it; rounding to
// bfloat16 keeps the sign, so relu and rounding commute.
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

// bfloat16 relu of two result fragments (units 4 g + e of tiles 2 kb and
// 2 kb + 1) as the B fragment of k block kb of the next layer.
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

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 lds_frag(const uint16_t *p)
{
    return *reinterpret_cast<const bf16x8 *>(p);
}

// Stage the network in LDS: W1 as is, W2 and W3 with their k order permuted
// inside every 32-unit block so that k slots 8 g .. 8 g + 3 hold units
// 4 g .. 4 g + 3 and slots 8 g + 4 .. 8 g + 7 hold units 16 + 4 g .. 16 + 4 g + 3:
// what lane group g holds of the two 16-unit result tiles of the previous
// layer (moved as 8-byte pieces: slots 8 g + 4 h .. + 3 <- units 16 h + 4 g .. + 3).
__device__ void stage_network(CorrectLds &S, const MlpDev &net, int tid)
{
    // every load of a thread first, then the stores (one memory latency)
    constexpr int kW1 = H * 4 / kThreads;             // 16-byte pieces of W1 per thread
    constexpr int kW23 = (H + 16) * 32 / kThreads;    // 8-byte pieces of W2 and W3 per thread
    const GLOBAL u32x4 *w1 = (const GLOBAL u32x4 *)(uintptr_t)net.w1;
    const GLOBAL u32x2 *w2 = (const GLOBAL u32x2 *)(uintptr_t)net.w2;
    const GLOBAL u32x2 *w3 = (const GLOBAL u32x2 *)(uintptr_t)net.w3;
    u32x4 a[kW1];
    u32x2 b[kW23];
#pragma unroll
    for (int q = 0; q < kW1; ++q)
        a[q] = w1[tid + kThreads * q];
#pragma unroll
    for (int q = 0; q < kW23; ++q) {
        const int i = tid + kThreads * q, row = i >> 5, piece = i & 31;
        const int kb = piece >> 3, g = (piece >> 1) & 3, h = piece & 1;
        const int src = 32 * kb + 16 * h + 4 * g;
        b[q] = row < H ? w2[(row * H + src) >> 2] : w3[((row - H) * H + src) >> 2];
    }
    float c[3];
    c[0] = tid < H ? net.b1[tid] : 0.f;
    c[1] = tid < H ? net.b2[tid] : 0.f;
    c[2] = tid < kMlpOutputs ? net.b3[tid] : 0.f;
#pragma unroll
    for (int q = 0; q < kW1; ++q) {
        const int i = tid + kThreads * q, u = i >> 2, k = i & 3;
        *reinterpret_cast<u32x4 *>(&S.w1[u * PF + 8 * k]) = a[q];
    }
#pragma unroll
    for (int q = 0; q < kW23; ++q) {
        const int i = tid + kThreads * q, row = i >> 5, piece = i & 31;
        const int kb = piece >> 3, g = (piece >> 1) & 3, h = piece & 1;
        const int dst = 32 * kb + 8 * g + 4 * h;
        uint16_t *base = row < H ? &S.w2[row * PW] : &S.w3[(row - H) * PW];
        *reinterpret_cast<u32x2 *>(base + dst) = b[q];
    }
    if (tid < H) {
        S.b1[tid] = c[0];
        S.b2[tid] = c[1];
    }
    if (tid < 16)
        S.b3[tid] = c[2];
    __syncthreads();
}

// Grid: persistent workgroups of 256 threads (kCorrectWorkgroupsPerCu per
// CU).  Wave w of the grid takes the work items w, w + total waves, ...; item
// k is particles C (k % G + c0) .. + C - 1 of environment k / G, C =
// kCorrectChunk, G = L.chunks, c0 = L.chunk0
// of the environment's mesh (chunks of pinned particles only are skipped).
// Reads the feature rows L.features and adds the correction to the predicted
// positions L.xhat of the free particles.
__global__ void __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(kCorrectWorkgroupsPerCu, kCorrectWorkgroupsPerCu)))
learned_correct_kernel(StepArgs A, LearnedArgs L, MlpDev net)
{
    extern __shared__ __align__(16) unsigned char smem[];
    CorrectLds &S = *reinterpret_cast<CorrectLds *>(smem);
    const int tid = threadIdx.x, lane = tid & 63;
    const int r = lane & 15, g = lane >> 4;
    const int NP = A.total_particles;
    stage_network(S, net, tid);
    float oshift[3], oscale[3];
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        oshift[o] = net.out_shift[o];
        oscale[o] = net.out_scale[o];
    }
    const int G = L.chunks;
    const int items = A.num_envs * G;
    const int waves = gridDim.x * (kThreads / 64);
    // the loads of a work item are issued one item ahead, so they are in
    // flight while the previous item's products run
    struct Item {
        bool ok;            // inside a mesh
        int V, off, p0;
        u32x4 w[kTiles];    // this lane's 16 bytes of each tile's feature rows
        float xh[kTiles][3];
        bool free_p[kTiles];
    };
    auto fetch = [&](int item, Item &d) {
        d.ok = false;
        if (item >= items)
            return;
        const int env = item / G;
        const EnvDev ed = A.envs[env];
        const MeshDev &md = A.meshes[ed.mesh];
        d.V = md.num_vertices;
        d.off = ed.particle_offset;
        d.p0 = (item % G + L.chunk0[ed.mesh]) * 16 * kTiles;
        if (d.p0 >= d.V)
            return;
        d.ok = true;
        const GLOBAL u32x4 *feat =
            (const GLOBAL u32x4 *)(uintptr_t)(L.features + (size_t)d.off * kMlpFeatPad);
        const GLOBAL float *xhat = (const GLOBAL float *)(uintptr_t)L.xhat;
        const GLOBAL float *inv_mass = (const GLOBAL float *)(uintptr_t)md.inv_mass;
#pragma unroll
        for (int t = 0; t < kTiles; ++t) {
            const int i = d.p0 + 16 * t + r;
            const u32x4 zero = {0u, 0u, 0u, 0u};
            d.w[t] = i < d.V ? feat[i * (kMlpFeatPad / 8) + g] : zero;
            d.free_p[t] = false;
            if (g == 0 && i < d.V) {
#pragma unroll
                for (int o = 0; o < 3; ++o)
                    d.xh[t][o] = xhat[(size_t)o * NP + d.off + i];
                d.free_p[t] = inv_mass[i] > 0.0f;
            }
        }
    };
    int item = __builtin_amdgcn_readfirstlane(blockIdx.x * (kThreads / 64) + (tid >> 6));
    Item cur;
    fetch(item, cur);
    for (; item < items; item += waves) {
        Item next;
        fetch(item + waves, next);
        if (cur.ok) {
            bf16x8 x[kTiles];
#pragma unroll
            for (int t = 0; t < kTiles; ++t)
                __builtin_memcpy(&x[t], &cur.w[t], sizeof x[t]);
            // layer 1: 8 unit tiles, one k block
            f32x4 acc[kTiles][8];
#pragma unroll
            for (int nt = 0; nt < 8; ++nt) {
                const f32x4 bias = *reinterpret_cast<const f32x4 *>(&S.b1[16 * nt + 4 * g]);
                const bf16x8 w = lds_frag(&S.w1[(16 * nt + r) * PF + 8 * g]);
#pragma unroll
                for (int t = 0; t < kTiles; ++t)
                    acc[t][nt] = mfma(w, x[t], bias);
            }
            bf16x8 hid[kTiles][4];
#pragma unroll
            for (int t = 0; t < kTiles; ++t)
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
                    hid[t][kb] = relu_pack(acc[t][2 * kb], acc[t][2 * kb + 1]);
            // layer 2: 8 unit tiles, four k blocks; independent accumulators innermost
#pragma unroll
            for (int mt = 0; mt < 8; ++mt) {
                const f32x4 bias = *reinterpret_cast<const f32x4 *>(&S.b2[16 * mt + 4 * g]);
#pragma unroll
                for (int t = 0; t < kTiles; ++t)
                    acc[t][mt] = bias;
            }
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
#pragma unroll
                for (int mt = 0; mt < 8; ++mt) {
                    const bf16x8 w = lds_frag(&S.w2[(16 * mt + r) * PW + 32 * kb + 8 * g]);
#pragma unroll
                    for (int t = 0; t < kTiles; ++t)
                        acc[t][mt] = mfma(w, hid[t][kb], acc[t][mt]);
                }
#pragma unroll
            for (int t = 0; t < kTiles; ++t)
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
                    hid[t][kb] = relu_pack(acc[t][2 * kb], acc[t][2 * kb + 1]);
            // layer 3: outputs 0..2 (rows 3..15 of W3 are zero)
            f32x4 y[kTiles];
            const f32x4 b3 = *reinterpret_cast<const f32x4 *>(&S.b3[4 * g]);
#pragma unroll
            for (int t = 0; t < kTiles; ++t)
                y[t] = b3;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const bf16x8 w = lds_frag(&S.w3[r * PW + 32 * kb + 8 * g]);
#pragma unroll
                for (int t = 0; t < kTiles; ++t)
                    y[t] = mfma(w, hid[t][kb], y[t]);
            }
            // lanes 0..15 hold outputs 0..2 of particle r of every tile
            if (g == 0) {
#pragma unroll
                for (int t = 0; t < kTiles; ++t) {
                    const int i = cur.p0 + 16 * t + r;
                    if (i >= cur.V)
                        continue;
#pragma unroll
                    for (int o = 0; o < 3; ++o) {
                        float p = cur.xh[t][o];
                        if (cur.free_p[t]) {
                            const float yc = fminf(fmaxf(y[t][o], -kMlpClip), kMlpClip);
                            p += oshift[o] + yc * oscale[o];
                        }
                        L.xhat[(size_t)o * NP + cur.off + i] = p;
                    }
                }
            }
        }
        cur = next;
    }
}

}  // namespace

uint32_t learned_correct_lds_bytes() { return (uint32_t)sizeof(CorrectLds); }

hipError_t launch_learned_correct(const StepArgs &args, const LearnedArgs &largs,
                                  const MlpDev &net, int num_workgroups, hipStream_t stream)
{
    if (args.num_envs <= 0)
        return hipSuccess;
    const uint32_t lds = learned_correct_lds_bytes();
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(learned_correct_kernel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess)
        return err;
    const int64_t items = (int64_t)args.num_envs * largs.chunks;
    const int64_t needed = (items + kThreads / 64 - 1) / (kThreads / 64);
    const int grid = (int)(needed < num_workgroups ? needed : num_workgroups);
    hipLaunchKernelGGL(learned_correct_kernel, dim3((unsigned)grid), dim3(kThreads), lds, stream,
                       args, largs, net);
    return hipGetLastError();
}

}  // namespace xpbd
