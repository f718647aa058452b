// Matrix-core kernels of the learned warm start (gfx950, v_mfma_f32_16x16x32_bf16).
//
// The network maps 27 normalised features of a particle's predicted state to a
// correction of its predicted position: a0 = bf16((f - in_shift) * in_scale),
// a1 = bf16(relu(a0 W1^T + b1)), a2 = bf16(relu(a1 W2^T + b2)),
// y = a2 W3^T + b3 (float32), correction = out_shift + clamp(y, -8, 8) * out_scale.
// Products take bfloat16 operands and accumulate in float32.
//
// A workgroup of 4 waves takes 64 samples.  MFMA 16x16x32 operand layout:
// lane l supplies row/column l % 16 and the 8 consecutive k values
// 8 (l / 16) .. 8 (l / 16) + 7 of both operands; it receives column l % 16,
// rows 4 (l / 16) .. 4 (l / 16) + 3 of the result.  Every operand is stored
// "k-contiguous" so each fragment is one 16-byte load: activations in LDS
// both sample-major ([sample][unit]) and unit-major ([unit][sample]), weights
// in global memory both [out][in] and [in][out].
#include <hip/hip_runtime.h>

#include "mlp_device.h"

namespace xpbd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int S = kMlpTile;        // samples per workgroup
constexpr int F = kMlpFeatPad;     // padded feature width (27 used, 31 = free flag)
constexpr int H = kMlpHidden;      // hidden units
constexpr int PS = S + 8;          // pitch of unit-major tiles [unit][sample]
constexpr int PF = F + 8;          // pitch of sample-major feature tiles
constexpr int PH = H + 8;          // pitch of sample-major hidden tiles

__device__ __forceinline__ uint16_t bf16_bits(float f)
{
    // round to nearest, ties to even
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// 16-byte fragment: row r0 + lane % 16, columns k0 + 8 (lane / 16) .. +7 of a
// k-contiguous bf16 matrix with the given pitch (elements)
__device__ __forceinline__ bf16x8 frag(const uint16_t *m, int pitch, int r0, int k0, int lane)
{
    return *reinterpret_cast<const bf16x8 *>(m + (r0 + (lane & 15)) * pitch + k0 + 8 * (lane >> 4));
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct MlpLds {
    uint16_t a0[S * PF];     // features, sample-major
    uint16_t a0t[F * PS];    // features, unit-major
    uint16_t a1[S * PH];     // layer-1 activations (later: output error, both layouts)
    uint16_t a1t[H * PS];    // (later: layer-1 error, unit-major)
    uint16_t a2[S * PH];     // layer-2 activations (later: layer-2 error, sample-major)
    uint16_t a2t[H * PS];    // (later: layer-2 error, unit-major)
    uint32_t m1[S * H / 32]; // relu masks: bit (s * H + u)
    uint32_t m2[S * H / 32];
    float red[4][H];         // per-wave partial column sums
    float loss[4];
};

// Inference needs only the sample-major activations (4 workgroups fit a CU).
struct MlpFwdLds {
    uint16_t a0[S * PF];
    uint16_t a1[S * PH];
    uint16_t a2[S * PH];
};

// The table row of sample j: with a row list, entry (start + j) mod count of
// the list (a window that may wrap around its end; start < count and
// j < count), else row j.
struct RowList {
    const int32_t *rows;
    int64_t start, count;
    __device__ int64_t operator()(int64_t j) const
    {
        if (!rows)
            return j;
        int64_t k = start + j;
        k = k >= count ? k - count : k;
        return (int64_t)rows[k];
    }
};

// Load the features of samples base .. base + S (rows beyond n are zero);
// sample j reads table row rows(j).  The unit-major copy only when a0t is
// given.
__device__ void load_features(uint16_t *a0, uint16_t *a0t, const uint16_t *feat,
                              const RowList &rows, int64_t base, int n, int tid)
{
    for (int i = tid; i < S * F / 8; i += 256) {
        const int s = i / (F / 8), c = (i % (F / 8)) * 8;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (base + s < n) {
            const int64_t r = rows(base + s);
            v = *reinterpret_cast<const uint4 *>(feat + r * F + c);
        }
        *reinterpret_cast<uint4 *>(&a0[s * PF + c]) = v;
        if (a0t) {
            const uint16_t *e = reinterpret_cast<const uint16_t *>(&v);
            for (int k = 0; k < 8; ++k)
                a0t[(c + k) * PS + s] = e[k];
        }
    }
}

// Hidden layer: out = relu(in W^T + b) for the S x H tile; wave w takes the
// output units 32 w .. 32 w + 31 of every sample.  Training also writes the
// unit-major copy and the relu mask.
template <int K, bool TRAIN>
__device__ void hidden_layer(const uint16_t *in, int in_pitch, const uint16_t *w, const float *b,
                             uint16_t *out, uint16_t *out_t, uint32_t *mask, int wave, int lane)
{
    for (int nt = 0; nt < 2; ++nt) {
        const int n0 = 32 * wave + 16 * nt;
        for (int mt = 0; mt < S / 16; ++mt) {
            const int m0 = 16 * mt;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k0 = 0; k0 < K; k0 += 32)
                acc = mfma(frag(in, in_pitch, m0, k0, lane), frag(w, K, n0, k0, lane), acc);
            const int u = n0 + (lane & 15);
            const float bias = b[u];
            uint16_t t[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int s = m0 + 4 * (lane >> 4) + e;
                const float z = acc[e] + bias;
                const uint16_t q = bf16_bits(z > 0.f ? z : 0.f);
                out[s * PH + u] = q;
                t[e] = q;
                if (TRAIN && z > 0.f)
                    atomicOr(&mask[(s * H + u) >> 5], 1u << ((s * H + u) & 31));
            }
            if (TRAIN)
                *reinterpret_cast<uint2 *>(&out_t[u * PS + m0 + 4 * (lane >> 4)]) =
                    make_uint2((uint32_t)t[0] | ((uint32_t)t[1] << 16),
                               (uint32_t)t[2] | ((uint32_t)t[3] << 16));
        }
    }
}

// Output layer for the 16 samples of wave w: y[s][o] for o < 16 (3 used).
__device__ f32x4 output_layer(const uint16_t *a2, const uint16_t *w3, int wave, int lane)
{
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < H; k0 += 32)
        acc = mfma(frag(a2, PH, 16 * wave, k0, lane), frag(w3, H, 0, k0, lane), acc);
    return acc;
}

__device__ void forward_train(MlpLds &L, const MlpDev &net, int tid, int wave, int lane)
{
    for (int i = tid; i < S * H / 32; i += 256) {
        L.m1[i] = 0u;
        L.m2[i] = 0u;
    }
    __syncthreads();
    hidden_layer<F, true>(L.a0, PF, net.w1, net.b1, L.a1, L.a1t, L.m1, wave, lane);
    __syncthreads();
    hidden_layer<H, true>(L.a1, PH, net.w2, net.b2, L.a2, L.a2t, L.m2, wave, lane);
    __syncthreads();
}

// Inference: y (float32 [n][4], MODE_OUT) or the correction added to the
// predicted positions of free particles (structure of arrays, MODE_CORRECT;
// row p of the features is particle p, feature 31 flags a free particle).
template <int MODE>
__global__ void __launch_bounds__(256) mlp_forward_kernel(MlpDev net, const uint16_t *feat, int n,
                                                          float *y_out, float *pos, int64_t np)
{
    __shared__ MlpFwdLds L;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t base = (int64_t)blockIdx.x * S;
    load_features(L.a0, nullptr, feat, RowList{nullptr, 0, 0}, base, n, tid);
    __syncthreads();
    hidden_layer<F, false>(L.a0, PF, net.w1, net.b1, L.a1, nullptr, nullptr, wave, lane);
    __syncthreads();
    hidden_layer<H, false>(L.a1, PH, net.w2, net.b2, L.a2, nullptr, nullptr, wave, lane);
    __syncthreads();
    const f32x4 acc = output_layer(L.a2, net.w3, wave, lane);
    const int o = lane & 15;
    if (o < 3) {
        const float bias = net.b3[o];
        for (int e = 0; e < 4; ++e) {
            const int s = 16 * wave + 4 * (lane >> 4) + e;
            if (base + s >= n)
                continue;
            const float y = acc[e] + bias;
            if (MODE == 0) {
                y_out[(base + s) * 4 + o] = y;
            } else if (bf16_float(L.a0[s * PF + 31]) > 0.f) {
                const float yc = fminf(fmaxf(y, -kMlpClip), kMlpClip);
                pos[(int64_t)o * np + base + s] += net.out_shift[o] + yc * net.out_scale[o];
            }
        }
    }
}

// Column sums of a 16 x 16 result fragment over its rows (samples), summed
// over the waves through LDS later: lanes l, l + 16, l + 32, l + 48 hold the
// same column.
__device__ __forceinline__ float column_sum(f32x4 v)
{
    float s = v[0] + v[1] + v[2] + v[3];
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    return s;
}

// Training: forward and backward of 64 samples; this workgroup's gradient sums
// (unnormalised) go to partial[blockIdx.x][param], its loss sum and sample
// count to stats[blockIdx.x][2].  targets: float32 [n][4] in scaled units.
__global__ void __launch_bounds__(256) mlp_grad_kernel(MlpDev net, const uint16_t *feat,
                                                       const float *targets, RowList rows,
                                                       int n, float *partial, float *stats)
{
    __shared__ MlpLds L;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t base = (int64_t)blockIdx.x * S;
    float *g = partial + (int64_t)blockIdx.x * kMlpParams;
    load_features(L.a0, L.a0t, feat, rows, base, n, tid);
    forward_train(L, net, tid, wave, lane);

    // output error dy = (y - t) * free for the 16 samples of this wave
    uint16_t *gy = L.a1;                      // sample-major [S][32] (pitch PF)
    uint16_t *gyt = L.a1 + S * PF;            // unit-major [32][S] (pitch PS)
    for (int i = tid; i < S * PF + 32 * PS; i += 256)
        L.a1[i] = 0;
    __syncthreads();
    {
        const f32x4 acc = output_layer(L.a2, net.w3, wave, lane);
        const int o = lane & 15;
        float dsum = 0.f, lsum = 0.f, cnt = 0.f;
        uint16_t t[4] = {0, 0, 0, 0};
        for (int e = 0; e < 4; ++e) {
            const int s = 16 * wave + 4 * (lane >> 4) + e;
            float d = 0.f;
            if (o < 3 && base + s < n && bf16_float(L.a0[s * PF + 31]) > 0.f) {
                const int64_t r = rows(base + s);
                d = acc[e] + net.b3[o] - targets[r * 4 + o];
                cnt += o == 0 ? 1.f : 0.f;
            }
            dsum += d;
            lsum += d * d;
            t[e] = bf16_bits(d);
            gy[s * PF + o] = t[e];
        }
        *reinterpret_cast<uint2 *>(&gyt[o * PS + 16 * wave + 4 * (lane >> 4)]) =
            make_uint2((uint32_t)t[0] | ((uint32_t)t[1] << 16), (uint32_t)t[2] | ((uint32_t)t[3] << 16));
        // db3 and the loss: sums over this wave's samples
        dsum += __shfl_xor(dsum, 16, 64);
        dsum += __shfl_xor(dsum, 32, 64);
        if (lane < 16)
            L.red[wave][lane] = dsum;
        for (int off = 32; off > 0; off >>= 1) {
            lsum += __shfl_xor(lsum, off, 64);
            cnt += __shfl_xor(cnt, off, 64);
        }
        if (lane == 0) {
            L.loss[wave] = lsum;
            L.red[wave][16] = cnt;
        }
    }
    __syncthreads();
    if (tid < 3)
        g[kMlpOffB3 + tid] = L.red[0][tid] + L.red[1][tid] + L.red[2][tid] + L.red[3][tid];
    if (tid == 0) {
        stats[2 * blockIdx.x] = L.loss[0] + L.loss[1] + L.loss[2] + L.loss[3];
        stats[2 * blockIdx.x + 1] = L.red[0][16] + L.red[1][16] + L.red[2][16] + L.red[3][16];
    }

    // dW3[o][u] = sum_s gy[s][o] a2[s][u]: M = 16 outputs, N = H, K = S
    for (int nt = 0; nt < 2; ++nt) {
        const int n0 = 32 * wave + 16 * nt;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < S; k0 += 32)
            acc = mfma(frag(gyt, PS, 0, k0, lane), frag(L.a2t, PS, n0, k0, lane), acc);
        for (int e = 0; e < 4; ++e) {
            const int o = 4 * (lane >> 4) + e;
            if (o < 3)
                g[kMlpOffW3 + o * H + n0 + (lane & 15)] = acc[e];
        }
    }
    __syncthreads();   // every read of a2t done before the layer-2 error overwrites it

    // d_a2[s][u] = sum_o gy[s][o] W3[o][u]; dz2 = d_a2 * [z2 > 0]; g2 = bf16(dz2)
    uint16_t *g2 = L.a2, *g2t = L.a2t;
    for (int nt = 0; nt < 2; ++nt) {
        const int n0 = 32 * wave + 16 * nt;
        float csum = 0.f;
        for (int mt = 0; mt < S / 16; ++mt) {
            const int m0 = 16 * mt;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma(frag(gy, PF, m0, 0, lane), frag(net.w3t, 32, n0, 0, lane), acc);
            const int u = n0 + (lane & 15);
            uint16_t t[4];
            for (int e = 0; e < 4; ++e) {
                const int s = m0 + 4 * (lane >> 4) + e;
                const bool on = (L.m2[(s * H + u) >> 5] >> ((s * H + u) & 31)) & 1u;
                const float dz = on ? acc[e] : 0.f;
                acc[e] = dz;
                t[e] = bf16_bits(dz);
                g2[s * PH + u] = t[e];
            }
            csum += column_sum(acc);
            *reinterpret_cast<uint2 *>(&g2t[u * PS + m0 + 4 * (lane >> 4)]) =
                make_uint2((uint32_t)t[0] | ((uint32_t)t[1] << 16), (uint32_t)t[2] | ((uint32_t)t[3] << 16));
        }
        if (lane < 16)
            g[kMlpOffB2 + n0 + lane] = csum;
    }
    __syncthreads();

    // dW2[v][u] = sum_s g2[s][v] a1[s][u]: M = H (v), N = H (u), K = S
    for (int mt = 0; mt < 2; ++mt) {
        const int m0 = 32 * wave + 16 * mt;
        for (int nt = 0; nt < H / 16; ++nt) {
            const int n0 = 16 * nt;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < S; k0 += 32)
                acc = mfma(frag(g2t, PS, m0, k0, lane), frag(L.a1t, PS, n0, k0, lane), acc);
            for (int e = 0; e < 4; ++e)
                g[kMlpOffW2 + (m0 + 4 * (lane >> 4) + e) * H + n0 + (lane & 15)] = acc[e];
        }
    }
    __syncthreads();   // every read of a1t done before the layer-1 error overwrites it

    // d_a1[s][u] = sum_v g2[s][v] W2[v][u]; dz1 = d_a1 * [z1 > 0]; g1 = bf16(dz1)
    uint16_t *g1t = L.a1t;
    for (int nt = 0; nt < 2; ++nt) {
        const int n0 = 32 * wave + 16 * nt;
        float csum = 0.f;
        for (int mt = 0; mt < S / 16; ++mt) {
            const int m0 = 16 * mt;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k0 = 0; k0 < H; k0 += 32)
                acc = mfma(frag(g2, PH, m0, k0, lane), frag(net.w2t, H, n0, k0, lane), acc);
            const int u = n0 + (lane & 15);
            uint16_t t[4];
            for (int e = 0; e < 4; ++e) {
                const int s = m0 + 4 * (lane >> 4) + e;
                const bool on = (L.m1[(s * H + u) >> 5] >> ((s * H + u) & 31)) & 1u;
                const float dz = on ? acc[e] : 0.f;
                acc[e] = dz;
                t[e] = bf16_bits(dz);
            }
            csum += column_sum(acc);
            *reinterpret_cast<uint2 *>(&g1t[u * PS + m0 + 4 * (lane >> 4)]) =
                make_uint2((uint32_t)t[0] | ((uint32_t)t[1] << 16), (uint32_t)t[2] | ((uint32_t)t[3] << 16));
        }
        if (lane < 16)
            g[kMlpOffB1 + n0 + lane] = csum;
    }
    __syncthreads();

    // dW1[u][f] = sum_s g1[s][u] a0[s][f]: M = H (u), N = F (f < 27 kept), K = S
    for (int mt = 0; mt < 2; ++mt) {
        const int m0 = 32 * wave + 16 * mt;
        for (int nt = 0; nt < F / 16; ++nt) {
            const int n0 = 16 * nt;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < S; k0 += 32)
                acc = mfma(frag(g1t, PS, m0, k0, lane), frag(L.a0t, PS, n0, k0, lane), acc);
            const int f = n0 + (lane & 15);
            if (f < kMlpFeatures)
                for (int e = 0; e < 4; ++e)
                    g[kMlpOffW1 + (m0 + 4 * (lane >> 4) + e) * kMlpFeatures + f] = acc[e];
        }
    }
}

// Reduce the workgroup partials (fixed order), normalise by the free-sample
// count, take one Adam step on the float32 master weights and refresh the
// bfloat16 operand copies.  One thread per parameter.  step = t (1-based).
__global__ void __launch_bounds__(256) mlp_adam_kernel(MlpDev net, const float *partial,
                                                       const float *stats, int groups, float lr,
                                                       float beta1, float beta2, float eps, int step,
                                                       float *grad_out, float *loss_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams)
        return;
    float count = 0.f, loss = 0.f, sum = 0.f;
    for (int w = 0; w < groups; ++w) {
        count += stats[2 * w + 1];
        loss += stats[2 * w];
        sum += partial[(int64_t)w * kMlpParams + p];
    }
    const float inv_n = 1.0f / fmaxf(count, 1.0f);
    const float grad = sum * inv_n;
    if (grad_out)
        grad_out[p] = grad;
    if (p == 0 && loss_out)
        loss_out[0] = 0.5f * loss * inv_n;
    if (lr == 0.f)
        return;
    float m = net.adam_m[p] * beta1 + (1.f - beta1) * grad;
    float v = net.adam_v[p] * beta2 + (1.f - beta2) * grad * grad;
    net.adam_m[p] = m;
    net.adam_v[p] = v;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    const float w = net.master[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    net.master[p] = w;
    mlp_store_operand(net, p, w);
}

// bfloat16 operand copies of every master weight (after create or write).
__global__ void mlp_sync_kernel(MlpDev net)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams)
        mlp_store_operand(net, p, net.master[p]);
}

}  // namespace

__device__ void mlp_store_operand(const MlpDev &net, int p, float w)
{
    const uint16_t q = bf16_bits(w);
    if (p < kMlpOffB1) {
        const int u = p / kMlpFeatures, f = p % kMlpFeatures;
        net.w1[u * kMlpFeatPad + f] = q;
    } else if (p < kMlpOffW2) {
        net.b1[p - kMlpOffB1] = w;
    } else if (p < kMlpOffB2) {
        const int i = p - kMlpOffW2, v = i / kMlpHidden, u = i % kMlpHidden;
        net.w2[v * kMlpHidden + u] = q;
        net.w2t[u * kMlpHidden + v] = q;
    } else if (p < kMlpOffW3) {
        net.b2[p - kMlpOffB2] = w;
    } else if (p < kMlpOffB3) {
        const int i = p - kMlpOffW3, o = i / kMlpHidden, u = i % kMlpHidden;
        net.w3[o * kMlpHidden + u] = q;
        net.w3t[u * 32 + o] = q;
    } else {
        net.b3[p - kMlpOffB3] = w;
    }
}

hipError_t launch_mlp_sync(const MlpDev &net, hipStream_t stream)
{
    hipLaunchKernelGGL(mlp_sync_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, stream, net);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDev &net, const uint16_t *feat, int n, float *y_out,
                              float *pos, int64_t np, hipStream_t stream)
{
    if (n <= 0)
        return hipSuccess;
    const dim3 grid((unsigned)((n + S - 1) / S));
    if (pos)
        hipLaunchKernelGGL(mlp_forward_kernel<1>, grid, dim3(256), 0, stream, net, feat, n, y_out,
                           pos, np);
    else
        hipLaunchKernelGGL(mlp_forward_kernel<0>, grid, dim3(256), 0, stream, net, feat, n, y_out,
                           pos, np);
    return hipGetLastError();
}

hipError_t launch_mlp_train(const MlpDev &net, const uint16_t *feat, const float *targets,
                            const int32_t *rows, int64_t rows_start, int64_t rows_count, int n,
                            float *partial, float *stats, float lr, float beta1, float beta2,
                            float eps, int step, float *grad_out, float *loss_out,
                            hipStream_t stream)
{
    const int groups = (n + S - 1) / S;
    RowList list;
    list.rows = rows;
    list.start = rows_start;
    list.count = rows_count;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)groups), dim3(256), 0, stream, net, feat,
                       targets, list, n, partial, stats);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, stream, net,
                       partial, stats, groups, lr, beta1, beta2, eps, step, grad_out, loss_out);
    return hipGetLastError();
}

}  // namespace xpbd
