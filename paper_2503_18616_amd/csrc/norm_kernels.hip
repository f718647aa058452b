// Normalisation statistics of the learned warm start's training rows: the
// mean and standard deviation, over the rows whose free flag (feature 31) is
// set, of the 27 features and of the 3 target columns.  Two passes in double
// precision (the sums, then the squared deviations from the means), each a
// fixed grid of workgroups writing partial sums that one workgroup then adds
// in workgroup order, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp_device.h"

namespace xpbd {
namespace {

constexpr int kNormThreads = 256;
constexpr int kNormGroups = 240;
constexpr int kNormFeatures = kMlpFeatures;   // 27
constexpr int kNormTargets = 3;
constexpr int kNormCols = kNormFeatures + kNormTargets;   // 30 (+ the free-row count)

__device__ __forceinline__ float bf16_value(uint16_t b)
{
    return __uint_as_float((uint32_t)b << 16);
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
    for (int d = 32; d > 0; d >>= 1)
        v += __shfl_xor(v, d, 64);
    return v;
}

// Column value c of row r: feature c (bfloat16) or target column c - 27.
__device__ __forceinline__ double column(const uint16_t *feat, const float *targets, int64_t r,
                                         int c)
{
    return c < kNormFeatures ? (double)bf16_value(feat[r * kMlpFeatPad + c])
                             : (double)targets[r * 4 + (c - kNormFeatures)];
}

// pass 0: sums of every column and the free-row count; pass 1: sums of the
// squared deviations from mean[] (device, written by the first reduction).
// partial: [kNormGroups][kNormCols + 1]
__global__ void __launch_bounds__(kNormThreads) norm_partial_kernel(
    const uint16_t *feat, const float *targets, int64_t n, int pass, const double *mean,
    double *partial)
{
    __shared__ double wsum[kNormThreads / 64][kNormCols + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double acc[kNormCols + 1];
#pragma unroll
    for (int c = 0; c <= kNormCols; ++c)
        acc[c] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * kNormThreads + threadIdx.x; r < n;
         r += (int64_t)kNormGroups * kNormThreads) {
        if (!(bf16_value(feat[r * kMlpFeatPad + 31]) > 0.0f))
            continue;
        acc[kNormCols] += 1.0;
#pragma unroll
        for (int c = 0; c < kNormCols; ++c) {
            const double v = column(feat, targets, r, c);
            const double d = pass == 0 ? v : v - mean[c];
            acc[c] += pass == 0 ? d : d * d;
        }
    }
#pragma unroll
    for (int c = 0; c <= kNormCols; ++c) {
        const double s = wave_sum_f64(acc[c]);
        if (lane == 0)
            wsum[wave][c] = s;
    }
    __syncthreads();
    if (threadIdx.x <= kNormCols) {
        double s = 0.0;
        for (int w = 0; w < kNormThreads / 64; ++w)
            s += wsum[w][threadIdx.x];
        partial[(int64_t)blockIdx.x * (kNormCols + 1) + threadIdx.x] = s;
    }
}

// The partial sums added in workgroup order.  pass 0: mean[c] = sum / count;
// pass 1: the outputs (float) [in_shift 27 | in_scale 27 | out_shift 3 |
// out_scale 3]: in_scale = 1 / std (1 where std is 0), out_scale =
// max(std, 1e-12).  One thread per column.
__global__ void norm_reduce_kernel(const double *partial, int pass, double *mean, float *out)
{
    const int c = threadIdx.x;
    if (c > kNormCols)
        return;
    double s = 0.0, count = 0.0;
    for (int g = 0; g < kNormGroups; ++g) {
        s += partial[(int64_t)g * (kNormCols + 1) + c];
        count += partial[(int64_t)g * (kNormCols + 1) + kNormCols];
    }
    if (c == kNormCols)
        return;
    const double n = count > 0.0 ? count : 1.0;
    if (pass == 0) {
        mean[c] = s / n;
        return;
    }
    const double sd = sqrt(s / n);
    if (c < kNormFeatures) {
        out[c] = (float)mean[c];
        out[kNormFeatures + c] = sd > 0.0 ? (float)(1.0 / (sd > 1e-30 ? sd : 1e-30)) : 1.0f;
    } else {
        const int k = c - kNormFeatures;
        out[2 * kNormFeatures + k] = (float)mean[c];
        out[2 * kNormFeatures + kNormTargets + k] = (float)(sd > 1e-12 ? sd : 1e-12);
    }
}

}  // namespace

size_t mlp_normalisation_workspace()
{
    return sizeof(double) * ((size_t)kNormGroups * (kNormCols + 1) + kNormCols) +
           sizeof(float) * (2 * kNormFeatures + 2 * kNormTargets);
}

hipError_t launch_mlp_normalisation(const uint16_t *feat, const float *targets, int64_t n,
                                    void *workspace, hipStream_t stream)
{
    double *partial = static_cast<double *>(workspace);
    double *mean = partial + (size_t)kNormGroups * (kNormCols + 1);
    float *out = reinterpret_cast<float *>(mean + kNormCols);
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(norm_partial_kernel, dim3(kNormGroups), dim3(kNormThreads), 0, stream,
                           feat, targets, n, pass, mean, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(norm_reduce_kernel, dim3(1), dim3(64), 0, stream, partial, pass, mean,
                           out);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace xpbd
