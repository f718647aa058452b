// Device-side layout of the learned warm start's network, shared by the
// runtime (host) and the matrix-core kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace xpbd {

constexpr int kMlpFeatures = 27;   // used features
constexpr int kMlpFeatPad = 32;    // row width of a feature record (bf16); column 31 flags a free particle
constexpr int kMlpHidden = 128;
constexpr int kMlpOutputs = 3;
constexpr int kMlpTile = 64;       // samples per workgroup
constexpr float kMlpClip = 8.0f;   // the correction clamps y to [-8, 8] (network units)
// The correction kernel: particles per work item (16-particle matrix tiles of
// one wave) and persistent workgroups per CU.
constexpr int kCorrectChunk = 32;
constexpr int kCorrectWorkgroupsPerCu = 3;

// Flat parameter order (float32): W1 [128][27], b1 [128], W2 [128][128], b2 [128],
// W3 [3][128], b3 [3]; weights are [out][in].
constexpr int kMlpOffW1 = 0;
constexpr int kMlpOffB1 = kMlpOffW1 + kMlpHidden * kMlpFeatures;
constexpr int kMlpOffW2 = kMlpOffB1 + kMlpHidden;
constexpr int kMlpOffB2 = kMlpOffW2 + kMlpHidden * kMlpHidden;
constexpr int kMlpOffW3 = kMlpOffB2 + kMlpHidden;
constexpr int kMlpOffB3 = kMlpOffW3 + kMlpOutputs * kMlpHidden;
constexpr int kMlpParams = kMlpOffB3 + kMlpOutputs;

// Device buffers of one network.  bfloat16 operand copies are padded with
// zeros: w1 [128][32], w2 [128][128] and its transpose w2t, w3 [16][128] and
// its transpose w3t [128][32].
struct MlpDev {
    float *master;      // [kMlpParams] float32 weights (Adam's copy)
    float *adam_m;      // [kMlpParams]
    float *adam_v;      // [kMlpParams]
    uint16_t *w1, *w2, *w2t, *w3, *w3t;
    float *b1, *b2, *b3;   // float32 biases used by the kernels
    float *out_shift;      // [4]  correction = out_shift + clamp(y) * out_scale
    float *out_scale;      // [4]
};

// Writes the bfloat16 (and bias) copies of master parameter p with value w.
__device__ void mlp_store_operand(const MlpDev &net, int p, float w);

hipError_t launch_mlp_sync(const MlpDev &net, hipStream_t stream);
// y_out: float32 [n][4] network outputs (pos == nullptr), or, with pos, the
// correction y * out_scale added to pos (structure of arrays [3][np]) of every
// row whose free flag is set.
hipError_t launch_mlp_forward(const MlpDev &net, const uint16_t *feat, int n, float *y_out,
                              float *pos, int64_t np, hipStream_t stream);
// Gradient of the masked mean squared error on n samples (sample j is row
// rows[(rows_start + j) mod rows_count] of feat / targets, with
// rows_start < rows_count and n <= rows_count, or row j without a row list),
// then one Adam step
// (skipped when lr == 0).  partial: [ceil(n / 64)][kMlpParams], stats:
// [ceil(n / 64)][2] scratch; grad_out (float32 [kMlpParams]) and loss_out may
// be null.
hipError_t launch_mlp_train(const MlpDev &net, const uint16_t *feat, const float *targets,
                            const int32_t *rows, int64_t rows_start, int64_t rows_count, int n,
                            float *partial, float *stats, float lr, float beta1, float beta2,
                            float eps, int step, float *grad_out, float *loss_out,
                            hipStream_t stream);

// Normalisation statistics of n training rows (features [n][32] bfloat16,
// targets [n][4]) over the rows whose free flag is set; workspace: device
// memory of mlp_normalisation_workspace() bytes, whose last 60 floats receive
// [in_shift 27 | in_scale 27 | out_shift 3 | out_scale 3].
size_t mlp_normalisation_workspace();
hipError_t launch_mlp_normalisation(const uint16_t *feat, const float *targets, int64_t n,
                                    void *workspace, hipStream_t stream);

}  // namespace xpbd
