// Shapes and launchers of the proposal-network kernels (mlp.hip).
#pragma once

#include "dcflow_internal.h"

namespace dcflow {

constexpr int kMlpDin = 96;    // padded feature width (86 used)
constexpr int kMlpH = 256;     // hidden width
constexpr int kMlpDmax = 14;   // incident-branch slots per action
constexpr int kMlpSlot = 5;    // values per slot
constexpr int kMlpPairs = 8;   // tracked (branch, contingency) pairs per snapshot
constexpr int kXPairs = 4 + kMlpDmax * kMlpSlot + 2;  // first pair-load feature
// FP32 master parameters, one flat array: w1 [96][256], b1 [256], w2 [256][256],
// b2 [256], w3 [256], b3 [1] (+3 padding)
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpDin * kMlpH;
constexpr int kOffW2 = kOffB1 + kMlpH;
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpH;
constexpr int kMlpParams = kOffB3 + 4;

constexpr int kEpiRelu = 1;   // max(x, 0)
constexpr int kEpiMask = 2;   // x * [mask > 0]
constexpr int kEpiAccum = 4;  // C += x

constexpr int kTopkMax = 1024;  // largest k of the top-k selection (power of two)

hipError_t launch_snapshot(const dcflow_plan *p, const double *X, int S, double *F,
                           double *n0max, hipStream_t s);
hipError_t launch_pairs(const dcflow_plan *p, const double *F, int S, int32_t *pairs,
                        double *loads, hipStream_t s);
hipError_t launch_features(const dcflow_plan *p, const double *Fs, const double *X,
                           const double *glob, const int32_t *worst, const int32_t *pairs,
                           int n_act, const int32_t *snap, const int32_t *bus,
                           const uint32_t *mask, const int32_t *side, float *out, hipStream_t s);
hipError_t launch_improvement(const double *max_load, const int32_t *snap, const double *glob,
                              int n, float *out, hipStream_t s);
hipError_t launch_gemm32(int M, int N, int K, const float *A, long sai, long sak, const float *B,
                         long sbk, long sbj, float *C, int ldc, const float *bias, int epi,
                         const float *mask, int ldm, hipStream_t s);
hipError_t launch_mse_grad(const float *y, const float *t, int B, float *dy, float *loss,
                           hipStream_t s);
hipError_t launch_colsum(const float *X, int rows, int cols, int ld, float *out, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s);
hipError_t launch_pack_bf16(const float *p, __bf16 *w1t, __bf16 *w2t, hipStream_t s);
hipError_t launch_mlp_infer(const float *X, int n, const float *p, const __bf16 *w1t,
                            const __bf16 *w2t, float *y, hipStream_t s);
hipError_t launch_colstats(const float *X, int rows, int cols, float *mean, float *inv_std,
                           hipStream_t s);
hipError_t launch_standardize(float *X, long rows, int cols, const float *mean,
                              const float *inv_std, hipStream_t s);
hipError_t launch_topk(const float *scores, int n, int k, int32_t *out, hipStream_t s);

}  // namespace dcflow
