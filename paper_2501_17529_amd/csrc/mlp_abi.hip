// Host side of the proposal-network entry points (declared in include/dcflow.h).
#include <cmath>
#include <cstdio>

#include "mlp.h"

using namespace dcflow;

namespace {

int fail(hipError_t e, const char *where) {
  fprintf(stderr, "dcflow: %s: %s\n", where, hipGetErrorString(e));
  return DCFLOW_E_HIP;
}

// training workspace: H1, H2, dZ2, dZ1 [B][H]; y, dy [B]
size_t ws_floats(int B) { return (size_t)4 * B * kMlpH + 2 * (size_t)B + 64; }

}  // namespace

extern "C" {

int dcflow_mlp_param_count(void) { return kMlpParams; }

size_t dcflow_mlp_bf16_bytes(void) {
  return sizeof(__bf16) * ((size_t)kMlpH * kMlpDin + (size_t)kMlpH * kMlpH);
}

size_t dcflow_mlp_workspace_bytes(int32_t batch) {
  return batch < 1 ? 0 : ws_floats(batch) * sizeof(float);
}

int dcflow_snapshot_flows(const dcflow_plan *p, const double *inj, int32_t n_snap, double *flows,
                          double *n0max, hipStream_t s) {
  if (!p || !inj || !flows || n_snap < 1) return DCFLOW_E_ARG;
  hipError_t e = launch_snapshot(p, inj, n_snap, flows, n0max, s);
  return e == hipSuccess ? DCFLOW_OK : fail(e, "dcflow_snapshot_flows");
}

int dcflow_snapshot_pairs(const dcflow_plan *p, const double *flows, int32_t n_snap,
                          int32_t *pairs, double *loads, hipStream_t s) {
  if (!p || !flows || !pairs || !loads || n_snap < 1) return DCFLOW_E_ARG;
  hipError_t e = launch_pairs(p, flows, n_snap, pairs, loads, s);
  return e == hipSuccess ? DCFLOW_OK : fail(e, "dcflow_snapshot_pairs");
}

int dcflow_action_features(const dcflow_plan *p, const double *flows, const double *inj,
                           const double *glob, const int32_t *worst, const int32_t *pairs,
                           int32_t n_act, const int32_t *snap, const int32_t *bus,
                           const uint32_t *mask, const int32_t *side, float *feat, hipStream_t s) {
  if (!p || !flows || !inj || !glob || !worst || !pairs || !snap || !bus || !mask || !side ||
      !feat)
    return DCFLOW_E_ARG;
  if (n_act < 0) return DCFLOW_E_SHAPE;
  if (n_act == 0) return DCFLOW_OK;
  hipError_t e =
      launch_features(p, flows, inj, glob, worst, pairs, n_act, snap, bus, mask, side, feat, s);
  return e == hipSuccess ? DCFLOW_OK : fail(e, "dcflow_action_features");
}

int dcflow_improvement_labels(const double *max_load, const int32_t *snap, const double *glob,
                              int32_t n, float *labels, hipStream_t s) {
  if (!max_load || !snap || !glob || !labels || n < 0) return DCFLOW_E_ARG;
  if (n == 0) return DCFLOW_OK;
  hipError_t e = launch_improvement(max_load, snap, glob, n, labels, s);
  return e == hipSuccess ? DCFLOW_OK : fail(e, "dcflow_improvement_labels");
}

int dcflow_mlp_forward(const float *prm, const float *x, int32_t n, float *y, void *ws,
                       size_t ws_bytes, hipStream_t s) {
  if (!prm || !x || !y || !ws || n < 1) return DCFLOW_E_ARG;
  if (ws_bytes < dcflow_mlp_workspace_bytes(n)) return DCFLOW_E_WORKSPACE;
  float *h1 = static_cast<float *>(ws), *h2 = h1 + (size_t)n * kMlpH;
  const float *w1 = prm + kOffW1, *b1 = prm + kOffB1, *w2 = prm + kOffW2, *b2 = prm + kOffB2;
  const float *w3 = prm + kOffW3, *b3 = prm + kOffB3;
  hipError_t e = launch_gemm32(n, kMlpH, kMlpDin, x, kMlpDin, 1, w1, kMlpH, 1, h1, kMlpH, b1,
                               kEpiRelu, nullptr, 0, s);
  if (e == hipSuccess)
    e = launch_gemm32(n, kMlpH, kMlpH, h1, kMlpH, 1, w2, kMlpH, 1, h2, kMlpH, b2, kEpiRelu,
                      nullptr, 0, s);
  if (e == hipSuccess)
    e = launch_gemm32(n, 1, kMlpH, h2, kMlpH, 1, w3, 1, 0, y, 1, b3, 0, nullptr, 0, s);
  return e == hipSuccess ? DCFLOW_OK : fail(e, "dcflow_mlp_forward");
}

int dcflow_mlp_grad(const float *prm, const float *x, const float *t, int32_t B, float *grad,
                    float *loss, void *ws, size_t ws_bytes, hipStream_t s) {
  if (!prm || !x || !t || !grad || !loss || !ws || B < 1) return DCFLOW_E_ARG;
  if (ws_bytes < dcflow_mlp_workspace_bytes(B)) return DCFLOW_E_WORKSPACE;
  float *h1 = static_cast<float *>(ws), *h2 = h1 + (size_t)B * kMlpH;
  float *dz2 = h2 + (size_t)B * kMlpH, *dz1 = dz2 + (size_t)B * kMlpH;
  float *y = dz1 + (size_t)B * kMlpH, *dy = y + B;
  const float *w1 = prm + kOffW1, *b1 = prm + kOffB1, *w2 = prm + kOffW2, *b2 = prm + kOffB2;
  const float *w3 = prm + kOffW3, *b3 = prm + kOffB3;
  float *gw1 = grad + kOffW1, *gb1 = grad + kOffB1, *gw2 = grad + kOffW2, *gb2 = grad + kOffB2;
  float *gw3 = grad + kOffW3, *gb3 = grad + kOffB3;
  const long H = kMlpH, D = kMlpDin;
  hipError_t e = hipSuccess;
#define STEP(call) \
  if (e == hipSuccess) e = (call)
  // forward: H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), y = H2 w3 + b3
  STEP(launch_gemm32(B, H, D, x, D, 1, w1, H, 1, h1, H, b1, kEpiRelu, nullptr, 0, s));
  STEP(launch_gemm32(B, H, H, h1, H, 1, w2, H, 1, h2, H, b2, kEpiRelu, nullptr, 0, s));
  STEP(launch_gemm32(B, 1, H, h2, H, 1, w3, 1, 0, y, 1, b3, 0, nullptr, 0, s));
  // dL/dy
  STEP(launch_mse_grad(y, t, B, dy, loss, s));
  // layer 3: g_w3 = H2^T dy, g_b3 = sum dy, dZ2 = (dy w3^T) * [H2 > 0]
  STEP(launch_gemm32(H, 1, B, h2, 1, H, dy, 1, 0, gw3, 1, nullptr, 0, nullptr, 0, s));
  STEP(launch_colsum(dy, B, 1, 1, gb3, s));
  STEP(launch_gemm32(B, H, 1, dy, 1, 0, w3, 0, 1, dz2, H, nullptr, kEpiMask, h2, H, s));
  // layer 2: g_W2 = H1^T dZ2, g_b2 = colsum dZ2, dZ1 = (dZ2 W2^T) * [H1 > 0]
  STEP(launch_gemm32(H, H, B, h1, 1, H, dz2, H, 1, gw2, H, nullptr, 0, nullptr, 0, s));
  STEP(launch_colsum(dz2, B, H, H, gb2, s));
  STEP(launch_gemm32(B, H, H, dz2, H, 1, w2, 1, H, dz1, H, nullptr, kEpiMask, h1, H, s));
  // layer 1: g_W1 = X^T dZ1, g_b1 = colsum dZ1
  STEP(launch_gemm32(D, H, B, x, 1, D, dz1, H, 1, gw1, H, nullptr, 0, nullptr, 0, s));
  STEP(launch_colsum(dz1, B, H, H, gb1, s));
#undef STEP
  return e == hipSuccess ? DCFLOW_OK : fail(e, "dcflow_mlp_grad");
}

int dcflow_mlp_adam(float *prm, const float *grad, float *m, float *v, int32_t step, float lr,
                    hipStream_t s) {
  if (!prm || !grad || !m || !v || step < 1 || !(lr > 0.f)) return DCFLOW_E_ARG;
  hipError_t e = launch_adam(prm, grad, m, v, kMlpParams, lr, 0.9f, 0.999f, 1e-8f, step, s);
  return e == hipSuccess ? DCFLOW_OK : fail(e, "dcflow_mlp_adam");
}

int dcflow_mlp_pack_bf16(const float *prm, void *bf16, hipStream_t s) {
  if (!prm || !bf16) return DCFLOW_E_ARG;
  __bf16 *w1t = static_cast<__bf16 *>(bf16);
  hipError_t e = launch_pack_bf16(prm, w1t, w1t + (size_t)kMlpH * kMlpDin, s);
  return e == hipSuccess ? DCFLOW_OK : fail(e, "dcflow_mlp_pack_bf16");
}

int dcflow_mlp_infer(const float *prm, const void *bf16, const float *x, int32_t n, float *y,
                     hipStream_t s) {
  if (!prm || !bf16 || !x || !y || n < 0) return DCFLOW_E_ARG;
  if (n == 0) return DCFLOW_OK;
  const __bf16 *w1t = static_cast<const __bf16 *>(bf16);
  hipError_t e = launch_mlp_infer(x, n, prm, w1t, w1t + (size_t)kMlpH * kMlpDin, y, s);
  return e == hipSuccess ? DCFLOW_OK : fail(e, "dcflow_mlp_infer");
}

int dcflow_topk_smallest(const float *scores, int32_t n, int32_t k, int32_t *idx, hipStream_t s) {
  if (!scores || !idx) return DCFLOW_E_ARG;
  if (n < 1 || k < 1 || k > n || k > kTopkMax) return DCFLOW_E_SHAPE;
  hipError_t e = launch_topk(scores, n, k, idx, s);
  return e == hipSuccess ? DCFLOW_OK : fail(e, "dcflow_topk_smallest");
}

int dcflow_column_stats(const float *x, int32_t rows, int32_t cols, float *mean, float *inv_std,
                        hipStream_t s) {
  if (!x || !mean || !inv_std) return DCFLOW_E_ARG;
  if (rows < 1 || cols < 1) return DCFLOW_E_SHAPE;
  hipError_t e = launch_colstats(x, rows, cols, mean, inv_std, s);
  return e == hipSuccess ? DCFLOW_OK : fail(e, "dcflow_column_stats");
}

int dcflow_standardize(float *x, int64_t rows, int32_t cols, const float *mean,
                       const float *inv_std, hipStream_t s) {
  if (!x || !mean || !inv_std) return DCFLOW_E_ARG;
  if (rows < 0 || cols < 1) return DCFLOW_E_SHAPE;
  if (rows == 0) return DCFLOW_OK;
  hipError_t e = launch_standardize(x, rows, cols, mean, inv_std, s);
  return e == hipSuccess ? DCFLOW_OK : fail(e, "dcflow_standardize");
}

}  // extern "C"
