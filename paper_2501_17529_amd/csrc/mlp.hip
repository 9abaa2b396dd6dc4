// Learned proposal network: ranks single-bus-split actions so the exact solver
// evaluates the most promising first.  (The paper leaves the proposing
// optimiser out of scope, Sec. III-A; this is an addition.)
//
// Kernels:
//   k_snapshot_flows  base-case flows of load snapshots on every branch
//                     (PTDF rows x injections, Eq. ptdf_times_nodal_inj) and the
//                     snapshot's largest N-0 relative load on the monitored set;
//   k_features        per-action feature vectors (FP32, 96 wide);
//   k_gemm32          FP32 MFMA GEMM with strided operands and epilogues
//                     (bias, ReLU, ReLU-mask of a forward activation) for the
//                     training forward and backward passes;
//   k_mse_grad        dL/dy of the mean squared error and the loss;
//   k_colsum          bias gradients;
//   k_adam            Adam update of FP32 master weights (Kingma & Ba);
//   k_pack_bf16       BF16 copies of the weights for inference;
//   k_mlp_infer       fused 3-layer inference on BF16 MFMA (16x16x32);
//   k_topk            the k smallest scores by radix select (one workgroup).
#include "dcflow_internal.h"
#include "mlp.h"

namespace dcflow {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------ snapshot flows
// One wave per (snapshot, branch): F[s][l] = H[l, :] . x_s.
__global__ void k_snapshot_flows(const double *__restrict__ Hb, int ld_h, int n, int m,
                                 const double *__restrict__ X, int S, double *__restrict__ F) {
  const int w = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (w >= S * m) return;
  const int s = w / m, l = w - s * m;
  double acc = 0.0;
  for (int x = lane; x < n; x += kWave) acc += Hb[(size_t)l * ld_h + x] * X[(size_t)s * n + x];
  acc = wave_sum(acc);
  if (lane == 0) F[(size_t)s * m + l] = acc;
}

// One workgroup per snapshot: max over monitored rows of |F| / r.
__global__ void k_snapshot_n0max(const double *__restrict__ F, int m, const int32_t *__restrict__ mon,
                                 const double *__restrict__ inv_r, int n_mon,
                                 double *__restrict__ out) {
  __shared__ double red[4];
  const int s = blockIdx.x, tid = threadIdx.x;
  double v = 0.0;
  for (int i = tid; i < n_mon; i += blockDim.x)
    v = fmax(v, fabs(F[(size_t)s * m + mon[i]]) * inv_r[i]);
  v = wave_max(v);
  if (tid % kWave == 0) red[tid / kWave] = v;
  __syncthreads();
  if (tid == 0) out[s] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// One thread per action.  With the snapshot's worst case of the unchanged grid
// (monitored branch l*, contingency c*, or c* = -1 for N-0), the row
// rho = PTDF[l*, :] + LODF[l*, c*] PTDF[c*, :] is the sensitivity of the
// critical post-contingency flow to nodal injections (Def. eq_lodf and
// Eq. lodf_delta applied to the PTDF).  Features:
//   [0] degree, [1] injection of the bus, [2] side bit, [3] rho[A];
//   slot q of the incident branches (ascending id, up to 14), 5 values:
//   [oriented flow / r_q, moved bit, present bit, sigma_q, sigma_q * oriented flow / r*]
//   with sigma_q = rho[A] - rho[far_q] (critical-flow change per unit moved
//   along branch q), r = scale |F_base| + offset, r* that of l*;
//   [74] snapshot max N-0 load, [75] snapshot max N-1 load.
//   [76..83] exact post-split loads of the snapshot's tracked pairs (below),
//   [84] their maximum, [85] 1 if the split islands the network (then 76..84 are 0).
//
// Pair loads.  Splitting bus A moves the masked branches to a new node B; the
// rest (the stay set) keeps A.  By the split factor of the paper (Def. eq_bsdf,
// Eq. bsdf_application) the post-split PTDF row of branch x is
//   H'_x = hx_x + v_x bbc,   v_x = (hx_x . p_shift + p_corr_x) / D,
//   D = 1 - bbc . p_shift,
// with hx the PTDF extended by column B := column A, bbc = e_A - sum_stay s_j hx_j
// (coupler row; slack column 0, shifted by -1 when A is the slack),
// p_shift = -e_B + sum_stay (b_j / beta) e_far_j, beta = sum_stay b_j, and
// p_corr_x = s_j b_j / beta for x = stay branch j.  The N-0 flow becomes
// F'_x = F_x + v_x f_cpl with the coupler flow f_cpl = bbc . p (injection left on A
// minus what the stay branches carry away).  The tracked pair (l, c) then loads
// |F'_l + LODF'_lc F'_c| / r_l with LODF'_lc = H'_l d / (1 - H'_c d), d the
// transfer between c's post-split terminals (Def. eq_lodf, Eq. lodf_delta);
// a contingency that islands the split network leaves the N-0 load.
__global__ void k_features(const int32_t *__restrict__ f, const int32_t *__restrict__ t,
                           const double *__restrict__ bsus, int slack,
                           const int32_t *__restrict__ adj_off,
                           const int32_t *__restrict__ adj_br, const double *__restrict__ fbase,
                           double rscale, double roffset, const double *__restrict__ Hb, int ld_h,
                           const double *__restrict__ hdo, int ld_o,
                           const int32_t *__restrict__ out, int n_out,
                           const int32_t *__restrict__ pos_of_br, const double *__restrict__ inv_r,
                           const double *__restrict__ Fs, int m,
                           const double *__restrict__ X, int n, int n_bus,
                           const double *__restrict__ glob,
                           const int32_t *__restrict__ worst, const int32_t *__restrict__ pairs,
                           int n_act, const int32_t *__restrict__ a_snap,
                           const int32_t *__restrict__ a_bus, const uint32_t *__restrict__ a_mask,
                           const int32_t *__restrict__ a_side, float *__restrict__ o_all) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_act) return;
  const int s = a_snap[a], A = a_bus[a];
  const uint32_t mk = a_mask[a];
  float *o = o_all + (size_t)a * kMlpDin;
  const int deg = adj_off[A + 1] - adj_off[A];
  // critical row: l* and the LODF weight of c* (0 for an N-0 worst case)
  const int ls = worst[2 * s + 0], cs = worst[2 * s + 1];
  int ci = -1;
  for (int c = 0; c < n_out; ++c)
    if (out[c] == cs) ci = c;
  double lw = 0.0;
  if (ci >= 0) {
    const double den = 1.0 - hdo[(size_t)cs * ld_o + ci];
    lw = fabs(den) > 1e-9 ? hdo[(size_t)ls * ld_o + ci] / den : 0.0;
  }
  const double *hl = Hb + (size_t)ls * ld_h;
  const double *hc = Hb + (size_t)(ci >= 0 ? cs : ls) * ld_h;
  const double rs = rscale * fabs(fbase[ls]) + roffset;
  const double rhoA = hl[A] + lw * hc[A];
  for (int q = 0; q < kMlpDin; ++q) o[q] = 0.f;
  o[0] = (float)deg;
  o[1] = (float)X[(size_t)s * n + A];
  o[2] = a_side[a] ? 1.f : 0.f;
  o[3] = (float)rhoA;
  for (int q = 0; q < deg && q < kMlpDmax; ++q) {
    const int br = adj_br[adj_off[A] + q];
    const bool leaves = f[br] == A;
    const int far = leaves ? t[br] : f[br];
    const double r = rscale * fabs(fbase[br]) + roffset;
    const double fo = (leaves ? 1.0 : -1.0) * Fs[(size_t)s * m + br];
    const double sig = rhoA - (hl[far] + lw * hc[far]);
    float *slot = o + 4 + q * kMlpSlot;
    slot[0] = (float)(fo / r);
    slot[1] = ((mk >> q) & 1u) ? 1.f : 0.f;
    slot[2] = 1.f;
    slot[3] = (float)sig;
    slot[4] = (float)(sig * fo / rs);
  }
  o[4 + kMlpDmax * kMlpSlot + 0] = (float)glob[2 * s + 0];
  o[4 + kMlpDmax * kMlpSlot + 1] = (float)glob[2 * s + 1];

  // ---- exact post-split loads of the tracked pairs
  const int a0 = adj_off[A];
  const double *Fv = Fs + (size_t)s * m;
  const double *xs = X + (size_t)s * n;
  double beta = 0.0;
  for (int q = 0; q < deg; ++q)
    if (!((mk >> q) & 1u)) beta += bsus[adj_br[a0 + q]];
  auto stay_s = [&](int br) { return f[br] == A ? 1.0 : -1.0; };
  auto stay_far = [&](int br) { return f[br] == A ? t[br] : f[br]; };
  auto hx = [&](int br, int x) { return Hb[(size_t)br * ld_h + (x < 0 ? A : x)]; };
  auto bbc = [&](int x) {  // coupler row at node x (x < 0: the new node B)
    double v = x == A ? 1.0 : 0.0;
    for (int q = 0; q < deg; ++q) {
      if ((mk >> q) & 1u) continue;
      const int br = adj_br[a0 + q];
      v -= stay_s(br) * hx(br, x);
    }
    if (A == slack) v -= 1.0;
    if (x >= 0 && x == slack) v = 0.0;
    return v;
  };
  double dsum = bbc(-1);
  for (int q = 0; q < deg; ++q) {
    if ((mk >> q) & 1u) continue;
    const int br = adj_br[a0 + q];
    dsum -= bsus[br] / beta * bbc(stay_far(br));
  }
  const double D = 1.0 + dsum;
  float *po = o + kXPairs;
  if (!(beta > 0.0) || fabs(D) < 1e-9) {  // the new node is cut off
    po[kMlpPairs + 1] = 1.f;
    return;
  }
  // injection left on A: the slack's own is minus the sum of the others
  double pA = xs[A];
  if (A == slack) {
    pA = 0.0;
    for (int x = 0; x < n_bus; ++x)
      if (x != slack) pA -= xs[x];
  }
  double fcpl = pA - (a_side[a] ? xs[A] : 0.0);
  for (int q = 0; q < deg; ++q) {
    if ((mk >> q) & 1u) continue;
    const int br = adj_br[a0 + q];
    fcpl -= stay_s(br) * Fv[br];
  }
  auto vrow = [&](int x) {  // v_x
    double hp = -hx(x, A);
    for (int q = 0; q < deg; ++q) {
      if ((mk >> q) & 1u) continue;
      const int br = adj_br[a0 + q];
      hp += bsus[br] / beta * hx(x, stay_far(br));
      if (br == x) hp += stay_s(br) * bsus[br] / beta;
    }
    return hp / D;
  };
  auto moved = [&](int br) {
    for (int q = 0; q < deg; ++q)
      if (adj_br[a0 + q] == br) return ((mk >> q) & 1u) != 0u;
    return false;
  };
  float pmax = 0.f;
  for (int k = 0; k < kMlpPairs; ++k) {
    const int l = pairs[((size_t)s * kMlpPairs + k) * 2 + 0];
    const int c = pairs[((size_t)s * kMlpPairs + k) * 2 + 1];
    double load = 0.0;
    if (l >= 0 && l != c) {
      const double ir = inv_r[pos_of_br[l]];
      const double vl = vrow(l);
      const double f0l = Fv[l] + vl * fcpl;
      load = fabs(f0l) * ir;
      if (c >= 0) {
        const double vc = vrow(c);
        const double f0c = Fv[c] + vc * fcpl;
        const bool mv = moved(c);
        const int fc = mv && f[c] == A ? -1 : f[c];
        const int tc = mv && t[c] == A ? -1 : t[c];
        const double dbb = bbc(fc) - bbc(tc);
        const double num = hx(l, fc) - hx(l, tc) + vl * dbb;
        const double den = 1.0 - (hx(c, fc) - hx(c, tc) + vc * dbb);
        if (fabs(den) >= 1e-9) load = fabs(f0l + num / den * f0c) * ir;
      }
    }
    po[k] = (float)load;
    pmax = fmaxf(pmax, (float)load);
  }
  po[kMlpPairs] = pmax;
}

// One workgroup per snapshot: the kMlpPairs largest relative N-0 / N-1 loads of
// the unchanged grid (Eq. lodf_delta with the base LODF, islanding
// contingencies excluded), ties to the lower position key = (c + 1) n_mon + row.
// Each thread keeps a sorted list of its best entries; thread 0 merges the lists.
__global__ void __launch_bounds__(256)
k_base_pairs(const double *__restrict__ F, int m, const int32_t *__restrict__ mon, int n_mon,
             const int32_t *__restrict__ out, int n_out, const double *__restrict__ hdo, int ld_o,
             const double *__restrict__ inv_r, int32_t *__restrict__ pairs,
             double *__restrict__ loads) {
  constexpr int K = kMlpPairs;
  __shared__ double sv[256][K];
  __shared__ long long sk[256][K];
  const int s = blockIdx.x, tid = threadIdx.x;
  const double *Fv = F + (size_t)s * m;
  double bv[K];
  long long bk[K];
  for (int i = 0; i < K; ++i) {
    bv[i] = -1.0;
    bk[i] = 0x7fffffffffffffffLL;
  }
  const long long total = (long long)(n_out + 1) * n_mon;
  for (long long e = tid; e < total; e += blockDim.x) {
    const int ci = (int)(e / n_mon) - 1, li = (int)(e % n_mon);
    const int l = mon[li];
    double v;
    if (ci < 0) {
      v = fabs(Fv[l]) * inv_r[li];
    } else {
      const int c = out[ci];
      const double den = 1.0 - hdo[(size_t)c * ld_o + ci];
      if (fabs(den) < 1e-9) continue;  // islanding contingency
      const double num = hdo[(size_t)l * ld_o + ci] - (l == c ? 1.0 : 0.0);
      v = fabs(Fv[l] + num / den * Fv[c]) * inv_r[li];
    }
    if (!(v > bv[K - 1] || (v == bv[K - 1] && e < bk[K - 1]))) continue;
    int j = K - 1;  // insertion into the sorted list
    while (j > 0 && (v > bv[j - 1] || (v == bv[j - 1] && e < bk[j - 1]))) {
      bv[j] = bv[j - 1];
      bk[j] = bk[j - 1];
      --j;
    }
    bv[j] = v;
    bk[j] = e;
  }
  for (int i = 0; i < K; ++i) {
    sv[tid][i] = bv[i];
    sk[tid][i] = bk[i];
  }
  __syncthreads();
  if (tid == 0) {
    int head[256];
    for (int i = 0; i < 256; ++i) head[i] = 0;
    for (int q = 0; q < K; ++q) {
      int bt = -1;
      for (int i = 0; i < (int)blockDim.x; ++i) {
        if (head[i] >= K) continue;
        const double v = sv[i][head[i]];
        const long long kk = sk[i][head[i]];
        if (kk == 0x7fffffffffffffffLL) continue;
        if (bt < 0 || v > sv[bt][head[bt]] || (v == sv[bt][head[bt]] && kk < sk[bt][head[bt]])) bt = i;
      }
      int32_t *pp = pairs + ((size_t)s * K + q) * 2;
      if (bt < 0) {  // fewer scored entries than K
        pp[0] = -1;
        pp[1] = -1;
        loads[(size_t)s * K + q] = 0.0;
        continue;
      }
      const long long e = sk[bt][head[bt]];
      const int ci = (int)(e / n_mon) - 1, li = (int)(e % n_mon);
      pp[0] = mon[li];
      pp[1] = ci < 0 ? -1 : out[ci];
      loads[(size_t)s * K + q] = sv[bt][head[bt]];
      ++head[bt];
    }
  }
}

// Training label: log(max_load / base maximum) clipped at 0, 0 for an islanded candidate.
__global__ void k_improvement(const double *__restrict__ max_load, const int32_t *__restrict__ snap,
                              const double *__restrict__ glob, int n, float *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = max_load[i];
  const uint64_t u = __double_as_longlong(v);
  const bool finite = ((u >> 52) & 0x7ff) != 0x7ff;
  out[i] = finite ? (float)fmin(log(v / glob[2 * snap[i] + 1]), 0.0) : 0.f;
}

// ------------------------------------------------------ FP32 GEMM
// C(i, j) = epi( sum_k A(i, k) B(k, j) ) with A(i, k) = A[i*sai + k*sak],
// B(k, j) = B[k*sbk + j*sbj], C row-major (ldc).  64 x 64 tile per workgroup
// (4 waves, 32 x 32 each = 2 x 2 MFMA 16x16x4 blocks), K staged 16 at a time.
// epi: + bias[j] (if bias), then ReLU (EPI_RELU) or multiply by [mask(i,j) > 0]
// (EPI_MASK, mask row-major with ldm), then C = out (+ C if accumulate).
constexpr int G_T = 64, G_K = 16;

__global__ void __launch_bounds__(256)
k_gemm32(int M, int N, int K, const float *__restrict__ A, long sai, long sak,
         const float *__restrict__ B, long sbk, long sbj, float *__restrict__ C, int ldc,
         const float *__restrict__ bias, int epi, const float *__restrict__ mask, int ldm) {
  __shared__ float As[G_T][G_K + 1];
  __shared__ float Bs[G_T][G_K + 1];  // Bs[j][k]
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, g = lane / 16, li = lane % 16;
  const int i0 = blockIdx.y * G_T, j0 = blockIdx.x * G_T;
  const int wi = (wv >> 1) * 32, wj = (wv & 1) * 32;
  f4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += G_K) {
    for (int e = tid; e < G_T * G_K; e += 256) {
      const int r = e / G_K, kk = e % G_K;
      const int i = i0 + r, k = k0 + kk, j = j0 + r;
      As[r][kk] = (i < M && k < K) ? A[i * sai + k * sak] : 0.f;
      Bs[r][kk] = (j < N && k < K) ? B[k * sbk + j * sbj] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < G_K / 4; ++ks) {
      float af[2], bf[2];
      for (int a = 0; a < 2; ++a) af[a] = As[wi + a * 16 + li][ks * 4 + g];
      for (int b = 0; b < 2; ++b) bf[b] = Bs[wj + b * 16 + li][ks * 4 + g];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int j = j0 + wj + b * 16 + li;
      if (j >= N) continue;
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wi + a * 16 + MfmaRow<float>::row(g, r);
        if (i >= M) continue;
        float v = acc[a][b][r];
        if (bias) v += bias[j];
        if (epi & kEpiRelu) v = v > 0.f ? v : 0.f;
        if (epi & kEpiMask) v = mask[(size_t)i * ldm + j] > 0.f ? v : 0.f;
        if (epi & kEpiAccum) v += C[(size_t)i * ldc + j];
        C[(size_t)i * ldc + j] = v;
      }
    }
}

// dL/dy = 2 (y - t) / B for the mean squared error; loss into out[0] (one block).
__global__ void k_mse_grad(const float *__restrict__ y, const float *__restrict__ t, int B,
                           float *__restrict__ dy, float *__restrict__ loss) {
  __shared__ float red[16];
  float acc = 0.f;
  for (int i = threadIdx.x; i < B; i += blockDim.x) {
    const float d = y[i] - t[i];
    dy[i] = 2.f * d / (float)B;
    acc += d * d;
  }
  acc = wave_sum(acc);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int w = 0; w < (int)blockDim.x / kWave; ++w) s += red[w];
    loss[0] = s / (float)B;
  }
}

// out[j] = sum_i X[i][j] (one thread per column; B is small).
__global__ void k_colsum(const float *__restrict__ X, int rows, int cols, int ld,
                         float *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int i = 0; i < rows; ++i) s += X[(size_t)i * ld + j];
  out[j] = s;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------ inference (BF16)
__global__ void k_pack_bf16(const float *__restrict__ p, __bf16 *__restrict__ w1t,
                            __bf16 *__restrict__ w2t) {
  // transposed copies: w1t[h][k] (k contiguous, 96 wide), w2t[h][k] (256 wide)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const float *w1 = p + kOffW1, *w2 = p + kOffW2;
  if (i < kMlpH * kMlpDin) {
    const int h = i / kMlpDin, k = i % kMlpDin;
    w1t[i] = (__bf16)w1[k * kMlpH + h];
  }
  if (i < kMlpH * kMlpH) {
    const int h = i / kMlpH, k = i % kMlpH;
    w2t[i] = (__bf16)w2[k * kMlpH + h];
  }
}

// One workgroup (4 waves) scores 64 actions; wave w owns actions [16w, 16w + 16).
// Layer l: D[act][h] = sum_k X[act][k] W[k][h] as 16 x 16 blocks of
// v_mfma_f32_16x16x32_bf16 (A = activations, 8 consecutive k per lane; B = W^T rows).
__global__ void __launch_bounds__(256)
k_mlp_infer(const float *__restrict__ X, int n, const float *__restrict__ p,
            const __bf16 *__restrict__ w1t, const __bf16 *__restrict__ w2t,
            float *__restrict__ y) {
  __shared__ __bf16 act[64][kMlpH + 8];   // activations of the block's 64 actions
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, g = lane / 16, li = lane % 16;
  const int a0 = blockIdx.x * 64;
  // stage the inputs as BF16
  for (int e = tid; e < 64 * kMlpDin; e += 256) {
    const int r = e / kMlpDin, k = e % kMlpDin;
    const int a = a0 + r;
    act[r][k] = (__bf16)(a < n ? X[(size_t)a * kMlpDin + k] : 0.f);
  }
  __syncthreads();
  const float *b1 = p + kOffB1, *b2 = p + kOffB2, *w3 = p + kOffW3, *b3 = p + kOffB3;
  const int rowA = wv * 16 + li;        // the action this lane feeds as A operand
  f4 h1[kMlpH / 16];
  // ---- layer 1 (K = 96 = 3 x 32)
  for (int hb = 0; hb < kMlpH / 16; ++hb) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kb = 0; kb < kMlpDin / 32; ++kb) {
      bf8 av, bv;
      for (int e = 0; e < 8; ++e) {
        av[e] = act[rowA][kb * 32 + g * 8 + e];
        bv[e] = w1t[(size_t)(hb * 16 + li) * kMlpDin + kb * 32 + g * 8 + e];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
    h1[hb] = acc;
  }
  __syncthreads();  // every wave has read its inputs; overwrite with layer-1 outputs
  for (int hb = 0; hb < kMlpH / 16; ++hb)
    for (int r = 0; r < 4; ++r) {
      const int rr = wv * 16 + MfmaRow<float>::row(g, r);
      const float v = h1[hb][r] + b1[hb * 16 + li];
      act[rr][hb * 16 + li] = (__bf16)(v > 0.f ? v : 0.f);
    }
  __syncthreads();
  // ---- layer 2 (K = 256 = 8 x 32) and the final dot product with w3
  float part[4] = {0.f, 0.f, 0.f, 0.f};
  for (int hb = 0; hb < kMlpH / 16; ++hb) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kb = 0; kb < kMlpH / 32; ++kb) {
      bf8 av, bv;
      for (int e = 0; e < 8; ++e) {
        av[e] = act[rowA][kb * 32 + g * 8 + e];
        bv[e] = w2t[(size_t)(hb * 16 + li) * kMlpH + kb * 32 + g * 8 + e];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    }
    const int h = hb * 16 + li;
    for (int r = 0; r < 4; ++r) {
      const float v = acc[r] + b2[h];
      part[r] += (v > 0.f ? v : 0.f) * w3[h];
    }
  }
  // sum over the 16 hidden columns held by the 16 lanes of a group
  for (int r = 0; r < 4; ++r) {
    float v = part[r];
    for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    part[r] = v;
  }
  if (li == 0)
    for (int r = 0; r < 4; ++r) {
      const int a = a0 + wv * 16 + MfmaRow<float>::row(g, r);
      if (a < n) y[a] = part[r] + b3[0];
    }
}

// ------------------------------------------------------ top-k
// The k smallest of n floats (ties: lowest index), indices written in
// ascending (score, index) order.  One workgroup of 1024 threads: radix select
// on order-preserving 32-bit keys (4 passes of 8 bits), then compaction and a
// bitonic sort of the selected (key, index) pairs in LDS.  k <= kTopkMax.
__device__ __forceinline__ uint32_t fkey(float x) {
  uint32_t u = x == 0.f ? 0u : __float_as_uint(x);  // -0 and +0 compare equal
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ void __launch_bounds__(1024)
k_topk(const float *__restrict__ s, int n, int k, int32_t *__restrict__ out) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t s_prefix, s_need;
  __shared__ unsigned long long pairs[kTopkMax];
  __shared__ uint32_t s_cnt;
  __shared__ uint32_t scan[1024];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_prefix = 0;
    s_need = (uint32_t)k;
  }
  // radix select: find the k-th smallest key
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    for (int b = tid; b < 256; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    const uint32_t pre = s_prefix;
    const uint32_t hmask = pass == 0 ? 0u : (0xffffffffu << (32 - 8 * pass));
    for (int i = tid; i < n; i += blockDim.x) {
      const uint32_t key = fkey(s[i]);
      if ((key & hmask) == (pre & hmask)) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t need = s_need, b = 0;
      while (b < 255 && hist[b] < need) need -= hist[b++];
      s_need = need;
      s_prefix = pre | (b << shift);
    }
    __syncthreads();
  }
  const uint32_t kth = s_prefix;  // keys < kth all selected; keys == kth: lowest indices
  if (tid == 0) s_cnt = 0;
  __syncthreads();
  for (int i = tid; i < n; i += blockDim.x) {
    const uint32_t key = fkey(s[i]);
    if (key < kth) {
      const uint32_t slot = atomicAdd(&s_cnt, 1u);
      pairs[slot] = ((unsigned long long)key << 32) | (uint32_t)i;
    }
  }
  __syncthreads();
  // ties at the threshold, lowest indices first: each thread counts the ties in
  // its contiguous index range, an exclusive scan over threads gives the slots
  const int per = (n + (int)blockDim.x - 1) / (int)blockDim.x;
  const int beg = tid * per, end = min(n, beg + per);
  uint32_t mine = 0;
  for (int i = beg; i < end; ++i) mine += fkey(s[i]) == kth ? 1u : 0u;
  scan[tid] = mine;
  __syncthreads();
  for (int o = 1; o < (int)blockDim.x; o <<= 1) {  // Hillis-Steele inclusive scan
    const uint32_t add = tid >= o ? scan[tid - o] : 0u;
    __syncthreads();
    scan[tid] += add;
    __syncthreads();
  }
  {
    const uint32_t base = s_cnt + scan[tid] - mine;
    uint32_t c = 0;
    for (int i = beg; i < end && base + c < (uint32_t)k; ++i)
      if (fkey(s[i]) == kth) {
        pairs[base + c] = ((unsigned long long)kth << 32) | (uint32_t)i;
        ++c;
      }
  }
  __syncthreads();
  for (int q = tid; q < kTopkMax; q += blockDim.x)
    if (q >= k) pairs[q] = ~0ull;
  __syncthreads();
  // bitonic sort of kTopkMax pairs
  for (int size = 2; size <= kTopkMax; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < kTopkMax; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const unsigned long long a = pairs[i], b = pairs[j];
          if ((a > b) == up) {
            pairs[i] = b;
            pairs[j] = a;
          }
        }
      }
      __syncthreads();
    }
  for (int i = tid; i < k; i += blockDim.x) out[i] = (int32_t)(pairs[i] & 0xffffffffu);
}

// Column mean and 1 / std (std floored at 1e-6) of X [rows][cols], one workgroup
// per column, two-pass in FP64.
__global__ void k_colstats(const float *__restrict__ X, int rows, int cols,
                           float *__restrict__ mean, float *__restrict__ inv_std) {
  __shared__ double red[4];
  __shared__ double s_mu;
  const int j = blockIdx.x, tid = threadIdx.x;
  double a = 0.0;
  for (int i = tid; i < rows; i += blockDim.x) a += X[(size_t)i * cols + j];
  a = wave_sum(a);
  if (tid % kWave == 0) red[tid / kWave] = a;
  __syncthreads();
  if (tid == 0) s_mu = (red[0] + red[1] + red[2] + red[3]) / rows;
  __syncthreads();
  const double mu = s_mu;
  double q = 0.0;
  for (int i = tid; i < rows; i += blockDim.x) {
    const double d = X[(size_t)i * cols + j] - mu;
    q += d * d;
  }
  q = wave_sum(q);
  __syncthreads();
  if (tid % kWave == 0) red[tid / kWave] = q;
  __syncthreads();
  if (tid == 0) {
    const double sd = sqrt((red[0] + red[1] + red[2] + red[3]) / rows);
    mean[j] = (float)mu;
    inv_std[j] = (float)(1.0 / fmax(sd, 1e-6));
  }
}

// X[i][j] = (X[i][j] - mean[j]) * inv_std[j]
__global__ void k_standardize(float *__restrict__ X, long rows, int cols,
                              const float *__restrict__ mean, const float *__restrict__ inv_std) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int j = (int)(e % cols);
  X[e] = (X[e] - mean[j]) * inv_std[j];
}

inline unsigned nblk(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_colstats(const float *X, int rows, int cols, float *mean, float *inv_std,
                           hipStream_t s) {
  k_colstats<<<cols, 256, 0, s>>>(X, rows, cols, mean, inv_std);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_standardize(float *X, long rows, int cols, const float *mean,
                              const float *inv_std, hipStream_t s) {
  k_standardize<<<nblk(rows * cols, 256), 256, 0, s>>>(X, rows, cols, mean, inv_std);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_snapshot(const dcflow_plan *p, const double *X, int S, double *F,
                           double *n0max, hipStream_t s) {
  k_snapshot_flows<<<nblk((long)S * p->m, 4), 256, 0, s>>>(p->d_hb, p->ld_h, p->n_inj, p->m, X, S, F);
  DCF_CHECK_LAUNCH();
  if (n0max) {
    k_snapshot_n0max<<<S, 256, 0, s>>>(F, p->m, p->d_mon, p->d_inv_r, p->n_mon, n0max);
    DCF_CHECK_LAUNCH();
  }
  return hipSuccess;
}

hipError_t launch_features(const dcflow_plan *p, const double *Fs, const double *X,
                           const double *glob, const int32_t *worst, const int32_t *pairs,
                           int n_act, const int32_t *snap, const int32_t *bus,
                           const uint32_t *mask, const int32_t *side, float *out, hipStream_t s) {
  k_features<<<nblk(n_act, 128), 128, 0, s>>>(
      p->d_f, p->d_t, p->d_b, p->slack, p->d_adj_off, p->d_adj_br, p->d_fbase, p->rating_scale,
      p->rating_offset, p->d_hb, p->ld_h, p->d_hdo, p->ld_o, p->d_out, p->n_out, p->d_pos_of_br,
      p->d_inv_r, Fs, p->m, X, p->n_inj, p->n, glob, worst, pairs, n_act, snap, bus, mask, side, out);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_pairs(const dcflow_plan *p, const double *F, int S, int32_t *pairs,
                        double *loads, hipStream_t s) {
  k_base_pairs<<<S, 256, 0, s>>>(F, p->m, p->d_mon, p->n_mon, p->d_out, p->n_out, p->d_hdo,
                                 p->ld_o, p->d_inv_r, pairs, loads);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_improvement(const double *max_load, const int32_t *snap, const double *glob,
                              int n, float *out, hipStream_t s) {
  k_improvement<<<nblk(n, 256), 256, 0, s>>>(max_load, snap, glob, n, out);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_gemm32(int M, int N, int K, const float *A, long sai, long sak, const float *B,
                         long sbk, long sbj, float *C, int ldc, const float *bias, int epi,
                         const float *mask, int ldm, hipStream_t s) {
  dim3 grid(nblk(N, G_T), nblk(M, G_T));
  k_gemm32<<<grid, 256, 0, s>>>(M, N, K, A, sai, sak, B, sbk, sbj, C, ldc, bias, epi, mask, ldm);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_mse_grad(const float *y, const float *t, int B, float *dy, float *loss,
                           hipStream_t s) {
  k_mse_grad<<<1, 1024, 0, s>>>(y, t, B, dy, loss);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_colsum(const float *X, int rows, int cols, int ld, float *out, hipStream_t s) {
  k_colsum<<<nblk(cols, 256), 256, 0, s>>>(X, rows, cols, ld, out);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  k_adam<<<nblk(n, 256), 256, 0, s>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_pack_bf16(const float *p, __bf16 *w1t, __bf16 *w2t, hipStream_t s) {
  k_pack_bf16<<<nblk(kMlpH * kMlpH, 256), 256, 0, s>>>(p, w1t, w2t);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_mlp_infer(const float *X, int n, const float *p, const __bf16 *w1t,
                            const __bf16 *w2t, float *y, hipStream_t s) {
  k_mlp_infer<<<nblk(n, 64), 256, 0, s>>>(X, n, p, w1t, w2t, y);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_topk(const float *scores, int n, int k, int32_t *out, hipStream_t s) {
  k_topk<<<1, 1024, 0, s>>>(scores, n, k, out);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

}  // namespace dcflow
