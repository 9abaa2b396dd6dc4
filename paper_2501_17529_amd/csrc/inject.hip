// Injection module step 8a (paper Sec. III-C): post-change N-0 flows of every
// injection variant, F' = PTDF' x  (Eq. ptdf_times_nodal_inj with the
// candidate's corrected PTDF), computed as
//
//   F'[i][v] = H_Er x_v + U_i z_i[:, v],
//   z_i = K_i^-1 (sigma_i . H x_v - pi_i . x_v)      (sensing rows, k x V)
//
// k_sense: per candidate, the sensing dot products sigma_j . H x_v as a small
//   FP64 MFMA product (sensing rows of the full PTDF x the candidate's
//   variants), then z = K^-1 h.
// k_gemm:  F = X He^T on MFMA (FP64 16x16x4 or FP32 16x16x4), 128x128 tiles,
//   LDS-staged operands with register prefetch, and the rank-k correction
//   U z fused into the epilogue.  He is the kept-row PTDF; X holds one
//   injection vector per output column (variant-major, K contiguous).
// k_bcast: shared-injection mode, F0 = X He^T computed once and corrected per
//   candidate.
#include "dcflow_internal.h"

namespace dcflow {
namespace {

// ---------------------------------------------------------------- sense
// One workgroup per candidate.  The sensing rows (signed rows of the full PTDF)
// times the candidate's variants is a small FP64 MFMA product: 16 rows x 16
// variants per block, K = n_bus split over the 4 waves, 4 independent
// accumulators per wave (one per K sub-step) so the MFMA chain does not
// serialise.  Row results are folded into per-element sums h[j][v] in LDS.
constexpr int kSenseUnroll = 4;
// four doubles at an 8-byte-aligned address (a row of X starts anywhere)
typedef double d4u __attribute__((ext_vector_type(4), aligned(8)));  // K chunks per wave whose loads are in flight together

// four waves per SIMD (at most 128 VGPRs): the occupancy hides the latency of
// the kSenseUnroll chunk loads
__global__ void __launch_bounds__(256, 4)
k_sense(const int32_t *__restrict__ off, const int32_t *__restrict__ kind,
        const int32_t *__restrict__ nsig, const int32_t *__restrict__ sig,
        const double *__restrict__ pnew, const double *__restrict__ kinv,
        const double *__restrict__ Hb, int ld_h, int n, const double *__restrict__ X, int nvar,
        int shared, double *__restrict__ z, int vmax, int cand0,
        const double *__restrict__ pnv) {
  __shared__ int rbr[kMaxRank * kMaxSig];
  __shared__ double rsg[kMaxRank * kMaxSig];
  __shared__ int relem[kMaxRank * kMaxSig];
  __shared__ double red[4][16][17];
  __shared__ double hacc[kMaxRank][16];
  __shared__ int s_R;
  const int cand = cand0 + blockIdx.x;
  const int e0 = off[cand];
  const int k = off[cand + 1] - e0;
  if (k == 0) return;
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, g = lane / 16, li = lane % 16;
  if (tid == 0) {
    int R = 0;
    for (int j = 0; j < k; ++j)
      for (int q = 0; q < nsig[e0 + j]; ++q) {
        int sb = sig[(size_t)(e0 + j) * kMaxSig + q];
        rbr[R] = sb > 0 ? sb - 1 : -sb - 1;
        rsg[R] = sb > 0 ? 1.0 : -1.0;
        relem[R] = j;
        ++R;
      }
    s_R = R;
  }
  __syncthreads();
  const int R = s_R;
  const int nch = (n + 15) / 16;
  for (int v0 = 0; v0 < nvar; v0 += 16) {
    if (tid < kMaxRank * 16) hacc[tid / 16][tid % 16] = 0.0;
    for (int r0 = 0; r0 < R; r0 += 16) {
      // Every lane reads valid memory (row 0 / the candidate's first variant
      // stand in for missing rows and variants, the last entry for k past n),
      // and the zeroing happens at the MFMA: the loads of kSenseUnroll chunks are
      // issued together instead of one wait per guarded load.
      const int row = r0 + li;
      const double *hp = Hb + (size_t)(row < R ? rbr[row] : 0) * ld_h;  // rows padded to
      const double sg = row < R ? rsg[row] : 0.0;                        // ld_h >= nch * 16
      const int v = v0 + li;
      const bool vok = v < nvar;
      const double *xp =
          X + (size_t)(shared ? (vok ? v : 0) : (size_t)cand * nvar + (vok ? v : 0)) * n;
      d4 acc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
      for (int ch0 = wv; ch0 < nch; ch0 += 4 * kSenseUnroll) {
        double a[kSenseUnroll][4], bq[kSenseUnroll][4];
#pragma unroll
        for (int u = 0; u < kSenseUnroll; ++u) {
          const int nb = min(ch0 + 4 * u, nch - 1) * 16 + 4 * g;
#pragma unroll
          for (int q = 0; q < 4; ++q) a[u][q] = hp[nb + q];
          if (n >= 4) {
            // four consecutive entries in one 32-byte load, its start clamped so that
            // it stays inside the row; past the row's end the shift drops them
            const int base = min(nb, n - 4), sh = nb - base;
            const d4u xv = *reinterpret_cast<const d4u *>(xp + base);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int i = q + sh;
              bq[u][q] = i == 0 ? xv[0] : i == 1 ? xv[1] : i == 2 ? xv[2] : xv[3];
            }
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) bq[u][q] = xp[min(nb + q, n - 1)];
          }
        }
#pragma unroll
        for (int u = 0; u < kSenseUnroll; ++u) {
          const int ch = ch0 + 4 * u;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int kk = ch * 16 + 4 * g + q;
            const double av = ch < nch ? sg * a[u][q] : 0.0;
            const double bv = ch < nch && vok && kk < n ? bq[u][q] : 0.0;
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        red[wv][MfmaRow<double>::row(g, r)][li] = acc[0][r] + acc[1][r] + acc[2][r] + acc[3][r];
      __syncthreads();
      if (tid < 16) {  // thread tid owns variant column tid of hacc
        for (int rt = 0; rt < 16 && r0 + rt < R; ++rt)
          hacc[relem[r0 + rt]][tid] += red[0][rt][tid] + red[1][rt][tid] + red[2][rt][tid] +
                                       red[3][rt][tid];
      }
      __syncthreads();
    }
    if (tid < 16) {
      const int v = v0 + tid;
      if (v < nvar) {
        // injection on the split's new busbar: per variant (injection topologies)
        // if given, else the candidate's fixed value
        const double *pbv = pnv ? pnv + (size_t)e0 * nvar + v : pnew + e0;
        const int pstride = pnv ? nvar : 1;
        double h[kMaxRank];
#pragma unroll
        for (int j = 0; j < kMaxRank; ++j) {
          h[j] = 0.0;
          if (j < k)
            h[j] = hacc[j][tid] - (kind[e0 + j] == DCFLOW_SPLIT ? pbv[(size_t)j * pstride] : 0.0);
        }
        const double *Ki = kinv + (size_t)cand * 64;
#pragma unroll
        for (int j = 0; j < kMaxRank; ++j) {
          if (j >= k) break;
          double s = 0.0;
#pragma unroll
          for (int i = 0; i < kMaxRank; ++i) s += Ki[j * 8 + i] * h[i];   // K^-1 zero-padded
          z[(size_t)(e0 + j) * vmax + v] = s;
        }
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------- GEMM
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

constexpr int BM = 128, BN = 128, KT = 16;
// K stages per FP32 partial sum before it is added into FP64 (64 and 128 terms)
constexpr int kFlush32 = 4, kFlushBf = 4;
// LDS row stride: 16-byte aligned rows so that stores and fragment reads are vector
// accesses (lane group g reads the 4 consecutive k it owns in one access)
template <typename T>
struct Ldk {
  static constexpr int v = KT + 16 / (int)sizeof(T);
};
template <typename T>
struct alignas(16) V4 {
  T x[4];
};

constexpr int kXcd = 8;  // MI355X: workgroups are dealt round-robin to 8 XCDs (own L2 each)

// F[col][m] = sum_k X[xrow(col)][k] He[m][k] (+ U z correction), T in {double, float}.
// 1-D grid, XCD-aware: the n_mt row tiles of one column tile run back to back on
// one XCD, so the column tile of X is read from HBM once and then hits that L2.
// 256 threads = 2 x 2 waves of 64 x 64.
// FL > 0 (FP32): the FP32 accumulators are emptied into FP64 ones every FL K stages,
// so FP32 rounding meets only partial sums over FL * KT terms; over the ten
// thousand terms of a large grid a running FP32 sum would carry the rounding of
// its full magnitude at every step (flows of heavily loaded corridors are sums of
// many same-signed terms).
template <typename T, int FL, bool PRE = false>
__global__ void __launch_bounds__(256, (sizeof(T) == 4 && FL == 0) ? 4 : 2)
k_gemm(const T *__restrict__ He, int ld_h, const double *__restrict__ X, int n, int ncols,
       int nvar, int shared, T *__restrict__ F, int ld_f, const int32_t *__restrict__ off,
       const double *__restrict__ U, int ld_er, const double *__restrict__ z, int vmax,
       int correct, int n_mt, int n_nt, const double *__restrict__ pbase,
       const double *__restrict__ fber, const float *__restrict__ Xf = nullptr, int ldx = 0) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int LDS_K = Ldk<T>::v;
  // FP64: two LDS stages (one barrier per K step; two workgroups per CU either way);
  // FP32: one stage, which keeps four workgroups per CU
  constexpr int NS = sizeof(T) == 8 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) T As[NS][BM][LDS_K];
  __shared__ __attribute__((aligned(16))) T Bs[NS][BN][LDS_K];
  const int xcd = blockIdx.x % kXcd, local = blockIdx.x / kXcd;
  const int n_tile = (local / n_mt) * kXcd + xcd, m_tile = local % n_mt;
  if (n_tile >= n_nt) return;
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, g = lane / 16, li = lane % 16;
  const int wm = wv >> 1, wn = wv & 1;
  const int n0 = n_tile * BN, m0 = m_tile * BM;
  // global -> register staging: thread loads 8 consecutive k of one row of A and of B
  const int lr = tid >> 1, lk = (tid & 1) * 8;
  const T *arow = He + (size_t)(m0 + lr) * ld_h;
  const int bcol = n0 + lr;
  const double *brow = nullptr;
  if (bcol < ncols) brow = X + (size_t)bcol * n;
  T ra[8], rb[8];
  const int nk = (n + KT - 1) / KT;
  // FP64: B goes to LDS as loaded (x) with p_base per k in Ps, subtracted from the
  // fragments: no instruction touches the next k-tile's loads before the MFMAs of
  // the current one, so they stay in flight under them.  The columns past ncols
  // read row 0 of X (never stored) and the last k-tile clamps its indices (He is
  // zero there).  FP32 (PRE) reads x - p_base rounded to FP32 by k_sub_f32 (rows of
  // ldx, zero past n; the columns past ncols read row 0): plain loads, consumed only
  // when stored.
  __shared__ double Ps[NS][KT];
  const double *xr = brow ? brow : X;
  double pv = 0.0;
  auto gload = [&](int kt) {
    const int kb = kt * KT + lk;
#pragma unroll
    for (int q = 0; q < 8; ++q) ra[q] = arow[kb + q];  // He padded to ld_h (multiple of 16)
    if constexpr (sizeof(T) == 8) {
      if (kt + 1 < nk) {  // uniform: a whole k-tile
#pragma unroll
        for (int q = 0; q < 8; ++q) rb[q] = xr[kb + q];
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) rb[q] = xr[min(kb + q, n - 1)];
      }
      if (tid < KT) pv = pbase[min(kt * KT + tid, n - 1)];
      return;
    }
    if constexpr (PRE) {
      const float *xf = Xf + (size_t)(bcol < ncols ? bcol : 0) * ldx;
#pragma unroll
      for (int q = 0; q < 8; ++q) rb[q] = xf[kb + q];  // kb + 8 <= n rounded to 16 <= ldx
      return;
    }
    if (brow && kb + 8 <= n) {
#pragma unroll
      for (int q = 0; q < 8; ++q) rb[q] = (T)(brow[kb + q] - pbase[kb + q]);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        rb[q] = (brow && kb + q < n) ? (T)(brow[kb + q] - pbase[kb + q]) : (T)0;
    }
  };
  auto sstore = [&](int st) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      V4<T> va, vb;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        va.x[q] = ra[4 * h + q];
        vb.x[q] = rb[4 * h + q];
      }
      *reinterpret_cast<V4<T> *>(&As[st][lr][lk + 4 * h]) = va;
      *reinterpret_cast<V4<T> *>(&Bs[st][lr][lk + 4 * h]) = vb;
    }
    if (sizeof(T) == 8 && tid < KT) Ps[st][tid] = pv;
  };
  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  d4 acc64[FL > 0 ? 4 : 1][FL > 0 ? 4 : 1];
  if constexpr (FL > 0) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc64[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  }
  auto flush = [&]() {
    if constexpr (FL > 0) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[a][b][r] += (double)acc[a][b][r];
          acc[a][b] = acc_t{0, 0, 0, 0};
        }
    }
  };

  // the next k-tile waits in registers while the current one is consumed; FP32 (one
  // LDS stage, measured faster there than two) stores it after a barrier, FP64 into
  // the other stage at once
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int st = NS == 2 ? (kt & 1) : 0;
    if (kt + 1 < nk) gload(kt + 1);
    // lane group g owns k = 4 g .. 4 g + 3 of the stage and feeds them to the 4 MFMA
    // steps in turn (A and B alike, so every k meets its partner)
    V4<T> af[4], bf[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      af[a] = *reinterpret_cast<const V4<T> *>(&As[st][wm * 64 + a * 16 + li][4 * g]);
#pragma unroll
    for (int b = 0; b < 4; ++b)
      bf[b] = *reinterpret_cast<const V4<T> *>(&Bs[st][wn * 64 + b * 16 + li][4 * g]);
    if constexpr (sizeof(T) == 8) {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const double pk = Ps[st][4 * g + ks];
#pragma unroll
        for (int b = 0; b < 4; ++b) bf[b].x[ks] -= pk;
      }
    }
    // FP64: the wave holds a raised issue priority through its MFMAs, so that the
    // other wave on the SIMD issues its loads and LDS traffic around them rather
    // than between (measured 2% faster in FP64, 1.5% slower in FP32)
    if constexpr (sizeof(T) == 8) __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int ks = 0; ks < KT / 4; ++ks)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<T>::op(af[a].x[ks], bf[b].x[ks], acc[a][b]);
    if constexpr (sizeof(T) == 8) __builtin_amdgcn_s_setprio(0);
    if constexpr (FL > 0) {
      if (kt % FL == FL - 1 || kt + 1 == nk) flush();
    }
    if constexpr (NS == 2) {
      // the other stage was last read in step kt - 1, before the previous barrier
      if (kt + 1 < nk) sstore(st ^ 1);
      __syncthreads();
    } else {
      __syncthreads();
      if (kt + 1 < nk) {
        sstore(0);
        __syncthreads();
      }
    }
  }
  // epilogue: rank-k correction and store
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int col = n0 + wn * 64 + b * 16 + li;
    if (col >= ncols) continue;
    int e0 = 0, e1 = 0, v = col;
    if (correct) {
      const int cand = col / nvar;
      v = col - cand * nvar;
      e0 = off[cand];
      e1 = off[cand + 1];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int mb = m0 + wm * 64 + a * 16;
      double o[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double sum;
        if constexpr (FL > 0)
          sum = acc64[a][b][r];
        else
          sum = (double)acc[a][b][r];
        o[r] = sum + fber[mb + MfmaRow<T>::row(g, r)];
      }
      for (int e = e0; e < e1; ++e) {
        const double ze = z[(size_t)e * vmax + v];
        const double *ue = U + (size_t)e * ld_er + mb;
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] += ue[MfmaRow<T>::row(g, r)] * ze;
      }
      T *dst = F + (size_t)col * ld_f + mb;
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[MfmaRow<T>::row(g, r)] = (T)o[r];
    }
  }
}

// ------------------------------------------------------------ BF16 GEMM
// F[col][m] = sum_k X[xrow(col)][k] He[m][k] (+ U z) on v_mfma_f32_16x16x32_bf16
// with FP32 accumulation.  NP = 1: one BF16 product (BF16 mode).  NP = 3: both
// operands are split into three BF16 parts (He's precomputed in the plan, X's in
// the staging), and the six cross products of order i + j <= 2 are summed
// (BF16X6 mode): every product of parts is exact in the FP32 accumulator, and
// the dropped terms are of order 2^-24 relative.  128 x 128 tile, K step 32;
// lane group g feeds k = 8 g .. 8 g + 7 of each 32-step (A and B alike).
constexpr int BKT = 32, BLD = BKT + 8;  // K step and LDS row stride (bf16)

// x - p_base split into NP BF16 parts, once per call (the GEMM's column tiles
// are read by every row tile): part q of column col at Xs[q * xpart + col * ldx
// + k], K padded with zeros to ldx (a multiple of BKT).  Each thread takes 8
// consecutive k of one column: 64 bytes read, 16 bytes written per part.
template <int NP>
__global__ void __launch_bounds__(256)
k_split_x(const double *__restrict__ X, int n, const double *__restrict__ pbase, int ncols,
          int ldx, __bf16 *__restrict__ Xs, size_t xpart) {
  const int groups = ldx / 8;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ncols * groups) return;
  const int col = (int)(idx / groups), k0 = (int)(idx - (size_t)col * groups) * 8;
  const double *src = X + (size_t)col * n;
  double xv[8];
  if (k0 + 8 <= n) {
#pragma unroll
    for (int e = 0; e < 8; ++e) xv[e] = src[k0 + e] - pbase[k0 + e];
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) xv[e] = k0 + e < n ? src[k0 + e] - pbase[k0 + e] : 0.0;
  }
  __bf16 *dst = Xs + (size_t)col * ldx + k0;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    bf8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const __bf16 b = (__bf16)(float)xv[e];
      v[e] = b;
      xv[e] -= (double)(float)b;
    }
    *reinterpret_cast<bf8 *>(dst + q * xpart) = v;
  }
}

// FP32 mode: x - p_base of every column rounded to FP32 once per call (the values
// the GEMM's B operand takes), rows of ldx, zero past n.  Eight k per thread.
__global__ void __launch_bounds__(256)
k_sub_f32(const double *__restrict__ X, int n, const double *__restrict__ pbase, int ncols,
          int ldx, float *__restrict__ Xf) {
  const int groups = ldx / 8;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ncols * groups) return;
  const int col = (int)(idx / groups), k0 = (int)(idx - (size_t)col * groups) * 8;
  const double *src = X + (size_t)col * n;
  float v[8];
  if (k0 + 8 <= n) {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (float)(src[k0 + e] - pbase[k0 + e]);
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = k0 + e < n ? (float)(src[k0 + e] - pbase[k0 + e]) : 0.0f;
  }
  float *dst = Xf + (size_t)col * ldx + k0;
#pragma unroll
  for (int e = 0; e < 8; ++e) dst[e] = v[e];
}

template <int NP, int FL>
__global__ void __launch_bounds__(256)
k_gemm_bf(const __bf16 *__restrict__ Hp, size_t part, int ld_h, const __bf16 *__restrict__ Xs,
          size_t xpart, int ldx, int n, int ncols, int nvar, int shared, float *__restrict__ F,
          int ld_f, const int32_t *__restrict__ off, const double *__restrict__ U, int ld_er,
          const double *__restrict__ z, int vmax, int correct, int n_mt, int n_nt,
          const double *__restrict__ fber) {
  __shared__ __attribute__((aligned(16))) __bf16 As[NP][BM * BLD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[NP][BN * BLD];
  const int xcd = blockIdx.x % kXcd, local = blockIdx.x / kXcd;
  const int n_tile = (local / n_mt) * kXcd + xcd, m_tile = local % n_mt;
  if (n_tile >= n_nt) return;
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, g = lane / 16, li = lane % 16;
  const int wm = wv >> 1, wn = wv & 1;
  const int n0 = n_tile * BN, m0 = m_tile * BM;
  // staging: each thread 16 consecutive k of one row of A and of B
  const int lr = tid >> 1, lk = (tid & 1) * 16;
  const int bcol = n0 + lr;
  const __bf16 *bsrc = bcol < ncols ? Xs + (size_t)bcol * ldx : nullptr;
  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  // FL > 0: FP32 partial sums over FL K steps, emptied into FP64 (see k_gemm)
  d4 acc64[FL > 0 ? 4 : 1][FL > 0 ? 4 : 1];
  if constexpr (FL > 0) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc64[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  }
  const int nk = (n + BKT - 1) / BKT;
  // register stage of the next K step: A parts (zero past the padded width; ld_h is a
  // multiple of 16) and the parts of 16 injections minus the base case (base flows
  // added in FP64; ldx covers every K step)
  bf8 ra[NP][2], rb[NP][2];
  auto gload = [&](int kt) {
    const int kb = kt * BKT + lk;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      if (kb < ld_h) {
        const bf8 *src = reinterpret_cast<const bf8 *>(Hp + q * part + (size_t)(m0 + lr) * ld_h + kb);
        ra[q][0] = src[0];
        ra[q][1] = src[1];
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          ra[q][0][e] = (__bf16)0.f;
          ra[q][1][e] = (__bf16)0.f;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      if (bsrc) {
        const bf8 *src = reinterpret_cast<const bf8 *>(bsrc + q * xpart + kb);
        rb[q][0] = src[0];
        rb[q][1] = src[1];
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          rb[q][0][e] = (__bf16)0.f;
          rb[q][1][e] = (__bf16)0.f;
        }
      }
    }
  };
  // register stage -> LDS
  auto sstore = [&]() {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      bf8 *da = reinterpret_cast<bf8 *>(&As[q][lr * BLD + lk]);
      da[0] = ra[q][0];
      da[1] = ra[q][1];
      bf8 *db = reinterpret_cast<bf8 *>(&Bs[q][lr * BLD + lk]);
      db[0] = rb[q][0];
      db[1] = rb[q][1];
    }
  };
  gload(0);
  for (int kt = 0; kt < nk; ++kt) {
    sstore();
    __syncthreads();
    if (kt + 1 < nk) gload(kt + 1);  // in flight during this step's MFMAs
    bf8 af[NP][4], bfr[NP][4];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
        af[q][a] = *reinterpret_cast<const bf8 *>(&As[q][(wm * 64 + a * 16 + li) * BLD + g * 8]);
#pragma unroll
      for (int b = 0; b < 4; ++b)
        bfr[q][b] = *reinterpret_cast<const bf8 *>(&Bs[q][(wn * 64 + b * 16 + li) * BLD + g * 8]);
    }
    // smallest terms first: (2,0), (0,2), (1,1), (1,0), (0,1), (0,0)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        f4 c = acc[a][b];
        if (NP == 3) {
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2 % NP][a], bfr[0][b], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][a], bfr[2 % NP][b], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1 % NP][a], bfr[1 % NP][b], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1 % NP][a], bfr[0][b], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][a], bfr[1 % NP][b], c, 0, 0, 0);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][a], bfr[0][b], c, 0, 0, 0);
        acc[a][b] = c;
      }
    if constexpr (FL > 0) {
      if (kt % FL == FL - 1 || kt + 1 == nk) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[a][b][r] += (double)acc[a][b][r];
            acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
          }
      }
    }
    __syncthreads();
  }
  // epilogue: rank-k correction and store (rows 4 g + r of each block)
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int col = n0 + wn * 64 + b * 16 + li;
    if (col >= ncols) continue;
    int e0 = 0, e1 = 0, v = col;
    if (correct) {
      const int cand = col / nvar;
      v = col - cand * nvar;
      e0 = off[cand];
      e1 = off[cand + 1];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int mb = m0 + wm * 64 + a * 16;
      double o[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double sum;
        if constexpr (FL > 0)
          sum = acc64[a][b][r];
        else
          sum = (double)acc[a][b][r];
        o[r] = sum + fber[mb + MfmaRow<float>::row(g, r)];
      }
      for (int e = e0; e < e1; ++e) {
        const double ze = z[(size_t)e * vmax + v];
        const double *ue = U + (size_t)e * ld_er + mb;
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] += ue[MfmaRow<float>::row(g, r)] * ze;
      }
      float *dst = F + (size_t)col * ld_f + mb;
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[MfmaRow<float>::row(g, r)] = (float)o[r];
    }
  }
  (void)shared;
}

// Shared injections: F[i][v][m] = F0[v][m] + sum_e U[e][m] z[e][v].
template <typename T>
__global__ void k_bcast(const T *__restrict__ F0, T *__restrict__ F, int ld_f, int nvar,
                        const int32_t *__restrict__ off, const double *__restrict__ U, int ld_er,
                        const double *__restrict__ z, int vmax) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y, cand = blockIdx.z;
  if (m >= ld_f) return;
  double o = (double)F0[(size_t)v * ld_f + m];
  for (int e = off[cand]; e < off[cand + 1]; ++e) o += U[(size_t)e * ld_er + m] * z[(size_t)e * vmax + v];
  F[((size_t)cand * nvar + v) * ld_f + m] = (T)o;
}

// The GEMM F = X He^T (+ U z) with T operands, or BF16 parts (np = 1 or 3) when T = float
// and np > 0.
// X, F and off are taken from column col0 (candidate col0 / nvar) on.
template <typename T>
hipError_t launch_gemm(const dcflow_plan *p, const T *He, int np, const double *X, int ncols,
                       int nvar, int shared, T *F, const dcflow_batch *bt, int correct,
                       const int32_t *off, size_t col0, hipStream_t s) {
  const int n_mt = p->ld_er / BM, n_nt = (ncols + BN - 1) / BN;
  dim3 grid(kXcd * ((n_nt + kXcd - 1) / kXcd) * n_mt);
  if constexpr (sizeof(T) == 4) {
    const size_t part = (size_t)p->ld_er * p->ld_h;
    if (np == 0) {
      // x - p_base in FP32 into the split buffer (it holds at least xs_cols columns of
      // ldx floats), then the GEMM with plain B loads; larger GEMMs in column blocks
      const int blk = (int)std::min<size_t>((size_t)ncols, bt->xs_cols / nvar * nvar);
      if (blk <= 0) return hipErrorInvalidValue;
      if (ncols > blk) {
        for (int cb = 0; cb < ncols; cb += blk) {
          const int nc = std::min(blk, ncols - cb);
          const hipError_t e = launch_gemm<T>(p, He, np, X + (size_t)cb * p->n_inj, nc, nvar, shared,
                                              F + (size_t)cb * p->ld_er, bt, correct,
                                              off + (correct ? cb / nvar : 0), 0, s);
          if (e != hipSuccess) return e;
        }
        return hipSuccess;
      }
      (void)col0;
      float *xf = reinterpret_cast<float *>(bt->d_xs);
      const size_t nthr = (size_t)ncols * (bt->ldx / 8);
      k_sub_f32<<<dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s>>>(X, p->n_inj, p->d_pbase,
                                                                          ncols, bt->ldx, xf);
      DCF_CHECK_LAUNCH();
      k_gemm<float, kFlush32, true><<<grid, dim3(256), 0, s>>>(
          He, p->ld_h, X, p->n_inj, ncols, nvar, shared, F, p->ld_er, off, bt->d_U, p->ld_er,
          bt->d_z, bt->vmax, correct, n_mt, n_nt, p->d_pbase, p->d_fber, xf, bt->ldx);
      DCF_CHECK_LAUNCH();
      return hipSuccess;
    }
    if (np == 3 || np == 1) {
      // the split buffer holds xs_cols columns: larger GEMMs run in blocks of whole
      // candidates (the parts of a block are written just before its GEMM)
      const size_t xpart = bt->xs_cols * (size_t)bt->ldx;
      const int blk = (int)std::min<size_t>((size_t)ncols, bt->xs_cols / nvar * nvar);
      if (blk <= 0) return hipErrorInvalidValue;
      if (ncols > blk) {
        for (int cb = 0; cb < ncols; cb += blk) {
          const int nc = std::min(blk, ncols - cb);
          const hipError_t e = launch_gemm<T>(p, He, np, X + (size_t)cb * p->n_inj, nc, nvar, shared,
                                              F + (size_t)cb * p->ld_er, bt, correct,
                                              off + (correct ? cb / nvar : 0), 0, s);
          if (e != hipSuccess) return e;
        }
        return hipSuccess;
      }
      (void)col0;
      __bf16 *xs = bt->d_xs;  // columns from 0: each launch splits its own columns first
      const size_t nthr = (size_t)ncols * (bt->ldx / 8);
      const dim3 sg((unsigned)((nthr + 255) / 256));
      if (np == 3) {
        k_split_x<3><<<sg, dim3(256), 0, s>>>(X, p->n_inj, p->d_pbase, ncols, bt->ldx, xs, xpart);
        DCF_CHECK_LAUNCH();
        k_gemm_bf<3, kFlushBf><<<grid, dim3(256), 0, s>>>(p->d_heb, part, p->ld_h, xs, xpart, bt->ldx,
                                                p->n_inj, ncols, nvar, shared, F, p->ld_er, off,
                                                bt->d_U, p->ld_er, bt->d_z, bt->vmax, correct,
                                                n_mt, n_nt, p->d_fber);
      } else {
        k_split_x<1><<<sg, dim3(256), 0, s>>>(X, p->n_inj, p->d_pbase, ncols, bt->ldx, xs, xpart);
        DCF_CHECK_LAUNCH();
        k_gemm_bf<1, 0><<<grid, dim3(256), 0, s>>>(p->d_heb, part, p->ld_h, xs, xpart, bt->ldx,
                                                p->n_inj, ncols, nvar, shared, F, p->ld_er, off,
                                                bt->d_U, p->ld_er, bt->d_z, bt->vmax, correct,
                                                n_mt, n_nt, p->d_fber);
      }
      DCF_CHECK_LAUNCH();
      return hipSuccess;
    }
  }
  // the GEMM takes x - p_base and the FP64 base flows are added back (the injections are
  // variants of the base case, so this keeps most cancellation out of the sums)
  k_gemm<T, sizeof(T) == 4 ? kFlush32 : 0><<<grid, dim3(256), 0, s>>>(He, p->ld_h, X, p->n_inj, ncols, nvar, shared, F, p->ld_er,
                                       off, bt->d_U, p->ld_er, bt->d_z, bt->vmax, correct, n_mt,
                                       n_nt, p->d_pbase, p->d_fber);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

// Candidates [c0, c1); the shared-injection mode takes the whole batch only.
template <typename T>
hipError_t run_injections(dcflow_batch *bt, const T *He, int np, const double *inj, int nvar,
                          int shared, T *flows, int c0, int c1, hipStream_t s) {
  dcflow_plan *p = bt->plan;
  const int ld_f = p->ld_er;
  if (c1 <= c0) return hipSuccess;
  if (shared && (c0 != 0 || c1 != bt->n_cand)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sense, dim3(c1 - c0), dim3(256), 0, s, bt->d_off, bt->d_kind, bt->d_nsig,
                     bt->d_sig, bt->d_pnew, bt->d_kinv, p->d_hb, p->ld_h, p->n_inj, inj, nvar, shared,
                     bt->d_z, bt->vmax, c0, bt->d_pnv);
  DCF_CHECK_LAUNCH();
  if (!shared) {
    const size_t col0 = (size_t)c0 * nvar;
    const hipError_t e =
        launch_gemm<T>(p, He, np, inj + col0 * p->n_inj, (c1 - c0) * nvar, nvar, 0,
                       flows + col0 * ld_f, bt, 1, bt->d_off + c0, col0, s);
    if (e != hipSuccess) return e;
  } else {
    T *f0 = reinterpret_cast<T *>(bt->d_f0);
    const hipError_t e = launch_gemm<T>(p, He, np, inj, nvar, nvar, 1, f0, bt, 0, bt->d_off, 0, s);
    if (e != hipSuccess) return e;
    dim3 g2((ld_f + 255) / 256, nvar, bt->n_cand);
    k_bcast<T><<<g2, dim3(256), 0, s>>>(f0, flows, ld_f, nvar, bt->d_off, bt->d_U, p->ld_er,
                                        bt->d_z, bt->vmax);
    DCF_CHECK_LAUNCH();
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_injections(dcflow_batch *bt, const double *inj, int nvar, int shared, int prec,
                             void *flows, int c0, int c1, hipStream_t s) {
  if (bt->n_cand == 0) return hipSuccess;
  if (prec == DCFLOW_FP64)
    return run_injections<double>(bt, bt->plan->d_he64, 0, inj, nvar, shared,
                                  static_cast<double *>(flows), c0, c1, s);
  const int np = prec == DCFLOW_BF16X6 ? 3 : prec == DCFLOW_BF16 ? 1 : 0;
  return run_injections<float>(bt, bt->plan->d_he32, np, inj, nvar, shared,
                               static_cast<float *>(flows), c0, c1, s);
}

}  // namespace dcflow
