// Injection module steps 8b and 8e (paper Sec. III-C, metric-first mode of
// Sec. IV-B): N-1 flows of every contingency (Eq. lodf_delta) reduced on chip
// to the maximum relative branch load per variant (agg_m), then the argmin
// over the variants (t_i*) and, for the winner only, the overload sum and the
// worst (branch, contingency).
//
// With ratings folded into the rows (tilde = divided by r_l) and the LODF
// denominators into the contingency flows, the N-1 flow of monitored row l
// under contingency c for variant v is
//
//     p~1[l, c, v] = F~[l, v] + L~[l, c] y[c, v]
//     L~ = (H_O[E_m, :] - [l == c]) / r  +  (U / r) W      (LODF' numerators, -den on the diagonal)
//     y[c, v] = F'[c, v] / den_c                         (0 for islanding / removed c)
//
// L~ is built per 16 x 16 block on the matrix cores: one FP64 MFMA
// (16x16x4, two when k > 4) with the shared seed Lsd as the accumulator input,
// U/r as A and W as B.  The block stays in registers (converted to T) and is
// reused for every variant of the chunk; the variants' F~ and y are staged in
// LDS.  The scan is VALU work: one FMA plus an absolute max per element.
#include "dcflow_internal.h"

namespace dcflow {
namespace {

__device__ __forceinline__ bool finite_bits(double x) {
  uint64_t u = __double_as_longlong(x);
  return ((u >> 52) & 0x7ff) != 0x7ff;
}

__device__ __forceinline__ float tabs(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double tabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float tmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double tmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float tfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// max(m, |a|, |b|) in one VALU instruction (the compiler does not fold the abs
// modifiers into v_max3_f32 on its own).  Inputs are FMA results (canonical).
__device__ __forceinline__ float absmax3(float m, float a, float b) {
  float r;
  asm("v_max3_f32 %0, %1, |%2|, |%3|" : "=v"(r) : "v"(m), "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double absmax3(double m, double a, double b) {
  return __builtin_fmax(__builtin_fmax(m, __builtin_fabs(a)), __builtin_fabs(b));
}
__device__ __forceinline__ double tfma(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
struct ScanCfg;
template <>
struct ScanCfg<float> {
  static constexpr int TN = 64;  // columns per wave tile
};
template <>
struct ScanCfg<double> {
  static constexpr int TN = 32;
};

// MODE 0: per-variant maxima for variants [vbeg, vbeg + VC).  MODE 1: winner pass.
template <typename T, int VC, int MODE>
__global__ void __launch_bounds__(256)
k_scan(const T *__restrict__ F, int ld_f, int nvar, const int32_t *__restrict__ off,
       const double *__restrict__ U, int ld_er, const double *__restrict__ W, int ld_o,
       const double *__restrict__ invden, const uint32_t *__restrict__ isl,
       const uint32_t *__restrict__ status, const double *__restrict__ lsd,
       const double *__restrict__ inv_r, int n_mon, int mon_pad,
       const int32_t *__restrict__ out_pos, int n_out, const int32_t *__restrict__ mon,
       const int32_t *__restrict__ out, double *__restrict__ vmaxbuf, int vmax_ld,
       dcflow_score *__restrict__ res, int rchunk, int single) {
  constexpr int TM = 64, TN = ScanCfg<T>::TN, NB = TN / 16;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T *ys = reinterpret_cast<T *>(smem_raw);       // [VC][ld_o]
  T *fs = ys + (size_t)VC * ld_o;                // [VC][rchunk]
  T *colw = fs + (size_t)VC * rchunk;            // [ld_o] (winner pass)
  __shared__ double s_red[4][VC];
  __shared__ long long s_key[4];
  __shared__ double s_ov[4];
  __shared__ int s_nf[VC];
  __shared__ int s_vstar;

  const int cand = blockIdx.x;
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, g = lane / 16, li = lane % 16;
  const int e0 = off[cand];
  const int k = off[cand + 1] - e0;
  const uint32_t st = status[cand];

  if (tid < VC) s_nf[tid] = 0;
  __syncthreads();

  // variants of this launch
  int vlist[VC];
  int nv = 0;
  if (MODE == 0) {
    const int vbeg = blockIdx.y * VC;
#pragma unroll
    for (int i = 0; i < VC; ++i) vlist[i] = vbeg + i < nvar ? vbeg + i : -1;
    nv = min(VC, nvar - vbeg);
  } else {
    if (tid == 0 && single) s_vstar = 0;
    if (tid == 0 && !single) {
      int best = 0;
      double bv = vmaxbuf[(size_t)cand * vmax_ld];
      bool any_inf = !finite_bits(bv);
      for (int v = 1; v < nvar; ++v) {
        double x = vmaxbuf[(size_t)cand * vmax_ld + v];
        any_inf |= !finite_bits(x);
        if (x < bv) {
          bv = x;
          best = v;
        }
      }
      s_vstar = best;
      // a variant whose flows were not finite was given +inf by the first pass
      if (any_inf && !(st & DCFLOW_ST_DISCONNECTED)) s_nf[0] = 2;
    }
    __syncthreads();
    vlist[0] = s_vstar;
    nv = 1;
  }

  // stage y = F'[c] / den_c for all contingencies
#pragma unroll
  for (int vi = 0; vi < VC; ++vi) {
    if (vi < nv) {
      const T *Fv = F + ((size_t)cand * nvar + vlist[vi]) * ld_f;
      for (int c = tid; c < ld_o; c += blockDim.x) {
        T y = (T)0;
        if (c < n_out) {
          const double fv = (double)Fv[out_pos[c]];
          if (!finite_bits(fv)) s_nf[vi] = 1;
          y = (T)(fv * invden[(size_t)cand * ld_o + c]);
        }
        ys[(size_t)vi * ld_o + c] = y;
      }
    }
  }
  if (MODE == 1) {
    for (int c = tid; c < ld_o; c += blockDim.x) {
      bool valid = c < n_out && !((isl[(size_t)cand * (ld_o / 32) + c / 32] >> (c % 32)) & 1u);
      colw[c] = valid ? (T)1 : (T)0;
    }
  }

  // per-lane running results
  T mx[VC];
#pragma unroll
  for (int i = 0; i < VC; ++i) mx[i] = (T)0;
  // winner pass: running maximum, the lowest (contingency, branch) key
  // attaining it (N-0 rows first: key = row), and the overload sum
  T bestv = (T)-1;
  long long bestk = 0x7fffffffffffffffLL;
  double ov = 0.0;

  const int ntc = ld_o / TN;
  for (int rc0 = 0; rc0 < mon_pad; rc0 += rchunk) {
    const int rows = min(rchunk, mon_pad - rc0);
    __syncthreads();
    // stage F~ = F' / r for the monitored rows of this chunk (N-0 loads)
#pragma unroll
    for (int vi = 0; vi < VC; ++vi) {
      if (vi < nv) {
        const T *Fv = F + ((size_t)cand * nvar + vlist[vi]) * ld_f;
        for (int rr = tid; rr < rows; rr += blockDim.x) {
          const int row = rc0 + rr;
          T fvs = (T)0;
          if (row < n_mon) {
            const double fv = (double)Fv[row];
            if (!finite_bits(fv)) s_nf[vi] = 1;
            fvs = (T)(fv * inv_r[row]);
          }
          // position p of each 16-row group holds row (p / 4) + 4 (p % 4): the rows an
          // FP64 MFMA block leaves in register r of lane group g sit at p = 4g + r
          const int i16 = rr & 15;
          fs[(size_t)vi * rchunk + (rr - i16) + (i16 >> 2) + 4 * (i16 & 3)] = fvs;
          const T a = tabs(fvs);
          if (MODE == 0) {
            mx[vi] = tmax(mx[vi], a);
          } else if (row < n_mon) {
            if (a > bestv || (a == bestv && (long long)row < bestk)) {
              bestv = a;
              bestk = row;
            }
            ov += fmax((double)a - 1.0, 0.0);
          }
        }
      }
    }
    __syncthreads();

    const int ntr = rows / TM;
    for (int tile = wv; tile < ntr * ntc; tile += 4) {
      const int tr = tile / ntc, tc = tile - tr * ntc;
      const int rowbase = rc0 + tr * TM, colbase = tc * TN;
      // A (U / r) and B (W) fragments of the k-column update
      double af[4][2], bfr[NB][2];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int row = rowbase + a * 16 + li;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int e = h * 4 + g;
          af[a][h] = e < k ? U[(size_t)(e0 + e) * ld_er + row] * inv_r[row] : 0.0;
        }
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int col = colbase + b * 16 + li;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int e = h * 4 + g;
          bfr[b][h] = e < k ? W[(size_t)(e0 + e) * ld_o + col] : 0.0;
        }
      }
      T L[4][NB][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double *src = lsd + (size_t)(rowbase + a * 16) * ld_o + colbase + b * 16 + li;
          d4 c4;
#pragma unroll
          for (int r = 0; r < 4; ++r) c4[r] = src[(size_t)MfmaRow<double>::row(g, r) * ld_o];
          if (k > 0) c4 = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a][0], bfr[b][0], c4, 0, 0, 0);
          if (k > 4) c4 = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a][1], bfr[b][1], c4, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) L[a][b][r] = (T)c4[r];
        }
      // scan the variants
#pragma unroll
      for (int vi = 0; vi < VC; ++vi) {
        if (vi >= nv) continue;
        const T *fsv = fs + (size_t)vi * rchunk + (rowbase - rc0) + 4 * g;
        const T *ysv = ys + (size_t)vi * ld_o + colbase + li;
        T fr[4][4], yc[NB];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) fr[a][r] = fsv[a * 16 + r];
#pragma unroll
        for (int b = 0; b < NB; ++b) yc[b] = ysv[b * 16];
        if (MODE == 0) {
          T m = mx[vi];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
              for (int r = 0; r < 4; r += 2) {
                const T p0 = tfma(L[a][b][r], yc[b], fr[a][r]);
                const T p1 = tfma(L[a][b][r + 1], yc[b], fr[a][r + 1]);
                m = absmax3(m, p0, p1);
              }
          mx[vi] = m;
        } else {
          T pv[4][NB][4];
          T m = (T)0;
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
              for (int r = 0; r < 4; r += 2) {
                pv[a][b][r] = tfma(L[a][b][r], yc[b], fr[a][r]);
                pv[a][b][r + 1] = tfma(L[a][b][r + 1], yc[b], fr[a][r + 1]);
                m = absmax3(m, pv[a][b][r], pv[a][b][r + 1]);
              }
          if (m > (T)1) {  // overloads in this lane's part of the tile
            T o = (T)0;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = 0; b < NB; ++b) {
                const T w = colw[colbase + b * 16 + li];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                  o = tfma(w, tmax(tabs(pv[a][b][r]) - (T)1, (T)0), o);
              }
            ov += (double)o;
          }
          if (m >= bestv) {  // a new (or tied) maximum in this tile: locate it
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = 0; b < NB; ++b) {
                const int c = colbase + b * 16 + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  const int row = rowbase + a * 16 + MfmaRow<double>::row(g, r);
                  const long long key = (long long)(c + 1) * n_mon + row;
                  const T av = tabs(pv[a][b][r]);
                  if (colw[c] != (T)0 && row < n_mon &&
                      (av > bestv || (av == bestv && key < bestk))) {
                    bestv = av;
                    bestk = key;
                  }
                }
              }
          }
        }
      }
    }
  }

  // ---- reductions
  if (MODE == 0) {
#pragma unroll
    for (int i = 0; i < VC; ++i) {
      T m = wave_max(mx[i]);
      if (lane == 0) s_red[wv][i] = (double)m;
    }
    __syncthreads();
    if (tid < nv) {
      double m = fmax(fmax(s_red[0][tid], s_red[1][tid]), fmax(s_red[2][tid], s_red[3][tid]));
      if (s_nf[tid] || (st & DCFLOW_ST_DISCONNECTED)) m = __builtin_inf();
      vmaxbuf[(size_t)cand * vmax_ld + blockIdx.y * VC + tid] = m;  // variant vbeg + tid
    }
  } else {
    // (max, lowest key) across the wave, then across waves; overload sum
    double bv = (double)bestv;
    long long bk = bestk;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double ov2 = __shfl_xor(bv, o);
      const long long ok2 = __shfl_xor(bk, o);
      const bool take = ov2 > bv || (ov2 == bv && ok2 < bk);
      bv = take ? ov2 : bv;
      bk = take ? ok2 : bk;
    }
    double os = wave_sum(ov);
    if (lane == 0) {
      s_red[wv][0] = bv;
      s_key[wv] = bk;
      s_ov[wv] = os;
    }
    __syncthreads();
    if (tid == 0) {
      double b2 = s_red[0][0];
      long long k2 = s_key[0];
      double osum = s_ov[0];
      for (int w = 1; w < 4; ++w) {
        if (s_red[w][0] > b2 || (s_red[w][0] == b2 && s_key[w] < k2)) {
          b2 = s_red[w][0];
          k2 = s_key[w];
        }
        osum += s_ov[w];
      }
      dcflow_score r;
      uint32_t stat = st | (s_nf[0] ? DCFLOW_ST_NONFINITE : 0u);
      r.status = stat;
      if (st & DCFLOW_ST_DISCONNECTED) {
        r.max_load = __builtin_inf();
        r.overload_sum = 0.0;
        r.best_variant = -1;
        r.worst_branch = -1;
        r.worst_outage = -1;
      } else {
        const bool found = k2 != 0x7fffffffffffffffLL;
        const int c = found ? (int)(k2 / n_mon) - 1 : -1;
        const int row = found ? (int)(k2 % n_mon) : -1;
        r.max_load = s_nf[0] == 1 ? __builtin_inf() : b2;
        r.overload_sum = osum;
        r.best_variant = vlist[0];
        r.worst_branch = found ? mon[row] : -1;
        r.worst_outage = c >= 0 ? out[c] : -1;
      }
      res[cand] = r;
      if (single) vmaxbuf[(size_t)cand * vmax_ld] = r.max_load;
    }
  }
}

template <typename T, int VC>
size_t scan_lds(int ld_o, int rchunk, int mode) {
  return sizeof(T) * ((size_t)VC * ld_o + (size_t)VC * rchunk + (mode ? ld_o : 0));
}

// rows per LDS chunk: as many as fit in the LDS budget, a multiple of 64
template <typename T, int VC>
int pick_rchunk(const dcflow_plan *p, int mode) {
  const size_t budget = 64 * 1024;
  size_t fixed = sizeof(T) * ((size_t)VC * p->ld_o + (mode ? p->ld_o : 0));
  if (fixed + sizeof(T) * VC * 64 > budget) return -1;
  int rc = (int)((budget - fixed) / (sizeof(T) * VC)) / 64 * 64;
  return min(rc, p->mon_pad);
}

template <typename T, int VC>
hipError_t run_scan(dcflow_batch *bt, const T *flows, int nvar, dcflow_score *out, hipStream_t s) {
  dcflow_plan *p = bt->plan;
  const int ld_f = p->ld_er;
  int rc0 = pick_rchunk<T, VC>(p, 0);
  int rc1 = pick_rchunk<T, 1>(p, 1);
  if (rc0 <= 0 || rc1 <= 0) return hipErrorInvalidValue;
  dim3 g0(bt->n_cand, (nvar + VC - 1) / VC);
  const size_t lds0 = scan_lds<T, VC>(p->ld_o, rc0, 0);
  const size_t lds1 = scan_lds<T, 1>(p->ld_o, rc1, 1);
  const int single = nvar == 1;  // one variant: the winner pass alone gives everything
  if (!single) {
    k_scan<T, VC, 0><<<g0, dim3(256), lds0, s>>>(
        flows, ld_f, nvar, bt->d_off, bt->d_U, p->ld_er, bt->d_W, p->ld_o, bt->d_invden,
        bt->d_isl, bt->d_status, p->d_lsd, p->d_inv_r, p->n_mon, p->mon_pad, p->d_out_pos,
        p->n_out, p->d_mon, p->d_out, bt->d_vmax, bt->vmax, out, rc0, 0);
    DCF_CHECK_LAUNCH();
  }
  k_scan<T, 1, 1><<<dim3(bt->n_cand), dim3(256), lds1, s>>>(
      flows, ld_f, nvar, bt->d_off, bt->d_U, p->ld_er, bt->d_W, p->ld_o, bt->d_invden, bt->d_isl,
      bt->d_status, p->d_lsd, p->d_inv_r, p->n_mon, p->mon_pad, p->d_out_pos, p->n_out, p->d_mon,
      p->d_out, bt->d_vmax, bt->vmax, out, rc1, single);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

}  // namespace

hipError_t launch_score(dcflow_batch *bt, const void *flows, int nvar, int prec, dcflow_score *out,
                        hipStream_t s) {
  if (bt->n_cand == 0) return hipSuccess;
  if (prec == DCFLOW_FP64) return run_scan<double, 8>(bt, static_cast<const double *>(flows), nvar, out, s);
  return run_scan<float, 16>(bt, static_cast<const float *>(flows), nvar, out, s);
}

}  // namespace dcflow
