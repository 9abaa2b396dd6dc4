// agg_i in two levels (paper Sec. IV-B): for the winning variant t_i* of every
// candidate, the top per_case loads inside each case (the N-0 case, each scored
// contingency column, each multi-outage case), then the top_k of that collection.
// A global top-k would let one dominant outage fill the whole list; the per-case
// cap keeps the other cases visible.
//
// With one row band, level 1 starts from the column-maximum sweep of the
// worst-case pass: only the hot columns (at most top_k of them) can place an entry
// in the result, and k_scan_hot builds their per-case lists on the tiles'
// arithmetic.  k_pc_sel adds the N-0 case and the columns that the FP32 scan's
// error guard computes in FP64 (one wave per case, rows over the lanes), and
// k_pc_multi the multi-outage cases (coefficients z = coef p1[S], the m entries of
// their branches summed).  Otherwise k_pc_cols walks every case, one thread each:
// an LODF' entry is Lsd[row, c] + (U / r)[row, :] W[:, c] (k FMAs), the N-1 flow
// F~ + L~ y_c, and a sorted list of the case's largest |p~|.  Level 2 (k_pc_fin)
// takes the top_k of the lists per candidate.
#include "percase.h"

namespace dcflow {
namespace {

struct PcEntry;

}  // namespace
size_t pc_list_bytes(int n_cand, int nslots, int per_case);
namespace {

struct PcEntry {  // one list entry: |p| / r and its key (case slot x n_mon + row)
  double v;
  int k, pad;
};

constexpr int kEmptyKey = 0x7fffffff;
constexpr int kFinRankCap = 256;  // k_pc_fin ranks up to this many entries in LDS

__device__ __forceinline__ float pc_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double pc_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ bool pc_better(T v, int k, T w, int kw) {
  return v > w || (v == w && k < kw);
}

template <typename T, int KM>
__device__ __forceinline__ void pc_insert(T (&lv)[KM], int (&lk)[KM], T v, int k) {
#pragma unroll
  for (int j = KM - 1; j > 0; --j) {
    const bool up = pc_better(v, k, lv[j - 1], lk[j - 1]);
    const bool here = pc_better(v, k, lv[j], lk[j]);
    lv[j] = up ? lv[j - 1] : (here ? v : lv[j]);
    lk[j] = up ? lk[j - 1] : (here ? k : lk[j]);
  }
  if (pc_better(v, k, lv[0], lk[0])) {
    lv[0] = v;
    lk[0] = k;
  }
}

struct PcArgs {
  const void *F;  // flows [n_cand][nvar][ld_f]
  int ld_f, nvar;
  const int32_t *off;
  const double *U;  // [n_elem][ld_er]
  int ld_er;
  const double *W;  // [n_elem][ld_o]
  const float *ur32, *w32;
  int ld_o, mon_pad, n_mon;
  const double *lsd;     // [mon_pad][ld_o]
  const double *lsdT;    // [ld_o][mon_pad] the same column-major
  const double *inv_r;   // [mon_pad]
  const double *invden;  // [n_cand][ld_o]
  const uint32_t *isl;   // [n_cand][ld_o / 32]
  const int32_t *out_pos;
  int n_out, n_ctg, n_gen;
  const double *gen_y;
  int n_multi;
  const int32_t *moff, *mcol;
  const double *lsdm;    // [n_msub][mon_pad]
  const double *mcoef;   // [n_cand][n_multi][16]
  const int32_t *mok;
  const int32_t *mon, *out;
  const dcflow_score *scores;
  int per_case, top_k, nslots;
  PcEntry *ws;  // [n_cand][nslots][per_case]
  const uint32_t *flag;  // [n_cand][ld_o / 32] columns the FP32 scan's error guard
                         // computes in FP64 (null: none)
  const double *cmx;     // [n_cand][ld_o + 2] the winner's column maxima (from the tiles),
                         // N-0 maximum and their top_k-th largest, or null: every slot
                         // is listed by k_pc_cols
  const int32_t *hotl;   // [n_cand][kHotLd] with cmx: the hot columns, whose lists
                         // k_scan_hot writes
  int32_t *sel;          // [n_cand][n_ctg + 2] with cmx: the number of slots that
                         // k_pc_sel lists (N-0 and guarded columns), then the slots
};

template <typename T>
struct PcOps;
template <>
struct PcOps<double> {
  static __device__ __forceinline__ double ur(const PcArgs &A, int e, int row) {
    return A.U[(size_t)e * A.ld_er + row] * A.inv_r[row];
  }
  static __device__ __forceinline__ double w(const PcArgs &A, int e, int c) {
    return A.W[(size_t)e * A.ld_o + c];
  }
};
template <>
struct PcOps<float> {
  static __device__ __forceinline__ float ur(const PcArgs &A, int e, int row) {
    return A.ur32[(size_t)e * A.mon_pad + row];
  }
  static __device__ __forceinline__ float w(const PcArgs &A, int e, int c) {
    return A.w32[(size_t)e * A.ld_o + c];
  }
};

__device__ __forceinline__ bool pc_skip(const PcArgs &A, int cand, int &vstar) {
  const dcflow_score sc = A.scores[cand];
  vstar = sc.best_variant;
  return (sc.status & (DCFLOW_ST_DISCONNECTED | DCFLOW_ST_NONFINITE)) != 0 || vstar < 0 ||
         vstar >= A.nvar;
}

template <typename T, int KM>
__device__ __forceinline__ void pc_store(const PcArgs &A, int cand, int slot, const T (&lv)[KM],
                                         const int (&lk)[KM]) {
  PcEntry *dst = A.ws + ((size_t)cand * A.nslots + slot) * A.per_case;
#pragma unroll
  for (int j = 0; j < KM; ++j)
    if (j < A.per_case) {
      PcEntry e;
      e.v = lk[j] == kEmptyKey ? -1.0 : (double)lv[j];
      e.k = lk[j];
      e.pad = 0;
      dst[j] = e;
    }
}

// Level 1, slots 0 .. n_ctg: slot 0 the N-0 case, slot 1 + c contingency column c.
template <typename T, int KM>
__global__ void __launch_bounds__(256) k_pc_cols(PcArgs A) {
  const int cand = blockIdx.x;
  const int slot = blockIdx.y * blockDim.x + threadIdx.x;
  if (slot > A.n_ctg) return;
  T lv[KM];
  int lk[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    lv[j] = (T)-1;
    lk[j] = kEmptyKey;
  }
  int vstar = 0;
  const int c = slot - 1;
  bool live = !pc_skip(A, cand, vstar);
  if (live && c >= 0)
    live = !((A.isl[(size_t)cand * (A.ld_o / 32) + c / 32] >> (c % 32)) & 1u);
  const bool guard = live && c >= 0 && A.flag != nullptr &&
                     ((A.flag[(size_t)cand * (A.ld_o / 32) + c / 32] >> (c % 32)) & 1u);
  if (guard) {
    // a column of the FP32 scan's error guard: the entries in FP64 from the FP64
    // factors, as the scan computes them
    const T *Fv = static_cast<const T *>(A.F) + ((size_t)cand * A.nvar + vstar) * A.ld_f;
    const int e0 = A.off[cand], k = A.off[cand + 1] - e0;
    const double inv = A.invden[(size_t)cand * A.ld_o + c];
    const double y = (c < A.n_out ? (double)Fv[A.out_pos[c]] : A.gen_y[c - A.n_out]) * inv;
    double w[kMaxRank];
#pragma unroll
    for (int e = 0; e < kMaxRank; ++e) w[e] = e < k ? PcOps<double>::w(A, e0 + e, c) : 0.0;
    for (int row = 0; row < A.n_mon; ++row) {
      double l = A.lsd[(size_t)row * A.ld_o + c];
#pragma unroll
      for (int e = 0; e < kMaxRank; ++e)
        if (e < k) l = pc_fma(PcOps<double>::ur(A, e0 + e, row), w[e], l);
      const double p = pc_fma(l, y, (double)Fv[row] * A.inv_r[row]);
      const T a = (T)(p < 0.0 ? -p : p);
      const int key = slot * A.n_mon + row;
      if (pc_better(a, key, lv[KM - 1], lk[KM - 1])) pc_insert(lv, lk, a, key);
    }
  } else if (live) {
    const T *Fv = static_cast<const T *>(A.F) + ((size_t)cand * A.nvar + vstar) * A.ld_f;
    const int e0 = A.off[cand], k = A.off[cand + 1] - e0;
    T y = (T)0, w[kMaxRank];
#pragma unroll
    for (int e = 0; e < kMaxRank; ++e) w[e] = (T)0;
    if (c >= 0) {
      const double inv = A.invden[(size_t)cand * A.ld_o + c];
      y = (T)(c < A.n_out ? (double)Fv[A.out_pos[c]] * inv : A.gen_y[c - A.n_out] * inv);
#pragma unroll
      for (int e = 0; e < kMaxRank; ++e)
        if (e < k) w[e] = PcOps<T>::w(A, e0 + e, c);
    }
    for (int row = 0; row < A.n_mon; ++row) {
      const T f = (T)((double)Fv[row] * A.inv_r[row]);
      T p = f;
      if (c >= 0) {
        T l = (T)A.lsd[(size_t)row * A.ld_o + c];
#pragma unroll
        for (int e = 0; e < kMaxRank; ++e)
          if (e < k) l = pc_fma(PcOps<T>::ur(A, e0 + e, row), w[e], l);
        p = pc_fma(l, y, f);
      }
      const T a = p < (T)0 ? -p : p;
      const int key = slot * A.n_mon + row;
      if (pc_better(a, key, lv[KM - 1], lk[KM - 1])) pc_insert(lv, lk, a, key);
    }
  }
  pc_store(A, cand, slot, lv, lk);
}

// Level 1 beside the hot columns (one row band): the N-0 case and the columns that
// the FP32 scan's error guard computes in FP64, one wave per case and the rows
// spread over its lanes.  Every other contingency column either is hot (its list
// comes from k_scan_hot, on the tiles' arithmetic) or has all its entries after
// top_k entries of other cases.  The block collects its slots in LDS and in sel;
// each lane keeps a sorted list of its rows' largest loads, and the wave's list is
// taken one entry per round from the lanes' heads.  The arithmetic is that of
// k_pc_cols (guarded columns in FP64).
template <typename T, int KM, bool STAGE>
__global__ void __launch_bounds__(256) k_pc_sel(PcArgs A) {
  // [n_ctg + 1] listed slots; with STAGE then the candidate's F~ on the monitored
  // rows ([mon_pad] of T)
  extern __shared__ __attribute__((aligned(16))) int s_sel[];
  __shared__ int s_n;
  const int cand = blockIdx.x, tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  int vstar = 0;
  if (pc_skip(A, cand, vstar)) return;
  if (tid == 0) s_n = 0;
  T *s_f = reinterpret_cast<T *>(s_sel + ((A.n_ctg + 1 + 3) / 4) * 4);
  if (STAGE) {
    const T *Fs = static_cast<const T *>(A.F) + ((size_t)cand * A.nvar + vstar) * A.ld_f;
    for (int row = tid; row < A.n_mon; row += blockDim.x)
      s_f[row] = (T)((double)Fs[row] * A.inv_r[row]);
  }
  __syncthreads();
  for (int slot = tid; slot <= A.n_ctg; slot += blockDim.x) {
    const int c = slot - 1;
    bool keep = c < 0;  // N-0
    if (c >= 0 && A.flag && ((A.flag[(size_t)cand * (A.ld_o / 32) + c / 32] >> (c % 32)) & 1u))
      keep = !((A.isl[(size_t)cand * (A.ld_o / 32) + c / 32] >> (c % 32)) & 1u);
    if (keep) s_sel[atomicAdd(&s_n, 1)] = slot;
  }
  __syncthreads();
  const int n_sel = s_n;
  int32_t *sl = A.sel + (size_t)cand * (A.n_ctg + 2);
  for (int q = tid; q < n_sel; q += blockDim.x) sl[1 + q] = s_sel[q];
  if (tid == 0) sl[0] = n_sel;
  const T *Fv = static_cast<const T *>(A.F) + ((size_t)cand * A.nvar + vstar) * A.ld_f;
  const int e0 = A.off[cand], k = A.off[cand + 1] - e0;
  // with the case maxima, only entries at or above tau can reach the final list
  const T thr = A.cmx ? (T)A.cmx[(size_t)cand * (A.ld_o + 2) + A.ld_o + 1] : (T)-1;
  for (int q = wv; q < n_sel; q += 4) {
    const int slot = s_sel[q], c = slot - 1;
    const bool guard = c >= 0 && A.flag != nullptr &&
                       ((A.flag[(size_t)cand * (A.ld_o / 32) + c / 32] >> (c % 32)) & 1u);
    T lv[KM];
    int lk[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      lv[j] = (T)-1;
      lk[j] = kEmptyKey;
    }
    double y64 = 0.0, w64[kMaxRank];
#pragma unroll
    for (int e = 0; e < kMaxRank; ++e) w64[e] = 0.0;
    if (guard) {
      const double inv = A.invden[(size_t)cand * A.ld_o + c];
      y64 = (c < A.n_out ? (double)Fv[A.out_pos[c]] : A.gen_y[c - A.n_out]) * inv;
#pragma unroll
      for (int e = 0; e < kMaxRank; ++e)
        if (e < k) w64[e] = PcOps<double>::w(A, e0 + e, c);
    }
    for (int row = lane; row < A.n_mon; row += kWave) {
      T a;
      if (!guard) {  // N-0
        const T f = STAGE ? s_f[row] : (T)((double)Fv[row] * A.inv_r[row]);
        a = f < (T)0 ? -f : f;
      } else {
        double l = A.lsdT[(size_t)c * A.mon_pad + row];
#pragma unroll
        for (int e = 0; e < kMaxRank; ++e)
          if (e < k) l = pc_fma(PcOps<double>::ur(A, e0 + e, row), w64[e], l);
        const double p = pc_fma(l, y64, (double)Fv[row] * A.inv_r[row]);
        a = (T)(p < 0.0 ? -p : p);
      }
      const int key = slot * A.n_mon + row;
      if (a >= thr && pc_better(a, key, lv[KM - 1], lk[KM - 1])) pc_insert(lv, lk, a, key);
    }
    // the case's list: per_case rounds of the best head over the wave
    PcEntry *dst = A.ws + ((size_t)cand * A.nslots + slot) * A.per_case;
    for (int j = 0; j < A.per_case; ++j) {
      T bv = lv[0];
      int bk = lk[0];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const T ov = __shfl_xor(bv, o);
        const int ok = __shfl_xor(bk, o);
        if (pc_better(ov, ok, bv, bk)) {
          bv = ov;
          bk = ok;
        }
      }
      if (lane == 0) {
        PcEntry e;
        e.v = bk == kEmptyKey ? -1.0 : (double)bv;
        e.k = bk;
        e.pad = 0;
        dst[j] = e;
      }
      if (bk != kEmptyKey && lk[0] == bk) {
#pragma unroll
        for (int t = 0; t < KM - 1; ++t) {
          lv[t] = lv[t + 1];
          lk[t] = lk[t + 1];
        }
        lv[KM - 1] = (T)-1;
        lk[KM - 1] = kEmptyKey;
      }
    }
  }
}

// Level 1, multi-outage cases: slot 1 + n_ctg + q, one thread per case.  The
// candidate's U / r rows and F~ (the same for all its cases) are staged in LDS 64
// rows at a time; each thread reads its case's seed entries for kPcRows rows at once.
template <typename T, int KM>
__global__ void __launch_bounds__(256) k_pc_multi(PcArgs A) {
  constexpr int MM = DCFLOW_MULTI_MAX, kRows = 64, kPcRows = 8;
  __shared__ T s_ur[kMaxRank][kRows];
  __shared__ T s_f[kRows];
  const int cand = blockIdx.x;
  const int q = blockIdx.y * blockDim.x + threadIdx.x;
  const bool act = q < A.n_multi;  // the threads past the last case still stage rows
  const int slot = 1 + A.n_ctg + q;
  T lv[KM];
  int lk[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    lv[j] = (T)-1;
    lk[j] = kEmptyKey;
  }
  int vstar = 0;
  const bool cand_live = !pc_skip(A, cand, vstar);  // block-uniform
  const bool live = cand_live && act && A.mok[(size_t)cand * A.n_multi + q] != 0;
  // with the case maxima, only entries at or above tau can reach the final list
  const T thr = A.cmx ? (T)A.cmx[(size_t)cand * (A.ld_o + 2) + A.ld_o + 1] : (T)-1;
  if (cand_live) {
    const T *Fv = static_cast<const T *>(A.F) + ((size_t)cand * A.nvar + vstar) * A.ld_f;
    const int e0 = A.off[cand], k = A.off[cand + 1] - e0;
    const int a = live ? A.moff[q] : 0, m = live ? A.moff[q + 1] - a : 0;
    T z[MM], w[MM][kMaxRank];
    {
      double p1s[MM];
#pragma unroll
      for (int j = 0; j < MM; ++j) p1s[j] = j < m ? (double)Fv[A.out_pos[A.mcol[a + j]]] : 0.0;
      const double *cq = A.mcoef + ((size_t)cand * A.n_multi + (live ? q : 0)) * 16;
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        double zz = 0.0;
#pragma unroll
        for (int t = 0; t < MM; ++t) zz += (j < m ? cq[j * 4 + t] : 0.0) * p1s[t];
        z[j] = (T)zz;
#pragma unroll
        for (int e = 0; e < kMaxRank; ++e)
          w[j][e] = (j < m && e < k) ? PcOps<T>::w(A, e0 + e, A.mcol[a + j]) : (T)0;
      }
    }
    for (int c0 = 0; c0 < A.n_mon; c0 += kRows) {
      __syncthreads();  // the previous chunk is consumed
      for (int i = threadIdx.x; i < kRows * (kMaxRank + 1); i += blockDim.x) {
        const int e = i / kRows, r = i - e * kRows, row = c0 + r;  // row < mon_pad
        if (e < kMaxRank)
          s_ur[e][r] = e < k ? PcOps<T>::ur(A, e0 + e, row) : (T)0;
        else
          s_f[r] = (T)((double)Fv[row] * A.inv_r[row]);
      }
      __syncthreads();
      if (!live) continue;
      const int rows = min(kRows, A.n_mon - c0);
      // branch-free: the sub-columns past m read the case's last one (finite) and
      // meet z = 0 and W = 0, which leaves p unchanged
      for (int r0 = 0; r0 < rows; r0 += kPcRows) {
        T l[kPcRows][MM];
#pragma unroll
        for (int u = 0; u < kPcRows; ++u)
#pragma unroll
          for (int j = 0; j < MM; ++j)
            l[u][j] = (T)A.lsdm[(size_t)(a + max(min(j, m - 1), 0)) * A.mon_pad + c0 + r0 + u];
#pragma unroll
        for (int u = 0; u < kPcRows; ++u) {
          const int r = r0 + u, row = c0 + r;
          T p = s_f[r];
#pragma unroll
          for (int j = 0; j < MM; ++j) {
            T lj = l[u][j];
#pragma unroll
            for (int e = 0; e < kMaxRank; ++e) lj = pc_fma(s_ur[e][r], w[j][e], lj);
            p = pc_fma(lj, z[j], p);
          }
          const T ab = p < (T)0 ? -p : p;
          const int key = slot * A.n_mon + row;
          if (r < rows && ab >= thr && pc_better(ab, key, lv[KM - 1], lk[KM - 1]))
            pc_insert(lv, lk, ab, key);
        }
      }
    }
  }
  if (act) pc_store(A, cand, slot, lv, lk);
}

// Level 2: one workgroup per candidate (one wave when the case maxima leave a few
// lists: the hot columns, N-0, guarded and multi-outage cases; four waves over
// every slot otherwise).  With the case maxima the listed slots' entries go to LDS
// and each counts the entries before it (up to kFinRankCap entries); else each
// thread keeps the top KM of the entries of its slots and the block takes one
// entry per round from the heads.
template <int KM>
__global__ void __launch_bounds__(256) k_pc_fin(PcArgs A, dcflow_case *out) {
  __shared__ double s_bv[4];
  __shared__ int s_bk[4];
  const int cand = blockIdx.x, tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  const int nw = blockDim.x / kWave;  // one wave after pruning (few lists), else four
  double lv[KM];
  int lk[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    lv[j] = -1.0;
    lk[j] = kEmptyKey;
  }
  const PcEntry *base = A.ws + (size_t)cand * A.nslots * A.per_case;
  int vstar = 0;
  // with the case maxima: the slots that k_pc_sel lists, the hot columns, then the
  // multi-outage slots (a skipped candidate has no lists); else every slot
  const int32_t *sl = A.cmx ? A.sel + (size_t)cand * (A.n_ctg + 2) : nullptr;
  const int32_t *hl = A.cmx ? A.hotl + (size_t)cand * kHotLd : nullptr;
  const bool skip = A.cmx != nullptr && pc_skip(A, cand, vstar);
  const int n_live = sl && !skip ? sl[0] : 0;
  const int n_hot = hl && !skip ? hl[0] : 0;
  const int n_iter = !sl ? A.nslots : (skip ? 0 : n_live + n_hot + A.n_multi);
  auto slot_of = [&](int i) __attribute__((always_inline)) {
    return !sl ? i
               : (i < n_live ? sl[1 + i]
                             : (i < n_live + n_hot ? 1 + hl[1 + i - n_live]
                                                   : 1 + A.n_ctg + (i - n_live - n_hot)));
  };
  auto emit = [&](int j, double v, int k) __attribute__((always_inline)) {
    dcflow_case e;
    if (k == kEmptyKey) {
      e.load = -1.0;
      e.branch = -1;
      e.outage = -1;
    } else {
      const int slot = k / A.n_mon, row = k - slot * A.n_mon;
      e.load = v;
      e.branch = A.mon[row];
      // slot 0: N-0; 1 + c: contingency column c (branch id, or -2 - g for a
      // generator); after them the multi-outage cases, -2 - n_gen - q
      e.outage = slot == 0 ? -1 : (slot - 1 < A.n_out ? A.out[slot - 1] : -2 - (slot - 1 - A.n_out));
    }
    out[(size_t)cand * A.top_k + j] = e;
  };
  if (A.cmx) {  // block-uniform
    // the listed slots' entries in LDS; a real entry's place is the number of
    // entries before it (the keys are unique); more than kFinRankCap: the rounds
    __shared__ PcEntry s_e[kFinRankCap];
    __shared__ int s_n;
    if (tid == 0) s_n = 0;
    __syncthreads();
    for (int i = tid; i < n_iter; i += blockDim.x) {
      const int s = slot_of(i);
      for (int j = 0; j < A.per_case; ++j) {
        const PcEntry e = base[(size_t)s * A.per_case + j];
        if (e.k == kEmptyKey) break;  // lists are sorted, empties last
        const int pos = atomicAdd(&s_n, 1);
        if (pos < kFinRankCap) s_e[pos] = e;
      }
    }
    __syncthreads();
    const int n = s_n;
    if (n > kFinRankCap) goto rounds;
    for (int i = tid; i < n; i += blockDim.x) {
      const PcEntry e = s_e[i];
      int rank = 0;
      for (int f = 0; f < n; ++f) {
        const PcEntry o = s_e[f];
        rank += pc_better(o.v, o.k, e.v, e.k) ? 1 : 0;
      }
      if (rank < A.top_k) emit(rank, e.v, e.k);
    }
    for (int j = n + tid; j < A.top_k; j += blockDim.x) emit(j, -1.0, kEmptyKey);
    return;
  }
rounds:
  for (int i = tid; i < n_iter; i += blockDim.x) {
    const int s = slot_of(i);
    for (int j = 0; j < A.per_case; ++j) {
      const PcEntry e = base[(size_t)s * A.per_case + j];
      if (e.k == kEmptyKey) break;  // lists are sorted, empties last
      if (!pc_better(e.v, e.k, lv[KM - 1], lk[KM - 1])) break;
      pc_insert(lv, lk, e.v, e.k);
    }
  }
  for (int j = 0; j < A.top_k; ++j) {
    double bv = lv[0];
    int bk = lk[0];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double ov = __shfl_xor(bv, o);
      const int ok = __shfl_xor(bk, o);
      if (pc_better(ov, ok, bv, bk)) {
        bv = ov;
        bk = ok;
      }
    }
    if (lane == 0) {
      s_bv[wv] = bv;
      s_bk[wv] = bk;
    }
    __syncthreads();
    double wbv = s_bv[0];
    int wbk = s_bk[0];
    for (int w = 1; w < nw; ++w)
      if (pc_better(s_bv[w], s_bk[w], wbv, wbk)) {
        wbv = s_bv[w];
        wbk = s_bk[w];
      }
    if (tid == 0) emit(j, wbv, wbk);
    if (wbk != kEmptyKey && lk[0] == wbk) {
#pragma unroll
      for (int t = 0; t < KM - 1; ++t) {
        lv[t] = lv[t + 1];
        lk[t] = lk[t + 1];
      }
      lv[KM - 1] = -1.0;
      lk[KM - 1] = kEmptyKey;
    }
    __syncthreads();
  }
}

template <typename T>
hipError_t run_pc(dcflow_batch *bt, const T *flows, int nvar, int prec, const dcflow_score *scores,
                  int per_case, int top_k, void *ws, dcflow_case *out, hipStream_t s) {
  const dcflow_plan *p = bt->plan;
  PcArgs a;
  a.F = flows;
  a.ld_f = p->ld_er;
  a.nvar = nvar;
  a.off = bt->d_off;
  a.U = bt->d_U;
  a.ld_er = p->ld_er;
  a.W = bt->d_W;
  a.ur32 = bt->d_ur32;
  a.w32 = bt->d_w32;
  a.ld_o = p->ld_o;
  a.mon_pad = p->mon_pad;
  a.n_mon = p->n_mon;
  a.lsd = p->d_lsd;
  a.lsdT = p->d_lsdT;
  a.inv_r = p->d_inv_r;
  a.invden = bt->d_invden;
  a.isl = bt->d_isl;
  a.out_pos = p->d_out_pos;
  a.n_out = p->n_out;
  a.n_ctg = p->n_out + p->n_gen;
  a.n_gen = p->n_gen;
  a.gen_y = p->d_gen_y;
  a.n_multi = p->n_multi;
  a.moff = p->d_moff;
  a.mcol = p->d_mcol;
  a.lsdm = p->d_lsdm;
  a.mcoef = bt->d_mcoef;
  a.mok = bt->d_mok;
  a.mon = p->d_mon;
  a.out = p->d_out;
  a.scores = scores;
  a.per_case = per_case;
  a.top_k = top_k;
  a.nslots = per_case_slots(p);
  a.ws = static_cast<PcEntry *>(ws);
  a.flag = sizeof(T) == 4 && bt->guard_valid ? bt->d_flag : nullptr;
  a.cmx = nullptr;
  a.hotl = nullptr;
  a.sel = nullptr;
  if (case_maxima_supported(p)) {
    // the case maxima of the winners and the hot columns' lists first (the maxima,
    // tau, the hot-column list and the kept slots after the lists in the workspace)
    double *cmx = reinterpret_cast<double *>(
        static_cast<char *>(ws) + pc_list_bytes(bt->n_cand, a.nslots, per_case));
    const hipError_t e = launch_case_maxima(bt, flows, nvar, prec, scores, top_k, cmx, a.ws,
                                            a.nslots, per_case, s);
    if (e != hipSuccess) return e;
    a.cmx = cmx;
    double *tau = cmx + (size_t)bt->n_cand * (p->ld_o + 2);
    a.hotl = reinterpret_cast<const int32_t *>(tau + bt->n_cand);
    a.sel = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(tau) +
                                        worst_aux_bytes(bt->n_cand, 1));
  }
  const unsigned nc = (unsigned)bt->n_cand;
  if (a.cmx) {
    const size_t sel = sizeof(int) * (size_t)((a.n_ctg + 1 + 3) / 4 * 4);
    const size_t staged = sel + sizeof(T) * (size_t)p->mon_pad;
    if (staged <= 64 * 1024) {
      if (per_case <= 4)
        k_pc_sel<T, 4, true><<<dim3(nc), dim3(256), staged, s>>>(a);
      else
        k_pc_sel<T, 16, true><<<dim3(nc), dim3(256), staged, s>>>(a);
    } else {
      if (per_case <= 4)
        k_pc_sel<T, 4, false><<<dim3(nc), dim3(256), sel, s>>>(a);
      else
        k_pc_sel<T, 16, false><<<dim3(nc), dim3(256), sel, s>>>(a);
    }
  } else {
    const dim3 gcols(nc, (unsigned)((a.n_ctg + 1 + 255) / 256));
    if (per_case <= 4)
      k_pc_cols<T, 4><<<gcols, dim3(256), 0, s>>>(a);
    else
      k_pc_cols<T, 16><<<gcols, dim3(256), 0, s>>>(a);
  }
  DCF_CHECK_LAUNCH();
  if (a.n_multi > 0) {
    const dim3 gm(nc, (unsigned)((a.n_multi + 255) / 256));
    if (per_case <= 4)
      k_pc_multi<T, 4><<<gm, dim3(256), 0, s>>>(a);
    else
      k_pc_multi<T, 16><<<gm, dim3(256), 0, s>>>(a);
    DCF_CHECK_LAUNCH();
  }
  const dim3 fin_block(a.cmx && a.n_multi <= 64 ? 64 : 256);
  if (top_k <= 8)
    k_pc_fin<8><<<dim3(nc), fin_block, 0, s>>>(a, out);
  else
    k_pc_fin<16><<<dim3(nc), fin_block, 0, s>>>(a, out);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

}  // namespace

int per_case_slots(const dcflow_plan *p) { return 1 + p->n_out + p->n_gen + p->n_multi; }

size_t pc_list_bytes(int n_cand, int nslots, int per_case) {
  return ((size_t)n_cand * nslots * per_case * sizeof(PcEntry) + 255) / 256 * 256;
}

size_t per_case_workspace(const dcflow_batch *bt, int per_case) {
  const dcflow_plan *p = bt->plan;
  // the lists; with one row band then the case maxima, tau and the hot columns,
  // and the slots of k_pc_sel
  return pc_list_bytes(bt->n_cand, per_case_slots(p), per_case) +
         (case_maxima_supported(p)
              ? (size_t)bt->n_cand * (p->ld_o + 2) * sizeof(double) +
                    worst_aux_bytes(bt->n_cand, 1) +
                    (size_t)bt->n_cand * (p->n_out + p->n_gen + 2) * sizeof(int32_t)
              : 0);
}

hipError_t launch_worst_per_case(dcflow_batch *bt, const void *flows, int nvar, int prec,
                                 const dcflow_score *scores, int per_case, int top_k, void *ws,
                                 dcflow_case *out, hipStream_t s) {
  if (bt->n_cand == 0) return hipSuccess;
  if (prec == DCFLOW_FP64)
    return run_pc<double>(bt, static_cast<const double *>(flows), nvar, prec, scores, per_case,
                          top_k, ws, out, s);
  return run_pc<float>(bt, static_cast<const float *>(flows), nvar, prec, scores, per_case, top_k,
                       ws, out, s);
}

}  // namespace dcflow
