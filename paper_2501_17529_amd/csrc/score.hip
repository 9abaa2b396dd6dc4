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
// Generator outages (step 8d, Eq. ptdf_delta) are further columns c >= n_out:
// L~[:, c] is the changed grid's PTDF column of the generator's bus over r, and
// y[c, v] = -P_g for every variant.
//
// L~ is built per 16 x 16 block on the matrix cores, with the shared seed Lsd as
// the accumulator input, U/r as A and W as B (k <= 4: one MFMA, k <= 8: two).
// The FP32 path seeds from an FP32 copy of Lsd stored in accumulator order (one
// 16-byte load per lane and block) and uses the FP32 16x16x4 MFMA; the FP64
// path uses FP64 Lsd and the FP64 16x16x4 MFMA.  A 64-row tile stays in
// registers and is reused for every variant of the launch; the variants' F~ and
// y are staged in LDS.  The scan is VALU work: one FMA plus half a three-way
// absolute maximum per element.
//
// Pass 1 (k_scan_max) writes the per-variant maxima.  Pass 2 (k_scan_win)
// rescans the winning variant once: overload sum, running maximum per lane and
// the tile where each lane first reached it; only the tiles that hold the final
// maximum are built a third time to find the lowest (contingency, branch) key.
// Both passes build tiles with the same code, so the maxima agree bit for bit.
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
__device__ __forceinline__ double tfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
// max(m, |a|, |b|) in one VALU instruction (the compiler does not fold the abs
// modifiers into v_max3_f32 on its own).  Inputs are FMA results (canonical).
__device__ __forceinline__ float absmax3(float m, float a, float b) {
  float r;
  asm("v_max3_f32 %0, %1, |%2|, |%3|" : "=v"(r) : "v"(m), "v"(a), "v"(b));
  return r;
}
// (FP64 has no three-operand maximum: the pair's maximum first, so that the
// running maximum waits on one instruction per pair, not two)
__device__ __forceinline__ double absmax3(double m, double a, double b) {
  return __builtin_fmax(m, __builtin_fmax(__builtin_fabs(a), __builtin_fabs(b)));
}

// acc + max(|a|, 1) + max(|b|, 1) in four VALU instructions (the compiler's fmax
// spends three per element, and it puts a wait state after each asm statement)
__device__ __forceinline__ float add_absmax1(float acc, float a, float b) {
  float t, u;
  asm("v_max_f32 %1, |%3|, 1.0\n\tv_max_f32 %2, |%4|, 1.0\n\t"
      "v_add_f32 %0, %0, %1\n\tv_add_f32 %0, %0, %2"
      : "+v"(acc), "=&v"(t), "=&v"(u) : "v"(a), "v"(b));
  return acc;
}
__device__ __forceinline__ double add_absmax1(double acc, double a, double b) {
  return acc + (__builtin_fmax(__builtin_fabs(a), 1.0) + __builtin_fmax(__builtin_fabs(b), 1.0));
}

// running maximum of non-negative values in LDS: their IEEE bit patterns order
// like the values, so an unsigned integer atomic max suffices
__device__ __forceinline__ void lds_max_nonneg(float *p, float v) {
  atomicMax(reinterpret_cast<unsigned int *>(p), __float_as_uint(v));
}
__device__ __forceinline__ void lds_max_nonneg(double *p, double v) {
  atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

// one entry of a band's worst-case list: load, key (row for N-0, (c + 1) n_mon + row)
struct WEntry {
  double v;
  int k, pad;
};

// kernel arguments shared by both passes
struct ScanArgs {
  const void *F;  // [n_cand][nvar][ld_f] flows of the kept rows (T)
  int ld_f, nvar;
  const int32_t *off;
  const double *U;  // [n_elem][ld_er]
  int ld_er;
  const double *W;  // [n_elem][ld_o]
  int ld_o;
  const double *invden;   // [n_cand][ld_o]
  const uint32_t *isl;    // [n_cand][ld_o / 32]
  const uint32_t *status; // [n_cand]
  const double *lsd;      // [mon_pad][ld_o]
  const float *lsd32;     // fragment-major FP32 copy
  const double *lsd64f;   // fragment-major FP64 copy
  const double *inv_r;    // [mon_pad]
  const float *ur32;      // [n_elem][mon_pad] FP32 U / r
  const float *w32;       // [n_elem][ld_o] FP32 W
  int n_mon, mon_pad;
  const int32_t *out_pos;
  int n_out;
  int n_ctg;              // n_out branch columns, then the generator columns
  const double *gen_y;    // [n_ctg - n_out] -P_g of each generator column
  const int32_t *mon, *out;
  double *vmax;  // [n_cand][vmax_ld]
  int vmax_ld;
  dcflow_score *res;
  int rchunk;     // rows per LDS chunk (multiple of 64)
  int band_rows;  // rows per work item (a multiple of rchunk)
  int single;     // one variant: pass 2 alone
  // work items: (candidate, band of rchunk monitored rows), band-major so that the
  // workgroups in flight share one band of the seed in L2; candidates in queue order
  // (descending rank) within a band
  int n_cand, nbands;
  const int32_t *order;  // [n_cand] queue order, or null: candidates cand0, cand0 + 1, ...
  int cand0;
  int persistent;        // resident workgroups take items from a queue
  int32_t *queue;        // counters: [variant group] for pass 1, [kQueueWin] for pass 2
  // per-band partial results of pass 2 ([n_cand][nbands])
  double *part_m;      // band maximum
  long long *part_k;   // lowest key attaining it in the band
  double *part_ov;     // overload sum of the band
  int32_t *part_nf;    // nonfinite flows of the winning variant seen in the band
  // worst-case lists (dcflow_n1_worst)
  const dcflow_score *scores;  // [n_cand] winners of a preceding n1_score
  int top_k;
  WEntry *wpart;       // [n_cand][nbt][top_k] band lists of dcflow_n1_worst
  double *cmx_out;     // k_scan_colmax, non-null: per candidate the column maxima [ld_o]
                       // (-1 for unscored columns), the N-0 maximum and tau ([ld_o + 2]);
                       // one band must cover every monitored row
  double *tau;         // [n_cand][nbands] lower bounds of the bands' top_k-th case
  int32_t *hotl;       // [n_cand][nbands][kHotLd] the band's hot columns: their number,
                       // then the columns (see scan_colmax_item)
  WEntry *pcl;         // two-level lists: [n_cand][pc_nslots][per_case] per-case lists
                       // (slot 1 + c for contingency column c), or null: one list
  int pc_nslots, per_case;
  // multi-outage N-1 cases (scanned apart, in row chunks of kMultiRows)
  int n_multi;
  const int32_t *moff, *mcol;   // case q: sub-columns moff[q] .. moff[q+1]-1
  const double *lsdm;           // [n_msub][mon_pad] seeds
  const float *lsdm32;
  const double *mcoef;          // [n_cand][n_multi][16]
  const int32_t *mok;           // [n_cand][n_multi]
  int nmb;                      // row chunks per candidate (0: no multi cases)
  int nbt;                      // partial slots per candidate: nbands row bands, then nmb
                                // chunks, then ng guard slots
  // error guard of the FP32 scan (null / 0 in FP64 and with the guard off)
  const uint32_t *flag;         // [n_cand][ld_o / 32] columns computed in FP64 instead
  const int32_t *nflag;         // [n_cand] their number
  int ng;                       // 1: the last partial slot holds the guarded columns
  // column-maximum record of the winner (see dcflow_batch::d_rec): [n_cand][ld_o + 1] T
  void *rec = nullptr;          // k_scan_win writes it, k_scan_colmax may read it
  int32_t *rec_var = nullptr;   // [n_cand] the variant each candidate's record describes
  int rec_atomic = 0;           // k_scan_win: several bands per candidate accumulate their
                                // maxima (the record was cleared first)
  int rec_use = 0;              // k_scan_colmax: take the maxima of the candidates whose
                                // record names their winner
  int rec_sel = 0;              // k_rec_select has done those candidates already
  int32_t *hot_q = nullptr;     // [1 + n_cand nbands] items whose entries at or above tau
                                // outgrew k_scan_hot's LDS: their number, then the items
  int hot_cap = 0;              // entries k_scan_hot keeps in LDS (at most kHotUnionCap)
};

constexpr int kHotUnionCap = 1024;

constexpr int kQueueWin = 15;  // counter slot of pass 2

// Resident workgroups per CU assumed by the persistent launches (the scan is
// shaped for four; more would only wait, fewer still drain the queue).
constexpr int kPersistPerCu = 4;

// Runs body(cand, band) for this workgroup's work items: its own (blockIdx.x) or,
// in persistent mode, queue positions taken one at a time until none are left.
template <typename F>
__device__ __forceinline__ void for_each_item(const ScanArgs &A, int slot, F body) {
  const int n_items = A.n_cand * A.nbands;
  auto run = [&](int q) __attribute__((always_inline)) {
    const int band = q / A.n_cand, i = q - band * A.n_cand;
    body(A.order ? A.order[i] : A.cand0 + i, band);
  };
  if (!A.persistent) {
    run(blockIdx.x);
    return;
  }
  __shared__ int s_pos;
  while (true) {
    __syncthreads();  // the previous item is done with shared memory
    if (threadIdx.x == 0) s_pos = atomicAdd(A.queue + slot, 1);
    __syncthreads();
    const int pos = s_pos;
    if (pos >= n_items) break;
    run(pos);
  }
}

// running maximum of non-negative doubles in global memory (bit patterns order
// like the values)
__device__ __forceinline__ void global_max_nonneg(double *p, double v) {
  atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ void global_max_nonneg(float *p, float v) {
  atomicMax(reinterpret_cast<unsigned int *>(p), __float_as_uint(v));
}

template <typename T>
struct ScanCfg;
// Wave tile: RB row blocks of 16 by TN columns (FP32 64 x 64, FP64 32 x 64: the
// same 32 accumulator values per lane; the FP64 shape reads 8 F~ and 4 y values
// per variant and lane instead of 16 and 2)
template <>
struct ScanCfg<float> {
  static constexpr int RB = 4, TN = 64;
};
template <>
struct ScanCfg<double> {
  static constexpr int RB = 2, TN = 64;
};

// Position of chunk row rr in the staged F~ array: the rows that a block leaves
// in register r of lane group g must sit at 16-row offset 4 g + r.
__device__ __forceinline__ int fs_pos(float *, int rr) { return rr; }
__device__ __forceinline__ int fs_pos(double *, int rr) {
  const int i16 = rr & 15;
  return (rr - i16) + (i16 >> 2) + 4 * (i16 & 3);
}

// A (U / r) and B (W) fragments of k-step h: lane group g supplies element
// 4 h + g.  The loads are unconditional (issued together, never waited on in a
// branch): every lane reads a valid element of the batch (clamped to the
// candidate's last one, and to the first element of the batch when the
// candidate has none), and frag_mask zeroes the fragments past k only where
// the MFMA consumes them.  The FP32 path reads U / r and W rounded to FP32 once
// per evaluation (the same values the FP64 products would round to).
template <int RB, int NB>
__device__ __forceinline__ void update_frags(double (&af)[RB], double (&bfr)[NB], const ScanArgs &A,
                                             int e0, int k, int h, int rowbase, int colbase, int g,
                                             int li) {
  const int e = h * 4 + g;
  const int es = max(e0 + (e < k ? e : k - 1), 0);
  const double *u = A.U + (size_t)es * A.ld_er;
  const double *w = A.W + (size_t)es * A.ld_o;
#pragma unroll
  for (int a = 0; a < RB; ++a) {
    const int row = rowbase + a * 16 + li;
    af[a] = u[row] * A.inv_r[row];
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) bfr[b] = w[colbase + b * 16 + li];
}
template <int RB, int NB>
__device__ __forceinline__ void update_frags(float (&af)[RB], float (&bfr)[NB], const ScanArgs &A,
                                             int e0, int k, int h, int rowbase, int colbase, int g,
                                             int li) {
  const int e = h * 4 + g;
  const int es = max(e0 + (e < k ? e : k - 1), 0);
  const float *u = A.ur32 + (size_t)es * A.mon_pad;
  const float *w = A.w32 + (size_t)es * A.ld_o;
#pragma unroll
  for (int a = 0; a < RB; ++a) af[a] = u[rowbase + a * 16 + li];
#pragma unroll
  for (int b = 0; b < NB; ++b) bfr[b] = w[colbase + b * 16 + li];
}
template <typename T, int RB, int NB>
__device__ __forceinline__ void frag_mask(T (&af)[RB], T (&bfr)[NB], int k, int h, int g) {
  const bool on = h * 4 + g < k;
#pragma unroll
  for (int a = 0; a < RB; ++a) af[a] = on ? af[a] : (T)0;
#pragma unroll
  for (int b = 0; b < NB; ++b) bfr[b] = on ? bfr[b] : (T)0;
}

// A tile of L~ in MFMA accumulator form (RB x NB blocks of 16 x 16: f4 in FP32,
// d4 in FP64).  L[a][b][r] is row 16 a + MfmaRow(g, r), column 16 b + li of the
// tile.
template <typename T>
struct TileOf;
template <>
struct TileOf<float> {
  typedef f4 blk;
  static constexpr int RB = ScanCfg<float>::RB, NB = ScanCfg<float>::TN / 16;
};
template <>
struct TileOf<double> {
  typedef d4 blk;
  static constexpr int RB = ScanCfg<double>::RB, NB = ScanCfg<double>::TN / 16;
};

// The seed blocks of a tile (fragment-major copies of Lsd: per 16 x 16 block the
// 64 lanes' accumulator values in a row), loaded into the MFMA accumulators.
template <typename B, int RB, int NB>
__device__ __forceinline__ void tile_load_seed(B (&c)[RB][NB], const B *base, int ld_o,
                                               int rowbase, int colbase, int lane) {
  const B *seed = base + ((size_t)(rowbase / 16) * (ld_o / 16) + colbase / 16) * kWave + lane;
  const size_t rstride = (size_t)(ld_o / 16) * kWave;
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) c[a][b] = seed[a * rstride + b * kWave];
}
__device__ __forceinline__ const f4 *seed_of(const ScanArgs &A, float) {
  return reinterpret_cast<const f4 *>(A.lsd32);
}
__device__ __forceinline__ const d4 *seed_of(const ScanArgs &A, double) {
  return reinterpret_cast<const d4 *>(A.lsd64f);
}
// One k step of L = seed + (U / r) W on the matrix cores.
__device__ __forceinline__ f4 mfma_step1(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4 mfma_step1(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename T, typename B, int RB, int NB>
__device__ __forceinline__ void tile_mfma_step(B (&c)[RB][NB], const T (&fa)[RB],
                                               const T (&fb)[NB]) {
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) c[a][b] = mfma_step1(fa[a], fb[b], c[a][b]);
}
// L~ for the tile at (rowbase, colbase): the seed blocks, then per k step (one
// for k <= 4, two for k <= 8; wave-uniform) its fragments and MFMAs.
template <typename T, int RB, int NB>
__device__ __forceinline__ void build_tile(T (&L)[RB][NB][4], const ScanArgs &A, int e0, int k,
                                           int rowbase, int colbase, int g, int li, int lane) {
  typename TileOf<T>::blk c[RB][NB];
  T fa[RB], fb[NB];
  tile_load_seed(c, seed_of(A, (T)0), A.ld_o, rowbase, colbase, lane);
  // raised issue priority through the fragment loads and MFMAs: the build of one
  // wave goes ahead of the VALU sweeps of the others on its SIMD, whose work then
  // fills the MFMA cycles (measured about 1% faster in both precisions)
  __builtin_amdgcn_s_setprio(1);
  for (int h = 0; h * 4 < k; ++h) {  // wave-uniform
    update_frags(fa, fb, A, e0, k, h, rowbase, colbase, g, li);
    frag_mask(fa, fb, k, h, g);
    tile_mfma_step(c, fa, fb);
  }
  __builtin_amdgcn_s_setprio(0);
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) L[a][b][r] = c[a][b][r];
}

// F~ of monitored row `row` for one variant (the same expression in every pass)
template <typename T>
__device__ __forceinline__ T ftilde(const T *Fv, const double *inv_r, int row, int n_mon,
                                    bool &nonfinite) {
  if (row >= n_mon) return (T)0;
  const double fv = (double)Fv[row];
  if (!finite_bits(fv)) nonfinite = true;
  return (T)(fv * inv_r[row]);
}

// y = F'[c] / den_c for a branch column, -P_g for a generator column (times the
// stored 1/den of 1, or 0 for a candidate whose correction failed)
template <typename T>
__device__ __forceinline__ T ycol(const T *Fv, const ScanArgs &A, int cand, int c, bool &nonfinite) {
  if (c >= A.n_out) {
    if (c >= A.n_ctg) return (T)0;
    return (T)(A.gen_y[c - A.n_out] * A.invden[(size_t)cand * A.ld_o + c]);
  }
  const double fv = (double)Fv[A.out_pos[c]];
  if (!finite_bits(fv)) nonfinite = true;
  return (T)(fv * A.invden[(size_t)cand * A.ld_o + c]);
}

// reported id of contingency column c: the branch id, -2 - g for generator g,
// -1 for the N-0 case (c < 0)
__device__ __forceinline__ int outage_id(const ScanArgs &A, int c) {
  if (c < 0) return -1;
  return c < A.n_out ? A.out[c] : -2 - (c - A.n_out);
}

// True for a contingency column that the error guard takes out of the FP32 tiles
// of this candidate (its y is zero there and its elements are not scored; the
// guard kernels compute the column in FP64).
__device__ __forceinline__ bool guarded(const ScanArgs &A, int cand, int c) {
  return A.flag != nullptr && ((A.flag[(size_t)cand * (A.ld_o / 32) + c / 32] >> (c % 32)) & 1u);
}

// ---------------------------------------------------------------- pass 1
// Row strides (in elements) of pass 1's variant-minor LDS arrays: y uses VC + 1
// (odd, so that the 16 columns a read touches fall in different banks); F~ uses
// VC + 1 too, or in FP64 with an even VC, VC + 2, so that each pair of variants is
// one aligned 16-byte read (ds_read_b128 takes a 16-bit offset: one base address
// per tile for all F~ reads; its 4 row groups read broadcast addresses).
template <typename T, int VC>
struct VStride {
  static constexpr bool pair = sizeof(T) == 8 && VC % 2 == 0;
  static constexpr int y = VC + 1;
  static constexpr int f = pair ? VC + 2 : VC + 1;
};

// One variant of a tile: p = L~ y + F~ and the running maximum of |p| (two
// maxima, even and odd row blocks, halve the dependent chain).
template <typename T, int RB, int NB>
__device__ __forceinline__ T sweep_variant(const T (&L)[RB][NB][4], const T (&fr)[RB][4],
                                           const T (&yc)[NB], T m) {
  T m0 = m, m1 = (T)0;
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; r += 2) {
        const T p0 = tfma(L[a][b][r], yc[b], fr[a][r]);
        const T p1 = tfma(L[a][b][r + 1], yc[b], fr[a][r + 1]);
        if (a % 2 == 0)
          m0 = absmax3(m0, p0, p1);
        else
          m1 = absmax3(m1, p0, p1);
      }
  return tmax(m0, m1);
}
// Item (cand, band): maxima of the band's N-0 rows and of its N-1 rows against
// every contingency, for the VC variants of blockIdx.y, merged into vmax by
// atomic maxima (vmax is cleared by k_clear first).
template <typename T, int VC>
__device__ __forceinline__ void scan_max_item(const ScanArgs &A, int cand, int band) {
  constexpr int RB = ScanCfg<T>::RB, TM = 16 * RB, TN = ScanCfg<T>::TN, NB = TN / 16;
  // y and F~ are stored variant-minor (strides VStride), so that every read of the
  // variant loop is one base address per tile plus a compile-time offset
  constexpr int VS = VStride<T, VC>::y, VF = VStride<T, VC>::f;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int ld_o = A.ld_o, rchunk = A.rchunk;
  T *ys = reinterpret_cast<T *>(smem_raw);  // [ld_o][VS]
  T *fs = ys + (size_t)VS * ld_o;           // [rchunk][VF] (ld_o even: 16-byte aligned)
  __shared__ double s_red[4][VC];
  __shared__ int s_nfm;  // bit vi: a non-finite flow of variant vi was read

  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, g = lane / 16, li = lane % 16;
  const int e0 = A.off[cand];
  const int k = A.off[cand + 1] - e0;
  const uint32_t st = A.status[cand];
  const int vbeg = blockIdx.y * VC;
  const int nv = min(VC, A.nvar - vbeg);
  double *vm = A.vmax + (size_t)cand * A.vmax_ld + vbeg;
  if (st & DCFLOW_ST_DISCONNECTED) {
    if (tid < nv && band == 0) global_max_nonneg(vm + tid, __builtin_inf());
    return;
  }
  if (tid == 0) s_nfm = 0;
  const T *F = static_cast<const T *>(A.F) + ((size_t)cand * A.nvar + vbeg) * A.ld_f;
  const int r0 = band * A.band_rows, r1 = min(r0 + A.band_rows, A.mon_pad);
  __syncthreads();

  // y for every contingency column and variant of the launch (0 for the variants
  // past nv), one thread per column with its VC flow reads issued together; the
  // expression is that of ycol
  unsigned nfm = 0;
  for (int c = tid; c < ld_o; c += blockDim.x) {
    T yv[VC];
    if (c >= A.n_out) {
      const T gy = c < A.n_ctg ? (T)(A.gen_y[c - A.n_out] * A.invden[(size_t)cand * ld_o + c])
                               : (T)0;
#pragma unroll
      for (int vi = 0; vi < VC; ++vi) yv[vi] = vi < nv ? gy : (T)0;
    } else {
      const double inv = A.invden[(size_t)cand * ld_o + c];
      const T *Fc = F + A.out_pos[c];
      T fv[VC];
#pragma unroll
      for (int vi = 0; vi < VC; ++vi) fv[vi] = vi < nv ? Fc[(size_t)vi * A.ld_f] : (T)0;
#pragma unroll
      for (int vi = 0; vi < VC; ++vi) {
        if (!finite_bits((double)fv[vi])) nfm |= 1u << vi;
        yv[vi] = (T)((double)fv[vi] * inv);
      }
    }
    const bool gd = guarded(A, cand, c);
#pragma unroll
    for (int vi = 0; vi < VC; ++vi) ys[(size_t)c * VS + vi] = gd ? (T)0 : yv[vi];
  }

  // running maxima of |p| per variant; the N-0 loads enter them while F~ is staged
  T mx[VC];
#pragma unroll
  for (int i = 0; i < VC; ++i) mx[i] = (T)0;
  const int ntc = ld_o / TN;
  for (int rc0 = r0; rc0 < r1; rc0 += rchunk) {
    const int rows = min(rchunk, r1 - rc0);
    __syncthreads();
    // F~ of the chunk's rows (the expression of ftilde), one thread per row with its
    // VC flow reads issued together; the N-0 loads enter the running maxima.  The
    // variants past nv get zeros: the FP64 sweep below runs all VC of them without
    // a branch, so that the compiler can interleave their loads and arithmetic.
    for (int rr = tid; rr < rows; rr += blockDim.x) {
      const int row = rc0 + rr;
      const bool on = row < A.n_mon;
      const double ir = on ? A.inv_r[row] : 0.0;
      T fv[VC];
#pragma unroll
      for (int vi = 0; vi < VC; ++vi) fv[vi] = (on && vi < nv) ? F[(size_t)vi * A.ld_f + row] : (T)0;
      T *dst = fs + (size_t)fs_pos(fs, rr) * VF;
#pragma unroll
      for (int vi = 0; vi < VC; ++vi) {
        if (!finite_bits((double)fv[vi])) nfm |= 1u << vi;
        const T f = (T)((double)fv[vi] * ir);
        dst[vi] = f;
        mx[vi] = tmax(mx[vi], tabs(f));
      }
    }
    __syncthreads();

    const int nt = (rows / TM) * ntc;
    for (int tile = wv; tile < nt; tile += 4) {
      const int tr = tile / ntc, tc = tile - tr * ntc;
      const int rowbase = rc0 + tr * TM, colbase = tc * TN;
      T L[RB][NB][4];
      build_tile(L, A, e0, k, rowbase, colbase, g, li, lane);
      const T *fsb = fs + (size_t)((rowbase - rc0) + 4 * g) * VF;
      const T *ysb = ys + (size_t)(colbase + li) * VS;
      if constexpr (VStride<T, VC>::pair) {
        // FP64: two variants per 16-byte read
#pragma unroll
        for (int vp = 0; vp < VC; vp += 2) {
          T fr[2][RB][4], yc[2][NB];
#pragma unroll
          for (int a = 0; a < RB; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const double2 q = *reinterpret_cast<const double2 *>(&fsb[(a * 16 + r) * VF + vp]);
              fr[0][a][r] = q.x;
              fr[1][a][r] = q.y;
            }
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            yc[0][b] = ysb[b * 16 * VS + vp];
            yc[1][b] = ysb[b * 16 * VS + vp + 1];
          }
          mx[vp] = sweep_variant(L, fr[0], yc[0], mx[vp]);
          mx[vp + 1] = sweep_variant(L, fr[1], yc[1], mx[vp + 1]);
        }
      } else {
#pragma unroll
        for (int vi = 0; vi < VC; ++vi) {
          // FP32 keeps a branch per variant: without it the hoisted LDS reads of the
          // 16 variants overflow its 128-register budget (four waves per SIMD)
          if (sizeof(T) == 4 && vi >= nv) continue;
          T fr[RB][4], yc[NB];
#pragma unroll
          for (int a = 0; a < RB; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) fr[a][r] = fsb[(a * 16 + r) * VF + vi];
#pragma unroll
          for (int b = 0; b < NB; ++b) yc[b] = ysb[b * 16 * VS + vi];
          mx[vi] = sweep_variant(L, fr, yc, mx[vi]);
        }
      }
    }
  }

#pragma unroll
  for (int i = 0; i < VC; ++i) {
    const T m = wave_max(mx[i]);
    if (lane == 0) s_red[wv][i] = (double)m;
  }
  if (nfm) atomicOr(&s_nfm, (int)nfm);
  __syncthreads();
  if (tid < nv) {
    double m = fmax(fmax(s_red[0][tid], s_red[1][tid]), fmax(s_red[2][tid], s_red[3][tid]));
    if ((s_nfm >> tid) & 1) m = __builtin_inf();
    global_max_nonneg(vm + tid, m);
  }
}

template <typename T, int VC, int MINW>
__global__ void __launch_bounds__(256, MINW) k_scan_max(ScanArgs A) {
  for_each_item(A, blockIdx.y, [&](int cand, int band) __attribute__((always_inline)) { scan_max_item<T, VC>(A, cand, band); });
}

// ---------------------------------------------------------------- pass 2
// Item (cand, band) of the winning variant v* (argmin of the pass-1 maxima, the
// lowest index on ties): the band's maximum, the lowest (contingency, branch)
// key attaining it (N-0 rows first: key = row), and its overload sum, written
// as partials that k_scan_fin combines.  Per lane: the running maximum, the
// first tile reaching it and whether a later tile reached it again; only the
// tiles where a lane first reached the band maximum are built again for the key.
// The tiles of a chunk are visited column tile first, so that a wave's consecutive
// tiles share their columns.
//   REC: the item also records the winner's column maxima over the band's rows and
//   its N-0 maximum (A.rec): each lane keeps the maxima of its 4 columns in
//   registers and adds them to the block's LDS maxima only when its column tile
//   changes.  The tile values are those of every other sweep.
template <typename T, bool REC>
__device__ __forceinline__ void scan_win_item(const ScanArgs &A, int cand, int band) {
  constexpr int RB = ScanCfg<T>::RB, TM = 16 * RB, TN = ScanCfg<T>::TN, NB = TN / 16;
  constexpr long long kNoKey = 0x7fffffffffffffffLL;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int ld_o = A.ld_o, rchunk = A.rchunk;
  T *ys = reinterpret_cast<T *>(smem_raw);  // [ld_o]
  T *colw = ys + ld_o;                      // [ld_o] 1 for scored contingencies
  T *fs = colw + ld_o;                      // [rchunk]
  T *cmx = fs + rchunk;                     // REC: [ld_o] the band's column maxima
  __shared__ double s_m0[4], s_m1[4], s_ov[4];
  __shared__ long long s_key[4];
  __shared__ int s_nf, s_vstar;

  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, g = lane / 16, li = lane % 16;
  const int e0 = A.off[cand];
  const int k = A.off[cand + 1] - e0;
  const uint32_t st = A.status[cand];
  const size_t pidx = (size_t)cand * A.nbt + band;
  if (st & DCFLOW_ST_DISCONNECTED) return;  // k_scan_fin writes the record

  if (tid == 0) {
    int best = 0;
    if (!A.single) {
      double bv = A.vmax[(size_t)cand * A.vmax_ld];
      for (int v = 1; v < A.nvar; ++v) {
        const double x = A.vmax[(size_t)cand * A.vmax_ld + v];
        if (x < bv) {
          bv = x;
          best = v;
        }
      }
    }
    s_vstar = best;
    s_nf = 0;
  }
  __syncthreads();
  const int vstar = s_vstar;
  const T *Fv = static_cast<const T *>(A.F) + ((size_t)cand * A.nvar + vstar) * A.ld_f;
  bool nf = false;
  for (int c = tid; c < ld_o; c += blockDim.x) {
    const T y = ycol(Fv, A, cand, c, nf);
    const bool gd = guarded(A, cand, c);
    ys[c] = gd ? (T)0 : y;
    const bool valid =
        c < A.n_ctg && !gd && !((A.isl[(size_t)cand * (ld_o / 32) + c / 32] >> (c % 32)) & 1u);
    colw[c] = valid ? (T)1 : (T)0;
    if (REC) cmx[c] = (T)0;
  }
  const int r0 = band * A.band_rows, r1 = min(r0 + A.band_rows, A.mon_pad);
  // REC: the lane's maxima of its columns of column tile acc_tc (wave-uniform)
  T cacc[NB];
  int acc_tc = -1;
  auto rec_flush = [&]() __attribute__((always_inline)) {
    if (acc_tc >= 0) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int c = acc_tc * TN + b * 16 + li;
        if (colw[c] != (T)0) lds_max_nonneg(&cmx[c], cacc[b]);
      }
    }
  };

  // N-0 rows of the band: maximum and the lowest row attaining it
  T b0 = (T)-1;
  int k0 = 0x7fffffff;
  double ov = 0.0;
  // N-1: running maximum per lane, the first tile (global id) where it was
  // reached, and whether a later tile reached it again
  T run = (T)-1;
  int first = -1, tie = 0;
  const int ntc = ld_o / TN;
  for (int rc0 = r0; rc0 < r1; rc0 += rchunk) {
    const int rows = min(rchunk, r1 - rc0);
    __syncthreads();
    for (int rr = tid; rr < rows; rr += blockDim.x) {
      const int row = rc0 + rr;
      const T fv = ftilde(Fv, A.inv_r, row, A.n_mon, nf);
      fs[fs_pos(fs, rr)] = fv;
      if (row < A.n_mon) {
        const T a = tabs(fv);
        if (a > b0) {  // rows are visited in increasing order per thread
          b0 = a;
          k0 = row;
        }
        ov += fmax((double)a - 1.0, 0.0);
      }
    }
    __syncthreads();

    const int ntr = rows / TM, nt = ntr * ntc;
    for (int tile = wv; tile < nt; tile += 4) {
      // column tile first (with or without the record, so that the overload sums
      // add the same tiles in the same order)
      const int tc = tile / ntr, tr = tile - tc * ntr;
      const int rowbase = rc0 + tr * TM, colbase = tc * TN;
      const int tid_tile = (rowbase / TM) * ntc + tc;
      T L[RB][NB][4];
      build_tile(L, A, e0, k, rowbase, colbase, g, li, lane);
      const T *fsv = fs + (rowbase - rc0) + 4 * g;
      T fr[RB][4], yc[NB];
#pragma unroll
      for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) fr[a][r] = fsv[a * 16 + r];
#pragma unroll
      for (int b = 0; b < NB; ++b) yc[b] = ys[colbase + b * 16 + li];
      // per column: the sum of max(|p|, 1) over the lane's 4 RB rows, less 4 RB, is its
      // overload sum (loads within the rating add exactly 1, so rounding enters only
      // where a row is overloaded, and the difference with 4 RB is exact; a tile
      // without overloads adds 0).  FP64 accumulates it as the elements are made (no
      // tile held in registers: four waves per SIMD); FP32 keeps the tile and sums it
      // only where the lane's part holds an overload (fewer instructions; the same bits)
      constexpr bool kInline = sizeof(T) == 8;
      T mt = (T)0, cm[NB], acc[NB], pv[RB][NB][4];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        cm[b] = (T)0;
        acc[b] = (T)0;
      }
#pragma unroll
      for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int r = 0; r < 4; r += 2) {
            const T p0 = tfma(L[a][b][r], yc[b], fr[a][r]);
            const T p1 = tfma(L[a][b][r + 1], yc[b], fr[a][r + 1]);
            if (REC)
              cm[b] = absmax3(cm[b], p0, p1);
            else
              mt = absmax3(mt, p0, p1);
            if (kInline) {
              acc[b] = add_absmax1(acc[b], p0, p1);
            } else {
              pv[a][b][r] = p0;
              pv[a][b][r + 1] = p1;
            }
          }
      if (REC) {
        const bool same = tc == acc_tc;
        if (!same) rec_flush();
        acc_tc = tc;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          cacc[b] = same ? tmax(cacc[b], cm[b]) : cm[b];
          mt = tmax(mt, cm[b]);
        }
      }
      const bool gt = mt > run;
      tie = gt ? 0 : (mt == run ? 1 : tie);
      first = gt ? tid_tile : first;
      run = gt ? mt : run;
      if (kInline || mt > (T)1) {
        if (!kInline) {
#pragma unroll
          for (int a = 0; a < RB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
              for (int r = 0; r < 4; r += 2)
                acc[b] = add_absmax1(acc[b], pv[a][b][r], pv[a][b][r + 1]);
        }
        T o = (T)0;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          o = tfma(colw[colbase + b * 16 + li], acc[b] - (T)(4 * RB), o);
        ov += (double)o;
      }
    }
  }

  if (REC) rec_flush();

  // ---- band maxima over the block
  {
    const T w0 = wave_max(b0), w1 = wave_max(run);
    const double os = wave_sum(ov);
    if (lane == 0) {
      s_m0[wv] = (double)w0;
      s_m1[wv] = (double)w1;
      s_ov[wv] = os;
    }
    if (nf) s_nf = 1;
  }
  __syncthreads();
  const T M0 = (T)fmax(fmax(s_m0[0], s_m0[1]), fmax(s_m0[2], s_m0[3]));
  const T M1 = (T)fmax(fmax(s_m1[0], s_m1[1]), fmax(s_m1[2], s_m1[3]));
  if (REC) {
    // the LDS maxima are complete after the barrier above
    T *rec = static_cast<T *>(A.rec) + (size_t)cand * (ld_o + 1);
    const T n0 = M0 > (T)0 ? M0 : (T)0;
    if (A.rec_atomic) {
      for (int c = tid; c < ld_o; c += blockDim.x)
        if (cmx[c] > (T)0) global_max_nonneg(&rec[c], cmx[c]);
      if (tid == 0) global_max_nonneg(&rec[ld_o], n0);
    } else {
      for (int c = tid; c < ld_o; c += blockDim.x) rec[c] = cmx[c];
      if (tid == 0) rec[ld_o] = n0;
    }
    if (tid == 0 && band == 0) A.rec_var[cand] = vstar;
  }

  // ---- lowest key attaining the band maximum
  long long bestk = kNoKey;
  if (M0 >= M1) {
    bestk = b0 == M0 ? (long long)k0 : kNoKey;
  } else {
    // a lane that reached the maximum again in a later tile may hide a lower
    // key anywhere: then the wave rebuilds every tile of the band (exact ties only)
    const int t_end = (r1 / TM) * ntc;
    const bool want = run == M1;
    const bool all = __any(want && tie);
    bool done = !want;
    int t = all ? (r0 / TM) * ntc : -1;
    while (true) {
      if (!all) {
        int c = done ? 0x7fffffff : first;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
          const int w = __shfl_xor(c, o);
          c = w < c ? w : c;
        }
        if (c == 0x7fffffff) break;
        t = c;
        done = done || first == t;
      } else if (t >= t_end) {
        break;
      }
      const int tr = t / ntc, tc = t - tr * ntc;
      const int rowbase = tr * TM, colbase = tc * TN;
      T L[RB][NB][4];
      build_tile(L, A, e0, k, rowbase, colbase, g, li, lane);
#pragma unroll
      for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rowbase + a * 16 + MfmaRow<T>::row(g, r);
          bool dummy = false;
          const T fv = ftilde(Fv, A.inv_r, row, A.n_mon, dummy);
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const int c = colbase + b * 16 + li;
            const T p = tfma(L[a][b][r], ys[c], fv);
            const long long key = (long long)(c + 1) * A.n_mon + row;
            if (tabs(p) == M1 && colw[c] != (T)0 && row < A.n_mon && key < bestk) bestk = key;
          }
        }
      if (all) ++t;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const long long w = __shfl_xor(bestk, o);
    bestk = w < bestk ? w : bestk;
  }
  if (lane == 0) s_key[wv] = bestk;
  __syncthreads();
  if (tid == 0) {
    long long k2 = s_key[0];
    for (int w = 1; w < 4; ++w) k2 = s_key[w] < k2 ? s_key[w] : k2;
    A.part_m[pidx] = (double)(M0 > M1 ? M0 : M1);
    A.part_k[pidx] = k2;
    A.part_ov[pidx] = s_ov[0] + s_ov[1] + s_ov[2] + s_ov[3];
    A.part_nf[pidx] = s_nf;
  }
}

template <typename T, int MINW, bool REC>
__global__ void __launch_bounds__(256, MINW) k_scan_win(ScanArgs A) {
  for_each_item(A, kQueueWin, [&](int cand, int band) __attribute__((always_inline)) { scan_win_item<T, REC>(A, cand, band); });
}

// One thread per candidate: combines the band partials into the score record.
__global__ void k_scan_fin(ScanArgs A) {
  const int local = blockIdx.x * blockDim.x + threadIdx.x;
  if (local >= A.n_cand) return;
  const int cand = A.cand0 + local;
  constexpr long long kNoKey = 0x7fffffffffffffffLL;
  const uint32_t st = A.status[cand];
  dcflow_score r;
  if (st & DCFLOW_ST_DISCONNECTED) {
    r.max_load = __builtin_inf();
    r.overload_sum = 0.0;
    r.best_variant = -1;
    r.worst_branch = -1;
    r.worst_outage = -1;
    r.status = st;
    A.res[cand] = r;
    if (A.single) A.vmax[(size_t)cand * A.vmax_ld] = r.max_load;
    return;
  }
  int best = 0, any_inf = 0;
  if (!A.single) {
    double bv = A.vmax[(size_t)cand * A.vmax_ld];
    any_inf = !finite_bits(bv);
    for (int v = 1; v < A.nvar; ++v) {
      const double x = A.vmax[(size_t)cand * A.vmax_ld + v];
      any_inf |= !finite_bits(x);
      if (x < bv) {
        bv = x;
        best = v;
      }
    }
  }
  const double *pm = A.part_m + (size_t)cand * A.nbt;
  const long long *pk = A.part_k + (size_t)cand * A.nbt;
  double M = pm[0], ov = 0.0;
  int nf = 0;
  // row bands, then the chunks of the multi-outage cases
  for (int b = 0; b < A.nbt; ++b) {
    M = fmax(M, pm[b]);
    ov += A.part_ov[(size_t)cand * A.nbt + b];
    nf |= A.part_nf[(size_t)cand * A.nbt + b];
  }
  long long key = kNoKey;
  for (int b = 0; b < A.nbt; ++b)
    if (pm[b] == M && pk[b] < key) key = pk[b];
  // a variant whose flows were not finite was given +inf by pass 1; the
  // winner's own non-finite flows make its maximum +inf
  r.status = st | ((nf || any_inf) ? DCFLOW_ST_NONFINITE : 0u) |
             ((A.nflag != nullptr && A.nflag[cand] > 0) ? DCFLOW_ST_GUARDED : 0u);
  const bool found = key != kNoKey;
  const int c = found ? (int)(key / A.n_mon) - 1 : -1;
  const int row = found ? (int)(key % A.n_mon) : -1;
  r.max_load = nf ? __builtin_inf() : M;
  r.overload_sum = ov;
  r.best_variant = best;
  r.worst_branch = found ? A.mon[row] : -1;
  r.worst_outage = outage_id(A, c);
  A.res[cand] = r;
  if (A.single) A.vmax[(size_t)cand * A.vmax_ld] = r.max_load;
}

// Zeroes n 32-bit words (a kernel, so that a captured graph clears them too).
__global__ void k_zero32(uint32_t *p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Whether n1_score writes the column-maximum record (see dcflow_batch::d_rec).
inline bool record_on(const dcflow_batch *bt) { return bt->tune.worst_record >= 0 && bt->d_rec; }

// Clears the work-queue counters and the per-variant maxima (a kernel, so that a
// captured graph clears them too).
__global__ void k_clear(int32_t *q, int nq, double *vmax, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (size_t)nq) q[i] = 0;
  if (i < n) vmax[i] = 0.0;
}

// ---------------------------------------------------------------- worst cases
// agg_i for the winner (metric-first recompute): the top_k largest loads of
// v* over the band's N-0 rows and valid N-1 cases, ordered by load descending,
// then key ascending (key = row for N-0, (c + 1) n_mon + row for N-1).  Each
// lane keeps a sorted list of KM entries in registers; a tile is examined
// element by element only when its lane maximum reaches the lane's last entry.
// The band's list is then taken from the lanes' heads, one entry per round.
template <typename T>
__device__ __forceinline__ bool better(T v, int k, T w, int kw) {
  return v > w || (v == w && k < kw);
}

template <typename T, int KM>
__device__ __forceinline__ void list_insert(T (&lv)[KM], int (&lk)[KM], T v, int k) {
#pragma unroll
  for (int j = KM - 1; j > 0; --j) {
    const bool up = better(v, k, lv[j - 1], lk[j - 1]);
    const bool here = better(v, k, lv[j], lk[j]);
    lv[j] = up ? lv[j - 1] : (here ? v : lv[j]);
    lk[j] = up ? lk[j - 1] : (here ? k : lk[j]);
  }
  if (better(v, k, lv[0], lk[0])) {
    lv[0] = v;
    lk[0] = k;
  }
}

// Item (cand, band) of the winning variant: the band's column maxima over the
// scored contingency columns and its N-0 maximum.  They are distinct elements, so
// the top_k-th largest of them, tau, bounds the band's top_k-th case from below,
// and they name the band's hot columns (k_scan_hot).  The tiles are built with the
// same code as there, so the values agree bit for bit.
template <typename T>
__device__ __forceinline__ void scan_colmax_item(const ScanArgs &A, int cand, int band) {
  constexpr int RB = ScanCfg<T>::RB, TM = 16 * RB, TN = ScanCfg<T>::TN, NB = TN / 16;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int ld_o = A.ld_o, rchunk = A.rchunk;
  T *ys = reinterpret_cast<T *>(smem_raw);  // [ld_o]
  T *colw = ys + ld_o;                      // [ld_o]
  T *fs = colw + ld_o;                      // [rchunk]
  T *cmx = fs + rchunk;                     // [ld_o] column maxima of the band
  __shared__ T s_n0max;

  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, g = lane / 16, li = lane % 16;
  const int e0 = A.off[cand];
  const int k = A.off[cand + 1] - e0;
  const dcflow_score sc = A.scores[cand];
  const bool skip = (sc.status & (DCFLOW_ST_DISCONNECTED | DCFLOW_ST_NONFINITE)) != 0 ||
                    sc.best_variant < 0 || sc.best_variant >= A.nvar;
  double *co = A.cmx_out ? A.cmx_out + (size_t)cand * (ld_o + 2) : nullptr;
  if (skip) {
    if (tid == 0) A.tau[(size_t)cand * A.nbands + band] = -1.0;
    if (A.hotl && tid == 0) A.hotl[((size_t)cand * A.nbands + band) * kHotLd] = 0;
    if (co)
      for (int c = tid; c < ld_o + 2; c += blockDim.x) co[c] = -1.0;
    return;
  }
  const T *Fv = static_cast<const T *>(A.F) + ((size_t)cand * A.nvar + sc.best_variant) * A.ld_f;
  // the winner pass's record of this winner holds the maxima already
  const bool from_rec = A.rec_use && A.rec_var[cand] == sc.best_variant;
  if (from_rec && A.rec_sel) return;
  const T *rec = from_rec ? static_cast<const T *>(A.rec) + (size_t)cand * (ld_o + 1) : nullptr;
  bool nf = false;
  for (int c = tid; c < ld_o; c += blockDim.x) {
    const bool gd = guarded(A, cand, c);
    if (!from_rec) {
      const T y = ycol(Fv, A, cand, c, nf);
      ys[c] = gd ? (T)0 : y;
    }
    const bool valid =
        c < A.n_ctg && !gd && !((A.isl[(size_t)cand * (ld_o / 32) + c / 32] >> (c % 32)) & 1u);
    colw[c] = valid ? (T)1 : (T)0;
    cmx[c] = from_rec ? rec[c] : (T)0;
  }
  if (tid == 0) s_n0max = from_rec ? rec[ld_o] : (T)0;
  const int r0 = band * A.band_rows, r1 = min(r0 + A.band_rows, A.mon_pad);
  const int ntc = ld_o / TN;
  for (int rc0 = r0; rc0 < (from_rec ? r0 : r1); rc0 += rchunk) {
    const int rows = min(rchunk, r1 - rc0);
    __syncthreads();
    for (int rr = tid; rr < rows; rr += blockDim.x) {
      const int row = rc0 + rr;
      const T fv = ftilde(Fv, A.inv_r, row, A.n_mon, nf);
      fs[fs_pos(fs, rr)] = fv;
      if (row < A.n_mon) lds_max_nonneg(&s_n0max, tabs(fv));
    }
    __syncthreads();
    const int nt = (rows / TM) * ntc;
    for (int tile = wv; tile < nt; tile += 4) {
      const int tr = tile / ntc, tc = tile - tr * ntc;
      const int rowbase = rc0 + tr * TM, colbase = tc * TN;
      T L[RB][NB][4];
      build_tile(L, A, e0, k, rowbase, colbase, g, li, lane);
      const T *fsv = fs + (rowbase - rc0) + 4 * g;
      T fr[RB][4];
#pragma unroll
      for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) fr[a][r] = fsv[a * 16 + r];
      // per column: the maximum over the lane's 16 rows, then over the 4 lane groups
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int c = colbase + b * 16 + li;
        const T yc = ys[c];
        T cm = (T)0;
#pragma unroll
        for (int a = 0; a < RB; ++a)
#pragma unroll
          for (int r = 0; r < 4; r += 2)
            cm = absmax3(cm, tfma(L[a][b][r], yc, fr[a][r]), tfma(L[a][b][r + 1], yc, fr[a][r + 1]));
        cm = tmax(cm, __shfl_xor(cm, 16));
        cm = tmax(cm, __shfl_xor(cm, 32));
        if (g == 0 && colw[c] != (T)0) lds_max_nonneg(&cmx[c], cm);
      }
    }
  }
  __syncthreads();
  // The selection is one wave's (k_scan_colmax runs one item per workgroup and no
  // barrier follows); lane l holds the values of columns l, l + 64, ... and the
  // N-0 maximum is index ld_o.
  if (wv != 0) return;
  const T n0 = s_n0max;
  // tau: top_k rounds of "the largest after the previous one" (ties by index); -1
  // when there are fewer values than top_k
  T prev = (T)0;
  int prev_i = -1;
  bool any = true;
  for (int j = 0; j < A.top_k && any; ++j) {
    T bv = (T)-1;
    int bi = 0x7fffffff;
    for (int c = lane; c <= ld_o; c += kWave) {
      const T v = c < ld_o ? (colw[c] != (T)0 ? cmx[c] : (T)-1) : n0;
      const bool after = j == 0 || v < prev || (v == prev && c > prev_i);
      if (v >= (T)0 && after && (v > bv || (v == bv && c < bi))) {
        bv = v;
        bi = c;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const T ov = __shfl_xor(bv, o);
      const int oi = __shfl_xor(bi, o);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    any = bv >= (T)0;
    prev = bv;
    prev_i = bi;
  }
  const double tau = any ? (double)prev : -1.0;
  if (lane == 0) A.tau[(size_t)cand * A.nbands + band] = tau;
  // The hot columns: the scored columns among the top_k of that order (all scored
  // ones when there are fewer values), in increasing order.  Any other column's
  // entries come after top_k distinct entries of the band (the chosen column
  // maxima and N-0 maximum) in the order of the lists (load descending, key
  // ascending; a column's keys grow with its index and the N-0 keys come first),
  // in either kind of list: the band's top_k, or the top_k of the per-case lists.
  if (A.hotl) {
    int32_t *hl = A.hotl + ((size_t)cand * A.nbands + band) * kHotLd;
    int nh = 0;
    for (int c0 = 0; c0 < ld_o; c0 += kWave) {
      const int c = c0 + lane;
      const bool hot = c < ld_o && colw[c] != (T)0 &&
                       (!any || cmx[c] > prev || (cmx[c] == prev && c <= prev_i));
      const unsigned long long m = __ballot(hot);
      const int pos = nh + __popcll(m & ((1ull << lane) - 1ull));
      if (hot && pos < DCFLOW_WORST_MAX) hl[1 + pos] = c;
      nh += __popcll(m);
    }
    if (lane == 0) hl[0] = min(nh, DCFLOW_WORST_MAX);
  }
  if (co) {
    for (int c = lane; c < ld_o; c += kWave) co[c] = colw[c] != (T)0 ? (double)cmx[c] : -1.0;
    if (lane == 0) {
      co[ld_o] = (double)n0;
      co[ld_o + 1] = tau;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256, 4) k_scan_colmax(ScanArgs A) {
  if (A.hot_q && blockIdx.x == 0 && threadIdx.x == 0) *A.hot_q = 0;  // k_scan_hot's queue
  for_each_item(A, kQueueWin, [&](int cand, int band) __attribute__((always_inline)) { scan_colmax_item<T>(A, cand, band); });
}

// The candidates whose column-maximum record names their winner (one band): the
// selection of scan_colmax_item straight from the record, one wave per candidate
// with the values in registers (lane l: columns l, l + 64, ..., at most 64 NJ;
// the N-0 maximum is index ld_o, lane 0's).  Same tau, hot columns and case
// maxima; the other candidates are left to k_scan_colmax.
//   tau by ranking instead of top_k rounds: the top_k-th of the 64 lane maxima, e,
// is at or before tau in the order (top_k distinct values reach it), so only the
// values at or before e (the survivors, at least top_k) can be tau; each survivor
// counts the survivors before it, and the one with top_k - 1 before it is tau.
// With fewer than top_k lane maxima every value survives.  (More than kSurv
// survivors: the rounds.)
template <typename T, int NJ>
__global__ void __launch_bounds__(256) k_rec_select(ScanArgs A) {
  constexpr int kSurv = 256;
  __shared__ T s_v[4][kSurv];
  __shared__ int s_i[4][kSurv];
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int cand = blockIdx.x * (blockDim.x / kWave) + wv;
  if (cand >= A.n_cand) return;
  const dcflow_score sc = A.scores[cand];
  const bool skip = (sc.status & (DCFLOW_ST_DISCONNECTED | DCFLOW_ST_NONFINITE)) != 0 ||
                    sc.best_variant < 0 || sc.best_variant >= A.nvar;
  if (skip || A.rec_var[cand] != sc.best_variant) return;  // wave-uniform
  const int ld_o = A.ld_o, top_k = A.top_k;
  const T *rec = static_cast<const T *>(A.rec) + (size_t)cand * (ld_o + 1);
  // the scored columns' maxima, -1 elsewhere
  T v[NJ];
#pragma unroll
  for (int q = 0; q < NJ; ++q) {
    const int c = lane + kWave * q;
    const bool valid = c < A.n_ctg && !guarded(A, cand, c) &&
                       !((A.isl[(size_t)cand * (ld_o / 32) + c / 32] >> (c % 32)) & 1u);
    v[q] = valid ? rec[c] : (T)-1;
  }
  const T n0 = rec[ld_o];
  auto val = [&](int q) __attribute__((always_inline)) {
    return q < NJ ? v[q] : (lane == 0 ? n0 : (T)-1);
  };
  auto idx = [&](int q) __attribute__((always_inline)) { return q < NJ ? lane + kWave * q : ld_o; };
  auto wave_sync = []() __attribute__((always_inline)) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  T *sv = s_v[wv];
  int *si = s_i[wv];

  // the lane's best value, its place among the 64, and the threshold e
  T lm = (T)-1;
  int lmi = 0x7fffffff;
#pragma unroll
  for (int q = 0; q <= NJ; ++q) {
    const T x = val(q);
    if (x >= (T)0 && (x > lm || (x == lm && idx(q) < lmi))) {
      lm = x;
      lmi = idx(q);
    }
  }
  sv[lane] = lm;
  si[lane] = lmi;
  wave_sync();
  int r = 0;
  for (int f = 0; f < kWave; ++f) {
    const T o = sv[f];
    const int oi = si[f];
    r += (o > lm || (o == lm && oi < lmi)) ? 1 : 0;
  }
  const bool thr = __popcll(__ballot(lm >= (T)0)) >= top_k;
  T ev = (T)-1;
  int ei = 0x7fffffff;
  if (thr) {
    const int wl = __ffsll((long long)__ballot(lm >= (T)0 && r == top_k - 1)) - 1;
    ev = __shfl(lm, wl);
    ei = __shfl(lmi, wl);
  }
  wave_sync();
  // the survivors, compacted into LDS
  int n_s = 0;
#pragma unroll
  for (int q = 0; q <= NJ; ++q) {
    const T x = val(q);
    const int c = idx(q);
    const bool keep = x >= (T)0 && (!thr || x > ev || (x == ev && c <= ei));
    const unsigned long long m = __ballot(keep);
    const int pos = n_s + __popcll(m & ((1ull << lane) - 1ull));
    if (keep && pos < kSurv) {
      sv[pos] = x;
      si[pos] = c;
    }
    n_s += __popcll(m);
  }
  wave_sync();
  T prev = (T)-1;
  int prev_i = -1;
  bool any;
  if (n_s <= kSurv) {
    any = n_s >= top_k;
    if (any) {
      int found = -1;
      for (int i0 = 0; i0 < n_s; i0 += kWave) {
        const int i = i0 + lane;
        int before = -1;
        if (i < n_s) {
          const T x = sv[i];
          const int c = si[i];
          before = 0;
          for (int f = 0; f < n_s; ++f) {
            const T o = sv[f];
            const int oi = si[f];
            before += (o > x || (o == x && oi < c)) ? 1 : 0;
          }
        }
        const unsigned long long m = __ballot(before == top_k - 1);
        if (m != 0ull && found < 0) found = i0 + __ffsll((long long)m) - 1;
      }
      prev = sv[found];
      prev_i = si[found];
    }
  } else {
    // rounds of "the largest after the previous one" (ties by index)
    prev = (T)0;
    any = true;
    for (int j = 0; j < top_k && any; ++j) {
      T bv = (T)-1;
      int bi = 0x7fffffff;
#pragma unroll
      for (int q = 0; q <= NJ; ++q) {
        const T x = val(q);
        const int c = idx(q);
        const bool after = j == 0 || x < prev || (x == prev && c > prev_i);
        if (x >= (T)0 && after && (x > bv || (x == bv && c < bi))) {
          bv = x;
          bi = c;
        }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const T ov = __shfl_xor(bv, o);
        const int oi = __shfl_xor(bi, o);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      any = bv >= (T)0;
      prev = bv;
      prev_i = bi;
    }
  }
  const double tau = any ? (double)prev : -1.0;
  if (lane == 0) A.tau[(size_t)cand * A.nbands] = tau;
  if (A.hotl) {
    int32_t *hl = A.hotl + (size_t)cand * A.nbands * kHotLd;
    int nh = 0;
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
      const int c = lane + kWave * q;
      const bool hot = v[q] >= (T)0 && (!any || v[q] > prev || (v[q] == prev && c <= prev_i));
      const unsigned long long m = __ballot(hot);
      const int pos = nh + __popcll(m & ((1ull << lane) - 1ull));
      if (hot && pos < DCFLOW_WORST_MAX) hl[1 + pos] = c;
      nh += __popcll(m);
    }
    if (lane == 0) hl[0] = min(nh, DCFLOW_WORST_MAX);
  }
  if (A.cmx_out) {
    double *co = A.cmx_out + (size_t)cand * (ld_o + 2);
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
      const int c = lane + kWave * q;
      if (c < ld_o) co[c] = (double)v[q];
    }
    if (lane == 0) {
      co[ld_o] = (double)n0;
      co[ld_o + 1] = tau;
    }
  }
}

// Item (cand, band) of the winning variant after k_scan_colmax: only the band's hot
// columns (at most 16) can place an entry in the list, so they are gathered into
// one 16-column block (lane column li = the li-th hot column; the padding lanes
// repeat a hot column and are masked) and built on the matrix cores from the same
// seed fragments, U / r and W values as the full tiles: every entry is bit for bit
// the value k_scan_colmax maximised (each MFMA output depends on its own row,
// column and accumulator only).  A wave takes its row blocks G at a time, their
// seed and U / r loads issued together (W is the same for all of them).  Only
// entries at or above tau can reach either kind of list: the chosen column
// maxima and N-0 maximum are top_k entries at or above it, in both.
//   One list (PC false): the N-0 rows (while F~ is staged) and the hot entries at
//   or above tau go to an LDS array, and each counts the entries before it in
//   the list order: its place in the band's list (the keys of real entries are
//   unique).  More than hot_cap such entries: the item is queued for
//   k_scan_hot_lists.
//   Two-level lists (PC true, one band): each lane keeps the KM best rows at or
//   above tau of its own column; the 16 lists of a column (4 row groups x 4 waves)
//   are merged into its per-case list of at most per_case entries (slot 1 + c);
//   the N-0 case is left to the per-case kernels.
template <typename T, int KM, bool PC>
__device__ __forceinline__ void scan_hot_item(const ScanArgs &A, int cand, int band) {
  constexpr int kEmpty = 0x7fffffff;
  constexpr int G = 4;
  constexpr int kUnionCap = PC ? 1 : kHotUnionCap;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int ld_o = A.ld_o, rchunk = A.rchunk;
  T *fs = reinterpret_cast<T *>(smem_raw);  // [rchunk]
  __shared__ T s_y[16], s_tau;
  __shared__ int s_col[16], s_nh, s_rn;
  __shared__ WEntry s_re[kUnionCap];

  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, g = lane / 16, li = lane % 16;
  const int e0 = A.off[cand];
  const int k = A.off[cand + 1] - e0;
  const dcflow_score sc = A.scores[cand];
  const bool skip = (sc.status & (DCFLOW_ST_DISCONNECTED | DCFLOW_ST_NONFINITE)) != 0 ||
                    sc.best_variant < 0 || sc.best_variant >= A.nvar;
  T lv[PC ? KM : 1];
  int lk[PC ? KM : 1];
#pragma unroll
  for (int j = 0; j < (PC ? KM : 1); ++j) {
    lv[j] = (T)-1;
    lk[j] = kEmpty;
  }
  const int32_t *hl = A.hotl + ((size_t)cand * A.nbands + band) * kHotLd;
  const T *Fv = skip ? nullptr
                     : static_cast<const T *>(A.F) + ((size_t)cand * A.nvar + sc.best_variant) * A.ld_f;
  if (tid == 0) {
    s_nh = skip ? 0 : hl[0];
    s_tau = (T)A.tau[(size_t)cand * A.nbands + band];
    s_rn = 0;
  }
  __syncthreads();
  const int nh = s_nh;
  if (tid < 16) {
    const int c = nh > 0 ? hl[1 + (tid < nh ? tid : 0)] : 0;
    bool nf = false;
    s_col[tid] = c;
    s_y[tid] = nh > 0 ? ycol(Fv, A, cand, c, nf) : (T)0;
  }
  // an entry at or above tau joins the LDS array (one list)
  auto keep = [&](T v, int key) __attribute__((always_inline)) {
    const int pos = atomicAdd(&s_rn, 1);
    if (pos < kUnionCap) {
      WEntry e;
      e.v = (double)v;
      e.k = key;
      e.pad = 0;
      s_re[pos] = e;
    }
  };
  if (!skip && (nh > 0 || !PC)) {
    const T tau = s_tau;
    const int r0 = band * A.band_rows, r1 = min(r0 + A.band_rows, A.mon_pad);
    const int steps = (k + 3) / 4;  // at most 2 (k <= DCFLOW_MAX_RANK)
    bool first = true;
    int col = 0;
    T yc = (T)0, b0 = (T)0, b1 = (T)0;
    bool live = false;
    for (int rc0 = r0; rc0 < r1; rc0 += rchunk) {
      const int rows = min(rchunk, r1 - rc0);
      __syncthreads();
      bool nf = false;
      for (int rr = tid; rr < rows; rr += blockDim.x) {
        const int row = rc0 + rr;
        const T fv = ftilde(Fv, A.inv_r, row, A.n_mon, nf);
        fs[fs_pos(fs, rr)] = fv;
        if (!PC && row < A.n_mon && tabs(fv) >= tau) keep(tabs(fv), row);
      }
      __syncthreads();
      if (nh == 0) continue;
      if (first) {
        // the hot column of lane column li and its W fragments (row-independent)
        first = false;
        col = s_col[li];
        yc = s_y[li];
        live = li < nh;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int e = h * 4 + g;
          const int es = max(e0 + (e < k ? e : k - 1), 0);
          T b = sizeof(T) == 4 ? (T)A.w32[(size_t)es * ld_o + col] : (T)A.W[(size_t)es * ld_o + col];
          b = (h < steps && e < k) ? b : (T)0;
          if (h == 0)
            b0 = b;
          else
            b1 = b;
        }
      }
      const typename TileOf<T>::blk *seed = reinterpret_cast<const typename TileOf<T>::blk *>(
          sizeof(T) == 4 ? (const void *)A.lsd32 : (const void *)A.lsd64f);
      const int nrb = rows / 16;
      for (int i0 = wv; i0 < nrb; i0 += 4 * G) {
        typename TileOf<T>::blk c4[G];
        T a0[G], a1[G];
#pragma unroll
        for (int q = 0; q < G; ++q) {
          const int rb = i0 + 4 * q < nrb ? i0 + 4 * q : i0;  // wave-uniform; in bounds
          const int rowbase = rc0 + rb * 16;
          c4[q] = seed[((size_t)(rowbase / 16) * (ld_o / 16) + col / 16) * kWave + g * 16 + col % 16];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int e = h * 4 + g;
            const int es = max(e0 + (e < k ? e : k - 1), 0);
            T a = (T)0;
            if (h < steps) {  // wave-uniform
              if (sizeof(T) == 4)
                a = (T)A.ur32[(size_t)es * A.mon_pad + rowbase + li];
              else
                a = (T)(A.U[(size_t)es * A.ld_er + rowbase + li] * A.inv_r[rowbase + li]);
              a = e < k ? a : (T)0;
            }
            if (h == 0)
              a0[q] = a;
            else
              a1[q] = a;
          }
        }
#pragma unroll
        for (int q = 0; q < G; ++q) {
          if (steps > 0) c4[q] = mfma_step1(a0[q], b0, c4[q]);
          if (steps > 1) c4[q] = mfma_step1(a1[q], b1, c4[q]);
        }
#pragma unroll
        for (int q = 0; q < G; ++q) {
          if (i0 + 4 * q >= nrb) break;  // wave-uniform
          const int rowbase = rc0 + (i0 + 4 * q) * 16;
          const T *fsv = fs + (rowbase - rc0) + 4 * g;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = rowbase + MfmaRow<T>::row(g, r);
            const T v = tabs(tfma(c4[q][r], yc, fsv[r]));
            if (live && row < A.n_mon && v >= tau) {
              if (PC) {
                if (better(v, row, lv[KM - 1], lk[KM - 1])) list_insert(lv, lk, v, row);
              } else {
                keep(v, (col + 1) * A.n_mon + row);
              }
            }
          }
        }
      }
    }
  }
  if (PC) {
    // merge the 16 lists of each hot column; a skipped candidate writes nothing
    if (skip || nh == 0) return;
    T *mv = fs + ((A.rchunk + 1) & ~1);  // [256 lanes][KM] after the F~ chunk
    int *mk = reinterpret_cast<int *>(mv + (size_t)blockDim.x * KM);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      mv[(size_t)tid * KM + j] = lv[j];
      mk[(size_t)tid * KM + j] = lk[j];
    }
    __syncthreads();
    if (tid < nh) {
      // lists of column tid: lanes tid + 16 g of each wave
      int pos[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) pos[q] = 0;
      const int c = s_col[tid];
      WEntry *dst = A.pcl + ((size_t)cand * A.pc_nslots + 1 + c) * A.per_case;
      for (int j = 0; j < A.per_case; ++j) {
        T bv = (T)-1;
        int bk = kEmpty, bq = -1;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int t = (q / 4) * kWave + (q % 4) * 16 + tid;
          if (pos[q] < KM) {
            const T v = mv[(size_t)t * KM + pos[q]];
            const int kk = mk[(size_t)t * KM + pos[q]];
            if (kk != kEmpty && better(v, kk, bv, bk)) {
              bv = v;
              bk = kk;
              bq = q;
            }
          }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (q == bq) ++pos[q];
        WEntry e;
        e.v = bk == kEmpty ? -1.0 : (double)bv;
        e.k = bk == kEmpty ? kEmpty : (1 + c) * A.n_mon + bk;
        e.pad = 0;
        dst[j] = e;
      }
    }
    return;
  }
  // the band's list: each entry of the array counts the entries before it
  __syncthreads();
  const int N = s_rn;
  if (N > A.hot_cap) {
    if (tid == 0) {
      const int q = atomicAdd(A.hot_q, 1);
      A.hot_q[1 + q] = cand * A.nbands + band;
    }
    return;
  }
  WEntry *dst = A.wpart + ((size_t)cand * A.nbt + band) * A.top_k;
  for (int i = tid; i < N; i += blockDim.x) {
    const WEntry e = s_re[i];
    int rank = 0;
    for (int f = 0; f < N; ++f) {
      const WEntry o = s_re[f];
      rank += better(o.v, o.k, e.v, e.k) ? 1 : 0;
    }
    if (rank < A.top_k) dst[rank] = e;
  }
  for (int j = N + tid; j < A.top_k; j += blockDim.x) {
    WEntry e;
    e.v = -1.0;
    e.k = kEmpty;
    e.pad = 0;
    dst[j] = e;
  }
}

// The items k_scan_hot queued (more entries at or above tau than its LDS array
// holds): each lane keeps its KM best entries at or above tau in registers; an
// entry's place in the union of the lanes' lists is its place in the band (a lane
// drops an entry only behind KM better ones of its own).
template <typename T, int KM>
__device__ __forceinline__ void scan_hot_lists_item(const ScanArgs &A, int cand, int band) {
  constexpr bool PC = false;
  constexpr int kEmpty = 0x7fffffff;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int ld_o = A.ld_o, rchunk = A.rchunk;
  T *fs = reinterpret_cast<T *>(smem_raw);  // [rchunk]
  __shared__ T s_bv[4], s_y[16], s_tau;
  __shared__ int s_bk[4], s_col[16], s_nh;

  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, g = lane / 16, li = lane % 16;
  const int e0 = A.off[cand];
  const int k = A.off[cand + 1] - e0;
  const dcflow_score sc = A.scores[cand];
  const bool skip = (sc.status & (DCFLOW_ST_DISCONNECTED | DCFLOW_ST_NONFINITE)) != 0 ||
                    sc.best_variant < 0 || sc.best_variant >= A.nvar;
  T lv[KM];
  int lk[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    lv[j] = (T)-1;
    lk[j] = kEmpty;
  }
  const int32_t *hl = A.hotl + ((size_t)cand * A.nbands + band) * kHotLd;
  const T *Fv = skip ? nullptr
                     : static_cast<const T *>(A.F) + ((size_t)cand * A.nvar + sc.best_variant) * A.ld_f;
  if (tid == 0) {
    s_nh = skip ? 0 : hl[0];
    s_tau = (T)A.tau[(size_t)cand * A.nbands + band];
  }
  __syncthreads();
  const int nh = s_nh;
  if (tid < 16) {
    const int c = nh > 0 ? hl[1 + (tid < nh ? tid : 0)] : 0;
    bool nf = false;
    s_col[tid] = c;
    s_y[tid] = nh > 0 ? ycol(Fv, A, cand, c, nf) : (T)0;
  }
  if (!skip && (nh > 0 || !PC)) {
    const T tau = s_tau;
    const int r0 = band * A.band_rows, r1 = min(r0 + A.band_rows, A.mon_pad);
    for (int rc0 = r0; rc0 < r1; rc0 += rchunk) {
      const int rows = min(rchunk, r1 - rc0);
      __syncthreads();
      bool nf = false;
      for (int rr = tid; rr < rows; rr += blockDim.x) {
        const int row = rc0 + rr;
        const T fv = ftilde(Fv, A.inv_r, row, A.n_mon, nf);
        fs[fs_pos(fs, rr)] = fv;
        if (!PC && row < A.n_mon && tabs(fv) >= tau && better(tabs(fv), row, lv[KM - 1], lk[KM - 1]))
          list_insert(lv, lk, tabs(fv), row);
      }
      __syncthreads();
      if (nh == 0) continue;
      const int col = s_col[li];
      const T yc = s_y[li];
      const bool live = li < nh;
      for (int rb = wv; rb < rows / 16; rb += 4) {
        const int rowbase = rc0 + rb * 16;
        // the seed block of (rowbase, col) in the MFMA accumulator layout, then the
        // k steps with the gathered W values
        typename TileOf<T>::blk c4;
        {
          const typename TileOf<T>::blk *seed =
              reinterpret_cast<const typename TileOf<T>::blk *>(sizeof(T) == 4 ? (const void *)A.lsd32
                                                                               : (const void *)A.lsd64f);
          c4 = seed[((size_t)(rowbase / 16) * (ld_o / 16) + col / 16) * kWave + g * 16 + col % 16];
        }
        for (int h = 0; h * 4 < k; ++h) {  // wave-uniform
          // row li of the block, element 4 h + g (as update_frags, one row and column block)
          const int e = h * 4 + g;
          const int es = max(e0 + (e < k ? e : k - 1), 0);
          T a, b;
          if (sizeof(T) == 4) {
            a = (T)A.ur32[(size_t)es * A.mon_pad + rowbase + li];
            b = (T)A.w32[(size_t)es * ld_o + col];
          } else {
            a = (T)(A.U[(size_t)es * A.ld_er + rowbase + li] * A.inv_r[rowbase + li]);
            b = (T)A.W[(size_t)es * ld_o + col];
          }
          const bool on = e < k;
          a = on ? a : (T)0;
          b = on ? b : (T)0;
          c4 = mfma_step1(a, b, c4);
        }
        const T *fsv = fs + (rowbase - rc0) + 4 * g;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rowbase + MfmaRow<T>::row(g, r);
          const T v = tabs(tfma(c4[r], yc, fsv[r]));
          if (PC) {
            if (live && row < A.n_mon && better(v, row, lv[KM - 1], lk[KM - 1]))
              list_insert(lv, lk, v, row);
          } else {
            const int key = (col + 1) * A.n_mon + row;
            if (live && row < A.n_mon && v >= tau && better(v, key, lv[KM - 1], lk[KM - 1]))
              list_insert(lv, lk, v, key);
          }
        }
      }
    }
  }
  // The band's list.  The lanes' lists hold every entry that can reach it (all at
  // or above tau; a lane drops an entry only behind KM better ones of its own), and
  // the keys of real entries are unique, so an entry's place in the union of the
  // lists is its place in the band: the union goes to LDS and each entry counts
  // the entries before it.  (More than kRankCap entries: rounds of "best head
  // over the block", the winning lane popping.)
  WEntry *dst = A.wpart + ((size_t)cand * A.nbt + band) * A.top_k;
  {
    constexpr int kRankCap = 512;
    __shared__ WEntry s_re[kRankCap];
    __shared__ int s_rn;
    if (tid == 0) s_rn = 0;
    __syncthreads();
    int n = 0;
#pragma unroll
    for (int j = 0; j < KM; ++j) n += lk[j] != kEmpty ? 1 : 0;
    const int base = n > 0 ? atomicAdd(&s_rn, n) : 0;
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j < n && base + j < kRankCap) {
        WEntry e;
        e.v = (double)lv[j];
        e.k = lk[j];
        e.pad = 0;
        s_re[base + j] = e;
      }
    __syncthreads();
    const int N = s_rn;
    if (N <= kRankCap) {
      for (int i = tid; i < N; i += blockDim.x) {
        const WEntry e = s_re[i];
        int rank = 0;
        for (int f = 0; f < N; ++f) {
          const WEntry o = s_re[f];
          rank += better(o.v, o.k, e.v, e.k) ? 1 : 0;
        }
        if (rank < A.top_k) dst[rank] = e;
      }
      for (int j = N + tid; j < A.top_k; j += blockDim.x) {
        WEntry e;
        e.v = -1.0;
        e.k = kEmpty;
        e.pad = 0;
        dst[j] = e;
      }
      return;
    }
  }
  for (int j = 0; j < A.top_k; ++j) {
    T bv = lv[0];
    int bk = lk[0];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const T ov = __shfl_xor(bv, o);
      const int ok = __shfl_xor(bk, o);
      if (better(ov, ok, bv, bk)) {
        bv = ov;
        bk = ok;
      }
    }
    if (lane == 0) {
      s_bv[wv] = bv;
      s_bk[wv] = bk;
    }
    __syncthreads();
    T wbv = s_bv[0];
    int wbk = s_bk[0];
#pragma unroll
    for (int w = 1; w < 4; ++w)
      if (better(s_bv[w], s_bk[w], wbv, wbk)) {
        wbv = s_bv[w];
        wbk = s_bk[w];
      }
    if (tid == 0) {
      WEntry e;
      e.v = wbk == kEmpty ? -1.0 : (double)wbv;
      e.k = wbk;
      e.pad = 0;
      dst[j] = e;
    }
    if (wbk != kEmpty && lk[0] == wbk) {
#pragma unroll
      for (int q = 0; q < KM - 1; ++q) {
        lv[q] = lv[q + 1];
        lk[q] = lk[q + 1];
      }
      lv[KM - 1] = (T)-1;
      lk[KM - 1] = kEmpty;
    }
    __syncthreads();
  }
}

template <typename T, int KM, bool PC>
__global__ void __launch_bounds__(256) k_scan_hot(ScanArgs A) {
  for_each_item(A, kQueueWin, [&](int cand, int band) __attribute__((always_inline)) { scan_hot_item<T, KM, PC>(A, cand, band); });
}

template <typename T, int KM>
__global__ void __launch_bounds__(256) k_scan_hot_lists(ScanArgs A) {
  const int n = *reinterpret_cast<volatile int32_t *>(A.hot_q);
  for (int q = blockIdx.x; q < n; q += gridDim.x) {
    __syncthreads();  // the previous item is done with shared memory
    const int item = A.hot_q[1 + q];
    scan_hot_lists_item<T, KM>(A, item / A.nbands, item % A.nbands);
  }
}

// One wave per candidate: merges the bands' sorted lists into the final list of
// top_k cases.  Up to kRankCap entries in all (the usual case) each real entry
// counts the real entries before it in LDS; else rounds of "best head", lane b
// walking bands b, b + 64, ..., at most kFinBands in all.
constexpr int kFinBandsPerLane = 8, kFinBands = 64 * kFinBandsPerLane;

__global__ void __launch_bounds__(64) k_worst_fin(ScanArgs A, dcflow_case *out) {
  constexpr int kEmpty = 0x7fffffff;
  constexpr int kRankCap = 256;
  __shared__ WEntry s_e[kRankCap];
  const int cand = blockIdx.x, lane = threadIdx.x;
  const WEntry *base = A.wpart + (size_t)cand * A.nbt * A.top_k;
  auto emit = [&](int j, double v, int k) __attribute__((always_inline)) {
    dcflow_case e;
    if (k == kEmpty) {
      e.load = -1.0;
      e.branch = -1;
      e.outage = -1;
    } else {
      const bool n0 = k < A.n_mon;
      const int row = n0 ? k : k % A.n_mon;
      const int c = n0 ? -1 : k / A.n_mon - 1;
      e.load = v;
      e.branch = A.mon[row];
      e.outage = outage_id(A, c);
    }
    out[(size_t)cand * A.top_k + j] = e;
  };
  const int m = A.nbt * A.top_k;
  if (m <= kRankCap) {
    // every list entry in LDS; a real entry's place is the number of real entries
    // before it (the keys are unique)
    for (int i = lane; i < m; i += kWave) s_e[i] = base[i];
    __syncthreads();
    int n_real = 0;
    for (int i0 = 0; i0 < m; i0 += kWave) {
      const int i = i0 + lane;
      const bool real = i < m && s_e[i].k != kEmpty;
      n_real += __popcll(__ballot(real));
      if (!real) continue;
      const WEntry e = s_e[i];
      int rank = 0;
      for (int f = 0; f < m; ++f) {
        const WEntry o = s_e[f];
        rank += (o.k != kEmpty && better(o.v, o.k, e.v, e.k)) ? 1 : 0;
      }
      if (rank < A.top_k) emit(rank, e.v, e.k);
    }
    for (int j = n_real + lane; j < A.top_k; j += kWave) emit(j, -1.0, kEmpty);
    return;
  }
  int pos[kFinBandsPerLane];
#pragma unroll
  for (int q = 0; q < kFinBandsPerLane; ++q) pos[q] = 0;
  for (int j = 0; j < A.top_k; ++j) {
    double bv = -1.0;
    int bk = kEmpty, bq = -1;
#pragma unroll
    for (int q = 0; q < kFinBandsPerLane; ++q) {
      const int b = lane + 64 * q;
      if (b < A.nbt && pos[q] < A.top_k) {
        const WEntry e = base[(size_t)b * A.top_k + pos[q]];
        if (e.k != kEmpty && better(e.v, e.k, bv, bk)) {
          bv = e.v;
          bk = e.k;
          bq = q;
        }
      }
    }
    double wv = bv;
    int wk = bk;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double ov = __shfl_xor(wv, o);
      const int ok = __shfl_xor(wk, o);
      if (better(ov, ok, wv, wk)) {
        wv = ov;
        wk = ok;
      }
    }
    if (bq >= 0 && bk == wk && wk != kEmpty) {
#pragma unroll
      for (int q = 0; q < kFinBandsPerLane; ++q)
        if (q == bq) ++pos[q];
    }
    if (lane == 0) emit(j, wv, wk);
  }
}

// ---------------------------------------------------------- multi-outage cases
// Injection-module step 8c (Sec. IV-D): the N-1 flows of multi-outage case q (branch set S,
// m = |S| <= 4) for variant v are p~ = F~ + sum_j L~[:, c_j] z_j with z = coef_q
// p1[S] (coef_q = -N^-1 from the branch module, c_j the contingency column of the
// j-th branch).  One thread per monitored row builds the m entries L~[row, c_j] =
// Lsd[row, c_j] + (U / r)[row, :] W[:, c_j] once per case and applies them to every
// variant of the workgroup; the cases' z and W columns are staged in LDS,
// kMultiQC cases at a time.
//   MODE 0: per-variant maxima merged into vmax (after pass 1, before pass 2);
//   MODE 1: for v* (the argmin of vmax, as in pass 2) the chunk's maximum, its
//           lowest key ((n_ctg + q + 1) n_mon + row) and overload sum, written to
//           the partial slot nbands + chunk that k_scan_fin combines;
//   MODE 2: for the winner of a score record the chunk's top-KM list, written
//           to the worst-case slot nbands + chunk that k_worst_fin merges.
// The N-0 rows are covered by the band passes.
constexpr int kMultiQC = 32;  // cases staged per round
template <typename T>
struct MultiVc {              // variants per workgroup of the maxima
  static constexpr int v = sizeof(T) == 4 ? 16 : 8;
};

template <typename T>
struct MultiOps;
template <>
struct MultiOps<double> {
  static __device__ __forceinline__ double seed(const ScanArgs &A, int sc, int row) {
    return A.lsdm[(size_t)sc * A.mon_pad + row];
  }
  static __device__ __forceinline__ double ur(const ScanArgs &A, int e, int row) {
    return A.U[(size_t)e * A.ld_er + row] * A.inv_r[row];
  }
  static __device__ __forceinline__ double w(const ScanArgs &A, int e, int c) {
    return A.W[(size_t)e * A.ld_o + c];
  }
};
template <>
struct MultiOps<float> {
  static __device__ __forceinline__ float seed(const ScanArgs &A, int sc, int row) {
    return A.lsdm32[(size_t)sc * A.mon_pad + row];
  }
  static __device__ __forceinline__ float ur(const ScanArgs &A, int e, int row) {
    return A.ur32[(size_t)e * A.mon_pad + row];
  }
  static __device__ __forceinline__ float w(const ScanArgs &A, int e, int c) {
    return A.w32[(size_t)e * A.ld_o + c];
  }
};

template <typename T, int MODE, int KM>
__global__ void __launch_bounds__(256) k_scan_multi(ScanArgs A) {
  constexpr int VC = MODE == 0 ? MultiVc<T>::v : 1;
  constexpr int QC = kMultiQC, MM = DCFLOW_MULTI_MAX;
  constexpr long long kNoKey = 0x7fffffffffffffffLL;
  constexpr int kEmpty = 0x7fffffff;
  __shared__ T zs[QC][VC][MM];
  __shared__ T wsm[QC][MM][kMaxRank];  // W[e][c_j] of the round's cases
  __shared__ int s_m[QC], s_a[QC];
  __shared__ double s_red[4][VC];
  __shared__ double s_ov[4];
  __shared__ long long s_key[4];
  __shared__ T s_bv[4];
  __shared__ int s_bk[4];
  __shared__ int s_vstar;

  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  const int local = blockIdx.x / A.nmb, chunk = blockIdx.x - local * A.nmb;
  const int cand = A.cand0 + local;
  const int e0 = A.off[cand], k = A.off[cand + 1] - e0;
  const int row = chunk * kMultiRows + tid;
  const bool has_row = row < A.n_mon;
  const uint32_t st = A.status[cand];
  const int vbeg = MODE == 0 ? blockIdx.y * VC : 0;
  const int nv = MODE == 0 ? min(VC, A.nvar - vbeg) : 1;
  const size_t slot = (size_t)cand * A.nbt + A.nbands + chunk;

  // the variant of MODE 1 and 2; skip = nothing to scan (the slot still gets
  // an empty partial, so that the merges never read stale values)
  bool skip = (st & DCFLOW_ST_DISCONNECTED) != 0;
  if (MODE == 2) {
    const dcflow_score sc = A.scores[cand];
    skip = skip || (sc.status & DCFLOW_ST_NONFINITE) != 0 || sc.best_variant < 0 ||
           sc.best_variant >= A.nvar;
    if (tid == 0) s_vstar = skip ? 0 : sc.best_variant;
  } else if (MODE == 1 && tid == 0) {
    int best = 0;
    if (!A.single) {
      double bv = A.vmax[(size_t)cand * A.vmax_ld];
      for (int v = 1; v < A.nvar; ++v) {
        const double x = A.vmax[(size_t)cand * A.vmax_ld + v];
        if (x < bv) {
          bv = x;
          best = v;
        }
      }
    }
    s_vstar = best;
  }
  if (MODE == 0 && skip) return;  // pass 1 gave the disconnected candidate +inf
  __syncthreads();
  const int v0 = MODE == 0 ? vbeg : s_vstar;

  T fv[VC];
  T ur[kMaxRank];
#pragma unroll
  for (int i = 0; i < VC; ++i) {
    fv[i] = (T)0;
    if (!skip && has_row && i < nv) {
      bool nf = false;
      fv[i] = ftilde(static_cast<const T *>(A.F) + ((size_t)cand * A.nvar + v0 + i) * A.ld_f,
                     A.inv_r, row, A.n_mon, nf);
    }
  }
#pragma unroll
  for (int e = 0; e < kMaxRank; ++e)
    ur[e] = (!skip && has_row && e < k) ? MultiOps<T>::ur(A, e0 + e, row) : (T)0;

  T mx[VC];
#pragma unroll
  for (int i = 0; i < VC; ++i) mx[i] = (T)-1;
  long long bkey = kNoKey;
  double ov = 0.0;
  T lv[KM];
  int lk[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    lv[j] = (T)-1;
    lk[j] = kEmpty;
  }
  const int n_ctg = A.n_ctg;
  T thr = (T)-1;  // MODE 2: the largest of the candidate's band thresholds
  if (MODE == 2 && A.tau) {
    double t = -1.0;
    for (int b = 0; b < A.nbands; ++b) t = fmax(t, A.tau[(size_t)cand * A.nbands + b]);
    thr = (T)t;
  }
  for (int q0 = 0; q0 < A.n_multi && !skip; q0 += QC) {
    __syncthreads();
    // z of the round's cases for the workgroup's variants
    for (int i = tid; i < QC * VC; i += blockDim.x) {
      const int qq = i / VC, vi = i - qq * VC, q = q0 + qq;
      const bool live = q < A.n_multi && vi < nv && A.mok[(size_t)cand * A.n_multi + q] != 0;
      const int a = live ? A.moff[q] : 0, m = live ? A.moff[q + 1] - a : 0;
      double p1s[MM];
      const T *Fv =
          static_cast<const T *>(A.F) + ((size_t)cand * A.nvar + v0 + (live ? vi : 0)) * A.ld_f;
#pragma unroll
      for (int j = 0; j < MM; ++j)
        p1s[j] = j < m ? (double)Fv[A.out_pos[A.mcol[a + j]]] : 0.0;
      const double *cq = A.mcoef + ((size_t)cand * A.n_multi + (live ? q : 0)) * 16;
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        double z = 0.0;
#pragma unroll
        for (int t = 0; t < MM; ++t) z += live ? cq[j * 4 + t] * p1s[t] : 0.0;
        zs[qq][vi][j] = (T)z;
      }
      if (vi == 0) {
        s_m[qq] = live ? m : 0;
        s_a[qq] = a;
      }
    }
    for (int i = tid; i < QC * MM * kMaxRank; i += blockDim.x) {
      const int qq = i / (MM * kMaxRank), j = (i / kMaxRank) % MM, e = i % kMaxRank;
      const int q = q0 + qq;
      T wv0 = (T)0;
      if (q < A.n_multi && e < k) {
        const int a = A.moff[q];
        if (j < A.moff[q + 1] - a) wv0 = MultiOps<T>::w(A, e0 + e, A.mcol[a + j]);
      }
      wsm[qq][j][e] = wv0;
    }
    __syncthreads();
    if (!has_row) continue;
    const int qn = min(QC, A.n_multi - q0);
    for (int qq = 0; qq < qn; ++qq) {
      const int m = s_m[qq];
      if (m == 0) continue;
      const int a = s_a[qq];
      T lt[MM];
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        lt[j] = (T)0;
        if (j < m) {
          T acc = MultiOps<T>::seed(A, a + j, row);
#pragma unroll
          for (int e = 0; e < kMaxRank; ++e) acc = tfma(ur[e], wsm[qq][j][e], acc);  // ur, W 0 past k
          lt[j] = acc;
        }
      }
      const int q = q0 + qq;
#pragma unroll
      for (int vi = 0; vi < VC; ++vi) {
        T p = fv[vi];
#pragma unroll
        for (int j = 0; j < MM; ++j) p = tfma(lt[j], zs[qq][vi][j], p);
        const T ap = tabs(p);
        if (MODE == 0) {
          mx[vi] = tmax(mx[vi], ap);
        } else if (MODE == 1) {
          if (ap > mx[0]) {  // cases in increasing order: the first hit has the lowest key
            mx[0] = ap;
            bkey = (long long)(n_ctg + q + 1) * A.n_mon + row;
          }
          ov += fmax((double)ap - 1.0, 0.0);
        } else {
          // only entries at or above the candidate's largest band threshold can
          // reach its list (each band has top_k entries at or above its tau)
          const int key = (n_ctg + q + 1) * A.n_mon + row;
          if (ap >= thr && better(ap, key, lv[KM - 1], lk[KM - 1])) list_insert(lv, lk, ap, key);
        }
      }
    }
  }

  if (MODE == 0) {
#pragma unroll
    for (int i = 0; i < VC; ++i) {
      const T m = wave_max(mx[i]);
      if (lane == 0) s_red[wv][i] = (double)m;
    }
    __syncthreads();
    if (tid < nv) {
      const double m = fmax(fmax(s_red[0][tid], s_red[1][tid]), fmax(s_red[2][tid], s_red[3][tid]));
      if (m >= 0.0) global_max_nonneg(A.vmax + (size_t)cand * A.vmax_ld + vbeg + tid, m);
    }
  } else if (MODE == 1) {
    const T wm = wave_max(mx[0]);
    const double os = wave_sum(ov);
    if (lane == 0) {
      s_red[wv][0] = (double)wm;
      s_ov[wv] = os;
    }
    __syncthreads();
    const double M = fmax(fmax(s_red[0][0], s_red[1][0]), fmax(s_red[2][0], s_red[3][0]));
    long long kk = (double)mx[0] == M ? bkey : kNoKey;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const long long w = __shfl_xor(kk, o);
      kk = w < kk ? w : kk;
    }
    if (lane == 0) s_key[wv] = kk;
    __syncthreads();
    if (tid == 0) {
      long long k2 = s_key[0];
      for (int w = 1; w < 4; ++w) k2 = s_key[w] < k2 ? s_key[w] : k2;
      A.part_m[slot] = M;   // -1 when the chunk has no scored case
      A.part_k[slot] = M >= 0.0 ? k2 : kNoKey;
      A.part_ov[slot] = s_ov[0] + s_ov[1] + s_ov[2] + s_ov[3];
      A.part_nf[slot] = 0;
    }
  } else {
    WEntry *dst = A.wpart + slot * A.top_k;
    // the chunk's list: the union of the lanes' lists ranked in LDS (each real entry
    // counts the entries before it; the keys are unique), else rounds
    {
      constexpr int kRankCap = 512;
      __shared__ WEntry s_re[kRankCap];
      __shared__ int s_rn;
      if (tid == 0) s_rn = 0;
      __syncthreads();
      int n = 0;
#pragma unroll
      for (int j = 0; j < KM; ++j) n += lk[j] != kEmpty ? 1 : 0;
      const int base = n > 0 ? atomicAdd(&s_rn, n) : 0;
#pragma unroll
      for (int j = 0; j < KM; ++j)
        if (j < n && base + j < kRankCap) {
          WEntry e;
          e.v = (double)lv[j];
          e.k = lk[j];
          e.pad = 0;
          s_re[base + j] = e;
        }
      __syncthreads();
      const int N = s_rn;
      if (N <= kRankCap) {
        for (int i = tid; i < N; i += blockDim.x) {
          const WEntry e = s_re[i];
          int rank = 0;
          for (int f = 0; f < N; ++f) {
            const WEntry o = s_re[f];
            rank += better(o.v, o.k, e.v, e.k) ? 1 : 0;
          }
          if (rank < A.top_k) dst[rank] = e;
        }
        for (int j = N + tid; j < A.top_k; j += blockDim.x) {
          WEntry e;
          e.v = -1.0;
          e.k = kEmpty;
          e.pad = 0;
          dst[j] = e;
        }
        return;
      }
    }
    for (int j = 0; j < A.top_k; ++j) {
      T bv = lv[0];
      int bk = lk[0];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const T ov2 = __shfl_xor(bv, o);
        const int ok = __shfl_xor(bk, o);
        if (better(ov2, ok, bv, bk)) {
          bv = ov2;
          bk = ok;
        }
      }
      if (lane == 0) {
        s_bv[wv] = bv;
        s_bk[wv] = bk;
      }
      __syncthreads();
      T wbv = s_bv[0];
      int wbk = s_bk[0];
#pragma unroll
      for (int w = 1; w < 4; ++w)
        if (better(s_bv[w], s_bk[w], wbv, wbk)) {
          wbv = s_bv[w];
          wbk = s_bk[w];
        }
      if (tid == 0) {
        WEntry e;
        e.v = wbk == kEmpty ? -1.0 : (double)wbv;
        e.k = wbk;
        e.pad = 0;
        dst[j] = e;
      }
      if (wbk != kEmpty && lk[0] == wbk) {
#pragma unroll
        for (int t = 0; t < KM - 1; ++t) {
          lv[t] = lv[t + 1];
          lk[t] = lk[t + 1];
        }
        lv[KM - 1] = (T)-1;
        lk[KM - 1] = kEmpty;
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- error guard
// The FP32 tile build rounds the seed, U / r and W to FP32 and sums k products
// in FP32: an LODF' entry L carries an error of at most (k + 3) u S (u = 2^-24,
// S = the sum of the magnitudes of its terms), and the N-1 element L y another
// u |L| |y| from y's rounding.  Where a candidate's heavy rerouting makes the
// terms large and cancelling, times a large y = F'[c] / den_c, that product can
// exceed the rating tolerance although every operand is accurate in FP64.
// k_guard bounds it per (candidate, contingency column): S_c <= max |Lsd[:, c]|
// + sum_j max |U_j / r| |W_j[c]| and |y_c| <= max over the variants, so
// E_c = (k + 4) u S_c max_v |y_cv|; columns with E_c above the tolerance are
// flagged.  The FP32 passes give them y = 0 and leave their elements unscored,
// and k_guard_fix computes them in FP64 (seed, U, W and y from the FP64
// factors, the flows as stored): per-variant maxima, the winner's maximum, key
// and overload sum (the last partial slot), or the winner's worst-case list.

// Iterates the flagged columns of a candidate (the same order in every thread).
template <typename F>
__device__ __forceinline__ void for_each_flagged(const ScanArgs &A, int cand, F body) {
  const uint32_t *fw = A.flag + (size_t)cand * (A.ld_o / 32);
  for (int w = 0; w < A.ld_o / 32; ++w) {
    uint32_t bits = fw[w];
    while (bits) {
      const int b = __builtin_ctz(bits);
      bits &= bits - 1;
      body(32 * w + b);
    }
  }
}

// y of a guarded column in FP64 (the stored flow of the contingency row or the
// generator's lost output, times the FP64 inverse denominator)
__device__ __forceinline__ double guard_y(const ScanArgs &A, const float *Fv, int cand, int c) {
  const double inv = A.invden[(size_t)cand * A.ld_o + c];
  return (c < A.n_out ? (double)Fv[A.out_pos[c]] : A.gen_y[c - A.n_out]) * inv;
}

// The LODF' entry of row `row`, column c in FP64 from the FP64 factors.
__device__ __forceinline__ double guard_l(const ScanArgs &A, int e0, int k, const double (&wc)[kMaxRank],
                                          int row, int c) {
  double l = A.lsd[(size_t)row * A.ld_o + c];
  const double ir = A.inv_r[row];
#pragma unroll
  for (int j = 0; j < kMaxRank; ++j)
    if (j < k) l = __builtin_fma(A.U[(size_t)(e0 + j) * A.ld_er + row] * ir, wc[j], l);
  return l;
}

__device__ __forceinline__ void guard_w(const ScanArgs &A, int e0, int k, int c, double (&wc)[kMaxRank]) {
#pragma unroll
  for (int j = 0; j < kMaxRank; ++j) wc[j] = j < k ? A.W[(size_t)(e0 + j) * A.ld_o + c] : 0.0;
}

// One workgroup per candidate of [cand0, cand0 + n_cand): the flag words and count.
__global__ void __launch_bounds__(256)
k_guard(ScanArgs A, const float *__restrict__ umax, const double *__restrict__ lsdmax, double tol,
        uint32_t *__restrict__ flag, int32_t *__restrict__ nflag) {
  __shared__ int s_cnt[4];
  const int cand = A.cand0 + blockIdx.x;
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  const int e0 = A.off[cand], k = A.off[cand + 1] - e0;
  const bool dead = (A.status[cand] & DCFLOW_ST_DISCONNECTED) != 0;
  const int nw = A.ld_o / 32;
  const float *F = static_cast<const float *>(A.F) + (size_t)cand * A.nvar * A.ld_f;
  const double coef = (k + 4) * 0x1p-24;
  int cnt = 0;
  for (int c0 = 0; c0 < A.ld_o; c0 += blockDim.x) {
    const int c = c0 + tid;  // ld_o is a multiple of 64: a wave is all in or all out
    if (c0 + wv * kWave >= A.ld_o) break;
    bool f = false;
    if (!dead && c < A.n_ctg) {
      const double inv = A.invden[(size_t)cand * A.ld_o + c];
      const bool isl = (A.isl[(size_t)cand * nw + c / 32] >> (c % 32)) & 1u;
      if (inv != 0.0 && !isl) {
        double S = lsdmax[c];
        for (int j = 0; j < k; ++j)
          S += (double)umax[e0 + j] * fabs(A.W[(size_t)(e0 + j) * A.ld_o + c]);
        double Y = 0.0;
        if (c < A.n_out) {
          const float *Fc = F + A.out_pos[c];
          for (int v = 0; v < A.nvar; ++v) Y = fmax(Y, fabs((double)Fc[(size_t)v * A.ld_f]));
          Y *= fabs(inv);
        } else {
          Y = fabs(A.gen_y[c - A.n_out] * inv);
        }
        const double E = coef * S * Y;
        // a non-finite bound (non-finite flows) stays in the FP32 passes, which flag it
        f = E > tol && E <= 1.7976931348623157e308;
      }
    }
    const unsigned long long bal = __ballot(f);
    if (lane == 0) {
      flag[(size_t)cand * nw + c / 32] = (uint32_t)bal;
      flag[(size_t)cand * nw + c / 32 + 1] = (uint32_t)(bal >> 32);
    }
    cnt += f ? 1 : 0;
  }
  cnt = wave_sum(cnt);
  if (lane == 0) s_cnt[wv] = cnt;
  __syncthreads();
  if (tid == 0) nflag[cand] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
}

// Per-variant maxima over the guarded columns (merged into vmax by atomic maxima,
// after pass 1 and before the winner is chosen).
__global__ void __launch_bounds__(256) k_guard_max(ScanArgs A) {
  constexpr int GV = 16;
  __shared__ double s_red[4][GV];
  const int cand = A.cand0 + blockIdx.x;
  if (A.nflag[cand] == 0 || (A.status[cand] & DCFLOW_ST_DISCONNECTED)) return;
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  const int e0 = A.off[cand], k = A.off[cand + 1] - e0;
  const float *F = static_cast<const float *>(A.F) + (size_t)cand * A.nvar * A.ld_f;
  for (int v0 = 0; v0 < A.nvar; v0 += GV) {
    const int nv = min(GV, A.nvar - v0);
    double vm[GV];
#pragma unroll
    for (int i = 0; i < GV; ++i) vm[i] = 0.0;
    for_each_flagged(A, cand, [&](int c) {
      double y[GV], wc[kMaxRank];
#pragma unroll
      for (int i = 0; i < GV; ++i) y[i] = i < nv ? guard_y(A, F + (size_t)(v0 + i) * A.ld_f, cand, c) : 0.0;
      guard_w(A, e0, k, c, wc);
      for (int row = tid; row < A.n_mon; row += blockDim.x) {
        const double l = guard_l(A, e0, k, wc, row, c);
        const double ir = A.inv_r[row];
#pragma unroll
        for (int i = 0; i < GV; ++i)
          if (i < nv) {
            const double p = __builtin_fma(l, y[i], (double)F[(size_t)(v0 + i) * A.ld_f + row] * ir);
            vm[i] = fmax(vm[i], fabs(p));
          }
      }
    });
#pragma unroll
    for (int i = 0; i < GV; ++i) {
      const double m = wave_max(vm[i]);
      if (lane == 0) s_red[wv][i] = m;
    }
    __syncthreads();
    if (tid < nv) {
      const double m = fmax(fmax(s_red[0][tid], s_red[1][tid]), fmax(s_red[2][tid], s_red[3][tid]));
      global_max_nonneg(A.vmax + (size_t)cand * A.vmax_ld + v0 + tid, m);
    }
    __syncthreads();
  }
}

// The winner's maximum, lowest key and overload sum over the guarded columns, in
// the candidate's last partial slot (neutral values without guarded columns).
__global__ void __launch_bounds__(256) k_guard_win(ScanArgs A) {
  constexpr long long kNoKey = 0x7fffffffffffffffLL;
  __shared__ double s_m[4], s_ov[4];
  __shared__ long long s_k[4];
  __shared__ int s_vstar;
  const int cand = A.cand0 + blockIdx.x;
  const size_t slot = (size_t)cand * A.nbt + (A.nbt - 1);
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  if (A.nflag[cand] == 0 || (A.status[cand] & DCFLOW_ST_DISCONNECTED)) {
    if (tid == 0) {
      A.part_m[slot] = 0.0;
      A.part_k[slot] = kNoKey;
      A.part_ov[slot] = 0.0;
      A.part_nf[slot] = 0;
    }
    return;
  }
  if (tid == 0) {
    int best = 0;
    if (!A.single) {
      double bv = A.vmax[(size_t)cand * A.vmax_ld];
      for (int v = 1; v < A.nvar; ++v) {
        const double x = A.vmax[(size_t)cand * A.vmax_ld + v];
        if (x < bv) {
          bv = x;
          best = v;
        }
      }
    }
    s_vstar = best;
  }
  __syncthreads();
  const int e0 = A.off[cand], k = A.off[cand + 1] - e0;
  const float *Fv = static_cast<const float *>(A.F) + ((size_t)cand * A.nvar + s_vstar) * A.ld_f;
  double bm = -1.0, ov = 0.0;
  long long bk = kNoKey;
  for_each_flagged(A, cand, [&](int c) {
    double wc[kMaxRank];
    const double y = guard_y(A, Fv, cand, c);
    guard_w(A, e0, k, c, wc);
    for (int row = tid; row < A.n_mon; row += blockDim.x) {
      const double p = __builtin_fma(guard_l(A, e0, k, wc, row, c), y, (double)Fv[row] * A.inv_r[row]);
      const double a = fabs(p);
      const long long key = (long long)(c + 1) * A.n_mon + row;
      if (a > bm || (a == bm && key < bk)) {
        bm = a;
        bk = key;
      }
      ov += fmax(a - 1.0, 0.0);
    }
  });
  const double M = wave_max(bm);
  long long kk = bm == M ? bk : kNoKey;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const long long w = __shfl_xor(kk, o);
    kk = w < kk ? w : kk;
  }
  const double os = wave_sum(ov);
  if (lane == 0) {
    s_m[wv] = M;
    s_k[wv] = kk;
    s_ov[wv] = os;
  }
  __syncthreads();
  if (tid == 0) {
    const double m = fmax(fmax(s_m[0], s_m[1]), fmax(s_m[2], s_m[3]));
    long long key = kNoKey;
    for (int w = 0; w < 4; ++w)
      if (s_m[w] == m && s_k[w] < key) key = s_k[w];
    A.part_m[slot] = m;
    A.part_k[slot] = key;
    A.part_ov[slot] = s_ov[0] + s_ov[1] + s_ov[2] + s_ov[3];
    A.part_nf[slot] = 0;
  }
}

// The winner's top_k cases over the guarded columns: a sorted list in the
// candidate's last band-list slot (empty entries without guarded columns).
template <int KM>
__global__ void __launch_bounds__(256) k_guard_worst(ScanArgs A) {
  constexpr int kEmpty = 0x7fffffff;
  __shared__ double s_bv[4];
  __shared__ int s_bk[4];
  const int cand = blockIdx.x;
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  WEntry *dst = A.wpart + ((size_t)cand * A.nbt + (A.nbt - 1)) * A.top_k;
  const dcflow_score sc = A.scores[cand];
  const bool skip = A.nflag == nullptr || A.nflag[cand] == 0 ||
                    (sc.status & (DCFLOW_ST_DISCONNECTED | DCFLOW_ST_NONFINITE)) != 0 ||
                    sc.best_variant < 0 || sc.best_variant >= A.nvar;
  if (skip) {  // block-uniform: the empty list
    for (int j = tid; j < A.top_k; j += blockDim.x) {
      WEntry e;
      e.v = -1.0;
      e.k = kEmpty;
      e.pad = 0;
      dst[j] = e;
    }
    return;
  }
  double lv[KM];
  int lk[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    lv[j] = -1.0;
    lk[j] = kEmpty;
  }
  {
    const int e0 = A.off[cand], k = A.off[cand + 1] - e0;
    const float *Fv =
        static_cast<const float *>(A.F) + ((size_t)cand * A.nvar + sc.best_variant) * A.ld_f;
    for_each_flagged(A, cand, [&](int c) {
      double wc[kMaxRank];
      const double y = guard_y(A, Fv, cand, c);
      guard_w(A, e0, k, c, wc);
      for (int row = tid; row < A.n_mon; row += blockDim.x) {
        const double p =
            __builtin_fma(guard_l(A, e0, k, wc, row, c), y, (double)Fv[row] * A.inv_r[row]);
        const double a = fabs(p);
        const int key = (c + 1) * A.n_mon + row;
        if (better(a, key, lv[KM - 1], lk[KM - 1])) list_insert(lv, lk, a, key);
      }
    });
  }
  for (int j = 0; j < A.top_k; ++j) {
    double bv = lv[0];
    int bk = lk[0];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double ov = __shfl_xor(bv, o);
      const int ok = __shfl_xor(bk, o);
      if (better(ov, ok, bv, bk)) {
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
#pragma unroll
    for (int w = 1; w < 4; ++w)
      if (better(s_bv[w], s_bk[w], wbv, wbk)) {
        wbv = s_bv[w];
        wbk = s_bk[w];
      }
    if (tid == 0) {
      WEntry e;
      e.v = wbk == kEmpty ? -1.0 : wbv;
      e.k = wbk;
      e.pad = 0;
      dst[j] = e;
    }
    if (wbk != kEmpty && lk[0] == wbk) {
#pragma unroll
      for (int q = 0; q < KM - 1; ++q) {
        lv[q] = lv[q + 1];
        lk[q] = lk[q + 1];
      }
      lv[KM - 1] = -1.0;
      lk[KM - 1] = kEmpty;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launch
constexpr size_t kLdsBudget = 64 * 1024;   // dynamic LDS per workgroup by default
// The wider FP64 variant group of pass 1 may use more where the device allows it
// (gfx950: 160 KB per compute unit); its workgroups then share a unit two at a time.
inline size_t lds_budget(const dcflow_batch *bt, int vc, size_t elem) {
  return (elem == 8 && vc == 16) ? bt->lds_max : kLdsBudget;
}
constexpr size_t kLdsOccupancy = 38 * 1024; // fits four workgroups per CU

// Rows per band: the requested count (a multiple of 64, capped at the padded
// monitored rows) or, by default, the largest multiple of 64 that keeps the
// block within `target` bytes (at least 64 rows).
inline int choose_rchunk(int req, size_t fixed, size_t per_row, int mon_pad, size_t target) {
  int rc = req;
  if (rc <= 0) {
    const size_t cap = target > fixed ? (target - fixed) / per_row : 0;
    rc = (int)(cap / 64 * 64);
    if (rc < 64) rc = 64;
  }
  return rc < mon_pad ? rc : mon_pad;
}

// Rows per work item (band) and per LDS chunk.  The band is the requested count
// or, by default, all monitored rows when the seed block (rows x ld_o values) fits
// a fraction of L2, else about kBandSeed bytes of seed, so that the candidates in
// flight, which all work on one band, share its seed in L2.  The chunk never
// exceeds the band, and the band is a whole number of chunks.
constexpr size_t kSeedL2 = 2u << 20, kBandSeed = 4u << 20;
inline void choose_rows(const dcflow_batch *bt, size_t fixed, size_t per_row, int mon_pad,
                        int ld_o, size_t elem, size_t lds_target, ScanArgs &a) {
  int band = bt->tune.scan_band;
  if (band <= 0) {
    const size_t seed = (size_t)mon_pad * ld_o * elem;
    band = seed <= kSeedL2 ? mon_pad : (int)(kBandSeed / ((size_t)ld_o * elem)) / 64 * 64;
  }
  if (band < 64) band = 64;
  if (band > mon_pad) band = mon_pad;
  int rc = choose_rchunk(bt->tune.scan_rchunk, fixed, per_row, mon_pad, lds_target);
  if (rc > band) rc = band;
  a.rchunk = rc;
  a.band_rows = band < mon_pad ? band / rc * rc : mon_pad;
  a.nbands = (mon_pad + a.band_rows - 1) / a.band_rows;
}

inline int grid_x(const dcflow_batch *bt, const ScanArgs &a) {
  const int items = a.n_cand * a.nbands;
  if (!a.persistent) return items;
  const int resident = bt->n_cu * kPersistPerCu;
  return items < resident ? items : resident;
}

template <typename T, int VC, int MINW>
hipError_t launch_max(const ScanArgs &a0, const dcflow_batch *bt, int nvar, hipStream_t s) {
  ScanArgs a = a0;
  // variant-minor LDS rows (see scan_max_item)
  constexpr int VS = VStride<T, VC>::y, VF = VStride<T, VC>::f;
  const size_t fixed = sizeof(T) * (size_t)VS * a.ld_o;
  choose_rows(bt, fixed, sizeof(T) * VF, a.mon_pad, a.ld_o, sizeof(T), kLdsOccupancy, a);
  const size_t lds = fixed + sizeof(T) * (size_t)VF * a.rchunk;
  if (lds > lds_budget(bt, VC, sizeof(T))) return kShapeMisfit;
  const int ny = (nvar + VC - 1) / VC;
  if (ny > kQueueWin) a.persistent = 0;  // one counter per variant group
  k_scan_max<T, VC, MINW><<<dim3(grid_x(bt, a), ny), dim3(256), lds, s>>>(a);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

// variant-group widths compiled per precision (pass 1)
template <typename T>
struct VcSet;
template <>
struct VcSet<float> {
  static constexpr int v[4] = {16, 8, 4, 1};
};
template <>
struct VcSet<double> {
  static constexpr int v[4] = {16, 8, 4, 1};
};

template <typename T>
hipError_t launch_max_vc(const ScanArgs &a, const dcflow_batch *bt, int nvar, int vc,
                         hipStream_t s) {
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int V0 = VcSet<T>::v[0], V1 = VcSet<T>::v[1], V2 = VcSet<T>::v[2];
  if (vc == V0) return launch_max<T, V0, F32 ? 4 : 2>(a, bt, nvar, s);
  if (vc == V1) return launch_max<T, V1, F32 ? 4 : 2>(a, bt, nvar, s);
  if (vc == V2) return launch_max<T, V2, F32 ? 1 : 2>(a, bt, nvar, s);
  return launch_max<T, 1, 1>(a, bt, nvar, s);
}

inline void set_multi(ScanArgs &a, const dcflow_plan *p, const dcflow_batch *bt) {
  a.n_multi = p->n_multi;
  a.moff = p->d_moff;
  a.mcol = p->d_mcol;
  a.lsdm = p->d_lsdm;
  a.lsdm32 = p->d_lsdm32;
  a.mcoef = bt->d_mcoef;
  a.mok = bt->d_mok;
  a.nmb = bt->nmb;
  a.nbt = 1 + bt->nmb;
  a.flag = nullptr;
  a.nflag = nullptr;
  a.ng = 0;
}

template <typename T>
hipError_t run_scan(dcflow_batch *bt, const T *flows, int nvar, dcflow_score *out, int c0, int c1,
                    hipStream_t s) {
  dcflow_plan *p = bt->plan;
  ScanArgs a;
  a.F = flows;
  a.ld_f = p->ld_er;
  a.nvar = nvar;
  a.off = bt->d_off;
  a.U = bt->d_U;
  a.ld_er = p->ld_er;
  a.W = bt->d_W;
  a.ld_o = p->ld_o;
  a.invden = bt->d_invden;
  a.isl = bt->d_isl;
  a.status = bt->d_status;
  a.lsd = p->d_lsd;
  a.lsd32 = p->d_lsd32;
  a.lsd64f = p->d_lsd64f;
  a.inv_r = p->d_inv_r;
  a.ur32 = bt->d_ur32;
  a.w32 = bt->d_w32;
  a.n_mon = p->n_mon;
  a.mon_pad = p->mon_pad;
  a.out_pos = p->d_out_pos;
  a.n_out = p->n_out;
  a.n_ctg = p->n_out + p->n_gen;
  a.gen_y = p->d_gen_y;
  a.mon = p->d_mon;
  a.out = p->d_out;
  a.vmax = bt->d_vmax;
  a.vmax_ld = bt->vmax;
  a.res = out;
  a.single = nvar == 1;  // one variant: the winner pass alone gives everything
  const bool whole = c0 == 0 && c1 == bt->n_cand;
  a.persistent = whole && bt->tune.persistent ? 1 : 0;
  a.n_cand = c1 - c0;
  a.order = whole ? bt->d_order : nullptr;
  a.cand0 = c0;
  a.queue = bt->d_queue;
  a.part_m = bt->d_part_m;
  a.part_k = bt->d_part_k;
  a.part_ov = bt->d_part_ov;
  a.part_nf = bt->d_part_nf;
  a.rchunk = 0;
  a.band_rows = 0;
  a.nbands = 1;
  a.cmx_out = nullptr;
  set_multi(a, p, bt);
  if (sizeof(T) == 4 && bt->tune.guard_tol >= 0.0) {
    // the error guard of the FP32 scan flags its columns first
    const double tol = bt->tune.guard_tol > 0.0 ? bt->tune.guard_tol : kGuardTolDefault;
    a.flag = bt->d_flag;
    a.nflag = bt->d_nflag;
    a.ng = 1;
    k_guard<<<dim3((unsigned)a.n_cand), dim3(256), 0, s>>>(a, bt->d_umax, p->d_lsdmax, tol,
                                                          bt->d_flag, bt->d_nflag);
    DCF_CHECK_LAUNCH();
  }
  bt->guard_valid = a.ng;
  {
    const size_t nv = a.single ? 0 : (size_t)a.n_cand * bt->vmax;
    const size_t n = nv > (size_t)(kQueueWin + 1) ? nv : (size_t)(kQueueWin + 1);
    k_clear<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(bt->d_queue, kQueueWin + 1,
                                                        bt->d_vmax + (size_t)c0 * bt->vmax, nv);
    DCF_CHECK_LAUNCH();
  }
  if (!a.single) {
    // the requested variant group, else the widest whose y fits the LDS budget
    // with one 64-row band and that the variants fill
    auto fits = [&](int vc) {
      return sizeof(T) * (size_t)(vc + 1) * (p->ld_o + 64) <= lds_budget(bt, vc, sizeof(T));
    };
    int vc = bt->tune.scan_vc;
    bool known = false;
    for (int i = 0; i < 4; ++i) known |= vc == VcSet<T>::v[i];
    if (!known || !fits(vc)) {
      vc = 1;
      for (int i = 2; i >= 0; --i) {
        const int c = VcSet<T>::v[i];
        if (fits(c) && (i == 2 ? nvar > 1 : nvar > VcSet<T>::v[i + 1])) vc = c;
      }
    }
    const hipError_t e = launch_max_vc<T>(a, bt, nvar, vc, s);
    if (e != hipSuccess) return e;
    if (a.nmb > 0) {
      const int ny = (nvar + MultiVc<T>::v - 1) / MultiVc<T>::v;
      k_scan_multi<T, 0, 1><<<dim3((unsigned)((size_t)a.n_cand * a.nmb), ny), dim3(256), 0, s>>>(a);
      DCF_CHECK_LAUNCH();
    }
    if (a.ng) {
      k_guard_max<<<dim3((unsigned)a.n_cand), dim3(256), 0, s>>>(a);
      DCF_CHECK_LAUNCH();
    }
  }
  // y, the column weights and, with the record, the band's column maxima
  const bool rec = record_on(bt);
  const size_t fixed = sizeof(T) * (rec ? 3 : 2) * (size_t)p->ld_o;
  choose_rows(bt, fixed, sizeof(T), p->mon_pad, p->ld_o, sizeof(T), kLdsOccupancy, a);
  if (a.nbands > bt->max_bands) return hipErrorInvalidValue;
  a.nbt = a.nbands + a.nmb + a.ng;
  const size_t lds = fixed + sizeof(T) * (size_t)a.rchunk;
  if (lds > kLdsBudget) return kShapeMisfit;
  constexpr int kWinWaves = 4;
  if (rec) {
    a.rec = bt->d_rec;
    a.rec_var = bt->d_rec_var;
    a.rec_atomic = a.nbands > 1;
    if (a.rec_atomic) {
      // the bands' maxima accumulate: the candidates' records start at zero
      const size_t n = (size_t)(c1 - c0) * (p->ld_o + 1) * sizeof(T) / 4;
      k_zero32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
          reinterpret_cast<uint32_t *>(static_cast<T *>(bt->d_rec) + (size_t)c0 * (p->ld_o + 1)), n);
      DCF_CHECK_LAUNCH();
    }
    k_scan_win<T, kWinWaves, true><<<dim3(grid_x(bt, a)), dim3(256), lds, s>>>(a);
  } else {
    k_scan_win<T, kWinWaves, false><<<dim3(grid_x(bt, a)), dim3(256), lds, s>>>(a);
  }
  DCF_CHECK_LAUNCH();
  if (a.nmb > 0) {
    k_scan_multi<T, 1, 1><<<dim3((unsigned)((size_t)a.n_cand * a.nmb)), dim3(256), 0, s>>>(a);
    DCF_CHECK_LAUNCH();
  }
  if (a.ng) {
    k_guard_win<<<dim3((unsigned)a.n_cand), dim3(256), 0, s>>>(a);
    DCF_CHECK_LAUNCH();
  }
  k_scan_fin<<<(a.n_cand + 255) / 256, 256, 0, s>>>(a);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

// Row bands of the worst-case pass: a fixed rule (all rows when the FP32 seed is
// small, else about kBandSeed of FP64 seed, at most kFinBands bands), so that the
// workspace size depends on the batch alone.
inline int worst_band_rows(const dcflow_plan *p) {
  const int mon_pad = p->mon_pad;
  if ((size_t)mon_pad * p->ld_o * sizeof(float) <= kSeedL2) return mon_pad;
  int band = (int)(kBandSeed / ((size_t)p->ld_o * sizeof(double))) / 64 * 64;
  if (band < 64) band = 64;
  const int least = (mon_pad + kFinBands - 1) / kFinBands;
  if (band < least) band = (least + 63) / 64 * 64;
  return band < mon_pad ? band : mon_pad;
}

template <typename T>
hipError_t run_worst(dcflow_batch *bt, const T *flows, int nvar, const dcflow_score *scores,
                     int top_k, bool rec_use, void *ws, dcflow_case *out, hipStream_t s,
                     double *cmx_out = nullptr, void *pcl = nullptr, int pc_nslots = 0,
                     int per_case = 0) {
  dcflow_plan *p = bt->plan;
  ScanArgs a;
  a.F = flows;
  a.ld_f = p->ld_er;
  a.nvar = nvar;
  a.off = bt->d_off;
  a.U = bt->d_U;
  a.ld_er = p->ld_er;
  a.W = bt->d_W;
  a.ld_o = p->ld_o;
  a.invden = bt->d_invden;
  a.isl = bt->d_isl;
  a.status = bt->d_status;
  a.lsd = p->d_lsd;
  a.lsd32 = p->d_lsd32;
  a.lsd64f = p->d_lsd64f;
  a.inv_r = p->d_inv_r;
  a.ur32 = bt->d_ur32;
  a.w32 = bt->d_w32;
  a.n_mon = p->n_mon;
  a.mon_pad = p->mon_pad;
  a.out_pos = p->d_out_pos;
  a.n_out = p->n_out;
  a.n_ctg = p->n_out + p->n_gen;
  a.gen_y = p->d_gen_y;
  a.mon = p->d_mon;
  a.out = p->d_out;
  a.vmax = nullptr;
  a.vmax_ld = 0;
  a.res = nullptr;
  a.single = 0;
  a.persistent = 0;
  a.n_cand = bt->n_cand;
  a.order = bt->d_order;
  a.cand0 = 0;
  a.queue = nullptr;
  a.part_m = nullptr;
  a.part_k = nullptr;
  a.part_ov = nullptr;
  a.part_nf = nullptr;
  a.scores = scores;
  a.top_k = top_k;
  a.wpart = static_cast<WEntry *>(ws);
  a.cmx_out = cmx_out;
  a.pcl = static_cast<WEntry *>(pcl);
  a.pc_nslots = pc_nslots;
  a.per_case = per_case;
  if (rec_use) {
    a.rec = bt->d_rec;
    a.rec_var = bt->d_rec_var;
    a.rec_use = 1;
  }
  set_multi(a, p, bt);
  const size_t fixed = sizeof(T) * 2 * (size_t)p->ld_o;  // k_scan_colmax: y and the weights
  int band = worst_band_rows(p);
  int rc = choose_rchunk(0, fixed, sizeof(T), p->mon_pad, kLdsOccupancy);
  if (rc > band) rc = band;
  a.rchunk = rc;
  a.band_rows = band;  // a multiple of 64; the last chunk of a band may be shorter
  a.nbands = worst_bands(p);
  // with the error guard's flags of the score call, a last slot holds the list of
  // the guarded columns (empty where a candidate has none)
  if (sizeof(T) == 4 && bt->guard_valid) {
    a.flag = bt->d_flag;
    a.nflag = bt->d_nflag;
  }
  a.ng = a.flag ? 1 : 0;
  a.nbt = a.nbands + a.nmb + a.ng;
  if (a.nbt > kFinBands) return hipErrorInvalidValue;
  const size_t lds = fixed + sizeof(T) * (size_t)rc;
  if (lds > kLdsBudget) return kShapeMisfit;
  const dim3 grid((unsigned)((size_t)a.n_cand * a.nbands));
  // the thresholds and hot-column lists first (after the band lists in the
  // workspace, or after the case maxima of the two-level lists)
  a.tau = cmx_out ? cmx_out + (size_t)bt->n_cand * (p->ld_o + 2)
                  : reinterpret_cast<double *>(static_cast<char *>(ws) +
                                               worst_list_bytes(bt->n_cand, a.nbt, top_k));
  a.hotl = reinterpret_cast<int32_t *>(a.tau + (size_t)bt->n_cand * a.nbands);
  a.hot_q = a.hotl + (size_t)bt->n_cand * a.nbands * kHotLd;
  // DCFLOW_HOT_CAP lowers the entries k_scan_hot keeps in LDS (tests use it to run
  // the queued list kernel on small batches)
  a.hot_cap = kHotUnionCap;
  if (const char *env = std::getenv("DCFLOW_HOT_CAP")) {
    const long long v = std::atoll(env);
    if (v >= 0 && v < kHotUnionCap) a.hot_cap = (int)v;
  }
  if (a.rec_use && a.nbands == 1 && p->ld_o <= 16 * kWave) {
    // the candidates whose record names their winner, one wave each
    const dim3 gs((unsigned)((bt->n_cand + 3) / 4));
    if (p->ld_o <= 4 * kWave)
      k_rec_select<T, 4><<<gs, dim3(256), 0, s>>>(a);
    else if (p->ld_o <= 8 * kWave)
      k_rec_select<T, 8><<<gs, dim3(256), 0, s>>>(a);
    else
      k_rec_select<T, 16><<<gs, dim3(256), 0, s>>>(a);
    DCF_CHECK_LAUNCH();
    a.rec_sel = 1;
  }
  k_scan_colmax<T><<<grid, dim3(256), lds + sizeof(T) * (size_t)p->ld_o, s>>>(a);
  DCF_CHECK_LAUNCH();
  // the hot columns: F~ in row chunks of at most 1024 (and the per-case merge area)
  a.rchunk = std::min(band, 1024);
  const size_t lhot = sizeof(T) * (size_t)(((a.rchunk + 1) & ~1));
  if (cmx_out) {
    if (!pcl) return hipSuccess;  // the case maxima only
    if (per_case <= 4)
      k_scan_hot<T, 4, true><<<grid, dim3(256), lhot + 256 * 4 * (sizeof(T) + 4), s>>>(a);
    else
      k_scan_hot<T, 16, true><<<grid, dim3(256), lhot + 256 * 16 * (sizeof(T) + 4), s>>>(a);
    DCF_CHECK_LAUNCH();
    return hipSuccess;
  }
  k_scan_hot<T, 1, false><<<grid, dim3(256), lhot, s>>>(a);
  DCF_CHECK_LAUNCH();
  // the items whose entries at or above tau outgrew the LDS array (usually none)
  if (top_k <= 8)
    k_scan_hot_lists<T, 8><<<dim3(64), dim3(256), lhot, s>>>(a);
  else
    k_scan_hot_lists<T, 16><<<dim3(64), dim3(256), lhot, s>>>(a);
  DCF_CHECK_LAUNCH();
  if (a.nmb > 0) {
    const dim3 gm((unsigned)((size_t)a.n_cand * a.nmb));
    if (top_k <= 8)
      k_scan_multi<T, 2, 8><<<gm, dim3(256), 0, s>>>(a);
    else
      k_scan_multi<T, 2, 16><<<gm, dim3(256), 0, s>>>(a);
    DCF_CHECK_LAUNCH();
  }
  if (a.ng) {
    if (top_k <= 8)
      k_guard_worst<8><<<dim3(bt->n_cand), dim3(256), 0, s>>>(a);
    else
      k_guard_worst<16><<<dim3(bt->n_cand), dim3(256), 0, s>>>(a);
    DCF_CHECK_LAUNCH();
  }
  k_worst_fin<<<dim3(bt->n_cand), dim3(64), 0, s>>>(a, out);
  DCF_CHECK_LAUNCH();
  return hipSuccess;
}

}  // namespace

size_t worst_list_bytes(int n_cand, int nbt, int top_k) {
  return ((size_t)n_cand * nbt * top_k * sizeof(WEntry) + 255) / 256 * 256;
}

int worst_bands(const dcflow_plan *p) {
  const int band = worst_band_rows(p);
  return (p->mon_pad + band - 1) / band;
}

// Whether the column-maximum record describes these flows and score records (the
// n1_score call that wrote it); candidates whose record names another variant than
// their score record are swept as without it.
bool record_matches(const dcflow_batch *bt, const void *flows, int nvar, int prec,
                    const dcflow_score *scores) {
  return bt->d_rec && bt->rec_valid && bt->rec_prec == prec && bt->rec_nvar == nvar &&
         bt->rec_flows == flows && bt->rec_scores == scores && worst_bands(bt->plan) == 1;
}

hipError_t launch_worst(dcflow_batch *bt, const void *flows, int nvar, int prec,
                        const dcflow_score *scores, int top_k, void *ws, dcflow_case *out,
                        hipStream_t s) {
  if (bt->n_cand == 0) return hipSuccess;
  const bool ru = record_matches(bt, flows, nvar, prec, scores);
  if (prec == DCFLOW_FP64)
    return run_worst<double>(bt, static_cast<const double *>(flows), nvar, scores, top_k, ru, ws,
                             out, s);
  return run_worst<float>(bt, static_cast<const float *>(flows), nvar, scores, top_k, ru, ws, out,
                          s);
}

bool case_maxima_supported(const dcflow_plan *p) { return worst_bands(p) == 1; }

hipError_t launch_case_maxima(dcflow_batch *bt, const void *flows, int nvar, int prec,
                              const dcflow_score *scores, int top_k, double *cmx_out,
                              void *pcl, int pc_nslots, int per_case, hipStream_t s) {
  if (bt->n_cand == 0) return hipSuccess;
  if (!case_maxima_supported(bt->plan)) return hipErrorInvalidValue;
  const bool ru = record_matches(bt, flows, nvar, prec, scores);
  if (prec == DCFLOW_FP64)
    return run_worst<double>(bt, static_cast<const double *>(flows), nvar, scores, top_k, ru,
                             nullptr, nullptr, s, cmx_out, pcl, pc_nslots, per_case);
  return run_worst<float>(bt, static_cast<const float *>(flows), nvar, scores, top_k, ru, nullptr,
                          nullptr, s, cmx_out, pcl, pc_nslots, per_case);
}

size_t worst_aux_bytes(int n_cand, int nbands) {
  // per band: tau (double), then the hot-column lists, then the queue of k_scan_hot
  const size_t items = (size_t)n_cand * nbands;
  return (items * (sizeof(double) + kHotLd * sizeof(int32_t)) + (items + 1) * sizeof(int32_t) +
          255) / 256 * 256;
}

hipError_t launch_score(dcflow_batch *bt, const void *flows, int nvar, int prec, dcflow_score *out,
                        int c0, int c1, hipStream_t s) {
  if (c1 <= c0) return hipSuccess;
  const hipError_t e =
      prec == DCFLOW_FP64
          ? run_scan<double>(bt, static_cast<const double *>(flows), nvar, out, c0, c1, s)
          : run_scan<float>(bt, static_cast<const float *>(flows), nvar, out, c0, c1, s);
  // the record describes these flows and records once every chunk of the batch is
  // enqueued (a part of the batch comes from dcflow_step, which scores them all)
  bt->rec_valid = e == hipSuccess && record_on(bt);
  bt->rec_prec = prec;
  bt->rec_nvar = nvar;
  bt->rec_flows = flows;
  bt->rec_scores = out;
  return e;
}

}  // namespace dcflow
