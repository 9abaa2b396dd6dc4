// Internal layout of the plan and batch objects, launch parameters and the
// small device helpers shared by the dcflow kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/dcflow.h"

namespace dcflow {

constexpr int kMaxRank = DCFLOW_MAX_RANK;
constexpr int kMaxSig = DCFLOW_MAX_SPLIT_DEG;  // sensing branches per element
constexpr int kWave = 64;
constexpr int kMaxStepChunks = 16;  // most candidate chunks of the overlapped step
constexpr size_t kXsMaxCols = size_t(1) << 20;  // columns of the BF16 split buffer
constexpr double kIslandTol = 1e-9;   // |LODF denominator| below this: islanding
constexpr int kMultiRows = 256;       // monitored rows per work item of the multi-outage scan
constexpr double kSingularTol = 1e-10; // relative pivot threshold of the k x k solve
// Error guard of the FP32 N-1 scan: a contingency column whose error bound
// (k + 4) u (max |Lsd| + sum_j max |U_j / r| |W_j|) max_v |y_v| (u = 2^-24) exceeds
// this many rating units is taken out of the FP32 tiles and computed in FP64.
constexpr double kGuardTolDefault = 4e-5;

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// True when the precision's flows (and N-1 scan) are FP32.
inline bool prec_is_f32(int prec) { return prec == DCFLOW_FP32 || prec == DCFLOW_BF16 || prec == DCFLOW_BF16X6; }
inline bool prec_valid(int prec) { return prec == DCFLOW_FP64 || prec_is_f32(prec); }

}  // namespace dcflow

// Host-side plan: shapes, index maps and device pointers into the caller's
// workspace.  All device matrices are row-major.
struct dcflow_plan {
  int n, m, slack, n_mon, n_out, n_er;
  int n_gen;   // generator outages: contingency columns n_out .. n_out + n_gen - 1
  int n_ctrl;  // control columns (phase shifters, then HVDC links)
  int n_inj;   // entries per injection vector: n + n_ctrl
  int ld_h;    // columns of Hb / He (n rounded up to 16, the GEMM K step)
  int ld_b;    // leading dimension of Binv (n rounded up to 64, the inversion's block)
  int ld_er;   // rows kept, rounded up to the GEMM M tile (128); U, F, Ht stride
  int ld_o;    // contingency columns rounded up to 64 (>= 64)
  int mon_pad; // monitored rows rounded up to 64
  double rating_scale, rating_offset;  // rating rule (also the feature normaliser)
  // device arrays (all inside the workspace)
  int32_t *d_f, *d_t, *d_adj_off, *d_adj_br;
  double *d_b;
  int32_t *d_mon, *d_out, *d_er, *d_pos_of_br, *d_out_pos;
  int32_t *d_out_f, *d_out_t;  // [n_out + n_gen] column terminals (generator: bus, -1)
  double *d_binv;   // [ld_b][ld_b] inverse of the slack-reduced Laplacian (slack row/col and
                    // the padding: unit)
  double *d_piv;    // [64][64] inverse of the current diagonal block of the inversion
  double *d_hb;     // [m][ld_h] PTDF, all branches
  double *d_ht;     // [n][ld_er] PTDF transposed, kept rows only (node-major)
  double *d_he64;   // [ld_er][ld_h] kept rows of the PTDF, GEMM operand
  float *d_he32;    // [ld_er][ld_h] same in FP32
  __bf16 *d_heb;    // [3][ld_er][ld_h] same split into three BF16 parts (sum = FP64 value to ~2^-24)
  double *d_hdo;    // [m][ld_o] PTDF[:, f_c] - PTDF[:, t_c]; generator columns PTDF[:, bus]
  double *d_lsd;    // [mon_pad][ld_o] (hdo[mon] - [mon == out]) / rating
  double *d_lsdmax; // [ld_o] max over the monitored rows of |d_lsd[:, c]| (error guard)
  float *d_lsd32;   // same in FP32, fragment-major: 16 x 16 blocks [mon_pad/16][ld_o/16], each
                    // 64 lanes x 4 rows in the FP32 MFMA accumulator order (rows 4 (lane/16) + r)
  double *d_lsd64f; // the FP64 values fragment-major the same way, in the FP64 accumulator
                    // order (rows lane/16 + 4 r)
  double *d_lsdT;   // [ld_o][mon_pad] the FP64 values column-major (walks down one column)
  double *d_fbase;  // [m]
  double *d_fber;   // [ld_er] base flows of the kept rows (0 on padding)
  double *d_pbase;  // [ld_h]
  double *d_rating; // [mon_pad]
  double *d_inv_r;  // [mon_pad]
  // control column q of the PTDF: w_q (PTDF[:, a_q] - PTDF[:, c_q]) + d_q e_{br_q}
  int32_t *d_ctl_a, *d_ctl_c, *d_ctl_br;
  double *d_ctl_w, *d_ctl_d;
  double *d_gen_y;  // [max(n_gen, 1)] N-1 coefficient of each generator column: -P_g
  // multi-outage N-1 cases: case q owns sub-columns moff[q] .. moff[q+1]-1, each the
  // contingency column of one of its branches
  int n_multi, n_msub;
  int32_t *d_moff;  // [n_multi + 1]
  int32_t *d_mcol;  // [max(n_msub, 1)] contingency column of each sub-column
  double *d_lsdm;   // [n_msub][mon_pad] seed Lsd of each sub-column, row-contiguous
  float *d_lsdm32;  // same in FP32
  // host copies used for validation and packing
  std::vector<int32_t> f, t, adj_off, adj_br, out, pos_of_br;
  std::vector<uint8_t> is_out;  // per branch: contingency?
};

struct dcflow_batch {
  dcflow_plan *plan;
  int n_cand, n_elem, vmax;
  int64_t packed, padded;
  int kmax;
  int32_t *d_off, *d_kind, *d_id, *d_order;
  uint32_t *d_mask;
  double *d_pnew;
  int32_t *d_nsig;  // [n_elem]
  int32_t *d_sig;   // [n_elem][kMaxSig] signed (branch + 1)
  double *d_U;      // [n_elem][ld_er]
  double *d_W;      // [n_elem][ld_o]
  float *d_ur32;    // [n_elem][mon_pad] FP32 U / r (monitored rows) for the FP32 scan
  float *d_w32;     // [n_elem][ld_o] FP32 W
  float *d_umax;    // [n_elem] max over the monitored rows of |U / r| (error guard)
  uint32_t *d_flag; // [n_cand][ld_o / 32] contingency columns the guard computes in FP64
  int32_t *d_nflag; // [n_cand] number of such columns
  double *d_kinv;   // [n_cand][64]
  double *d_invden; // [n_cand][ld_o]
  uint32_t *d_isl;  // [n_cand][ld_o / 32] islanding contingency bits
  uint32_t *d_status; // [n_cand]
  double *d_z;      // [n_elem][vmax]
  double *d_vmax;   // [n_cand][vmax]
  double *d_f0;     // [vmax][ld_er] shared-injection GEMM output
  __bf16 *d_xs;     // [3][xs_cols][ldx] BF16 parts of x - p_base (BF16 GEMM modes)
  int ldx;          // n_inj rounded up to 32
  size_t xs_cols;   // min(n_cand * vmax, kXsMaxCols)
  int32_t *d_queue; // [16] work-queue counters of the persistent scan
  int max_bands;    // mon_pad / 64: most row bands of one candidate
  double *d_part_m, *d_part_ov;  // [n_cand][max_bands] band partials of the winner pass
  long long *d_part_k;
  int32_t *d_part_nf;
  int nmb;          // row chunks of the multi-outage scan (0 without multi cases); the
                    // band partials hold max_bands + nmb + 1 slots per candidate (the
                    // last for the error guard's FP64 columns)
  double *d_mcoef;  // [n_cand][n_multi][16] -N^-1 of each multi case (z = coef p1_S)
  int32_t *d_mok;   // [n_cand][n_multi] 1 = scored, 0 = islanding or failed candidate
  dcflow_tuning tune;
  hipStream_t aux;                 // second stream of the chunked step (default priority)
  hipEvent_t step_ev[dcflow::kMaxStepChunks + 1];  // fork points and the join of the chunked step
  int n_cu;               // compute units of the device the batch was created on
  size_t lds_max;         // its largest LDS allocation per workgroup (bytes)
  hipGraph_t graph;       // captured step (dcflow_graph_capture), or null
  hipGraphExec_t graph_exec;
  int factored;     // eval_topologies enqueued
  const double *d_pnv;  // [n_elem][pnv_nvar] per-variant new-busbar injections, or null
  int pnv_nvar;
  int flows_prec;   // precision of the last eval_injections (-1 none)
  int flows_nvar;
  int guard_valid;  // d_flag / d_nflag describe the current flows (set by an FP32
                    // n1_score with the guard on, cleared by a new evaluation)
  // column-maximum record of the winner pass (tune.worst_record, plans whose
  // worst-case pass has one row band): per candidate the winner's maxima over
  // the monitored rows of every scored contingency column (0 for the others),
  // then its N-0 maximum, in the scan's element type, and the variant they
  // describe; n1_worst and n1_worst_per_case read them instead of sweeping the
  // winner's tiles again when called with the flows and score records of the
  // n1_score call that wrote them
  void *d_rec;         // [n_cand][ld_o + 1] (8-byte slots), or null
  int32_t *d_rec_var;  // [n_cand]
  int rec_valid;       // set by n1_score with the record on, cleared by a new evaluation
  int rec_prec, rec_nvar;
  const void *rec_flows;
  const void *rec_scores;
  // the host-side state a captured step leaves (restored on each replay)
  struct StepState {
    int factored, flows_prec, flows_nvar, guard_valid, rec_valid, rec_prec, rec_nvar;
    const void *rec_flows;
    const void *rec_scores;
  } graph_state;
};

// What the launch code returns when the tuning's launch shape needs more LDS per
// workgroup than the budget (the entry points report it as DCFLOW_E_TUNING).
constexpr hipError_t kShapeMisfit = hipErrorInvalidConfiguration;

// Returns the launch error of the kernel just enqueued (HIP's last-error slot is
// overwritten by later successful calls, so every launch is checked at once).
#define DCF_CHECK_LAUNCH()                      \
  do {                                          \
    hipError_t e_ = hipGetLastError();          \
    if (e_ != hipSuccess) return e_;            \
  } while (0)

namespace dcflow {

// ------------------------------------------------------------ kernels
// build (a1)
hipError_t launch_build(dcflow_plan *p, hipStream_t s, const double *h_rating,
                        double rscale, double roffset);
// factors (a3)
hipError_t launch_factors(dcflow_batch *b, hipStream_t s);
// injections (a4)
// candidates [c0, c1) (the shared-injection mode: the whole batch only)
hipError_t launch_injections(dcflow_batch *b, const double *inj, int nvar, int shared,
                             int prec, void *flows, int c0, int c1, hipStream_t s);
// score (a5)
// worst-case lists (agg_i) of the winners; worst_bands = row bands of that pass, and
// its workspace: the band lists (worst_list_bytes), then per band a threshold and a
// hot-column list (worst_aux_bytes)
int worst_bands(const dcflow_plan *p);
size_t worst_list_bytes(int n_cand, int nbt, int top_k);
size_t worst_aux_bytes(int n_cand, int nbands);
constexpr int kHotLd = 1 + DCFLOW_WORST_MAX;  // a band's hot columns: number, columns
hipError_t launch_worst(dcflow_batch *b, const void *flows, int nvar, int prec,
                        const dcflow_score *scores, int top_k, void *ws, dcflow_case *out,
                        hipStream_t s);
// The winners' maxima of every contingency column, the N-0 maximum and the top_k-th
// largest of them (the first sweep of the worst-case pass), per candidate in cmx
// [n_cand][ld_o + 2], followed by worst_aux_bytes(n_cand, 1); with pcl, then the
// per-case lists of the hot columns ([n_cand][pc_nslots][per_case] 16-byte entries,
// slot 1 + c).  Only when one row band covers the monitored rows.
bool case_maxima_supported(const dcflow_plan *p);
hipError_t launch_case_maxima(dcflow_batch *b, const void *flows, int nvar, int prec,
                              const dcflow_score *scores, int top_k, double *cmx, void *pcl,
                              int pc_nslots, int per_case, hipStream_t s);
// candidates [c0, c1); a part of the batch runs without the persistent queue and in
// candidate order
hipError_t launch_score(dcflow_batch *b, const void *flows, int nvar, int prec,
                        dcflow_score *out, int c0, int c1, hipStream_t s);

// ------------------------------------------------------ device helpers
// Row of a 16x16 MFMA accumulator block held by lane group g (= lane / 16) in
// register r; the column is lane % 16.  Measured on gfx950: the FP32 16x16x4
// form keeps four consecutive rows per lane group (4g + r), the FP64 16x16x4
// form interleaves them (g + 4r).  The A operand row is lane % 16 and the
// B operand column is lane % 16 (k = lane / 16) for both.
template <typename T>
struct MfmaRow;
template <>
struct MfmaRow<float> {
  static __device__ __forceinline__ constexpr int row(int g, int r) { return 4 * g + r; }
};
template <>
struct MfmaRow<double> {
  static __device__ __forceinline__ constexpr int row(int g, int r) { return g + 4 * r; }
};

// Each shuffle is taken once, by every lane, before any select: a shuffle
// evaluated under divergent control flow reads 0 from inactive partner lanes.
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const T w = __shfl_xor(v, o);
    v = v > w ? v : w;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

}  // namespace dcflow
