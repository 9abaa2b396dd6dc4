/*
 * dcflow — batched DC loadflow over grid-topology candidates on one MI355X.
 *
 * C ABI of the solver library (libdcflow.so, gfx950).  The operations follow
 * Westerbeck et al., "Accelerated DC loadflow solver for topology
 * optimization":
 *
 *   dcflow_build_ptdf       Sec. II, Def. of the PTDF (PTDF' B' = C_w', slack
 *                           column zero) restricted to the rows the screen
 *                           needs, plus base flows (Eq. ptdf_times_nodal_inj).
 *   dcflow_eval_topologies  Sec. III-C branch module: per candidate, the PTDF
 *                           corrections for bus splits (Def. eq_bsdf,
 *                           Eq. bsdf_application) and remedial outages
 *                           (Def. eq_modf), joined into one k x k solve, and
 *                           the LODF denominators of every contingency in the
 *                           changed grid (Def. eq_lodf); for multi-outage N-1
 *                           cases the inverse of each case's MODF system
 *                           (step 5).
 *   dcflow_eval_injections  Sec. III-C injection module step 8a: post-change
 *                           N-0 flows F' = PTDF' P for every injection
 *                           variant (Eq. ptdf_times_nodal_inj).
 *   dcflow_n1_score         Steps 8b-8e: N-1 flows p0 + LODF[:,c] p0[c]
 *                           (Eq. lodf_delta), multi-outage cases through a
 *                           per-case MODF (Def. eq_modf), and p0 - P_g
 *                           PTDF'[:, bus_g] for generator outages (Eq.
 *                           ptdf_delta), reduced to agg_m (maximum
 *                           relative load), t_i* = argmin over the variants,
 *                           then (metric-first, Sec. IV-B) the winner's
 *                           overload sum and worst (branch, contingency).
 *   dcflow_n1_worst         agg_i: the k worst N-1 cases of the winning
 *                           variant, recomputed after the score (Sec. IV-B).
 *   dcflow_n1_worst_per_case  agg_i in two levels (a top list per N-1 case,
 *                           then the top of their collection; Sec. IV-B).
 *   dcflow_fold_stubs       host preprocessing: radial stubs replaced by their
 *                           injections at the station (Sec. IV-A).
 *   Together: Eq. solver_end_to_end, (t_b, t_d, T_i) -> (agg_m, agg_i, t_i*).
 *
 * Conventions
 *   - Memory: the caller allocates every device buffer (sizes come from the
 *     *_bytes queries); the library never allocates or frees device memory.
 *     Host structs hold host pointers that are read during the call only.
 *   - Asynchrony: every call validates its arguments on the host and returns a
 *     negative dcflow_status on error without launching anything; otherwise it
 *     enqueues work on `stream` and returns DCFLOW_OK.  Device faults show up
 *     as DCFLOW_E_HIP from a later call (or from the caller's own sync).
 *   - Per-candidate problems (islanded candidate, singular correction, non-
 *     finite values) are status bits in the result, never errors.
 *   - Threading: a plan and its batches must not be used from two host
 *     threads at once; separate plans are independent.  No global state.
 *   - Indices are 0-based.  Node n_bus + j is the new busbar of the j-th split
 *     of a candidate (element order).
 */
#ifndef DCFLOW_H
#define DCFLOW_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DCFLOW_OK = 0,
  DCFLOW_E_ARG = -1,          /* null pointer, negative size, bad enum        */
  DCFLOW_E_SHAPE = -2,        /* index out of range, duplicate id, size cap   */
  DCFLOW_E_DISCONNECTED = -3, /* base grid is not connected                   */
  DCFLOW_E_WORKSPACE = -4,    /* caller buffer smaller than the query said    */
  DCFLOW_E_HIP = -5,          /* a HIP runtime call failed                    */
  DCFLOW_E_CAND = -6,         /* malformed candidate record (see bad_index)   */
  DCFLOW_E_SCRATCH = -7,      /* input exceeds DCFLOW_NOALLOC_SCRATCH_BYTES   */
  DCFLOW_E_TUNING = -8        /* the tuning's launch shape needs more LDS per
                                 workgroup than this batch allows; nothing was
                                 enqueued after the failing launch (others of
                                 the call may have run)                        */
} dcflow_status;

typedef enum {
  DCFLOW_FP64 = 0,   /* every step in FP64 (plain path)                         */
  DCFLOW_FP32 = 1,   /* injection GEMM on FP32 MFMA, LODF' tile build and N-1
                        scan in FP32; the k x k solve, U, W, z and the LODF
                        denominators in FP64.  The GEMM of every mode takes
                        x - p_base and adds the FP64 base flows back
                        (Eq. ptdf_times_nodal_inj is linear), which keeps the
                        cancellation of large grids out of the FP32 sums        */
  DCFLOW_BF16 = 2,   /* as FP32, but the injection GEMM takes BF16 operands
                        (FP32 accumulation): fast and coarse (flow errors of the
                        order of 0.1 of the smallest ratings), for pre-screening */
  DCFLOW_BF16X6 = 3  /* as FP32, but the injection GEMM splits each operand into
                        three BF16 parts and sums the six cross products of
                        order <= 2 on BF16 MFMA with FP32 accumulation: FP32-level
                        flow accuracy at a fraction of the FP32 MFMA time         */
} dcflow_prec;

/* Candidate element kinds. */
#define DCFLOW_OUTAGE 0 /* remedial disconnection of branch `id` (t_d)          */
#define DCFLOW_SPLIT 1  /* two-way split of bus `id` (t_b)                      */

#define DCFLOW_MAX_RANK 8       /* elements per candidate                       */
#define DCFLOW_MAX_SPLIT_DEG 32 /* incident branches of a splittable bus        */
#define DCFLOW_MULTI_MAX 4      /* branches per multi-outage N-1 case           */

/* Status bits of dcflow_score.status. */
#define DCFLOW_ST_DISCONNECTED 0x1u /* candidate grid islanded: max_load=+inf  */
#define DCFLOW_ST_SINGULAR 0x2u     /* k x k correction singular (implies 0x1) */
#define DCFLOW_ST_NONFINITE 0x4u    /* NaN/Inf met in the injections or flows  */
#define DCFLOW_ST_GUARDED 0x8u      /* reduced precision: some contingency columns
                                       were computed in FP64 by the error guard
                                       (see dcflow_tuning.guard_tol)              */
#define DCFLOW_ST_ISLAND_SHIFT 8    /* bits 8..31: number of islanding N-1 cases */

/* Grid description (host pointers, read during dcflow_build_ptdf only). */
typedef struct {
  int32_t n_bus;      /* >= 2                                                   */
  int32_t n_branch;   /* >= 1                                                   */
  int32_t slack;      /* slack bus, 0 <= slack < n_bus                          */
  const int32_t *from;/* [n_branch] from bus                                    */
  const int32_t *to;  /* [n_branch] to bus, != from                             */
  const double *b;    /* [n_branch] susceptance 1/x, finite and > 0             */
  int32_t n_mon;      /* monitored branches E_m (>= 1)                          */
  const int32_t *mon; /* [n_mon] distinct branch ids                            */
  int32_t n_out;      /* N-1 contingencies O (>= 0)                             */
  const int32_t *out; /* [n_out] distinct branch ids                            */
  const double *p_base;   /* [n_bus] base injections (base flows, rating rule)  */
  const double *rating;   /* [n_mon] > 0, or NULL: rating_scale*|F_base| + rating_offset */
  double rating_scale;
  double rating_offset;
  /* Controls (optional: zero counts and NULL pointers for none).  Each control is
   * one more entry of every injection vector, after the n_bus nodal injections:
   * injection vectors have n_inj = n_bus + n_pst + n_hvdc entries, the phase
   * shifters first.  Their flow sensitivities (PSDF, DCDF; named at the end of
   * Sec. II) become extra PTDF columns:
   *   phase shifter on branch l (from f to t), value a:  p_l = b_l (theta_f -
   *     theta_t - pst_scale a), column pst_scale b_l (PTDF[:, f] - PTDF[:, t] - e_l);
   *   HVDC link from bus i to bus j, value P: moves hvdc_scale P from i to j,
   *     column hvdc_scale (PTDF[:, j] - PTDF[:, i]).
   * The base case has all controls at 0.  Phase-shifter branches may be
   * contingencies, outaged or moved by a split: the shift's direct term is part
   * of the flows that the low-rank corrections and the LODF act on, so a shifter
   * on a removed branch contributes nothing and one on a moved branch keeps its
   * shift between the branch's post-change terminals (Sec. II end; the tripping
   * of a branch is a transfer of its N-0 flow, whatever fixed shifts it carries). */
  int32_t n_pst;
  const int32_t *pst_branch;   /* [n_pst] distinct branch ids                    */
  double pst_scale;            /* radians per unit (pi / 180 for degrees)        */
  int32_t n_hvdc;
  const int32_t *hvdc_from;    /* [n_hvdc] bus ids                               */
  const int32_t *hvdc_to;      /* [n_hvdc] bus ids, != hvdc_from                 */
  double hvdc_scale;           /* p.u. per unit                                  */
  /* Generator outages (optional: 0 and NULLs for none).  N-1 case g loses the
   * output gen_p[g] of a generator at bus gen_bus[g] and the slack takes it up:
   * the flows change by -gen_p[g] PTDF'[:, gen_bus[g]] (Eq. ptdf_delta, Sec.
   * III-C step 8d), PTDF' being the candidate grid's.  The generator stays on
   * busbar A when its bus is split (the lost output leaves A).  Generator cases
   * come after the n_out branch contingencies in every contingency-indexed
   * array and are reported with outage id -2 - g.  A generator at the slack
   * changes no flow.  Several generators may share a bus. */
  int32_t n_gen_out;
  const int32_t *gen_bus;      /* [n_gen_out] bus ids                            */
  const double *gen_p;         /* [n_gen_out] lost output (p.u.), finite         */
  /* Multi-outage N-1 cases (optional: 0 and NULLs for none), such as a busbar
   * or a three-winding transformer: case q trips the branches multi_br[
   * multi_off[q]] .. multi_br[multi_off[q+1] - 1] together (Def. eq_modf; Sec.
   * III-C branch-module step 5 and injection-module step 8c; Sec. IV-D: the MODF
   * terms are formed in the branch module and applied in the injection module).  Each case has 1
   * to DCFLOW_MULTI_MAX branches, distinct, each one of the n_out contingencies.
   * A case that islands the candidate grid is excluded and counted like an
   * islanding contingency; branches the candidate removed drop out of the case.
   * Multi cases come after the generator outages in the case order and are
   * reported with outage id -2 - n_gen_out - q. */
  int32_t n_multi_out;
  const int32_t *multi_off;    /* [n_multi_out + 1], multi_off[0] = 0            */
  const int32_t *multi_br;     /* [multi_off[n_multi_out]] branch ids            */
} dcflow_grid_desc;

/* Topology candidates in CSR form (host pointers).  Candidate i owns
 * elements off[i] .. off[i+1]-1 (0 to DCFLOW_MAX_RANK of them; 0 = the
 * unchanged grid).  For a split, bit q of mask moves the q-th incident branch
 * of the bus (incident branches in ascending branch id) to the new busbar;
 * at least one bit set, not every incident branch moved, at most one split
 * per bus per candidate.  Outage ids are distinct within a candidate.
 * p_new (may be NULL = all zero) is the injection that moves with a split's
 * new busbar; the injection left on busbar A is the variant's value minus it. */
typedef struct {
  int32_t n_cand;
  const int32_t *off;     /* [n_cand + 1], off[0] = 0, non-decreasing           */
  const int8_t *kind;     /* [n_elem] DCFLOW_OUTAGE or DCFLOW_SPLIT             */
  const int32_t *id;      /* [n_elem] branch id (outage) or bus id (split)      */
  const uint32_t *mask;   /* [n_elem] split mask (ignored for outages)          */
  const double *p_new;    /* [n_elem] or NULL                                   */
} dcflow_cands;

/* Result of one candidate (device array of n_cand, written by dcflow_n1_score). */
typedef struct {
  double max_load;       /* agg_m at t_i*: max over N-0 and valid N-1 of |p|/r  */
  double overload_sum;   /* sum of max(0, |p|/r - 1) over the same set at t_i*  */
  int32_t best_variant;  /* t_i* (lowest index on ties); -1 if disconnected     */
  int32_t worst_branch;  /* monitored branch id of the maximum                  */
  int32_t worst_outage;  /* contingency branch id of the maximum, -1 for N-0,
                            -2 - g for generator outage g, -2 - n_gen_out - q
                            for multi-outage case q                             */
  uint32_t status;       /* DCFLOW_ST_* bits, island count in bits 8..31       */
} dcflow_score;

/* Device pointers into the plan workspace, for inspection and tests.  All
 * matrices are row-major with the given leading dimensions (elements). */
typedef struct {
  int32_t n_bus, n_branch, n_mon, n_out, n_er; /* n_er = |E_m u O| rows kept   */
  int32_t ld_h;      /* leading dim of ptdf (>= n_bus)                          */
  int32_t ld_o;      /* leading dim of hdo  (>= n_out + n_gen_out)              */
  const double *ptdf;    /* [n_branch][ld_h] full PTDF, slack column 0         */
  const double *hdo;     /* [n_branch][ld_o] PTDF[:, f_c] - PTDF[:, t_c], c in O;
                            column n_out + g: PTDF[:, gen_bus[g]]              */
  const double *f_base;  /* [n_branch] base flows PTDF p_base                   */
  const double *rating;  /* [n_mon] ratings used by the score                   */
  const int32_t *er;     /* [n_er] kept rows: E_m first, then O \ E_m          */
  int32_t n_inj;         /* entries per injection vector (n_bus + controls)    */
  int32_t n_gen_out;     /* generator outages (columns after the n_out ones)   */
  int32_t n_multi_out;   /* multi-outage N-1 cases                             */
} dcflow_plan_view;

typedef struct dcflow_plan dcflow_plan;
typedef struct dcflow_batch dcflow_batch;

/* Bytes of device workspace that dcflow_build_ptdf needs for this grid. */
int dcflow_plan_workspace_bytes(const dcflow_grid_desc *grid, size_t *bytes);

/* One-time FP64 base build (Def. eq_ptdf with row restriction): reduced
 * nodal susceptance matrix, its inverse (Gauss-Jordan, SPD), the full PTDF,
 * node-major rows E_r, the contingency transfer columns PTDF[:,f_c]-PTDF[:,t_c],
 * base flows and ratings.  `dev_ws` (>= dcflow_plan_workspace_bytes, 256-byte
 * aligned) must stay allocated until dcflow_plan_destroy.  Returns
 * DCFLOW_E_DISCONNECTED if the base grid is not connected.  The plan (host
 * object) is owned by the caller and freed by dcflow_plan_destroy. */
int dcflow_build_ptdf(const dcflow_grid_desc *grid, void *dev_ws, size_t ws_bytes,
                      hipStream_t stream, dcflow_plan **plan_out);

int dcflow_plan_view_get(const dcflow_plan *plan, dcflow_plan_view *view);
void dcflow_plan_destroy(dcflow_plan *plan);

/* Host-only validation of candidate records against a grid; touches no GPU.
 * On DCFLOW_E_CAND, *bad_index (if non-NULL) is the offending element index,
 * or -(candidate index)-1 for a bad offset.  *packed_slots receives the sum of
 * candidate ranks (elements processed with no padding) and *padded_slots the
 * slots a depth-padded batch would use (n_cand * max rank). */
int dcflow_validate_candidates(const dcflow_grid_desc *grid, const dcflow_cands *cands,
                               int32_t *bad_index, int64_t *packed_slots,
                               int64_t *padded_slots);

/* Stub folding (host only; Sec. IV-A): radial stubs hanging off the meshed grid
 * (a bus of degree one, repeatedly, so that whole radial trees go) are replaced
 * by their injections at the bus they hang from.  In DC the flows on the rest
 * of the grid are unchanged, a folded branch carries the sum of the injections
 * beyond it, and the station gains injections that injection topologies can
 * regroup.  The slack and buses with protect[b] != 0 (protect may be NULL; e.g.
 * buses that candidates split) are never folded; parallel branches count
 * towards a bus's degree.  Outputs, caller-allocated host arrays:
 *   bus_new [n_bus]     index of a kept bus in the folded grid; for a folded bus,
 *                       that of the kept bus its tree hangs from;
 *   branch_new [n_branch] index of a kept branch in the folded grid, -1 if folded;
 *   up_branch [n_bus]   for a folded bus the branch towards the kept grid, else -1;
 *   *n_bus_out, *n_branch_out  sizes of the folded grid (kept order preserved;
 *                       its slack is bus_new[slack]).
 * E_ARG for null pointers, E_SHAPE for bad sizes or terminals. */
int dcflow_fold_stubs(int32_t n_bus, int32_t n_branch, int32_t slack, const int32_t *from,
                      const int32_t *to, const uint8_t *protect, int32_t *bus_new,
                      int32_t *branch_new, int32_t *up_branch, int32_t *n_bus_out,
                      int32_t *n_branch_out);

/* Injections of the folded grid (host): x_out[v][bus_new[b]] = sum of x[v][b]
 * over the buses b mapped there; x [n_var][n_bus], x_out [n_var][n_bus_out]. */
int dcflow_fold_injections(int32_t n_bus, const int32_t *bus_new, int32_t n_bus_out,
                           const double *x, int32_t n_var, double *x_out);

/* Flows of the folded branches (host) for injections x [n_var][n_bus]: the sum of
 * x over the buses beyond the branch, positive when it leaves them towards the
 * kept grid in the branch's from -> to direction; 0 on kept branches.
 * flow [n_var][n_branch]. */
int dcflow_stub_flows(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to,
                      const int32_t *up_branch, const double *x, int32_t n_var, double *flow);

/* Device bytes for a batch of these candidates with up to n_var_max
 * injection variants per candidate. */
int dcflow_batch_bytes(const dcflow_plan *plan, const dcflow_cands *cands,
                       int32_t n_var_max, size_t *bytes);

/* Validate and pack the candidates (uneven ranks, no padding; work queue in
 * descending rank) and upload them into `dev_buf` (>= dcflow_batch_bytes,
 * 256-byte aligned, kept until dcflow_batch_destroy). */
int dcflow_batch_create(dcflow_plan *plan, const dcflow_cands *cands, int32_t n_var_max,
                        void *dev_buf, size_t bytes, hipStream_t stream,
                        dcflow_batch **batch_out);
void dcflow_batch_destroy(dcflow_batch *batch);

/* Branch module (Sec. III-C steps 2-4): for every candidate the joint k x k
 * correction (bus splits as in Def. eq_bsdf, outages as in Def. eq_modf),
 * factors U (kept rows x k), K^-1 and W = K^-1 R (k x |O|), and the LODF
 * denominators of the contingencies in the changed grid; |den| < 1e-9 marks
 * an islanding contingency. */
int dcflow_eval_topologies(dcflow_batch *batch, hipStream_t stream);

/* Bytes of the flow buffer for n_var variants: [n_cand][n_var][ld_f] of
 * double (FP64) or float (FP32). */
int dcflow_flow_bytes(const dcflow_batch *batch, int32_t n_var, dcflow_prec prec,
                      size_t *bytes, int32_t *ld_f);

/* Injection module step 8a: post-change N-0 flows on the kept rows,
 * F'[i][v][r] = (PTDF x_v)[E_r[r]] + U_i K_i^-1 (sigma_i . PTDF x_v - p_new_i).
 * dev_inj (device, FP64): [n_cand][n_var][n_bus] or, if inj_shared,
 * [n_var][n_bus]; injections are in base bus numbering (the slack entry is
 * ignored).  dev_flows: see dcflow_flow_bytes.  Needs eval_topologies first. */
int dcflow_eval_injections(dcflow_batch *batch, const double *dev_inj, int32_t n_var,
                           int32_t inj_shared, dcflow_prec prec, void *dev_flows,
                           size_t flow_bytes, hipStream_t stream);

/* Steps 8b/8e: N-1 flows over the monitored rows and contingencies, per
 * variant maximum relative load, t_i* = argmin, then the winner's overload
 * sum and worst case.  dev_out: [n_cand] dcflow_score (device). */
int dcflow_n1_score(dcflow_batch *batch, const void *dev_flows, int32_t n_var,
                    dcflow_prec prec, dcflow_score *dev_out, hipStream_t stream);

/* Injection topologies (T_i of Sec. III-A): per split element and variant, the
 * injection placed on the split's new busbar, replacing the candidate's fixed
 * p_new in every later dcflow_eval_injections / dcflow_step (and graphs captured
 * after this call).  A variant can then regroup the injections of a split
 * substation between its two busbars while the nodal injection vector, in base
 * numbering, stays the same; the argmin over the variants is t_i*.  dev_pnew:
 * device array [n_elem][n_var] in the candidates' element order (values of
 * outage elements are ignored), read during each evaluation; NULL restores the
 * fixed p_new.  E_SHAPE unless 1 <= n_var <= n_var_max; evaluations with another
 * n_var then fail with E_SHAPE. */
int dcflow_set_busbar_injections(dcflow_batch *batch, const double *dev_pnew, int32_t n_var);

/* One case of the worst-case list (agg_i of Sec. III-A). */
typedef struct {
  double load;      /* |p| / rating; -1 for an unused entry                      */
  int32_t branch;   /* monitored branch id; -1 for an unused entry               */
  int32_t outage;   /* contingency branch id, -1 for the N-0 case (or unused),
                       -2 - g for generator outage g, -2 - n_gen_out - q for
                       multi-outage case q                                      */
} dcflow_case;

#define DCFLOW_WORST_MAX 16 /* most cases per candidate in one call */

/* Device bytes of the workspace of dcflow_n1_worst for top_k cases. */
int dcflow_n1_worst_workspace_bytes(const dcflow_batch *batch, int32_t top_k, size_t *bytes);

/* agg_i (Sec. III-A) in metric-first mode (Sec. IV-B: the details are computed
 * for the chosen variant only): for every candidate, the top_k largest relative
 * loads of its winning variant over the monitored branches in N-0 and in every
 * scored N-1 case (islanding contingencies excluded, as in the score), ordered
 * by load descending, ties by case (N-0 first, then contingencies in the
 * order of the grid's list, then generator outages, then multi-outage cases)
 * and then by the branch's position in the monitored
 * list.  The winner is dev_scores[i].best_variant from a dcflow_n1_score call on
 * the same batch and flows (device array, read on the stream); the entry with
 * the largest load equals that call's (max_load, worst_branch, worst_outage).
 * Candidates that are disconnected or have non-finite flows, and entries past
 * the number of scored cases, are unused (load -1).  dev_ws: workspace of
 * dcflow_n1_worst_workspace_bytes bytes; dev_out: [n_cand][top_k] (device).
 * E_ARG for top_k outside 1..DCFLOW_WORST_MAX, or if (n_out + n_gen_out +
 * n_multi_out + 1) * n_mon
 * exceeds 2^31 - 1 (the case keys are 32-bit); E_WORKSPACE if ws_bytes is too
 * small. */
int dcflow_n1_worst(dcflow_batch *batch, const void *dev_flows, int32_t n_var, dcflow_prec prec,
                    const dcflow_score *dev_scores, int32_t top_k, void *dev_ws, size_t ws_bytes,
                    dcflow_case *dev_out, hipStream_t stream);

/* Capacity of the library's fixed scratch array (bytes, per device). */
#define DCFLOW_NOALLOC_SCRATCH_BYTES (32u << 20)

/* dcflow_n1_worst for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same results as dcflow_n1_worst, with the band lists kept in a fixed
 * device array of the library instead of a caller workspace.  Nothing is
 * allocated; the caller passes inputs and outputs as for dcflow_n1_worst.
 * Every device the library runs on holds one such array of
 * DCFLOW_NOALLOC_SCRATCH_BYTES until the process ends; its address is looked up
 * on the first call on each device (call with the batch's device current).
 * All calls on one device share the array: calls that overlap in time on one
 * device (different streams or host threads) race and must be serialised by
 * the caller.  Returns DCFLOW_E_SCRATCH, before launching anything, when
 * dcflow_n1_worst_workspace_bytes for this batch and top_k exceeds the
 * capacity; other errors as dcflow_n1_worst. */
int dcflow_n1_worst_noalloc(dcflow_batch *batch, const void *dev_flows, int32_t n_var,
                            dcflow_prec prec, const dcflow_score *dev_scores, int32_t top_k,
                            dcflow_case *dev_out, hipStream_t stream);

/* Bytes of device workspace for dcflow_n1_worst_per_case with this per-case cap. */
int dcflow_n1_worst_per_case_workspace_bytes(const dcflow_batch *batch, int32_t per_case,
                                             size_t *bytes);

/* agg_i in the paper's two-level form (Sec. IV-B): the top per_case loads of every
 * case of the winning variant (the N-0 case, each scored contingency, generator
 * outage and multi-outage case; over the monitored branches), then the top_k of
 * that collection, so that no single case fills the list.  Same winner, order,
 * ids and output layout as dcflow_n1_worst; with per_case >= top_k it returns the
 * same cases (with one row band, loads bit for bit except the FP32 scan's guarded
 * columns and the multi-outage cases, which are summed in another order; with
 * several bands every entry is built by k FMAs, equal to rounding).  per_case in
 * 1..DCFLOW_WORST_MAX; dev_ws:
 * dcflow_n1_worst_per_case_workspace_bytes bytes.  Errors as dcflow_n1_worst. */
int dcflow_n1_worst_per_case(dcflow_batch *batch, const void *dev_flows, int32_t n_var,
                             dcflow_prec prec, const dcflow_score *dev_scores, int32_t per_case,
                             int32_t top_k, void *dev_ws, size_t ws_bytes, dcflow_case *dev_out,
                             hipStream_t stream);

/* Per-variant maxima of the last n1_score call: device pointer to
 * [n_cand][n_var_max] double (valid after the stream reaches it). */
const double *dcflow_batch_variant_max(const dcflow_batch *batch);

const char *dcflow_strerror(int status);

/* ---------------------------------------------------------------------------
 * Orchestration.  Launch shapes of the N-1 scan, chosen per batch (the
 * package's autotuner times them and caches the fastest), and capture of one
 * whole step (eval_topologies -> eval_injections -> n1_score) into a HIP graph
 * that is replayed with one launch.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t scan_vc;     /* variants per pass-1 workgroup: 0 = automatic; FP32 runs accept
                          16, 8, 4, 1 and FP64 runs 16, 8, 4, 1 (others: automatic;
                          16 in FP64 needs more than 64 KB of LDS per workgroup) */
  int32_t scan_rchunk; /* monitored rows per LDS chunk, a multiple of 64; 0 = automatic */
  int32_t persistent;  /* nonzero: the scan runs as resident workgroups (4 per compute
                          unit) that take work items from a queue                    */
  int32_t scan_band;   /* monitored rows per work item (a multiple of 64, rounded to the
                          row chunk); 0 = automatic: all rows when the scan's seed block
                          is small, else bands whose seed slice stays in L2          */
  int32_t step_chunks; /* dcflow_step and captured steps: 0 or 1 = eval_injections then
                          n1_score over the batch; 2..16 = that many candidate chunks,
                          the injections of chunk i + 1 running beside the scan of
                          chunk i on a second stream of the batch (per-candidate
                          injections only; the results are the same)               */
  int32_t worst_record; /* 0 (default) or positive: the winner pass of n1_score also
                          records, per candidate, the winner's maximum load of every
                          scored contingency column and of N-0 (plans whose monitored
                          rows form one band of the worst-case pass, the case of
                          dcflow_n1_worst_per_case; nothing otherwise).  A following
                          n1_worst or n1_worst_per_case call with the same flows and
                          score array reads them instead of sweeping the winner's
                          LODF' tiles again (same results, bit for bit); a new
                          evaluation or score call replaces the record.  Costs one
                          [n_cand][ld_o + 1] array of the batch (reserved for such
                          plans) and about 1% of n1_score.  Negative: off (the
                          worst-case calls sweep)                                    */
  double guard_tol;    /* error guard of the reduced-precision scan (FP32, BF16,
                          BF16X6), in rating units: per candidate, a contingency column
                          whose FP32 error bound (k + 4) 2^-24 S_c max_v |y_cv| exceeds
                          it (S_c = max_l |Lsd[l, c]| + sum_j max_l |U_j[l] / r_l|
                          |W_j[c]|, a bound of the LODF' entries' magnitude sums; y_cv
                          = F'[c, v] / den_c) is left out of the FP32 tiles and computed
                          in FP64 from the FP64 factors (U, W, seed) and the flows, in
                          n1_score, n1_worst and n1_worst_per_case alike; such
                          candidates carry DCFLOW_ST_GUARDED.  0 = the default 4e-5;
                          negative = off (every column in FP32)                     */
} dcflow_tuning;

/* Sets / reads the batch's launch shapes (defaults: all zero).  E_ARG for a
 * negative value, a row chunk or band that is not a multiple of 64, or more
 * than 16 step chunks.  The scan runs over work items (candidate, band of
 * monitored rows), band-major, with the candidates of a band in descending rank
 * (candidate order within a step chunk).  Asking for step chunks creates the
 * batch's second stream (default priority) and its events here. */
int dcflow_batch_set_tuning(dcflow_batch *batch, const dcflow_tuning *tuning);
int dcflow_batch_get_tuning(const dcflow_batch *batch, dcflow_tuning *tuning);

/* One whole step on `stream`: dcflow_eval_topologies, dcflow_eval_injections and
 * dcflow_n1_score with these arguments (same results, same errors), split into
 * the tuning's step_chunks candidate chunks so that the injection GEMM of one
 * chunk runs beside the N-1 scan of the previous one.  Returns when enqueued;
 * the stream waits for the second stream's work before anything enqueued after. */
int dcflow_step(dcflow_batch *batch, const double *dev_inj, int32_t n_var, int32_t inj_shared,
                dcflow_prec prec, void *dev_flows, size_t flow_bytes, dcflow_score *dev_out,
                hipStream_t stream);

/* Captures one step (dcflow_step) with exactly these arguments from `stream`
 * into a graph held by the batch, replacing any earlier one.
 * Nothing runs during the capture.  The stream must not be the null stream.
 * The buffers named here must stay valid while the graph is used; tuning
 * changes need a new capture.  Errors as for the three calls, E_HIP if the
 * runtime refuses the capture. */
int dcflow_graph_capture(dcflow_batch *batch, const double *dev_inj, int32_t n_var,
                         int32_t inj_shared, dcflow_prec prec, void *dev_flows,
                         size_t flow_bytes, dcflow_score *dev_out, hipStream_t stream);
/* Replays the captured step on `stream` (E_ARG if nothing was captured). */
int dcflow_graph_launch(dcflow_batch *batch, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Learned proposal network (an addition: the paper leaves the optimiser that
 * proposes candidates out of scope, Sec. III-A).  A 96 -> 256 -> 256 -> 1 ReLU
 * perceptron scores single-bus-split actions; the exact screen verifies the
 * best-scored ones and exhaustive screening stays the fallback and arbiter.
 * All pointers are device pointers; buffers are caller-owned.
 * ------------------------------------------------------------------------- */
#define DCFLOW_MLP_DIN 96     /* feature width (86 used, rest zero)            */
#define DCFLOW_MLP_PAIRS 8    /* tracked (branch, contingency) pairs per snapshot */
#define DCFLOW_MLP_HIDDEN 256
#define DCFLOW_TOPK_MAX 1024

/* Number of FP32 parameters: w1 [96][256], b1 [256], w2 [256][256], b2 [256],
 * w3 [256], b3 [1], 3 floats of padding (this order, one flat array). */
int dcflow_mlp_param_count(void);
/* Bytes of the BF16 weight copies used by dcflow_mlp_infer. */
size_t dcflow_mlp_bf16_bytes(void);
/* Bytes of training/forward workspace for a batch of `batch` samples. */
size_t dcflow_mlp_workspace_bytes(int32_t batch);

/* Base-case flows of load snapshots on every branch (Eq. ptdf_times_nodal_inj):
 * inj [n_snap][n_bus] -> flows [n_snap][n_branch]; n0max [n_snap] (or NULL)
 * receives the largest N-0 load |p|/r over the monitored branches. */
int dcflow_snapshot_flows(const dcflow_plan *plan, const double *inj, int32_t n_snap,
                          double *flows, double *n0max, hipStream_t stream);

/* The DCFLOW_MLP_PAIRS largest relative loads of each snapshot's unchanged
 * grid over N-0 rows and N-1 cases (Eq. lodf_delta, islanding contingencies
 * excluded; ties to the lower position, N-0 rows first, then contingency-major):
 * flows [n_snap][n_branch] from dcflow_snapshot_flows -> pairs [n_snap][8][2] =
 * (monitored branch id, contingency branch id or -1) and their loads
 * [n_snap][8] (double).  Unused slots (fewer scored cases) hold (-1, -1), 0. */
int dcflow_snapshot_pairs(const dcflow_plan *plan, const double *flows, int32_t n_snap,
                          int32_t *pairs, double *loads, hipStream_t stream);

/* Feature vectors [n_act][96] (FP32) of split actions: action a splits bus
 * bus[a] with mask[a] (incident-branch bits as in dcflow_cands) in snapshot
 * snap[a]; side[a] != 0 moves the bus injection to the new busbar.  worst
 * [n_snap][2] = (monitored branch id l*, contingency branch id c* or -1) of the
 * snapshot's unchanged grid; rho = PTDF[l*,:] + LODF[l*,c*] PTDF[c*,:] (Def.
 * eq_lodf) is the critical flow's sensitivity to injections.  Features:
 * [0] degree, [1] bus injection, [2] side bit, [3] rho[bus]; per incident
 * branch (ascending id, up to 14), 5 values from [4]: flow oriented out of the
 * bus / r, moved bit, present bit, sigma = rho[bus] - rho[far end],
 * sigma * oriented flow / r(l*), with r = rating_scale |F_base| + rating_offset;
 * [74], [75] = glob[2 s], glob[2 s + 1]; [76..83] the exact loads after the split
 * of the snapshot's pairs (from dcflow_snapshot_pairs), by the split factor of
 * Def. eq_bsdf / Eq. bsdf_application and the post-split LODF (Def. eq_lodf),
 * normalised by the monitored ratings; [84] their maximum; [85] = 1 when the
 * split cuts the new busbar off (then [76..84] are 0). */
int dcflow_action_features(const dcflow_plan *plan, const double *flows, const double *inj,
                           const double *glob, const int32_t *worst, const int32_t *pairs,
                           int32_t n_act, const int32_t *snap, const int32_t *bus,
                           const uint32_t *mask, const int32_t *side, float *feat,
                           hipStream_t stream);

/* Training labels of exact-screen results: labels[i] = min(log(max_load[i] /
 * glob[2 snap[i] + 1]), 0), the gain over the unchanged grid's maximum load
 * (0 = none, also for an islanded candidate with max_load = +inf). */
int dcflow_improvement_labels(const double *max_load, const int32_t *snap, const double *glob,
                              int32_t n, float *labels, hipStream_t stream);

/* FP32 forward pass y [n] of x [n][96] (ws >= dcflow_mlp_workspace_bytes(n)). */
int dcflow_mlp_forward(const float *params, const float *x, int32_t n, float *y, void *ws,
                       size_t ws_bytes, hipStream_t stream);
/* Gradient of the mean squared error mean((y - t)^2) over a batch: grad has
 * the parameter layout; loss [1] receives the batch loss. */
int dcflow_mlp_grad(const float *params, const float *x, const float *t, int32_t batch,
                    float *grad, float *loss, void *ws, size_t ws_bytes, hipStream_t stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 master weights;
 * m, v are the moment buffers (zero before step 1); step counts from 1. */
int dcflow_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr,
                    hipStream_t stream);
/* BF16 copies of w1, w2 for inference (bf16 >= dcflow_mlp_bf16_bytes()). */
int dcflow_mlp_pack_bf16(const float *params, void *bf16, hipStream_t stream);
/* Fused inference on BF16 MFMA with FP32 accumulation: y [n] for x [n][96]. */
int dcflow_mlp_infer(const float *params, const void *bf16, const float *x, int32_t n, float *y,
                     hipStream_t stream);
/* Per-column mean and 1 / standard deviation (floored at 1e-6) of x [rows][cols]. */
int dcflow_column_stats(const float *x, int32_t rows, int32_t cols, float *mean, float *inv_std,
                        hipStream_t stream);
/* In place: x[i][j] = (x[i][j] - mean[j]) * inv_std[j]. */
int dcflow_standardize(float *x, int64_t rows, int32_t cols, const float *mean,
                       const float *inv_std, hipStream_t stream);
/* Indices of the k smallest of scores [n] (ties: lowest index), in ascending
 * (score, index) order; 1 <= k <= min(n, DCFLOW_TOPK_MAX). */
int dcflow_topk_smallest(const float *scores, int32_t n, int32_t k, int32_t *idx,
                         hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* DCFLOW_H */
