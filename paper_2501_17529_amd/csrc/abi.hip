// Host side of the C ABI: argument validation, workspace layout, candidate
// packing (uneven ranks, no padding, descending-rank work order) and the
// entry points declared in include/dcflow.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>

#include <cstdlib>
#include <mutex>

#include "dcflow_internal.h"
#include "percase.h"

using namespace dcflow;

namespace {

// Sub-allocator over a caller-provided device buffer (256-byte aligned chunks).
struct Arena {
  char *base;
  size_t used = 0;
  explicit Arena(void *p) : base(static_cast<char *>(p)) {}
  template <typename T>
  T *take(size_t count) {
    size_t bytes = (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
    T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
    used += bytes;
    return p;
  }
};

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_grid(const dcflow_grid_desc *g) {
  if (!g || !g->from || !g->to || !g->b || !g->mon || !g->p_base) return DCFLOW_E_ARG;
  if (g->n_bus < 2 || g->n_branch < 1 || g->n_mon < 1 || g->n_out < 0) return DCFLOW_E_SHAPE;
  if (g->n_out > 0 && !g->out) return DCFLOW_E_ARG;
  if (g->slack < 0 || g->slack >= g->n_bus) return DCFLOW_E_SHAPE;
  for (int l = 0; l < g->n_branch; ++l) {
    if (g->from[l] < 0 || g->from[l] >= g->n_bus || g->to[l] < 0 || g->to[l] >= g->n_bus ||
        g->from[l] == g->to[l])
      return DCFLOW_E_SHAPE;
    if (!finite_pos(g->b[l])) return DCFLOW_E_ARG;
  }
  std::vector<uint8_t> seen(g->n_branch, 0);
  for (int i = 0; i < g->n_mon; ++i) {
    int l = g->mon[i];
    if (l < 0 || l >= g->n_branch || seen[l]) return DCFLOW_E_SHAPE;
    seen[l] = 1;
  }
  std::fill(seen.begin(), seen.end(), 0);
  for (int i = 0; i < g->n_out; ++i) {
    int l = g->out[i];
    if (l < 0 || l >= g->n_branch || seen[l]) return DCFLOW_E_SHAPE;
    seen[l] = 1;
  }
  for (int i = 0; i < g->n_bus; ++i)
    if (!std::isfinite(g->p_base[i])) return DCFLOW_E_ARG;
  if (g->n_pst < 0 || g->n_hvdc < 0) return DCFLOW_E_SHAPE;
  if (g->n_pst > 0) {
    if (!g->pst_branch || !std::isfinite(g->pst_scale)) return DCFLOW_E_ARG;
    std::vector<uint8_t> is_pst(g->n_branch, 0);
    for (int q = 0; q < g->n_pst; ++q) {
      const int l = g->pst_branch[q];
      if (l < 0 || l >= g->n_branch || is_pst[l]) return DCFLOW_E_SHAPE;
      is_pst[l] = 1;
    }
  }
  if (g->n_hvdc > 0) {
    if (!g->hvdc_from || !g->hvdc_to || !std::isfinite(g->hvdc_scale)) return DCFLOW_E_ARG;
    for (int q = 0; q < g->n_hvdc; ++q) {
      const int i = g->hvdc_from[q], j = g->hvdc_to[q];
      if (i < 0 || i >= g->n_bus || j < 0 || j >= g->n_bus || i == j) return DCFLOW_E_SHAPE;
    }
  }
  if (g->n_multi_out < 0) return DCFLOW_E_SHAPE;
  if (g->n_multi_out > 0) {
    if (!g->multi_off || !g->multi_br || g->multi_off[0] != 0) return DCFLOW_E_ARG;
    std::vector<uint8_t> is_out(g->n_branch, 0);
    for (int i = 0; i < g->n_out; ++i) is_out[g->out[i]] = 1;
    for (int q = 0; q < g->n_multi_out; ++q) {
      const int a = g->multi_off[q], b = g->multi_off[q + 1];
      if (b - a < 1 || b - a > DCFLOW_MULTI_MAX) return DCFLOW_E_SHAPE;
      for (int i = a; i < b; ++i) {
        const int l = g->multi_br[i];
        if (l < 0 || l >= g->n_branch || !is_out[l]) return DCFLOW_E_SHAPE;
        for (int j = a; j < i; ++j)
          if (g->multi_br[j] == l) return DCFLOW_E_SHAPE;
      }
    }
    if (g->multi_off[g->n_multi_out] > 65535) return DCFLOW_E_SHAPE;  // sub-columns
  }
  if (g->n_gen_out < 0) return DCFLOW_E_SHAPE;
  if (g->n_gen_out > 0) {
    if (!g->gen_bus || !g->gen_p) return DCFLOW_E_ARG;
    for (int q = 0; q < g->n_gen_out; ++q) {
      if (g->gen_bus[q] < 0 || g->gen_bus[q] >= g->n_bus) return DCFLOW_E_SHAPE;
      if (!std::isfinite(g->gen_p[q])) return DCFLOW_E_ARG;
    }
  }
  if (g->rating) {
    for (int i = 0; i < g->n_mon; ++i)
      if (!finite_pos(g->rating[i])) return DCFLOW_E_ARG;
  } else if (!std::isfinite(g->rating_scale) || !std::isfinite(g->rating_offset)) {
    return DCFLOW_E_ARG;
  }
  return DCFLOW_OK;
}

bool grid_connected(const dcflow_grid_desc *g) {
  std::vector<int> par(g->n_bus);
  std::iota(par.begin(), par.end(), 0);
  auto find = [&](int a) {
    while (par[a] != a) a = par[a] = par[par[a]];
    return a;
  };
  int comps = g->n_bus;
  for (int l = 0; l < g->n_branch; ++l) {
    int a = find(g->from[l]), c = find(g->to[l]);
    if (a != c) {
      par[a] = c;
      --comps;
    }
  }
  return comps == 1;
}

struct Dims {
  int n, m, n_mon, n_out, n_gen, n_multi, n_msub, n_er, ld_h, ld_er, ld_o, mon_pad, n_ctrl, ld_b;
};

Dims grid_dims(const dcflow_grid_desc *g) {
  Dims d;
  d.n = g->n_bus;
  d.m = g->n_branch;
  d.n_mon = g->n_mon;
  d.n_out = g->n_out;
  d.n_gen = g->n_gen_out;
  d.n_multi = g->n_multi_out;
  d.n_msub = d.n_multi > 0 ? g->multi_off[d.n_multi] : 0;
  std::vector<uint8_t> inmon(d.m, 0);
  for (int i = 0; i < g->n_mon; ++i) inmon[g->mon[i]] = 1;
  int extra = 0;
  for (int i = 0; i < g->n_out; ++i) extra += inmon[g->out[i]] ? 0 : 1;
  d.n_er = d.n_mon + extra;
  d.n_ctrl = g->n_pst + g->n_hvdc;
  d.ld_h = round_up(d.n + d.n_ctrl, 16);
  d.ld_b = round_up(d.n, 64);
  d.ld_er = round_up(d.n_er, 128);
  d.ld_o = std::max(64, round_up(d.n_out + d.n_gen, 64));
  d.mon_pad = round_up(d.n_mon, 64);
  return d;
}

// Places every plan array in the arena (base may be null: size query).
void plan_layout(dcflow_plan *p, const Dims &d, Arena &a) {
  p->d_f = a.take<int32_t>(d.m);
  p->d_t = a.take<int32_t>(d.m);
  p->d_b = a.take<double>(d.m);
  p->d_adj_off = a.take<int32_t>(d.n + 1);
  p->d_adj_br = a.take<int32_t>(2 * (size_t)d.m);
  p->d_mon = a.take<int32_t>(d.n_mon);
  p->d_out = a.take<int32_t>(d.n_out);
  p->d_er = a.take<int32_t>(d.n_er);
  p->d_pos_of_br = a.take<int32_t>(d.m);
  p->d_out_pos = a.take<int32_t>(d.n_out);
  p->d_out_f = a.take<int32_t>(d.n_out + d.n_gen);
  p->d_out_t = a.take<int32_t>(d.n_out + d.n_gen);
  p->d_gen_y = a.take<double>(std::max(d.n_gen, 1));
  p->d_moff = a.take<int32_t>(d.n_multi + 1);
  p->d_mcol = a.take<int32_t>(std::max(d.n_msub, 1));
  p->d_lsdm = a.take<double>((size_t)d.n_msub * d.mon_pad);
  p->d_lsdm32 = a.take<float>((size_t)d.n_msub * d.mon_pad);
  p->d_binv = a.take<double>((size_t)d.ld_b * d.ld_b);
  p->d_piv = a.take<double>(64 * 64);
  p->d_hb = a.take<double>((size_t)d.m * d.ld_h);
  p->d_ht = a.take<double>((size_t)d.n * d.ld_er);
  p->d_he64 = a.take<double>((size_t)d.ld_er * d.ld_h);
  p->d_he32 = a.take<float>((size_t)d.ld_er * d.ld_h);
  p->d_heb = a.take<__bf16>(3 * (size_t)d.ld_er * d.ld_h);
  p->d_hdo = a.take<double>((size_t)d.m * d.ld_o);
  p->d_lsd = a.take<double>((size_t)d.mon_pad * d.ld_o);
  p->d_lsdmax = a.take<double>(d.ld_o);
  p->d_lsd32 = a.take<float>((size_t)d.mon_pad * d.ld_o);
  p->d_lsd64f = a.take<double>((size_t)d.mon_pad * d.ld_o);
  p->d_lsdT = a.take<double>((size_t)d.mon_pad * d.ld_o);
  p->d_fbase = a.take<double>(d.m);
  p->d_fber = a.take<double>(d.ld_er);
  p->d_pbase = a.take<double>(d.ld_h);
  p->d_rating = a.take<double>(d.mon_pad);
  p->d_inv_r = a.take<double>(d.mon_pad);
  const size_t nc = std::max(d.n_ctrl, 1);
  p->d_ctl_a = a.take<int32_t>(nc);
  p->d_ctl_c = a.take<int32_t>(nc);
  p->d_ctl_br = a.take<int32_t>(nc);
  p->d_ctl_w = a.take<double>(nc);
  p->d_ctl_d = a.take<double>(nc);
}

struct BatchDims {
  int n_cand, n_elem, vmax;
};

void batch_layout(dcflow_batch *b, const dcflow_plan *p, const BatchDims &d, Arena &a) {
  const size_t ne = std::max(d.n_elem, 1), nc = std::max(d.n_cand, 1);
  b->d_off = a.take<int32_t>(nc + 1);
  b->d_kind = a.take<int32_t>(ne);
  b->d_id = a.take<int32_t>(ne);
  b->d_order = a.take<int32_t>(nc);
  b->d_mask = a.take<uint32_t>(ne);
  b->d_pnew = a.take<double>(ne);
  b->d_nsig = a.take<int32_t>(ne);
  b->d_sig = a.take<int32_t>(ne * kMaxSig);
  b->d_U = a.take<double>(ne * p->ld_er);
  b->d_W = a.take<double>(ne * p->ld_o);
  b->d_ur32 = a.take<float>(ne * p->mon_pad);
  b->d_w32 = a.take<float>(ne * p->ld_o);
  b->d_umax = a.take<float>(ne);
  b->d_flag = a.take<uint32_t>(nc * (p->ld_o / 32));
  b->d_nflag = a.take<int32_t>(nc);
  b->d_kinv = a.take<double>(nc * 64);
  b->d_invden = a.take<double>(nc * p->ld_o);
  b->d_isl = a.take<uint32_t>(nc * (p->ld_o / 32));
  b->d_status = a.take<uint32_t>(nc);
  b->d_z = a.take<double>(ne * d.vmax);
  b->d_vmax = a.take<double>(nc * d.vmax);
  b->d_f0 = a.take<double>((size_t)d.vmax * p->ld_er);
  b->ldx = (p->n_inj + 31) / 32 * 32;
  // BF16 parts of x - p_base for at most kXsMaxCols columns (larger GEMMs run in
  // blocks of whole candidates); DCFLOW_SPLIT_COLS lowers the cap (tests use it to
  // run the blocked path on small batches)
  size_t cap = kXsMaxCols;
  if (const char *env = std::getenv("DCFLOW_SPLIT_COLS")) {
    const long long v = std::atoll(env);
    if (v > 0 && (size_t)v < cap) cap = (size_t)v;
  }
  b->xs_cols = std::min(nc * (size_t)d.vmax, cap);
  b->d_xs = a.take<__bf16>(3 * b->xs_cols * (size_t)b->ldx);
  b->d_queue = a.take<int32_t>(16);
  const size_t nmb = p->n_multi > 0 ? (p->n_mon + kMultiRows - 1) / kMultiRows : 0;
  const size_t np = nc * (size_t)(p->mon_pad / 64 + nmb + 1);  // + the guard's slot
  b->d_part_m = a.take<double>(np);
  b->d_part_ov = a.take<double>(np);
  b->d_part_k = a.take<long long>(np);
  b->d_part_nf = a.take<int32_t>(np);
  b->d_mcoef = a.take<double>(nc * (size_t)p->n_multi * 16);
  b->d_mok = a.take<int32_t>(nc * (size_t)p->n_multi);
  // the winner pass's column-maximum record, for plans whose worst-case pass has
  // one row band
  if (case_maxima_supported(p)) {
    b->d_rec = a.take<double>(nc * (size_t)(p->ld_o + 1));
    b->d_rec_var = a.take<int32_t>(nc);
  } else {
    b->d_rec = nullptr;
    b->d_rec_var = nullptr;
  }
}

// Candidate records against the grid (element kinds, ids, split masks, ranks).
// Phase-shifter branches may be contingencies, outaged or moved by a split like
// any other: the shift's direct term is part of the flows the corrections act on.
int check_cands(int n_bus, int n_branch, const std::vector<int32_t> &adj_off,
                const dcflow_cands *c, int32_t *bad, int64_t *packed, int64_t *padded,
                int *kmax_out) {
  if (bad) *bad = 0;
  if (!c || c->n_cand < 0) return DCFLOW_E_ARG;
  if (c->n_cand > 0 && !c->off) return DCFLOW_E_ARG;
  if (c->n_cand == 0) {
    if (packed) *packed = 0;
    if (padded) *padded = 0;
    if (kmax_out) *kmax_out = 0;
    return DCFLOW_OK;
  }
  if (c->off[0] != 0) {
    if (bad) *bad = -1;
    return DCFLOW_E_CAND;
  }
  int kmax = 0;
  int64_t tot = 0;
  for (int i = 0; i < c->n_cand; ++i) {
    int k = c->off[i + 1] - c->off[i];
    if (k < 0 || k > kMaxRank) {
      if (bad) *bad = -i - 1;
      return DCFLOW_E_CAND;
    }
    kmax = std::max(kmax, k);
    tot += k;
  }
  if (tot > 0 && (!c->kind || !c->id || !c->mask)) return DCFLOW_E_ARG;
  for (int i = 0; i < c->n_cand; ++i) {
    int a = c->off[i], e = c->off[i + 1];
    for (int j = a; j < e; ++j) {
      bool ok = true;
      if (c->kind[j] == DCFLOW_OUTAGE) {
        ok = c->id[j] >= 0 && c->id[j] < n_branch;
      } else if (c->kind[j] == DCFLOW_SPLIT) {
        ok = c->id[j] >= 0 && c->id[j] < n_bus;
        if (ok) {
          int deg = adj_off[c->id[j] + 1] - adj_off[c->id[j]];
          uint32_t mk = c->mask[j];
          uint64_t full = deg >= 32 ? 0xffffffffull : ((1ull << deg) - 1);
          ok = deg >= 2 && deg <= kMaxSig && mk != 0 && (uint64_t)mk <= full && (uint64_t)mk != full;
        }
      } else {
        ok = false;
      }
      if (ok && c->p_new && !std::isfinite(c->p_new[j])) ok = false;
      for (int q = a; ok && q < j; ++q)
        if (c->kind[q] == c->kind[j] && c->id[q] == c->id[j]) ok = false;  // duplicate
      if (!ok) {
        if (bad) *bad = j;
        return DCFLOW_E_CAND;
      }
    }
  }
  if (packed) *packed = tot;
  if (padded) *padded = (int64_t)kmax * c->n_cand;
  if (kmax_out) *kmax_out = kmax;
  return DCFLOW_OK;
}

std::vector<int32_t> host_adj_off(const dcflow_grid_desc *g) {
  std::vector<int32_t> off(g->n_bus + 1, 0);
  for (int l = 0; l < g->n_branch; ++l) {
    off[g->from[l] + 1]++;
    off[g->to[l] + 1]++;
  }
  for (int i = 0; i < g->n_bus; ++i) off[i + 1] += off[i];
  return off;
}

// Maps a HIP failure to DCFLOW_E_HIP and names it on stderr (the status code
// alone cannot say which runtime error it was).
int hip_fail(hipError_t e, const char *where) {
  if (e == kShapeMisfit) return DCFLOW_E_TUNING;  // a status, not a runtime failure
  fprintf(stderr, "dcflow: %s: %s\n", where, hipGetErrorString(e));
  return DCFLOW_E_HIP;
}

}  // namespace

extern "C" {

int dcflow_plan_workspace_bytes(const dcflow_grid_desc *grid, size_t *bytes) {
  if (!bytes) return DCFLOW_E_ARG;
  int rc = check_grid(grid);
  if (rc != DCFLOW_OK) return rc;
  dcflow_plan tmp;
  Arena a(nullptr);
  plan_layout(&tmp, grid_dims(grid), a);
  *bytes = a.used;
  return DCFLOW_OK;
}

int dcflow_build_ptdf(const dcflow_grid_desc *g, void *dev_ws, size_t ws_bytes, hipStream_t s,
                      dcflow_plan **plan_out) {
  if (!plan_out || !dev_ws) return DCFLOW_E_ARG;
  *plan_out = nullptr;
  int rc = check_grid(g);
  if (rc != DCFLOW_OK) return rc;
  if (reinterpret_cast<uintptr_t>(dev_ws) % 256) return DCFLOW_E_ARG;
  if (!grid_connected(g)) return DCFLOW_E_DISCONNECTED;
  Dims d = grid_dims(g);
  dcflow_plan *p = new (std::nothrow) dcflow_plan();
  if (!p) return DCFLOW_E_ARG;
  Arena a(dev_ws);
  plan_layout(p, d, a);
  if (a.used > ws_bytes) {
    delete p;
    return DCFLOW_E_WORKSPACE;
  }
  p->n = d.n;
  p->m = d.m;
  p->slack = g->slack;
  p->n_mon = d.n_mon;
  p->n_out = d.n_out;
  p->n_gen = d.n_gen;
  p->n_multi = d.n_multi;
  p->n_msub = d.n_msub;
  p->n_er = d.n_er;
  p->ld_h = d.ld_h;
  p->ld_b = d.ld_b;
  p->ld_er = d.ld_er;
  p->ld_o = d.ld_o;
  p->mon_pad = d.mon_pad;
  p->n_ctrl = d.n_ctrl;
  p->n_inj = d.n + d.n_ctrl;
  p->rating_scale = g->rating ? 1.2 : g->rating_scale;
  p->rating_offset = g->rating ? 0.1 : g->rating_offset;
  p->f.assign(g->from, g->from + d.m);
  p->t.assign(g->to, g->to + d.m);
  p->adj_off = host_adj_off(g);
  p->adj_br.assign(2 * (size_t)d.m, 0);
  {
    std::vector<int32_t> fill(p->adj_off.begin(), p->adj_off.end() - 1);
    for (int l = 0; l < d.m; ++l) {  // ascending branch id per bus
      p->adj_br[fill[g->from[l]]++] = l;
      p->adj_br[fill[g->to[l]]++] = l;
    }
  }
  p->out.assign(g->out, g->out + d.n_out);
  std::vector<int32_t> er(g->mon, g->mon + d.n_mon);
  p->pos_of_br.assign(d.m, -1);
  for (int i = 0; i < d.n_mon; ++i) p->pos_of_br[g->mon[i]] = i;
  std::vector<int32_t> out_pos(std::max(d.n_out, 1), 0), of(std::max(d.n_out + d.n_gen, 1), 0),
      ot(std::max(d.n_out + d.n_gen, 1), 0);
  std::vector<double> gen_y(std::max(d.n_gen, 1), 0.0);
  for (int q = 0; q < d.n_gen; ++q) {  // generator column: PTDF[:, bus], coefficient -P_g
    of[d.n_out + q] = g->gen_bus[q];
    ot[d.n_out + q] = -1;
    gen_y[q] = -g->gen_p[q];
  }
  p->is_out.assign(d.m, 0);
  for (int c = 0; c < d.n_out; ++c) {
    int l = g->out[c];
    p->is_out[l] = 1;
    if (p->pos_of_br[l] < 0) {
      p->pos_of_br[l] = (int)er.size();
      er.push_back(l);
    }
    out_pos[c] = p->pos_of_br[l];
    of[c] = g->from[l];
    ot[c] = g->to[l];
  }
  // multi-outage sub-columns: the contingency column of each branch of each case
  std::vector<int32_t> moff(d.n_multi + 1, 0), mcol(std::max(d.n_msub, 1), 0);
  {
    std::vector<int32_t> col_of(d.m, -1);
    for (int c = 0; c < d.n_out; ++c) col_of[g->out[c]] = c;
    for (int q = 0; q <= d.n_multi && d.n_multi > 0; ++q) moff[q] = g->multi_off[q];
    for (int i = 0; i < d.n_msub; ++i) mcol[i] = col_of[g->multi_br[i]];
  }
  std::vector<double> pb(d.ld_h, 0.0);  // controls of the base case: 0
  std::copy(g->p_base, g->p_base + d.n, pb.begin());
  // control columns: phase shifter on l = f -> t: pst_scale b_l (e_f - e_t) injection pattern
  // and -pst_scale b_l on l itself; HVDC i -> j: hvdc_scale (e_j - e_i)
  std::vector<int32_t> ca, cc, cbr;
  std::vector<double> cw, cd;
  for (int q = 0; q < g->n_pst; ++q) {
    const int l = g->pst_branch[q];
    ca.push_back(g->from[l]);
    cc.push_back(g->to[l]);
    cbr.push_back(l);
    cw.push_back(g->pst_scale * g->b[l]);
    cd.push_back(-g->pst_scale * g->b[l]);
  }
  for (int q = 0; q < g->n_hvdc; ++q) {
    ca.push_back(g->hvdc_to[q]);
    cc.push_back(g->hvdc_from[q]);
    cbr.push_back(-1);
    cw.push_back(g->hvdc_scale);
    cd.push_back(0.0);
  }

  // uploads; the first failing call's error is kept and named
  hipError_t up_err = hipSuccess;
  auto up = [&](void *dst, const void *src, size_t bytes) {
    const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess && up_err == hipSuccess) up_err = e;
    return e;
  };
  if (up(p->d_f, g->from, 4 * (size_t)d.m) != hipSuccess ||
      up(p->d_t, g->to, 4 * (size_t)d.m) != hipSuccess ||
      up(p->d_b, g->b, 8 * (size_t)d.m) != hipSuccess ||
      up(p->d_adj_off, p->adj_off.data(), 4 * p->adj_off.size()) != hipSuccess ||
      up(p->d_adj_br, p->adj_br.data(), 4 * p->adj_br.size()) != hipSuccess ||
      up(p->d_mon, g->mon, 4 * (size_t)d.n_mon) != hipSuccess ||
      (d.n_out > 0 && up(p->d_out, g->out, 4 * (size_t)d.n_out) != hipSuccess) ||
      up(p->d_er, er.data(), 4 * er.size()) != hipSuccess ||
      up(p->d_pos_of_br, p->pos_of_br.data(), 4 * (size_t)d.m) != hipSuccess ||
      up(p->d_out_pos, out_pos.data(), 4 * out_pos.size()) != hipSuccess ||
      up(p->d_out_f, of.data(), 4 * of.size()) != hipSuccess ||
      up(p->d_out_t, ot.data(), 4 * ot.size()) != hipSuccess ||
      up(p->d_gen_y, gen_y.data(), 8 * gen_y.size()) != hipSuccess ||
      up(p->d_moff, moff.data(), 4 * moff.size()) != hipSuccess ||
      up(p->d_mcol, mcol.data(), 4 * mcol.size()) != hipSuccess ||
      up(p->d_pbase, pb.data(), 8 * pb.size()) != hipSuccess ||
      (d.n_ctrl > 0 && (up(p->d_ctl_a, ca.data(), 4 * ca.size()) != hipSuccess ||
                        up(p->d_ctl_c, cc.data(), 4 * cc.size()) != hipSuccess ||
                        up(p->d_ctl_br, cbr.data(), 4 * cbr.size()) != hipSuccess ||
                        up(p->d_ctl_w, cw.data(), 8 * cw.size()) != hipSuccess ||
                        up(p->d_ctl_d, cd.data(), 8 * cd.size()) != hipSuccess))) {
    delete p;
    return hip_fail(up_err, "dcflow_build_ptdf (upload)");
  }
  hipError_t e = launch_build(p, s, g->rating, g->rating_scale, g->rating_offset);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // host staging vectors die here
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "dcflow_build_ptdf");
  }
  *plan_out = p;
  return DCFLOW_OK;
}

int dcflow_plan_view_get(const dcflow_plan *p, dcflow_plan_view *v) {
  if (!p || !v) return DCFLOW_E_ARG;
  v->n_bus = p->n;
  v->n_branch = p->m;
  v->n_mon = p->n_mon;
  v->n_out = p->n_out;
  v->n_gen_out = p->n_gen;
  v->n_multi_out = p->n_multi;
  v->n_er = p->n_er;
  v->ld_h = p->ld_h;
  v->ld_o = p->ld_o;
  v->ptdf = p->d_hb;
  v->hdo = p->d_hdo;
  v->f_base = p->d_fbase;
  v->rating = p->d_rating;
  v->er = p->d_er;
  v->n_inj = p->n_inj;
  return DCFLOW_OK;
}

void dcflow_plan_destroy(dcflow_plan *p) { delete p; }

int dcflow_validate_candidates(const dcflow_grid_desc *g, const dcflow_cands *c,
                               int32_t *bad_index, int64_t *packed, int64_t *padded) {
  int rc = check_grid(g);
  if (rc != DCFLOW_OK) return rc;
  return check_cands(g->n_bus, g->n_branch, host_adj_off(g), c, bad_index, packed, padded,
                     nullptr);
}

int dcflow_batch_bytes(const dcflow_plan *p, const dcflow_cands *c, int32_t n_var_max,
                       size_t *bytes) {
  if (!p || !c || !bytes || n_var_max < 1) return DCFLOW_E_ARG;
  if (c->n_cand < 0 || (c->n_cand > 0 && !c->off)) return DCFLOW_E_ARG;
  BatchDims d{c->n_cand, c->n_cand ? c->off[c->n_cand] : 0, n_var_max};
  dcflow_batch tmp;
  Arena a(nullptr);
  batch_layout(&tmp, p, d, a);
  *bytes = a.used;
  return DCFLOW_OK;
}

int dcflow_batch_create(dcflow_plan *p, const dcflow_cands *c, int32_t n_var_max, void *dev_buf,
                        size_t bytes, hipStream_t s, dcflow_batch **out) {
  if (!p || !c || !out || !dev_buf || n_var_max < 1) return DCFLOW_E_ARG;
  *out = nullptr;
  if (reinterpret_cast<uintptr_t>(dev_buf) % 256) return DCFLOW_E_ARG;
  int32_t bad = 0;
  int64_t packed = 0, padded = 0;
  int kmax = 0;
  int rc = check_cands(p->n, p->m, p->adj_off, c, &bad, &packed, &padded, &kmax);
  if (rc != DCFLOW_OK) return rc;
  BatchDims d{c->n_cand, c->n_cand ? c->off[c->n_cand] : 0, n_var_max};
  dcflow_batch *b = new (std::nothrow) dcflow_batch();
  if (!b) return DCFLOW_E_ARG;
  Arena a(dev_buf);
  batch_layout(b, p, d, a);
  if (a.used > bytes) {
    delete b;
    return DCFLOW_E_WORKSPACE;
  }
  b->plan = p;
  b->n_cand = d.n_cand;
  b->n_elem = d.n_elem;
  b->vmax = n_var_max;
  b->packed = packed;
  b->padded = padded;
  b->kmax = kmax;
  b->factored = 0;
  b->flows_prec = -1;
  b->flows_nvar = 0;
  b->guard_valid = 0;
  b->rec_valid = 0;
  b->rec_prec = -1;
  b->rec_nvar = 0;
  b->rec_flows = nullptr;
  b->rec_scores = nullptr;
  b->graph_state = dcflow_batch::StepState{};
  b->d_pnv = nullptr;
  b->pnv_nvar = 0;
  b->tune = dcflow_tuning{0, 0, 0, 0, 0, 0, 0.0};
  b->aux = nullptr;
  for (int i = 0; i <= kMaxStepChunks; ++i) b->step_ev[i] = nullptr;
  b->max_bands = p->mon_pad / 64;
  b->nmb = p->n_multi > 0 ? (p->n_mon + kMultiRows - 1) / kMultiRows : 0;
  b->graph = nullptr;
  b->graph_exec = nullptr;
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu < 1)
      ncu = 256;
    b->n_cu = ncu;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        lds < 64 * 1024)
      lds = 64 * 1024;
    b->lds_max = (size_t)lds;
  }
  if (d.n_cand > 0) {
    // work queue: descending rank, stable
    std::vector<int32_t> order(d.n_cand);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return (c->off[x + 1] - c->off[x]) > (c->off[y + 1] - c->off[y]);
    });
    const size_t ne = std::max(d.n_elem, 1);
    std::vector<int32_t> kind(ne, 0), id(ne, 0);
    std::vector<uint32_t> mask(ne, 0);
    std::vector<double> pn(ne, 0.0);
    for (int j = 0; j < d.n_elem; ++j) {
      kind[j] = c->kind[j];
      id[j] = c->id[j];
      mask[j] = c->mask[j];
      pn[j] = c->p_new ? c->p_new[j] : 0.0;
    }
    hipError_t e = hipMemcpyAsync(b->d_off, c->off, 4 * (size_t)(d.n_cand + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_order, order.data(), 4 * order.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_kind, kind.data(), 4 * ne, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_id, id.data(), 4 * ne, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_mask, mask.data(), 4 * ne, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_pnew, pn.data(), 8 * ne, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // host staging vectors die here
    if (e != hipSuccess) {
      delete b;
      return hip_fail(e, "dcflow_batch_create (upload)");
    }
  }
  *out = b;
  return DCFLOW_OK;
}

namespace {
void drop_graph(dcflow_batch *b) {
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->graph_exec = nullptr;
  b->graph = nullptr;
}
}  // namespace

void dcflow_batch_destroy(dcflow_batch *b) {
  if (!b) return;
  drop_graph(b);
  for (int i = 0; i <= kMaxStepChunks; ++i)
    if (b->step_ev[i]) (void)hipEventDestroy(b->step_ev[i]);
  if (b->aux) (void)hipStreamDestroy(b->aux);
  delete b;
}

namespace {
// the second stream and the events of the chunked step, made once per batch
// (outside any capture when the tuning asks for chunks)
hipError_t ensure_step_streams(dcflow_batch *b) {
  hipError_t e = hipSuccess;
  if (!b->aux) e = hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking);
  for (int i = 0; e == hipSuccess && i <= kMaxStepChunks; ++i)
    if (!b->step_ev[i]) e = hipEventCreateWithFlags(&b->step_ev[i], hipEventDisableTiming);
  return e;
}

// One whole step: eval_topologies, then eval_injections and n1_score over the
// batch, or over step_chunks candidate chunks with the injections of chunk i + 1
// (stream s) running beside the scan of chunk i (the batch's second stream).
int run_step(dcflow_batch *b, const double *inj, int nvar, int shared, int prec, void *flows,
             dcflow_score *out, hipStream_t s) {
  hipError_t e = launch_factors(b, s);
  if (e != hipSuccess) return hip_fail(e, "dcflow_step");
  b->factored = 1;
  b->guard_valid = 0;
  b->rec_valid = 0;
  int nch = b->tune.step_chunks;
  if (shared || nch > b->n_cand) nch = shared ? 1 : b->n_cand;
  if (nch <= 1) {
    e = launch_injections(b, inj, nvar, shared, prec, flows, 0, b->n_cand, s);
    if (e == hipSuccess) e = launch_score(b, flows, nvar, prec, out, 0, b->n_cand, s);
  } else {
    e = ensure_step_streams(b);
    for (int i = 0; e == hipSuccess && i < nch; ++i) {
      const int c0 = (int)((int64_t)b->n_cand * i / nch), c1 = (int)((int64_t)b->n_cand * (i + 1) / nch);
      e = launch_injections(b, inj, nvar, 0, prec, flows, c0, c1, s);
      if (e == hipSuccess) e = hipEventRecord(b->step_ev[i], s);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->aux, b->step_ev[i], 0);
      if (e == hipSuccess) e = launch_score(b, flows, nvar, prec, out, c0, c1, b->aux);
    }
    if (e == hipSuccess) e = hipEventRecord(b->step_ev[nch], b->aux);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, b->step_ev[nch], 0);
  }
  if (e != hipSuccess) return hip_fail(e, "dcflow_step");
  b->flows_prec = prec;
  b->flows_nvar = nvar;
  return DCFLOW_OK;
}

int check_step(dcflow_batch *b, const double *dev_inj, int32_t n_var, dcflow_prec prec,
               void *dev_flows, size_t flow_bytes, dcflow_score *dev_out) {
  if (!b || !dev_inj || !dev_flows || !dev_out) return DCFLOW_E_ARG;
  if (n_var < 1 || n_var > b->vmax) return DCFLOW_E_SHAPE;
  if (!prec_valid(prec)) return DCFLOW_E_ARG;
  if (b->d_pnv && b->pnv_nvar != n_var) return DCFLOW_E_SHAPE;
  size_t need = 0;
  dcflow_flow_bytes(b, n_var, prec, &need, nullptr);
  if (flow_bytes < need) return DCFLOW_E_WORKSPACE;
  return DCFLOW_OK;
}
}  // namespace

int dcflow_batch_set_tuning(dcflow_batch *b, const dcflow_tuning *t) {
  if (!b || !t) return DCFLOW_E_ARG;
  if (t->scan_vc < 0 || t->scan_rchunk < 0 || t->scan_rchunk % 64 || t->persistent < 0 ||
      t->scan_band < 0 || t->scan_band % 64 || t->step_chunks < 0 ||
      t->step_chunks > kMaxStepChunks || !std::isfinite(t->guard_tol))
    return DCFLOW_E_ARG;
  if (t->step_chunks > 1) {
    const hipError_t e = ensure_step_streams(b);
    if (e != hipSuccess) return hip_fail(e, "dcflow_batch_set_tuning");
  }
  b->tune = *t;
  return DCFLOW_OK;
}

int dcflow_step(dcflow_batch *b, const double *dev_inj, int32_t n_var, int32_t inj_shared,
                dcflow_prec prec, void *dev_flows, size_t flow_bytes, dcflow_score *dev_out,
                hipStream_t s) {
  const int rc = check_step(b, dev_inj, n_var, prec, dev_flows, flow_bytes, dev_out);
  if (rc != DCFLOW_OK) return rc;
  return run_step(b, dev_inj, n_var, inj_shared ? 1 : 0, prec, dev_flows, dev_out, s);
}

int dcflow_batch_get_tuning(const dcflow_batch *b, dcflow_tuning *t) {
  if (!b || !t) return DCFLOW_E_ARG;
  *t = b->tune;
  return DCFLOW_OK;
}

int dcflow_graph_capture(dcflow_batch *b, const double *dev_inj, int32_t n_var,
                         int32_t inj_shared, dcflow_prec prec, void *dev_flows, size_t flow_bytes,
                         dcflow_score *dev_out, hipStream_t s) {
  if (!b || !s) return DCFLOW_E_ARG;
  int rc = check_step(b, dev_inj, n_var, prec, dev_flows, flow_bytes, dev_out);
  if (rc != DCFLOW_OK) return rc;
  drop_graph(b);
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_fail(e, "dcflow_graph_capture");
  rc = run_step(b, dev_inj, n_var, inj_shared ? 1 : 0, prec, dev_flows, dev_out, s);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  if (rc != DCFLOW_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "dcflow_graph_capture");
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, "dcflow_graph_capture");
  }
  b->graph = g;
  b->graph_exec = x;
  b->graph_state = dcflow_batch::StepState{b->factored,  b->flows_prec, b->flows_nvar,
                                            b->guard_valid, b->rec_valid, b->rec_prec,
                                            b->rec_nvar,   b->rec_flows,  b->rec_scores};
  return DCFLOW_OK;
}

int dcflow_graph_launch(dcflow_batch *b, hipStream_t s) {
  if (!b || !b->graph_exec) return DCFLOW_E_ARG;
  hipError_t e = hipGraphLaunch(b->graph_exec, s);
  if (e != hipSuccess) return hip_fail(e, "dcflow_graph_launch");
  // the replayed step leaves the batch as the captured one did
  const dcflow_batch::StepState &g = b->graph_state;
  b->factored = g.factored;
  b->flows_prec = g.flows_prec;
  b->flows_nvar = g.flows_nvar;
  b->guard_valid = g.guard_valid;
  b->rec_valid = g.rec_valid;
  b->rec_prec = g.rec_prec;
  b->rec_nvar = g.rec_nvar;
  b->rec_flows = g.rec_flows;
  b->rec_scores = g.rec_scores;
  return DCFLOW_OK;
}

int dcflow_eval_topologies(dcflow_batch *b, hipStream_t s) {
  if (!b) return DCFLOW_E_ARG;
  hipError_t e = launch_factors(b, s);
  if (e != hipSuccess) return hip_fail(e, "dcflow_eval_topologies");
  b->factored = 1;
  b->guard_valid = 0;
  b->rec_valid = 0;
  return DCFLOW_OK;
}

int dcflow_flow_bytes(const dcflow_batch *b, int32_t n_var, dcflow_prec prec, size_t *bytes,
                      int32_t *ld_f) {
  if (!b || !bytes || n_var < 1) return DCFLOW_E_ARG;
  if (!prec_valid(prec)) return DCFLOW_E_ARG;
  size_t el = prec == DCFLOW_FP64 ? 8 : 4;
  *bytes = std::max<size_t>((size_t)b->n_cand * n_var * b->plan->ld_er * el, 256);
  if (ld_f) *ld_f = b->plan->ld_er;
  return DCFLOW_OK;
}

int dcflow_eval_injections(dcflow_batch *b, const double *dev_inj, int32_t n_var,
                           int32_t inj_shared, dcflow_prec prec, void *dev_flows,
                           size_t flow_bytes, hipStream_t s) {
  if (!b || !dev_inj || !dev_flows) return DCFLOW_E_ARG;
  if (n_var < 1 || n_var > b->vmax) return DCFLOW_E_SHAPE;
  if (!prec_valid(prec)) return DCFLOW_E_ARG;
  if (!b->factored) return DCFLOW_E_ARG;
  if (b->d_pnv && b->pnv_nvar != n_var) return DCFLOW_E_SHAPE;
  size_t need = 0;
  dcflow_flow_bytes(b, n_var, prec, &need, nullptr);
  if (flow_bytes < need) return DCFLOW_E_WORKSPACE;
  hipError_t e =
      launch_injections(b, dev_inj, n_var, inj_shared ? 1 : 0, prec, dev_flows, 0, b->n_cand, s);
  if (e != hipSuccess) return hip_fail(e, "dcflow_eval_injections");
  b->flows_prec = prec;
  b->guard_valid = 0;
  b->rec_valid = 0;
  b->flows_nvar = n_var;
  return DCFLOW_OK;
}

int dcflow_n1_score(dcflow_batch *b, const void *dev_flows, int32_t n_var, dcflow_prec prec,
                    dcflow_score *dev_out, hipStream_t s) {
  if (!b || !dev_flows || !dev_out) return DCFLOW_E_ARG;
  if (n_var < 1 || n_var > b->vmax) return DCFLOW_E_SHAPE;
  if (!prec_valid(prec)) return DCFLOW_E_ARG;
  if (!b->factored) return DCFLOW_E_ARG;
  if (b->flows_prec != prec || b->flows_nvar != n_var) return DCFLOW_E_ARG;
  hipError_t e = launch_score(b, dev_flows, n_var, prec, dev_out, 0, b->n_cand, s);
  if (e != hipSuccess) return hip_fail(e, "dcflow_n1_score");
  return DCFLOW_OK;
}

int dcflow_n1_worst_workspace_bytes(const dcflow_batch *b, int32_t top_k, size_t *bytes) {
  if (!b || !bytes || top_k < 1 || top_k > DCFLOW_WORST_MAX) return DCFLOW_E_ARG;
  // one 16-byte entry (load, key) per list place, band and candidate (the bands, the
  // multi-outage chunks and the guard's list), then per band a threshold and the
  // band's hot columns
  const int nb = worst_bands(b->plan);
  *bytes = worst_list_bytes(b->n_cand, nb + b->nmb + 1, top_k) + worst_aux_bytes(b->n_cand, nb);
  return DCFLOW_OK;
}

}  // extern "C"

namespace {
// Arguments of dcflow_n1_worst and its allocation-free variant (all but the workspace).
int check_worst_args(const dcflow_batch *b, const void *dev_flows, int32_t n_var,
                     dcflow_prec prec, const dcflow_score *dev_scores, int32_t top_k,
                     const dcflow_case *dev_out) {
  if (!b || !dev_flows || !dev_scores || !dev_out) return DCFLOW_E_ARG;
  if (top_k < 1 || top_k > DCFLOW_WORST_MAX) return DCFLOW_E_ARG;
  if (n_var < 1 || n_var > b->vmax) return DCFLOW_E_SHAPE;
  if (!prec_valid(prec)) return DCFLOW_E_ARG;
  if (!b->factored) return DCFLOW_E_ARG;
  if (b->flows_prec != prec || b->flows_nvar != n_var) return DCFLOW_E_ARG;
  if (((int64_t)b->plan->n_out + b->plan->n_gen + b->plan->n_multi + 1) * b->plan->n_mon >
      0x7fffffffLL)
    return DCFLOW_E_ARG;
  return DCFLOW_OK;
}
}  // namespace

extern "C" {

int dcflow_n1_worst(dcflow_batch *b, const void *dev_flows, int32_t n_var, dcflow_prec prec,
                    const dcflow_score *dev_scores, int32_t top_k, void *dev_ws, size_t ws_bytes,
                    dcflow_case *dev_out, hipStream_t s) {
  if (!dev_ws) return DCFLOW_E_ARG;
  const int st = check_worst_args(b, dev_flows, n_var, prec, dev_scores, top_k, dev_out);
  if (st != DCFLOW_OK) return st;
  size_t need = 0;
  dcflow_n1_worst_workspace_bytes(b, top_k, &need);
  if (ws_bytes < need) return DCFLOW_E_WORKSPACE;
  hipError_t e = launch_worst(b, dev_flows, n_var, prec, dev_scores, top_k, dev_ws, dev_out, s);
  if (e != hipSuccess) return hip_fail(e, "dcflow_n1_worst");
  return DCFLOW_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Scratch of the allocation-free worst-case call: a file-scope device array,
// one copy per device, held until the process ends.  In host code `scratch`
// only names the host-side stand-in of the symbol; its device address is looked
// up once per device (with that device current) and kept, and only that
// address reaches kernels.
static __device__ __align__(256) unsigned char scratch[DCFLOW_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices];

// Device address of the current device's scratch array (looked up on first use).
hipError_t scratch_of_current_device(void **ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" {

int dcflow_n1_worst_noalloc(dcflow_batch *b, const void *dev_flows, int32_t n_var,
                            dcflow_prec prec, const dcflow_score *dev_scores, int32_t top_k,
                            dcflow_case *dev_out, hipStream_t s) {
  const int st = check_worst_args(b, dev_flows, n_var, prec, dev_scores, top_k, dev_out);
  if (st != DCFLOW_OK) return st;
  size_t need = 0;
  dcflow_n1_worst_workspace_bytes(b, top_k, &need);
  if (need > (size_t)DCFLOW_NOALLOC_SCRATCH_BYTES) {
    fprintf(stderr,
            "dcflow_n1_worst_noalloc: %zu bytes of scratch needed (%d candidates, top %d), "
            "the fixed array holds %zu\n",
            need, b->n_cand, top_k, (size_t)DCFLOW_NOALLOC_SCRATCH_BYTES);
    return DCFLOW_E_SCRATCH;
  }
  void *ws = nullptr;
  hipError_t e = scratch_of_current_device(&ws);
  if (e != hipSuccess) return hip_fail(e, "dcflow_n1_worst_noalloc (scratch address)");
  e = launch_worst(b, dev_flows, n_var, prec, dev_scores, top_k, ws, dev_out, s);
  if (e != hipSuccess) return hip_fail(e, "dcflow_n1_worst_noalloc");
  return DCFLOW_OK;
}

int dcflow_n1_worst_per_case_workspace_bytes(const dcflow_batch *b, int32_t per_case,
                                             size_t *bytes) {
  if (!b || !bytes || per_case < 1 || per_case > DCFLOW_WORST_MAX) return DCFLOW_E_ARG;
  // one 16-byte entry (load, key) per list place, case and candidate, then the case
  // maxima of the pruning sweep
  *bytes = std::max<size_t>(per_case_workspace(b, per_case), 256);
  return DCFLOW_OK;
}

int dcflow_n1_worst_per_case(dcflow_batch *b, const void *dev_flows, int32_t n_var,
                             dcflow_prec prec, const dcflow_score *dev_scores, int32_t per_case,
                             int32_t top_k, void *dev_ws, size_t ws_bytes, dcflow_case *dev_out,
                             hipStream_t s) {
  if (!b || !dev_flows || !dev_scores || !dev_ws || !dev_out) return DCFLOW_E_ARG;
  if (top_k < 1 || top_k > DCFLOW_WORST_MAX) return DCFLOW_E_ARG;
  if (per_case < 1 || per_case > DCFLOW_WORST_MAX) return DCFLOW_E_ARG;
  if (n_var < 1 || n_var > b->vmax) return DCFLOW_E_SHAPE;
  if (!prec_valid(prec)) return DCFLOW_E_ARG;
  if (!b->factored) return DCFLOW_E_ARG;
  if (b->flows_prec != prec || b->flows_nvar != n_var) return DCFLOW_E_ARG;
  if ((int64_t)per_case_slots(b->plan) * b->plan->n_mon > 0x7fffffffLL) return DCFLOW_E_ARG;
  size_t need = 0;
  dcflow_n1_worst_per_case_workspace_bytes(b, per_case, &need);
  if (ws_bytes < need) return DCFLOW_E_WORKSPACE;
  hipError_t e = launch_worst_per_case(b, dev_flows, n_var, prec, dev_scores, per_case, top_k,
                                       dev_ws, dev_out, s);
  if (e != hipSuccess) return hip_fail(e, "dcflow_n1_worst_per_case");
  return DCFLOW_OK;
}

int dcflow_set_busbar_injections(dcflow_batch *b, const double *dev_pnew, int32_t n_var) {
  if (!b) return DCFLOW_E_ARG;
  if (dev_pnew && (n_var < 1 || n_var > b->vmax)) return DCFLOW_E_SHAPE;
  b->d_pnv = dev_pnew;
  b->pnv_nvar = dev_pnew ? n_var : 0;
  return DCFLOW_OK;
}

const double *dcflow_batch_variant_max(const dcflow_batch *b) { return b ? b->d_vmax : nullptr; }

// Stub folding: leaves of the branch graph (degree one, not the slack, not
// protected) are pruned one after another; each pruned bus remembers the branch
// that connected it, whose other end is its parent.
int dcflow_fold_stubs(int32_t n_bus, int32_t n_branch, int32_t slack, const int32_t *from,
                      const int32_t *to, const uint8_t *protect, int32_t *bus_new,
                      int32_t *branch_new, int32_t *up_branch, int32_t *n_bus_out,
                      int32_t *n_branch_out) {
  if (!from || !to || !bus_new || !branch_new || !up_branch || !n_bus_out || !n_branch_out)
    return DCFLOW_E_ARG;
  if (n_bus < 1 || n_branch < 0 || slack < 0 || slack >= n_bus) return DCFLOW_E_SHAPE;
  for (int l = 0; l < n_branch; ++l)
    if (from[l] < 0 || from[l] >= n_bus || to[l] < 0 || to[l] >= n_bus || from[l] == to[l])
      return DCFLOW_E_SHAPE;
  std::vector<int> deg(n_bus, 0), off(n_bus + 1, 0), adj(2 * (size_t)n_branch);
  for (int l = 0; l < n_branch; ++l) {
    ++deg[from[l]];
    ++deg[to[l]];
  }
  for (int b = 0; b < n_bus; ++b) off[b + 1] = off[b] + deg[b];
  {
    std::vector<int> fill(off.begin(), off.end() - 1);
    for (int l = 0; l < n_branch; ++l) {
      adj[fill[from[l]]++] = l;
      adj[fill[to[l]]++] = l;
    }
  }
  std::vector<uint8_t> br_cut(n_branch, 0), bus_cut(n_bus, 0);
  auto foldable = [&](int b) { return b != slack && !(protect && protect[b]) && deg[b] == 1; };
  std::vector<int> stack, order;
  for (int b = 0; b < n_bus; ++b)
    if (foldable(b)) stack.push_back(b);
  for (int b = 0; b < n_bus; ++b) up_branch[b] = -1;
  while (!stack.empty()) {
    const int b = stack.back();
    stack.pop_back();
    if (bus_cut[b] || !foldable(b)) continue;
    int l = -1;
    for (int i = off[b]; i < off[b + 1]; ++i)
      if (!br_cut[adj[i]]) l = adj[i];
    const int p = from[l] == b ? to[l] : from[l];
    bus_cut[b] = 1;
    br_cut[l] = 1;
    up_branch[b] = l;
    order.push_back(b);
    --deg[b];
    if (--deg[p] == 1 && foldable(p)) stack.push_back(p);
  }
  int nb = 0, nl = 0;
  for (int b = 0; b < n_bus; ++b) bus_new[b] = bus_cut[b] ? -1 : nb++;
  for (int l = 0; l < n_branch; ++l) branch_new[l] = br_cut[l] ? -1 : nl++;
  // a pruned bus's parent is kept or was pruned later: walk the pruning order backwards
  for (size_t i = order.size(); i-- > 0;) {
    const int b = order[i], l = up_branch[b];
    bus_new[b] = bus_new[from[l] == b ? to[l] : from[l]];
  }
  *n_bus_out = nb;
  *n_branch_out = nl;
  return DCFLOW_OK;
}

int dcflow_fold_injections(int32_t n_bus, const int32_t *bus_new, int32_t n_bus_out,
                           const double *x, int32_t n_var, double *x_out) {
  if (!bus_new || !x || !x_out) return DCFLOW_E_ARG;
  if (n_bus < 1 || n_bus_out < 1 || n_var < 0) return DCFLOW_E_SHAPE;
  for (int b = 0; b < n_bus; ++b)
    if (bus_new[b] < 0 || bus_new[b] >= n_bus_out) return DCFLOW_E_SHAPE;
  for (int v = 0; v < n_var; ++v) {
    double *o = x_out + (size_t)v * n_bus_out;
    std::fill(o, o + n_bus_out, 0.0);
    for (int b = 0; b < n_bus; ++b) o[bus_new[b]] += x[(size_t)v * n_bus + b];
  }
  return DCFLOW_OK;
}

int dcflow_stub_flows(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to,
                      const int32_t *up_branch, const double *x, int32_t n_var, double *flow) {
  if (!from || !to || !up_branch || !x || !flow) return DCFLOW_E_ARG;
  if (n_bus < 1 || n_branch < 0 || n_var < 0) return DCFLOW_E_SHAPE;
  // children before parents: folded buses by decreasing depth below the kept grid
  std::vector<int> depth(n_bus, -1), folded;
  for (int b = 0; b < n_bus; ++b) {
    const int l = up_branch[b];
    if (l < -1 || l >= n_branch || (l >= 0 && from[l] != b && to[l] != b)) return DCFLOW_E_SHAPE;
    if (l >= 0) folded.push_back(b);
  }
  for (int b : folded) {
    int d = 0, c = b;
    while (up_branch[c] >= 0) {
      const int l = up_branch[c];
      c = from[l] == c ? to[l] : from[l];
      if (++d > n_bus) return DCFLOW_E_SHAPE;  // a cycle: not a pruning forest
    }
    depth[b] = d;
  }
  std::sort(folded.begin(), folded.end(), [&](int a, int b) { return depth[a] > depth[b]; });
  std::vector<double> sub(n_bus);
  for (int v = 0; v < n_var; ++v) {
    const double *xv = x + (size_t)v * n_bus;
    double *fv = flow + (size_t)v * n_branch;
    std::fill(fv, fv + n_branch, 0.0);
    std::copy(xv, xv + n_bus, sub.begin());
    for (int b : folded) {
      const int l = up_branch[b], p = from[l] == b ? to[l] : from[l];
      fv[l] = from[l] == b ? sub[b] : -sub[b];
      sub[p] += sub[b];
    }
  }
  return DCFLOW_OK;
}

const char *dcflow_strerror(int st) {
  switch (st) {
    case DCFLOW_OK: return "ok";
    case DCFLOW_E_ARG: return "invalid argument";
    case DCFLOW_E_SHAPE: return "index or size out of range";
    case DCFLOW_E_DISCONNECTED: return "base grid is not connected";
    case DCFLOW_E_WORKSPACE: return "device buffer too small";
    case DCFLOW_E_HIP: return "HIP runtime error";
    case DCFLOW_E_CAND: return "malformed candidate record";
    case DCFLOW_E_SCRATCH: return "input too large for the fixed scratch array";
    case DCFLOW_E_TUNING: return "launch shape of the tuning does not fit this batch";
    default: return "unknown status";
  }
}

}  // extern "C"
