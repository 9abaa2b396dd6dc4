// Branch module: per-candidate low-rank factors (paper Sec. III-C steps 2-4).
//
// The paper applies each bus split by a BSDF update (Def. eq_bsdf,
// Eq. bsdf_application), remedial outages by a MODF update (Def. eq_modf) and
// then forms the LODF of the changed grid (Def. eq_lodf).  Here all k <= 8
// changes of a candidate are joined into one k x k system (the same updates,
// solved together instead of in sequence), and the changed PTDF is never
// materialised:
//
//   element j  injection pattern a_j, flow correction c_j, sensing row sigma_j
//     outage o       a = e_f - e_t,            c = e_o,        sigma = e_o
//     split of A     a = e_A - sum_M w_l e_far(l),  c = sum_M s_l w_l e_l,
//     moving M to B  sigma = sum_M s_l e_l,    w_l = b_l / sum_M b,
//                    s_l = +1 if the branch leaves A, -1 if it enters A
//                    (branches of M that are also outaged are left out)
//   u_j = H a_j - c_j,  K = -[sigma_i . u_j],  PTDF' x = H x + U K^-1 (sigma . H x - pi . x)
//   with pi_j . x the injection on the new busbar of split j.  The constraints
//   are zero flow on outaged branches and Kirchhoff's law on each new busbar;
//   K is singular exactly when the candidate grid is islanded.
//
//   For a contingency c (post-change terminals) the LODF column of the changed
//   grid is col_c = H_O[:, c] + U W[:, c], W = K^-1 R,
//   R[i, c] = sigma_i . H_O[:, c] - pi_i . d_c, den_c = 1 - col_c[c].
//   A generator outage (Eq. ptdf_delta, Sec. III-C step 8d) is one more column
//   with H_O[:, g] = H e_bus and d_g = e_bus: col_g is the changed grid's PTDF
//   column of the bus, with no denominator (1/den stored as 1).
//
// Outputs per candidate (element-major, no padding between uneven ranks):
//   U [elem][ld_er], W [elem][ld_o], K^-1 (8 x 8), 1/den_c (0 for islanding
//   or already-removed contingencies), islanding bits, status, sensing lists.
#include "dcflow_internal.h"

namespace dcflow {
namespace {

struct Elem {
  int kind, id, nsig, na;
  int sig_br[kMaxSig];
  double sig_s[kMaxSig];
  double sig_w[kMaxSig];
  int a_node[kMaxSig + 1];
  double a_val[kMaxSig + 1];
};

__global__ void __launch_bounds__(256)
k_factors(const int32_t *__restrict__ order, const int32_t *__restrict__ off,
          const int32_t *__restrict__ kind, const int32_t *__restrict__ id,
          const uint32_t *__restrict__ mask, const int32_t *__restrict__ f,
          const int32_t *__restrict__ t, const double *__restrict__ b,
          const int32_t *__restrict__ adj_off, const int32_t *__restrict__ adj_br,
          const double *__restrict__ Hb, int ld_h, const double *__restrict__ Ht, int ld_er,
          int n_er, const double *__restrict__ hdo, int ld_o, const int32_t *__restrict__ out,
          const int32_t *__restrict__ out_pos, int n_out, int n_ctg,
          const int32_t *__restrict__ pos_of_br,
          int32_t *__restrict__ nsig_g, int32_t *__restrict__ sig_g, double *__restrict__ U,
          double *__restrict__ W, double *__restrict__ kinv_g, double *__restrict__ invden,
          uint32_t *__restrict__ isl, uint32_t *__restrict__ status) {
  __shared__ Elem E[kMaxRank];
  __shared__ double K[kMaxRank][2 * kMaxRank];
  __shared__ double Ki[kMaxRank][kMaxRank];
  __shared__ int s_flags;
  __shared__ int s_island;

  const int cand = order[blockIdx.x];
  const int e0 = off[cand];
  const int k = off[cand + 1] - e0;
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  if (tid == 0) {
    s_flags = 0;
    s_island = 0;
  }
  __syncthreads();

  // ---- decode elements
  if (tid < k) {
    Elem &el = E[tid];
    el.kind = kind[e0 + tid];
    el.id = id[e0 + tid];
    if (el.kind == DCFLOW_OUTAGE) {
      int o = el.id;
      el.nsig = 1;
      el.sig_br[0] = o;
      el.sig_s[0] = 1.0;
      el.sig_w[0] = 1.0;
      el.na = 2;
      el.a_node[0] = f[o];
      el.a_val[0] = 1.0;
      el.a_node[1] = t[o];
      el.a_val[1] = -1.0;
    } else {
      int A = el.id;
      uint32_t mk = mask[e0 + tid];
      int deg = adj_off[A + 1] - adj_off[A];
      double beta = 0.0;
      int ns = 0;
      for (int q = 0; q < deg; ++q) {
        if (!((mk >> q) & 1u)) continue;
        int br = adj_br[adj_off[A] + q];
        bool removed = false;
        for (int j = 0; j < k; ++j)
          if (kind[e0 + j] == DCFLOW_OUTAGE && id[e0 + j] == br) removed = true;
        if (removed) continue;
        double s = f[br] == A ? 1.0 : -1.0;
        el.sig_br[ns] = br;
        el.sig_s[ns] = s;
        el.sig_w[ns] = b[br];
        el.a_node[1 + ns] = s > 0 ? t[br] : f[br];
        beta += b[br];
        ++ns;
      }
      el.nsig = ns;
      el.na = ns + 1;
      el.a_node[0] = A;
      el.a_val[0] = 1.0;
      for (int q = 0; q < ns; ++q) {
        el.sig_w[q] /= beta;
        el.a_val[1 + q] = -el.sig_w[q];
      }
      if (ns == 0) atomicOr(&s_flags, (int)(DCFLOW_ST_DISCONNECTED));
    }
    nsig_g[e0 + tid] = el.nsig;
    for (int q = 0; q < kMaxSig; ++q)
      sig_g[(size_t)(e0 + tid) * kMaxSig + q] =
          q < el.nsig ? (el.sig_s[q] > 0 ? el.sig_br[q] + 1 : -(el.sig_br[q] + 1)) : 0;
  }
  __syncthreads();

  // ---- K = -G, G_ij = sigma_i . H a_j - sigma_i . c_j   (one wave per entry)
  for (int p = wv; p < k * k; p += 4) {
    int i = p / k, j = p % k;
    const Elem &ei = E[i];
    const Elem &ej = E[j];
    int terms = ei.nsig * ej.na;
    double acc = 0.0;
    for (int q = lane; q < terms; q += kWave) {
      int qi = q / ej.na, qj = q % ej.na;
      acc += ei.sig_s[qi] * ej.a_val[qj] * Hb[(size_t)ei.sig_br[qi] * ld_h + ej.a_node[qj]];
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      double sc = 0.0;  // sigma_i . c_j
      for (int qi = 0; qi < ei.nsig; ++qi)
        for (int qj = 0; qj < ej.nsig; ++qj)
          if (ei.sig_br[qi] == ej.sig_br[qj]) sc += ei.sig_s[qi] * ej.sig_s[qj] * ej.sig_w[qj];
      K[i][j] = -(acc - sc);
    }
  }
  __syncthreads();

  // ---- K^-1 by Gauss-Jordan with partial pivoting (k <= 8, one thread)
  if (tid == 0) {
    double scale = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        scale = fmax(scale, fabs(K[i][j]));
        K[i][k + j] = i == j ? 1.0 : 0.0;
      }
    bool sing = false;
    for (int c = 0; c < k && !sing; ++c) {
      int pr = c;
      for (int r = c + 1; r < k; ++r)
        if (fabs(K[r][c]) > fabs(K[pr][c])) pr = r;
      if (!(fabs(K[pr][c]) > kSingularTol * fmax(scale, 1.0))) {
        sing = true;
        break;
      }
      if (pr != c)
        for (int q = 0; q < 2 * k; ++q) {
          double tmp = K[c][q];
          K[c][q] = K[pr][q];
          K[pr][q] = tmp;
        }
      double ip = 1.0 / K[c][c];
      for (int q = 0; q < 2 * k; ++q) K[c][q] *= ip;
      for (int r = 0; r < k; ++r) {
        if (r == c) continue;
        double fr = K[r][c];
        if (fr != 0.0)
          for (int q = 0; q < 2 * k; ++q) K[r][q] -= fr * K[c][q];
      }
    }
    if (sing) s_flags |= (int)(DCFLOW_ST_DISCONNECTED | DCFLOW_ST_SINGULAR);
    bool bad = s_flags != 0;
    for (int i = 0; i < kMaxRank; ++i)
      for (int j = 0; j < kMaxRank; ++j)
        Ki[i][j] = (!bad && i < k && j < k) ? K[i][k + j] : 0.0;
  }
  __syncthreads();
  const bool bad = s_flags != 0;
  if (tid < 64) kinv_g[(size_t)cand * 64 + tid] = Ki[tid / 8][tid % 8];

  // ---- U columns over the kept rows: u_j = H a_j (node-major gathers)
  for (int j = 0; j < k; ++j) {
    const Elem &ej = E[j];
    double *Uj = U + (size_t)(e0 + j) * ld_er;
    for (int pos = tid; pos < ld_er; pos += blockDim.x) {
      double u = 0.0;
      if (pos < n_er && !bad)
        for (int r = 0; r < ej.na; ++r) u += ej.a_val[r] * Ht[(size_t)ej.a_node[r] * ld_er + pos];
      Uj[pos] = u;
    }
  }
  __syncthreads();
  // ... minus c_j on the kept rows (each (j, branch) entry is touched once)
  if (!bad && tid < k * kMaxSig) {
    int j = tid / kMaxSig, q = tid % kMaxSig;
    if (q < E[j].nsig) {
      int pos = pos_of_br[E[j].sig_br[q]];
      if (pos >= 0) U[(size_t)(e0 + j) * ld_er + pos] -= E[j].sig_s[q] * E[j].sig_w[q];
    }
  }
  __syncthreads();

  // ---- W = K^-1 R and LODF denominators per contingency
  int nisl = 0;
  for (int c = tid; c < ld_o; c += blockDim.x) {
    double r[kMaxRank];
    double w[kMaxRank];
    bool removed = false;
    if (c < n_ctg && !bad) {
      // generator column (c >= n_out): no branch of its own; the lost output is
      // taken from busbar A, so the busbar-B term pi_i . d_c is zero as well
      const int oc = c < n_out ? out[c] : -1;
      for (int i = 0; i < k; ++i) {
        const Elem &ei = E[i];
        double acc = 0.0;
        for (int q = 0; q < ei.nsig; ++q) {
          int br = ei.sig_br[q];
          acc += ei.sig_s[q] * (hdo[(size_t)br * ld_o + c] - (br == oc ? 1.0 : 0.0));
        }
        r[i] = acc;
        if (ei.kind == DCFLOW_OUTAGE && ei.id == oc) removed = true;
      }
      for (int j = 0; j < k; ++j) {
        double acc = 0.0;
        for (int i = 0; i < k; ++i) acc += Ki[j][i] * r[i];
        w[j] = acc;
      }
    } else {
      for (int j = 0; j < k; ++j) w[j] = 0.0;
    }
    for (int j = 0; j < k; ++j) W[(size_t)(e0 + j) * ld_o + c] = w[j];
    double inv = 0.0;
    bool island = false;
    if (c < n_out && !bad && !removed) {
      int pc = out_pos[c];
      double col = hdo[(size_t)out[c] * ld_o + c];
      for (int j = 0; j < k; ++j) col += U[(size_t)(e0 + j) * ld_er + pc] * w[j];
      double den = 1.0 - col;
      if (fabs(den) < kIslandTol) {
        island = true;
        ++nisl;
      } else {
        inv = 1.0 / den;
      }
    } else if (c >= n_out && c < n_ctg && !bad) {
      inv = 1.0;  // generator outage: no denominator, never islanding
    }
    invden[(size_t)cand * ld_o + c] = inv;
    // islanding bits, one 32-bit word per 32 contingencies (ballot within the wave)
    unsigned long long bal = __ballot(island);
    if ((c % 32) == 0) {
      int sh = lane & 32;
      isl[(size_t)cand * (ld_o / 32) + c / 32] = (uint32_t)(bal >> sh);
    }
  }
  nisl = wave_sum(nisl);
  if (lane == 0) atomicAdd(&s_island, nisl);
  __syncthreads();
  if (tid == 0) status[cand] = (uint32_t)s_flags | ((uint32_t)s_island << DCFLOW_ST_ISLAND_SHIFT);
}

}  // namespace

// Operands of the FP32 scan's tile build, rounded once per evaluation instead
// of once per tile: U / r on the padded monitored rows and W, in FP32 (the same
// FP64 products the tile build would round).  One workgroup per element (grid-
// stride); it also records the element's largest |U / r| over the monitored rows
// (inv_r is zero on the padding), which the error guard of the FP32 scan uses.
__global__ void __launch_bounds__(256)
k_frags(const double *__restrict__ U, int ld_er, const double *__restrict__ inv_r, int mon_pad,
        const double *__restrict__ W, int ld_o, size_t n_elem, float *__restrict__ ur32,
        float *__restrict__ w32, float *__restrict__ umax) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  for (size_t e = blockIdx.x; e < n_elem; e += gridDim.x) {
    const double *u = U + e * ld_er;
    float *ur = ur32 + e * mon_pad;
    double m = 0.0;
    for (int r = tid; r < mon_pad; r += blockDim.x) {
      const double v = u[r] * inv_r[r];
      ur[r] = (float)v;
      m = fmax(m, fabs(v));
    }
    const double *w = W + e * ld_o;
    float *wf = w32 + e * ld_o;
    for (int c = tid; c < ld_o; c += blockDim.x) wf[c] = (float)w[c];
    m = wave_max(m);
    if (tid % kWave == 0) red[tid / kWave] = m;
    __syncthreads();
    if (tid == 0) umax[e] = (float)fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
  }
}

namespace {

// Branch-module step 5 for multi-outage N-1 cases (Sec. IV-D: formed once per
// candidate here, applied to every injection variant by the scan).  With the LODF' numerator
// columns n_j = col_{s_j} - e_{s_j} of the changed grid (col as above), tripping
// the branch set S of a case gives p = p1 + sum_j n_j z_j with z = -N^-1 p1[S] and
// N[i][j] = n_j[s_i]: the flows on every branch of S become zero (Def. eq_modf,
// one system per case).  N singular: S islands the candidate grid.  A branch the
// candidate already removed drops out (identity row and column of N, z_j = 0); a
// branch whose single outage islands makes the whole case island.
// One thread per (candidate, case); coef holds -N^-1 (row j: coefficients of z_j).
__global__ void __launch_bounds__(64) k_multi_prep(
    const int32_t *__restrict__ off, const double *__restrict__ U, int ld_er,
    const double *__restrict__ W, int ld_o, const double *__restrict__ hdo,
    const int32_t *__restrict__ out, const int32_t *__restrict__ out_pos,
    const double *__restrict__ invden, const uint32_t *__restrict__ isl,
    uint32_t *__restrict__ status, const int32_t *__restrict__ moff,
    const int32_t *__restrict__ mcol, int n_multi, double *__restrict__ coef,
    int32_t *__restrict__ mok) {
  __shared__ int s_isl;
  const int cand = blockIdx.x;
  const int e0 = off[cand], k = off[cand + 1] - e0;
  const uint32_t st = status[cand];
  const bool bad = (st & (DCFLOW_ST_DISCONNECTED | DCFLOW_ST_SINGULAR)) != 0;
  if (threadIdx.x == 0) s_isl = 0;
  __syncthreads();
  constexpr int MM = DCFLOW_MULTI_MAX;
  for (int q = threadIdx.x; q < n_multi; q += blockDim.x) {
    const int a = moff[q], m = moff[q + 1] - a;
    // all loops below run over MM with guards, so that the arrays stay in registers
    int col[MM], pos[MM];
    bool rem[MM];
    bool island = false;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      col[j] = j < m ? mcol[a + j] : 0;
      pos[j] = out_pos[col[j]];
      const bool ib = ((isl[(size_t)cand * (ld_o / 32) + col[j] / 32] >> (col[j] % 32)) & 1u) != 0;
      rem[j] = j < m && !ib && invden[(size_t)cand * ld_o + col[j]] == 0.0;
      island = island || (j < m && ib);
    }
    double A[MM][MM], Bi[MM][MM];  // N, then its inverse by Gauss-Jordan on [N | I]
    bool ok = !bad && !island;
#pragma unroll
    for (int i = 0; i < MM; ++i)
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        double v = i == j ? 1.0 : 0.0;  // identity outside the case and for removed branches
        if (ok && i < m && j < m && !rem[i] && !rem[j]) {
          v = hdo[(size_t)out[col[i]] * ld_o + col[j]] - v;
          for (int e = 0; e < k; ++e)
            v += U[(size_t)(e0 + e) * ld_er + pos[i]] * W[(size_t)(e0 + e) * ld_o + col[j]];
        }
        A[i][j] = v;
        Bi[i][j] = i == j ? 1.0 : 0.0;
      }
#pragma unroll
    for (int c = 0; c < MM; ++c) {
      // partial pivoting: the largest |A[r][c]| among r >= c, swapped into row c
      int pr = c;
      double pv = fabs(A[c][c]);
#pragma unroll
      for (int r = c + 1; r < MM; ++r)
        if (fabs(A[r][c]) > pv) {
          pv = fabs(A[r][c]);
          pr = r;
        }
      if (c < m && pv < kIslandTol) ok = false;
#pragma unroll
      for (int r = c + 1; r < MM; ++r)
        if (r == pr)
#pragma unroll
          for (int x = 0; x < MM; ++x) {
            double t = A[c][x];
            A[c][x] = A[r][x];
            A[r][x] = t;
            t = Bi[c][x];
            Bi[c][x] = Bi[r][x];
            Bi[r][x] = t;
          }
      const double inv = pv > 0.0 ? 1.0 / A[c][c] : 0.0;
#pragma unroll
      for (int x = 0; x < MM; ++x) {
        A[c][x] *= inv;
        Bi[c][x] *= inv;
      }
#pragma unroll
      for (int r = 0; r < MM; ++r) {
        if (r == c) continue;
        const double f = A[r][c];
#pragma unroll
        for (int x = 0; x < MM; ++x) {
          A[r][x] -= f * A[c][x];
          Bi[r][x] -= f * Bi[c][x];
        }
      }
    }
    if (!bad && !ok) island = true;
    if (!bad && island) atomicAdd(&s_isl, 1);
    double *cq = coef + ((size_t)cand * n_multi + q) * 16;
#pragma unroll
    for (int j = 0; j < MM; ++j)
#pragma unroll
      for (int i = 0; i < MM; ++i)
        cq[j * 4 + i] = (ok && j < m && i < m && !rem[j]) ? -Bi[j][i] : 0.0;
    mok[(size_t)cand * n_multi + q] = ok ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0 && s_isl > 0) status[cand] = st + ((uint32_t)s_isl << DCFLOW_ST_ISLAND_SHIFT);
}

}  // namespace

hipError_t launch_factors(dcflow_batch *bt, hipStream_t s) {
  dcflow_plan *p = bt->plan;
  if (bt->n_cand == 0) return hipSuccess;
  hipLaunchKernelGGL(k_factors, dim3(bt->n_cand), dim3(256), 0, s, bt->d_order, bt->d_off,
                     bt->d_kind, bt->d_id, bt->d_mask, p->d_f, p->d_t, p->d_b, p->d_adj_off,
                     p->d_adj_br, p->d_hb, p->ld_h, p->d_ht, p->ld_er, p->n_er, p->d_hdo, p->ld_o,
                     p->d_out, p->d_out_pos, p->n_out, p->n_out + p->n_gen, p->d_pos_of_br,
                     bt->d_nsig, bt->d_sig,
                     bt->d_U, bt->d_W, bt->d_kinv, bt->d_invden, bt->d_isl, bt->d_status);
  DCF_CHECK_LAUNCH();
  const size_t n_elem = bt->n_elem;
  if (n_elem) {
    const size_t nb = std::min<size_t>(n_elem, 16384);
    k_frags<<<dim3((unsigned)nb), dim3(256), 0, s>>>(bt->d_U, p->ld_er, p->d_inv_r, p->mon_pad,
                                                     bt->d_W, p->ld_o, n_elem, bt->d_ur32,
                                                     bt->d_w32, bt->d_umax);
    DCF_CHECK_LAUNCH();
  }
  if (p->n_multi > 0) {
    k_multi_prep<<<dim3(bt->n_cand), dim3(64), 0, s>>>(
        bt->d_off, bt->d_U, p->ld_er, bt->d_W, p->ld_o, p->d_hdo, p->d_out, p->d_out_pos,
        bt->d_invden, bt->d_isl, bt->d_status, p->d_moff, p->d_mcol, p->n_multi, bt->d_mcoef,
        bt->d_mok);
    DCF_CHECK_LAUNCH();
  }
  return hipSuccess;
}

}  // namespace dcflow
