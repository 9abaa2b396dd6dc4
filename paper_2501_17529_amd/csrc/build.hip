// One-time FP64 base build (the paper's Sec. II, Def. eq_ptdf with the row
// restriction that follows it, and Eq. ptdf_times_nodal_inj for base flows).
//
//   B'  : slack-reduced nodal susceptance matrix (Laplacian), assembled per bus
//         from the adjacency lists (no atomics, deterministic);
//   B'^-1 by in-place blocked Gauss-Jordan (B' is symmetric positive definite
//         for a connected grid, so no pivoting is needed; the trailing updates
//         run on the FP64 matrix cores); the slack row/column are a unit so the
//         matrix stays n x n;
//   PTDF rows H[l, x] = b_l (B'^-1[f_l, x] - B'^-1[t_l, x]), slack column 0,
//         which is PTDF' = C_w' B'^-1 written out per row;
//   derived operands: node-major kept rows (column gathers of the branch
//         module), the GEMM operand in FP64/FP32, contingency transfer columns
//         H[:, f_c] - H[:, t_c], base flows, ratings and the rating-scaled
//         LODF seed Lsd = (hdo[mon] - [mon == c]) / r used by the N-1 scan.
#include "dcflow_internal.h"

namespace dcflow {
namespace {

__global__ void k_fill(double *p, size_t n, double v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_f(float *p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.f;
}

// Row i of the reduced Laplacian is written by thread i only.
__global__ void k_assemble(double *B, int ld, int n, int slack, const int32_t *adj_off,
                           const int32_t *adj_br, const int32_t *f, const int32_t *t,
                           const double *b) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double *row = B + (size_t)i * ld;
  if (i == slack) {
    row[i] = 1.0;
    return;
  }
  double diag = 0.0;
  for (int q = adj_off[i]; q < adj_off[i + 1]; ++q) {
    int br = adj_br[q];
    int other = f[br] == i ? t[br] : f[br];
    diag += b[br];
    if (other != slack) row[other] -= b[br];
  }
  row[i] += diag;
}

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan inversion in place (B' is symmetric positive definite,
// so the pivots need no search).  With the matrix split into 64-wide blocks and
// K the current diagonal block, one step is
//   P = A[K, K]^-1                       (k_bgj_panel: one workgroup, in LDS)
//   A[K, J] <- P A[K, J]          J != K (k_bgj_rows)
//   A[I, J] <- A[I, J] - A[I, K] A[K, J]   I, J != K (k_bgj_update, FP64 MFMA)
//   A[I, K] <- -A[I, K] P,  A[K, K] <- P   (k_bgj_cols)
// and after the last block A holds the inverse.  The matrix is padded to a
// multiple of 64 with unit diagonal (its inverse stays unit there).
constexpr int kGjB = 64;

// P = inverse of the 64 x 64 diagonal block at p0 by Gauss-Jordan, the block in
// registers: thread t holds row t / 4, columns 16 (t % 4) .. + 15.  Per pivot q the
// owners of row q and of column q post them to LDS (two buffers, so that one
// barrier per pivot suffices) and every thread updates its 16 values.
__global__ void __launch_bounds__(256) k_bgj_panel(const double *A, int ld, int p0, double *P) {
  __shared__ double prow[2][kGjB], pcol[2][kGjB];
  const int tid = threadIdx.x, r = tid >> 2, c0 = (tid & 3) * 16;
  double v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = A[(size_t)(p0 + r) * ld + p0 + c0 + j];
#pragma unroll
  for (int q = 0; q < kGjB; ++q) {
    const int bf = q & 1;
    if (r == q)
#pragma unroll
      for (int j = 0; j < 16; ++j) prow[bf][c0 + j] = v[j];
    if ((tid & 3) == q / 16) pcol[bf][r] = v[q % 16];
    __syncthreads();
    const double ip = 1.0 / prow[bf][q];
    const double pc = pcol[bf][r];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int c = c0 + j;
      const double pr = prow[bf][c];
      double x;
      if (r == q)
        x = c == q ? ip : pr * ip;
      else if (c == q)
        x = -pc * ip;
      else
        x = v[j] - pc * (pr * ip);
      v[j] = x;
    }
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) P[r * kGjB + c0 + j] = v[j];
}

// A[K, J] <- P A[K, J] for the 64-column block J = blockIdx.x (skipping K).
__global__ void __launch_bounds__(256) k_bgj_rows(double *A, int ld, int p0, const double *P) {
  __shared__ double Ps[kGjB][kGjB + 1];
  __shared__ double X[kGjB][kGjB + 1];
  const int j0 = blockIdx.x * kGjB;
  if (j0 == p0) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < kGjB * kGjB; e += blockDim.x) {
    const int r = e / kGjB, c = e % kGjB;
    Ps[r][c] = P[e];
    X[r][c] = A[(size_t)(p0 + r) * ld + j0 + c];
  }
  __syncthreads();
  for (int e = tid; e < kGjB * kGjB; e += blockDim.x) {
    const int r = e / kGjB, c = e % kGjB;
    double v = 0.0;
#pragma unroll 8
    for (int q = 0; q < kGjB; ++q) v = __builtin_fma(Ps[r][q], X[q][c], v);
    A[(size_t)(p0 + r) * ld + j0 + c] = v;
  }
}

// A[I, K] <- -A[I, K] P for the 64-row block I = blockIdx.x; the block I = K gets P.
__global__ void __launch_bounds__(256) k_bgj_cols(double *A, int ld, int p0, const double *P) {
  __shared__ double Ps[kGjB][kGjB + 1];
  __shared__ double X[kGjB][kGjB + 1];
  const int i0 = blockIdx.x * kGjB;
  const int tid = threadIdx.x;
  if (i0 == p0) {
    for (int e = tid; e < kGjB * kGjB; e += blockDim.x)
      A[(size_t)(p0 + e / kGjB) * ld + p0 + e % kGjB] = P[e];
    return;
  }
  for (int e = tid; e < kGjB * kGjB; e += blockDim.x) {
    const int r = e / kGjB, c = e % kGjB;
    Ps[r][c] = P[e];
    X[r][c] = A[(size_t)(i0 + r) * ld + p0 + c];
  }
  __syncthreads();
  for (int e = tid; e < kGjB * kGjB; e += blockDim.x) {
    const int r = e / kGjB, c = e % kGjB;
    double v = 0.0;
#pragma unroll 8
    for (int q = 0; q < kGjB; ++q) v = __builtin_fma(X[r][q], Ps[q][c], v);
    A[(size_t)(i0 + r) * ld + p0 + c] = -v;
  }
}

// Trailing update A[I, J] -= A[I, K] A[K, J] over 128 x 128 tiles (4 waves of
// 64 x 64, FP64 16x16x4 MFMA, the tile's rows of A[I, K] staged in LDS, the
// A[K, J] fragments read from global memory: 16 consecutive doubles per lane
// group).  Rows and columns of K are left alone (the other kernels own them).
__global__ void __launch_bounds__(256) k_bgj_update(double *A, int ld, int p0) {
  __shared__ double As[128][kGjB + 1];
  const int i0 = blockIdx.y * 128, j0 = blockIdx.x * 128;
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, g = lane / 16, li = lane % 16;
  for (int e = tid; e < 128 * kGjB; e += blockDim.x) {
    const int r = e / kGjB, c = e % kGjB;
    const int i = i0 + r;
    As[r][c] = i < ld ? A[(size_t)i * ld + p0 + c] : 0.0;
  }
  __syncthreads();
  const int wr = (wv / 2) * 64, wc = (wv % 2) * 64;  // this wave's 64 x 64 sub-tile
  if (i0 + wr >= ld || j0 + wc >= ld) return;
  if (i0 + wr == p0 || j0 + wc == p0) return;  // a K row or column block
  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        acc[a][b][r] = A[(size_t)(i0 + wr + a * 16 + g + 4 * r) * ld + j0 + wc + b * 16 + li];
  for (int h = 0; h < kGjB / 4; ++h) {
    const int kk = 4 * h + g;
    double fa[4], fb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) fa[a] = -As[wr + a * 16 + li][kk];
#pragma unroll
    for (int b = 0; b < 4; ++b) fb[b] = A[(size_t)(p0 + kk) * ld + j0 + wc + b * 16 + li];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        A[(size_t)(i0 + wr + a * 16 + g + 4 * r) * ld + j0 + wc + b * 16 + li] = acc[a][b][r];
}

// Unit diagonal on the padding rows n .. ld - 1.
__global__ void k_pad_diag(double *A, int ld, int n) {
  const int i = n + blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ld) A[(size_t)i * ld + i] = 1.0;
}

__global__ void k_ptdf_rows(double *H, int ld, int n, int m, int slack, const double *Binv,
                            int lb, const int32_t *f, const int32_t *t, const double *b) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  int l = blockIdx.y;
  if (x >= ld || l >= m) return;
  double v = 0.0;
  if (x < n && x != slack)
    v = b[l] * (Binv[(size_t)f[l] * lb + x] - Binv[(size_t)t[l] * lb + x]);
  H[(size_t)l * ld + x] = v;
}

// Ht[x][pos] = H[er[pos]][x] via 32 x 32 LDS tiles (coalesced on both sides).
__global__ void k_rows_transpose(double *Ht, int ld_er, const double *H, int ld_h, int n,
                                 const int32_t *er, int n_er) {
  __shared__ double tile[32][33];
  int x0 = blockIdx.x * 32, p0 = blockIdx.y * 32;
  int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    int pos = p0 + r, x = x0 + tx;
    double v = 0.0;
    if (pos < n_er && x < n) v = H[(size_t)er[pos] * ld_h + x];
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    int x = x0 + r, pos = p0 + tx;
    if (x < n && pos < ld_er) Ht[(size_t)x * ld_er + pos] = tile[tx][r];
  }
}

// Kept PTDF rows as GEMM operands: FP64, FP32 and three BF16 parts whose sum
// reproduces the FP64 value to about 2^-24 relative (each part rounds what the
// previous ones left).
__global__ void k_copy_he(double *He, float *He32, __bf16 *Heb, int ld_h, const double *H,
                          const int32_t *er, int n_er, int ld_er) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  int pos = blockIdx.y;
  if (x >= ld_h || pos >= ld_er) return;
  double v = pos < n_er ? H[(size_t)er[pos] * ld_h + x] : 0.0;
  const size_t i = (size_t)pos * ld_h + x;
  He[i] = v;
  He32[i] = (float)v;
  const size_t part = (size_t)ld_er * ld_h;
  for (int q = 0; q < 3; ++q) {
    const __bf16 b = (__bf16)(float)v;
    Heb[q * part + i] = b;
    v -= (double)(float)b;
  }
}

// Contingency columns: PTDF[:, f_c] - PTDF[:, t_c] for a branch, PTDF[:, bus_g]
// for a generator outage (ot = -1: the slack takes up the lost output).
__global__ void k_hdo(double *hdo, int ld_o, const double *H, int ld_h, int m,
                      const int32_t *of, const int32_t *ot, int n_ctg) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  int l = blockIdx.y;
  if (c >= ld_o || l >= m) return;
  double v = 0.0;
  if (c < n_ctg) {
    v = H[(size_t)l * ld_h + of[c]];
    if (ot[c] >= 0) v -= H[(size_t)l * ld_h + ot[c]];
  }
  hdo[(size_t)l * ld_o + c] = v;
}

// One wave per branch: F_base[l] = H[l, :] . p_base.
__global__ void k_fbase(double *fb, const double *H, int ld_h, const double *p, int m) {
  int l = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  int lane = threadIdx.x % kWave;
  if (l >= m) return;
  double s = 0.0;
  for (int x = lane; x < ld_h; x += kWave) s += H[(size_t)l * ld_h + x] * p[x];
  s = wave_sum(s);
  if (lane == 0) fb[l] = s;
}

__global__ void k_rating(double *r, double *inv_r, int mon_pad, const int32_t *mon, int n_mon,
                         const double *fb, int use_given, double scale, double offset) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mon_pad) return;
  if (i < n_mon) {
    double v = use_given ? r[i] : scale * fabs(fb[mon[i]]) + offset;
    r[i] = v;
    inv_r[i] = 1.0 / v;
  } else {
    r[i] = 1.0;
    inv_r[i] = 0.0;
  }
}

// Largest magnitude of each column of Lsd over the monitored rows (one thread
// per column, rows walked in order: neighbouring threads read neighbouring
// columns).  The error guard of the FP32 scan bounds the seed by it.
// Column maxima of |Lsd| (cmax cleared to 0 first): blockIdx.y takes a chunk of
// kColmaxRows rows, and the chunk maxima meet in 64-bit integer atomic maxima on
// the non-negative bit patterns.
constexpr int kColmaxRows = 128;
__global__ void k_colmax(const double *lsd, int ld_o, int n_mon, double *cmax) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r0 = blockIdx.y * kColmaxRows, r1 = min(r0 + kColmaxRows, n_mon);
  if (c >= ld_o) return;
  double m = 0.0;
  for (int r = r0; r < r1; ++r) m = fmax(m, fabs(lsd[(size_t)r * ld_o + c]));
  atomicMax(reinterpret_cast<unsigned long long *>(cmax + c),
            (unsigned long long)__double_as_longlong(m));
}

__global__ void k_lsd(double *lsd, int ld_o, const double *hdo, const int32_t *mon, int n_mon,
                      const int32_t *out, int n_out, int n_ctg, const double *inv_r,
                      int mon_pad) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y;
  if (c >= ld_o || i >= mon_pad) return;
  double v = 0.0;
  if (i < n_mon && c < n_ctg) {
    // a branch contingency's own row carries -1 (LODF[c, c] = -1); a generator
    // column has no such entry
    int l = mon[i];
    v = (hdo[(size_t)l * ld_o + c] - (c < n_out && l == out[c] ? 1.0 : 0.0)) * inv_r[i];
  }
  lsd[(size_t)i * ld_o + c] = v;
}

// Seeds of the multi-outage sub-columns, each contiguous over the monitored rows
// (the multi-outage scan reads one row per thread): lsdm[s][i] = lsd[i][mcol[s]].
__global__ void k_lsd_multi(double *lsdm, float *lsdm32, const double *lsd, int ld_o,
                            const int32_t *mcol, int n_msub, int mon_pad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int sc = blockIdx.y;
  if (i >= mon_pad || sc >= n_msub) return;
  const double v = lsd[(size_t)i * ld_o + mcol[sc]];
  lsdm[(size_t)sc * mon_pad + i] = v;
  lsdm32[(size_t)sc * mon_pad + i] = (float)v;
}

// Control columns of the PTDF (phase-shifter and HVDC distribution factors):
// column n + q of row l = w_q (PTDF[l, a_q] - PTDF[l, c_q]) + [l == br_q] d_q.
__global__ void k_ctrl_cols(double *Hb, int ld_h, int m, int n, int n_ctrl, const int32_t *ca,
                            const int32_t *cc, const int32_t *cbr, const double *cw,
                            const double *cd) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (l >= m || q >= n_ctrl) return;
  double *row = Hb + (size_t)l * ld_h;
  row[n + q] = cw[q] * (row[ca[q]] - row[cc[q]]) + (l == cbr[q] ? cd[q] : 0.0);
}

// Base flows of the kept rows (the offset of the reduced-precision GEMM).
__global__ void k_fber(double *fber, const double *fb, const int32_t *er, int n_er, int ld_er) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ld_er) fber[i] = i < n_er ? fb[er[i]] : 0.0;
}

// FP32 copy of Lsd in the accumulator order of the FP32 16x16x4 MFMA, so that the
// scan seeds each block with one 16-byte load per lane.
// The FP64 seed in the same block order, each lane's four values in the FP64
// 16x16x4 accumulator order (rows g + 4 r of its lane group g): one 32-byte read
// per lane and block in the FP64 scan.
__global__ void k_lsd64f(d4 *dst, const double *lsd, int ld_o, int mon_pad) {
  const int ncb = ld_o / 16;
  const size_t total = (size_t)(mon_pad / 16) * ncb * kWave;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int lane = (int)(idx % kWave);
  const size_t blk = idx / kWave;
  const int cb = (int)(blk % ncb), rb = (int)(blk / ncb);
  const int g = lane / 16, col = cb * 16 + lane % 16;
  d4 v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = lsd[(size_t)(rb * 16 + MfmaRow<double>::row(g, r)) * ld_o + col];
  dst[idx] = v;
}

// dst[c][r] = src[r][c] for an R x C row-major matrix (32 x 32 LDS tiles).
__global__ void k_transpose(double *dst, const double *src, int R, int C) {
  __shared__ double tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  for (int r = ty; r < 32; r += 8)
    if (r0 + r < R && c0 + tx < C) tile[r][tx] = src[(size_t)(r0 + r) * C + c0 + tx];
  __syncthreads();
  for (int c = ty; c < 32; c += 8)
    if (c0 + c < C && r0 + tx < R) dst[(size_t)(c0 + c) * R + r0 + tx] = tile[tx][c];
}

__global__ void k_lsd32(float *dst, const double *lsd, int ld_o, int mon_pad) {
  const int ncb = ld_o / 16;
  const size_t total = (size_t)(mon_pad / 16) * ncb * kWave;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int lane = (int)(idx % kWave);
  const size_t blk = idx / kWave;
  const int cb = (int)(blk % ncb), rb = (int)(blk / ncb);
  const int row0 = rb * 16 + 4 * (lane / 16), col = cb * 16 + lane % 16;
  f4 v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = (float)lsd[(size_t)(row0 + r) * ld_o + col];
  reinterpret_cast<f4 *>(dst)[idx] = v;
}

inline unsigned nblk(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_build(dcflow_plan *p, hipStream_t s, const double *h_rating, double rscale,
                        double roffset) {
  const int n = p->n, m = p->m, ld = p->ld_h, lb = p->ld_b;
  // reduced Laplacian (padded to a multiple of 64 with unit diagonal) and its
  // inverse by blocked Gauss-Jordan
  hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, p->d_binv, (size_t)lb * lb, 0.0);
  DCF_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_assemble, dim3(nblk(n, 256)), dim3(256), 0, s, p->d_binv, lb, n, p->slack,
                     p->d_adj_off, p->d_adj_br, p->d_f, p->d_t, p->d_b);
  DCF_CHECK_LAUNCH();
  if (lb > n) {
    hipLaunchKernelGGL(k_pad_diag, dim3(1), dim3(64), 0, s, p->d_binv, lb, n);
    DCF_CHECK_LAUNCH();
  }
  const int nbk = lb / kGjB, nt = (lb + 127) / 128;
  for (int q = 0; q < nbk; ++q) {
    const int p0 = q * kGjB;
    hipLaunchKernelGGL(k_bgj_panel, dim3(1), dim3(256), 0, s, p->d_binv, lb, p0, p->d_piv);
    DCF_CHECK_LAUNCH();
    if (nbk > 1) {
      hipLaunchKernelGGL(k_bgj_rows, dim3(nbk), dim3(256), 0, s, p->d_binv, lb, p0, p->d_piv);
      DCF_CHECK_LAUNCH();
      hipLaunchKernelGGL(k_bgj_update, dim3(nt, nt), dim3(256), 0, s, p->d_binv, lb, p0);
      DCF_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_bgj_cols, dim3(nbk), dim3(256), 0, s, p->d_binv, lb, p0, p->d_piv);
    DCF_CHECK_LAUNCH();
  }
  // PTDF and derived operands
  hipLaunchKernelGGL(k_ptdf_rows, dim3(nblk(ld, 256), m), dim3(256), 0, s, p->d_hb, ld, n, m,
                     p->slack, p->d_binv, lb, p->d_f, p->d_t, p->d_b);
  DCF_CHECK_LAUNCH();
  if (p->n_ctrl > 0) {
    hipLaunchKernelGGL(k_ctrl_cols, dim3(nblk(m, 256), p->n_ctrl), dim3(256), 0, s, p->d_hb, ld,
                       m, n, p->n_ctrl, p->d_ctl_a, p->d_ctl_c, p->d_ctl_br, p->d_ctl_w,
                       p->d_ctl_d);
    DCF_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_rows_transpose, dim3(nblk(n, 32), nblk(p->ld_er, 32)), dim3(32, 8), 0, s,
                     p->d_ht, p->ld_er, p->d_hb, ld, n, p->d_er, p->n_er);
  DCF_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_copy_he, dim3(nblk(ld, 256), p->ld_er), dim3(256), 0, s, p->d_he64,
                     p->d_he32, p->d_heb, ld, p->d_hb, p->d_er, p->n_er, p->ld_er);
  DCF_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_hdo, dim3(nblk(p->ld_o, 256), m), dim3(256), 0, s, p->d_hdo, p->ld_o,
                     p->d_hb, ld, m, p->d_out_f, p->d_out_t, p->n_out + p->n_gen);
  DCF_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_fbase, dim3(nblk(m, 4)), dim3(256), 0, s, p->d_fbase, p->d_hb, ld,
                     p->d_pbase, m);
  DCF_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_fber, dim3(nblk(p->ld_er, 256)), dim3(256), 0, s, p->d_fber, p->d_fbase,
                     p->d_er, p->n_er, p->ld_er);
  DCF_CHECK_LAUNCH();
  if (h_rating) {
    hipError_t e = hipMemcpyAsync(p->d_rating, h_rating, sizeof(double) * p->n_mon,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_rating, dim3(nblk(p->mon_pad, 256)), dim3(256), 0, s, p->d_rating,
                     p->d_inv_r, p->mon_pad, p->d_mon, p->n_mon, p->d_fbase, h_rating ? 1 : 0,
                     rscale, roffset);
  DCF_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_lsd, dim3(nblk(p->ld_o, 256), p->mon_pad), dim3(256), 0, s, p->d_lsd,
                     p->ld_o, p->d_hdo, p->d_mon, p->n_mon, p->d_out, p->n_out,
                     p->n_out + p->n_gen, p->d_inv_r, p->mon_pad);
  DCF_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_fill, dim3(nblk(p->ld_o, 256)), dim3(256), 0, s, p->d_lsdmax,
                     (size_t)p->ld_o, 0.0);
  DCF_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_colmax, dim3(nblk(p->ld_o, 256), nblk(p->n_mon, kColmaxRows)), dim3(256), 0,
                     s, p->d_lsd, p->ld_o, p->n_mon, p->d_lsdmax);
  DCF_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_lsd32, dim3(nblk((size_t)p->mon_pad * p->ld_o / 4, 256)), dim3(256), 0, s,
                     p->d_lsd32, p->d_lsd, p->ld_o, p->mon_pad);
  DCF_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_lsd64f, dim3(nblk((size_t)p->mon_pad * p->ld_o / 4, 256)), dim3(256), 0, s,
                     reinterpret_cast<d4 *>(p->d_lsd64f), p->d_lsd, p->ld_o, p->mon_pad);
  DCF_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_transpose, dim3(nblk(p->ld_o, 32), nblk(p->mon_pad, 32)), dim3(32, 8), 0, s,
                     p->d_lsdT, p->d_lsd, p->mon_pad, p->ld_o);
  DCF_CHECK_LAUNCH();
  if (p->n_msub > 0) {
    hipLaunchKernelGGL(k_lsd_multi, dim3(nblk(p->mon_pad, 256), p->n_msub), dim3(256), 0, s,
                       p->d_lsdm, p->d_lsdm32, p->d_lsd, p->ld_o, p->d_mcol, p->n_msub,
                       p->mon_pad);
    DCF_CHECK_LAUNCH();
  }
  return hipSuccess;
}

}  // namespace dcflow
