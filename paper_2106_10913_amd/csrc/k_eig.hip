// Batched dense symmetric eigensolver for the low end of the spectrum (gfx950).
//
// Used for both local eigenproblems of the method: the non-positive
// eigenpairs of each B^s (splitting of B^s, Section 3.2) and the GenEO
// eigenpairs below tau after a Cholesky reduction of the pencil (Definition of
// Y_L, Section 3.4).  Steps:
//   1. Householder reduction to tridiagonal form, Q^T A Q = T.  One pass over
//      the trailing matrix per column: the rank-2 update of the previous step
//      and the product with the new reflector are fused.
//   2. Sturm-sequence counts on T give the exact number of eigenvalues below
//      the threshold (Sylvester inertia); bisection gives each eigenvalue.
//   3. Inverse iteration on T (LU with partial pivoting, fixed number of
//      sweeps) with modified Gram-Schmidt against the vectors already found,
//      so that clustered and repeated eigenvalues give an orthonormal basis.
//   4. Back-transformation Z <- Q Z.
#include "awg_common.h"

#include <float.h>

#include <algorithm>

namespace awg {

constexpr int TRD_ROWS = 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// Blocked Householder tridiagonalisation (lower, full symmetric storage).
// Panels of TRD_NB columns; inside a panel the trailing matrix is not
// updated: column j is brought up to date from the panel's reflectors V and
// vectors W, and A22 v is corrected by V (W^T v) + W (V^T v).  After the
// panel, A22 -= V W^T + W V^T as two MFMA products.
// Work layout (sumns = total rows of all blocks): V at [0, sumns*NB),
// W at [sumns*NB, 2 sumns*NB) (block b at off[b]*NB, n_b x NB, ld n_b),
// p (A22 v) at 2 sumns*NB + off[b].
struct TrdWork {
  double* V;
  double* W;
  double* p;
  __device__ TrdWork(double* work, long sumns, long o) {
    V = work + o * TRD_NB;
    W = work + sumns * TRD_NB + o * TRD_NB;
    p = work + 2 * sumns * TRD_NB + o;
  }
};

// p = A22 v reading only the lower triangle of A22 = A[j+1:, j+1:] (the
// trailing matrix is kept up to date in its lower triangle only).  A22 is cut
// into 64 x 64 tiles (I, C), I >= C; an off-diagonal tile gives the row part
// A_IC v_C and, by symmetry, the column part A_IC^T v_I; a diagonal tile is
// mirrored in LDS.  Partial vectors go to part[(I * ntmax + C) * 64 + r] and
// are summed over C in a fixed order by k_trd_wx (deterministic).
constexpr int SYMV_T = 64;

constexpr int TRD_RB = 256;     // rows per workgroup
constexpr int TRD_YCH = 512;    // rows per workgroup of the dot products

// partial dot products y[q] = W[:, q]^T v, y[NB + q] = V[:, q]^T v over chunk
// ch of the rows below j (TRD_YCH rows; matrix b of the batch)
constexpr int TRD_WYG = 4;      // workgroups per row chunk (each a quarter of the columns)

__device__ inline void trd_wy_chunk(const MatDesc& M, int b, int ch, int cg, int p0, int jj, const long* off,
                                    double* work, long sumns, double* ypart, int nchmax) {
  const int n = M.n;
  const int j = p0 + jj;
  if (j > n - 3 || ch * TRD_YCH >= n - j - 1) return;
  TrdWork T(work, sumns, off[b]);
  const double* __restrict__ v = T.V + (long)jj * n;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r0 = j + 1 + ch * TRD_YCH, r1 = min(n, r0 + TRD_YCH);
  // column q of [W | V] goes to wave slot q % (4 TRD_WYG); a column's sum is
  // each lane's rows in order and then the wavefront reduction, whichever
  // wavefront takes it
  constexpr int NS = 4 * TRD_WYG;
  constexpr int QW = 2 * TRD_NB / NS;
  const int slot = cg * 4 + wid;
  double acc[QW];
#pragma unroll
  for (int k = 0; k < QW; ++k) acc[k] = 0.0;
  for (int i = r0 + lane; i < r1; i += 64) {
    const double vi = v[i];
#pragma unroll
    for (int k = 0; k < QW; ++k) {
      const int q = slot + NS * k;
      if (q < 2 * jj) {
        const double* __restrict__ c = (q < jj) ? T.W + (long)q * n : T.V + (long)(q - jj) * n;
        acc[k] += c[i] * vi;
      }
    }
  }
  double* yp = ypart + ((long)b * nchmax + ch) * 2 * TRD_NB;
#pragma unroll
  for (int k = 0; k < QW; ++k) {
    const int q = slot + NS * k;
    if (q < 2 * jj) {
      const double a = wave_sum(acc[k]);
      if (lane == 0) yp[q < jj ? q : TRD_NB + (q - jj)] = a;
    }
  }
}

// A workgroup walks tiles t = bx, bx + gxs, ... of its
// matrix and loads the next tile into registers while it works on the current
// one in LDS (loads stay in flight).
__device__ inline void symv_tile_decode(int t, int& I, int& C) {
  I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  C = t - I * (I + 1) / 2;
}

// The first gwy workgroups of the launch compute the panel dot products of
// the column (trd_wy_chunk), which do not depend on the product; they are
// dispatched first so that they overlap the product instead of trailing it.
__global__ __launch_bounds__(256) void k_trd_symv_pipe(const MatDesc* mats, int p0, int jj, const long* off,
                                                       double* work, long sumns, double* part, int ntmax, int gxs,
                                                       double* ypart, int nchmax, int gwy) {
  const MatDesc M = mats[blockIdx.y];
  if ((int)blockIdx.x < gwy) {
    trd_wy_chunk(M, blockIdx.y, blockIdx.x / TRD_WYG, blockIdx.x % TRD_WYG, p0, jj, off, work, sumns, ypart,
                 nchmax);
    return;
  }
  const int bx = (int)blockIdx.x - gwy;
  const int n = M.n;
  const int j = p0 + jj;
  if (j > n - 3) return;
  const int base = j + 1, m = n - base;
  const int nt = (m + SYMV_T - 1) / SYMV_T;
  const int ntiles = nt * (nt + 1) / 2;
  int t = bx;
  if (t >= ntiles) return;
  TrdWork T(work, sumns, off[blockIdx.y]);
  const double* v = T.V + (long)jj * n;
  __shared__ double L[SYMV_T][SYMV_T + 1];
  __shared__ double vr[SYMV_T], vc[SYMV_T];
  __shared__ double red[4][SYMV_T];
  const int tid = threadIdx.x, lane = tid & 63, g = tid >> 6;
  double* out = part + (long)blockIdx.y * ntmax * ntmax * SYMV_T;
  double cur[16];
  auto load = [&](int tt, double* buf) {
    int I, C;
    symv_tile_decode(tt, I, C);
    const int r0 = base + I * SYMV_T, c0 = base + C * SYMV_T;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + q * 256;
      const int r = e % SYMV_T, c = e / SYMV_T;
      const int gr = r0 + r, gc = c0 + c;
      buf[q] = (gr < n && gc < n && (I != C || r >= c)) ? M.A[gr + (long)gc * M.ld] : 0.0;
    }
  };
  load(t, cur);
  for (;;) {
    int I, C;
    symv_tile_decode(t, I, C);
    const int r0 = base + I * SYMV_T, c0 = base + C * SYMV_T;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + q * 256;
      L[e % SYMV_T][e / SYMV_T] = cur[q];
    }
    if (tid < SYMV_T) {
      vr[tid] = (r0 + tid < n) ? v[r0 + tid] : 0.0;
      vc[tid] = (c0 + tid < n) ? v[c0 + tid] : 0.0;
    }
    const int tn = t + gxs;
    if (tn < ntiles) load(tn, cur);      // next tile in flight during the work below
    __syncthreads();
    if (I == C) {
      for (int e = tid; e < SYMV_T * SYMV_T; e += 256) {
        const int r = e % SYMV_T, c = e / SYMV_T;
        if (r < c) L[r][c] = L[c][r];
      }
      __syncthreads();
    }
    double a = 0.0;
    for (int c = g; c < SYMV_T; c += 4) a += L[lane][c] * vc[c];
    red[g][lane] = a;
    __syncthreads();
    if (g == 0) out[((long)I * ntmax + C) * SYMV_T + lane] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    __syncthreads();
    if (I != C) {
      a = 0.0;
      for (int r = g; r < SYMV_T; r += 4) a += L[r][lane] * vr[r];
      red[g][lane] = a;
      __syncthreads();
      if (g == 0)
        out[((long)C * ntmax + I) * SYMV_T + lane] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
      __syncthreads();
    }
    if (tn >= ntiles) break;
    t = tn;
  }
}

// ---------------------------------------------------------------------------
// Row-parallel per-column steps (many workgroups per matrix).  Reductions go
// through per-block partial sums added in a fixed order.
// ---------------------------------------------------------------------------

// column j updated from the panel (rows j..n-1); partial sums of squares of
// rows >= j + 2; block 0 keeps d_j = A[j][j] and alpha = A[j+1][j].
// pend: W[:, jj-1] still lacks its final term w += -tau/2 (w.v) v
// (k_trd_wfix); it is added here, to the rows below j, before use (row j of
// that column is never read again, so it is corrected on the fly only).  The
// correction is also made for a matrix whose last reflector was column j-1.
__global__ __launch_bounds__(256) void k_trd_cu(const MatDesc* mats, int p0, int jj, const long* off, double* work,
                                                long sumns, double* red, double* aux, int nblkmax, int pend,
                                                const double* tau, const double* svpart) {
  const MatDesc M = mats[blockIdx.y];
  const int n = M.n;
  const int j = p0 + jj;
  const bool active = j <= n - 3;
  const bool fix = pend && j - 1 <= n - 3;
  if ((!active && !fix) || (int)blockIdx.x * TRD_RB >= n - j) return;
  __shared__ double sh[4];
  __shared__ double alpha_s;
  const long o = off[blockIdx.y];
  TrdWork T(work, sumns, o);
  double alpha = 0.0;
  if (fix) {
    if (threadIdx.x == 0) {
      const int nb = (n - j + TRD_RB - 1) / TRD_RB;    // blocks of k_trd_wx for column j - 1
      double sv = 0.0;
      for (int b = 0; b < nb; ++b) sv += svpart[(long)blockIdx.y * nblkmax + b];
      alpha_s = -0.5 * tau[o + j - 1] * sv;
    }
    __syncthreads();
    alpha = alpha_s;
  }
  const int i = j + blockIdx.x * TRD_RB + threadIdx.x;
  const int tp = jj - 1;            // the pending column
  double* wp = T.W + (long)tp * n;
  const double* vp = T.V + (long)tp * n;
  // corrected W[i, tp]; written back below row j, and at row j too when
  // column j is past this matrix's last reflector (the panel update then
  // reads that row, and no thread here reads it)
  double wpi = 0.0;
  if (fix && i < n) {
    wpi = wp[i];
    wpi += alpha * vp[i];
    if (i > j || !active) wp[i] = wpi;
  }
  if (!active) return;
  double* col = M.A + (long)j * M.ld;
  double ss = 0.0;
  if (i < n) {
    double wj = 0.0;                // corrected W[j, tp], read by every row
    if (fix) {
      wj = wp[j];
      wj += alpha * vp[j];
    }
    double a = col[i];
    for (int t = 0; t < jj; ++t) {
      const bool p = fix && t == tp;
      const double wjt = p ? wj : T.W[j + (long)t * n];
      const double wit = p ? wpi : T.W[i + (long)t * n];
      a -= T.V[i + (long)t * n] * wjt + wit * T.V[j + (long)t * n];
    }
    col[i] = a;
    if (i >= j + 2) ss = a * a;
    if (i == j) aux[2 * blockIdx.y] = a;
    if (i == j + 1) aux[2 * blockIdx.y + 1] = a;
  }
  ss = block_sum256(ss, sh);
  if (threadIdx.x == 0) red[(long)blockIdx.y * nblkmax + blockIdx.x] = ss;
}

// Householder vector of column j: d_j, e_j, tau_j; v (unit first entry)
// replaces rows j+1.. of the column and is stored as V[:, jj] (zero above)
__global__ __launch_bounds__(256) void k_trd_cf(const MatDesc* mats, int p0, int jj, double* dd, double* ee,
                                                double* tau, const long* off, double* work, long sumns,
                                                const double* red, const double* aux, int nblkmax) {
  const MatDesc M = mats[blockIdx.y];
  const int n = M.n;
  const int j = p0 + jj;
  if (j > n - 3 || (int)blockIdx.x * TRD_RB >= n) return;
  __shared__ double scale_s;
  const long o = off[blockIdx.y];
  TrdWork T(work, sumns, o);
  if (threadIdx.x == 0) {
    const int nb = (n - j + TRD_RB - 1) / TRD_RB;
    double ss = 0.0;
    for (int b = 0; b < nb; ++b) ss += red[(long)blockIdx.y * nblkmax + b];
    const double dkk = aux[2 * blockIdx.y], alpha = aux[2 * blockIdx.y + 1];
    double sc;
    if (ss == 0.0) {
      sc = 0.0;
      if (blockIdx.x == 0) {
        ee[o + j] = alpha;
        tau[o + j] = 0.0;
      }
    } else {
      const double beta = -copysign(sqrt(alpha * alpha + ss), alpha);
      sc = 1.0 / (alpha - beta);
      if (blockIdx.x == 0) {
        tau[o + j] = (beta - alpha) / beta;
        ee[o + j] = beta;
      }
    }
    if (blockIdx.x == 0) dd[o + j] = dkk;
    scale_s = sc;
  }
  __syncthreads();
  const double scale = scale_s;
  const int i = blockIdx.x * TRD_RB + threadIdx.x;
  if (i >= n) return;
  double* col = M.A + (long)j * M.ld;
  if (i <= j) {
    T.V[i + (long)jj * n] = 0.0;
  } else {
    const double v = (i == j + 1) ? 1.0 : col[i] * scale;
    col[i] = v;
    T.V[i + (long)jj * n] = v;
  }
}

// x = tau (p - V y_W - W y_V) on a block of rows, p summed from the symv
// partials; partial sums of x . v
__global__ __launch_bounds__(256) void k_trd_wx(const MatDesc* mats, int p0, int jj, const double* tau,
                                                const long* off, double* work, long sumns, const double* part,
                                                int ntmax, const double* ypart, int nchmax, double* svpart,
                                                int nblkmax) {
  const MatDesc M = mats[blockIdx.y];
  const int n = M.n;
  const int j = p0 + jj;
  if (j > n - 3 || (int)blockIdx.x * TRD_RB >= n - j - 1) return;
  __shared__ double y[2 * TRD_NB];
  __shared__ double sh[4];
  const long o = off[blockIdx.y];
  TrdWork T(work, sumns, o);
  const int nch = (n - j - 1 + TRD_YCH - 1) / TRD_YCH;
  if (threadIdx.x < 2 * TRD_NB) {
    const int q = threadIdx.x;
    const bool used = (q < TRD_NB) ? q < jj : (q - TRD_NB) < jj;
    double a = 0.0;
    if (used)
      for (int ch = 0; ch < nch; ++ch) a += ypart[((long)blockIdx.y * nchmax + ch) * 2 * TRD_NB + q];
    y[q] = a;
  }
  __syncthreads();
  const double t = tau[o + j];
  const double* __restrict__ v = T.V + (long)jj * n;
  double* __restrict__ w = T.W + (long)jj * n;
  const double* pp = part + (long)blockIdx.y * ntmax * ntmax * SYMV_T;
  const int nt = (n - j - 1 + SYMV_T - 1) / SYMV_T;
  const int i = j + 1 + blockIdx.x * TRD_RB + threadIdx.x;
  double sv = 0.0;
  if (i < n) {
    const int I = (i - j - 1) / SYMV_T, r = (i - j - 1) % SYMV_T;
    double x = 0.0;
    for (int C = 0; C < nt; ++C) x += pp[((long)I * ntmax + C) * SYMV_T + r];
    for (int q = 0; q < jj; ++q) x -= T.V[i + (long)q * n] * y[q] + T.W[i + (long)q * n] * y[TRD_NB + q];
    x *= t;
    w[i] = x;
    sv = x * v[i];
  }
  sv = block_sum256(sv, sh);
  if (threadIdx.x == 0) svpart[(long)blockIdx.y * nblkmax + blockIdx.x] = sv;
}

// w += -tau/2 (x . v) v below row j, zero at and above it
__global__ __launch_bounds__(256) void k_trd_wfix(const MatDesc* mats, int p0, int jj, const double* tau,
                                                  const long* off, double* work, long sumns, const double* svpart,
                                                  int nblkmax) {
  const MatDesc M = mats[blockIdx.y];
  const int n = M.n;
  const int j = p0 + jj;
  if (j > n - 3 || (int)blockIdx.x * TRD_RB >= n) return;
  __shared__ double alpha_s;
  const long o = off[blockIdx.y];
  TrdWork T(work, sumns, o);
  if (threadIdx.x == 0) {
    const int nb = (n - j - 1 + TRD_RB - 1) / TRD_RB;
    double sv = 0.0;
    for (int b = 0; b < nb; ++b) sv += svpart[(long)blockIdx.y * nblkmax + b];
    alpha_s = -0.5 * tau[o + j] * sv;
  }
  __syncthreads();
  const int i = blockIdx.x * TRD_RB + threadIdx.x;
  if (i >= n) return;
  double* w = T.W + (long)jj * n;
  if (i <= j) w[i] = 0.0;
  else w[i] += alpha_s * T.V[i + (long)jj * n];
}

// last 2x2 (or 1x1) block after every reflector has been applied
__global__ void k_trd_fin(const MatDesc* mats, double* dd, double* ee, double* tau, const long* off, int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const MatDesc M = mats[b];
  const int n = M.n;
  const long o = off[b];
  if (n == 1) {
    dd[o] = M.A[0];
    tau[o] = 0.0;
    return;
  }
  const int k = n - 2;
  dd[o + k] = M.A[k + (long)k * M.ld];
  dd[o + k + 1] = M.A[(k + 1) + (long)(k + 1) * M.ld];
  ee[o + k] = M.A[(k + 1) + (long)k * M.ld];
  tau[o + k] = 0.0;
  tau[o + k + 1] = 0.0;
  M.A[(k + 1) + (long)k * M.ld] = 1.0;     // unit reflector slot read by the back-transformation
}

void sytrd_batched(const MatDesc* d_mats, const std::vector<int>& h_n, double* d, double* e, double* tau,
                   const long* d_off, double* work, hipStream_t s) {
  const int batch = (int)h_n.size();
  int maxn = 0;
  long sumns = 0;
  for (int v : h_n) {
    maxn = v > maxn ? v : maxn;
    sumns += v;
  }
  if (batch == 0 || maxn == 0) return;
  const int ntmax = (maxn + SYMV_T - 1) / SYMV_T;
  DBuf<double> part;
  part.alloc((size_t)batch * ntmax * ntmax * SYMV_T);
  const int nblkmax = (int)cdiv(maxn, TRD_RB) + 1;
  const int nchmax = (int)cdiv(maxn, TRD_YCH) + 1;
  DBuf<double> red, aux, ypart, svpart;
  red.alloc((size_t)batch * nblkmax);
  aux.alloc((size_t)batch * 2);
  ypart.alloc((size_t)batch * nchmax * 2 * TRD_NB);
  svpart.alloc((size_t)batch * nblkmax);
  for (int p0 = 0; p0 <= maxn - 3; p0 += TRD_NB) {
    const int nbp = std::min(TRD_NB, maxn - 2 - p0);
    for (int jj = 0; jj < nbp; ++jj) {
      const int j = p0 + jj;
      const unsigned gb = cdiv(maxn, TRD_RB);
      {
        KScope kt("k_trd_col", s, 0.0, 0.0);
        hipLaunchKernelGGL(k_trd_cu, dim3(gb, batch), dim3(256), 0, s, d_mats, p0, jj, d_off, work, sumns, red.p,
                           aux.p, nblkmax, jj > 0 ? 1 : 0, tau, svpart.p);
        hipLaunchKernelGGL(k_trd_cf, dim3(gb, batch), dim3(256), 0, s, d_mats, p0, jj, d, e, tau, d_off, work, sumns,
                           red.p, aux.p, nblkmax);
        AWG_LAUNCH_CHECK();
      }
      const int rows = maxn - j - 1;
      double tb = 0.0;
      if (ktimer_on())
        for (int nbk : h_n)
          if (j <= nbk - 3) tb += 8.0 * (double)(nbk - j - 1) * (nbk - j - 1);
      {
        const int ntr = (rows + SYMV_T - 1) / SYMV_T;
        const int ntiles = std::max(1, ntr * (ntr + 1) / 2);
        // 2 or 3 tiles per workgroup once the trailing matrices are large
        const int gx = ntiles <= 64 ? ntiles : ntiles <= 256 ? (ntiles + 1) / 2 : (ntiles + 2) / 3;
        // plus the workgroups of the panel dot products (none for the first column)
        const int gwy = jj > 0 ? TRD_WYG * (int)cdiv(std::max(1, rows), TRD_YCH) : 0;
        KScope kt("k_trd_symv", s, 0.5 * tb, tb / 4.0);
        hipLaunchKernelGGL(k_trd_symv_pipe, dim3(gx + gwy, batch), dim3(256), 0, s, d_mats, p0, jj, d_off, work,
                           sumns, part.p, ntmax, gx, ypart.p, nchmax, gwy);
        AWG_LAUNCH_CHECK();
      }
      {
        KScope ktw("k_trd_w", s, 0.0, 0.0);
        hipLaunchKernelGGL(k_trd_wx, dim3(cdiv(std::max(1, rows), TRD_RB), batch), dim3(256), 0, s, d_mats, p0, jj,
                           tau, d_off, work, sumns, part.p, ntmax, ypart.p, nchmax, svpart.p, nblkmax);
        // the last column of the panel gets its final term here, the others
        // in the next column's k_trd_cu
        if (jj == nbp - 1)
          hipLaunchKernelGGL(k_trd_wfix, dim3(gb, batch), dim3(256), 0, s, d_mats, p0, jj, tau, d_off, work, sumns,
                             svpart.p, nblkmax);
        AWG_LAUNCH_CHECK();
      }
    }
    const int rem = maxn - p0 - nbp;
    double fl = 0.0;
    if (ktimer_on())
      for (int nbk : h_n) {
        const int kb = std::min(TRD_NB, nbk - 2 - p0);
        if (kb > 0) fl += 4.0 * (double)(nbk - p0 - kb) * (nbk - p0 - kb) * kb;
      }
    if (rem > 0)
      syr2k_panel_update(d_mats, work, work + sumns * TRD_NB, d_off, p0, TRD_NB, rem, batch, s, fl);
  }
  hipLaunchKernelGGL(k_trd_fin, dim3(cdiv(batch, 64)), dim3(64), 0, s, d_mats, d, e, tau, d_off, batch);
  AWG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// tridiagonal eigenvalues by Sturm counts
// ---------------------------------------------------------------------------
// number of eigenvalues of T strictly below x
__device__ int sturm_count(const double* d, const double* e, int n, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

struct TriInfo {
  double gl, gu, pivmin, tnorm;
};

__device__ TriInfo tri_info(const double* d, const double* e, int n) {
  double gl = d[0], gu = d[0], emax = 0.0, tn = 0.0;
  for (int i = 0; i < n; ++i) {
    const double el = i > 0 ? fabs(e[i - 1]) : 0.0;
    const double er = i < n - 1 ? fabs(e[i]) : 0.0;
    gl = fmin(gl, d[i] - el - er);
    gu = fmax(gu, d[i] + el + er);
    tn = fmax(tn, fabs(d[i]) + el + er);
    if (i < n - 1) emax = fmax(emax, e[i] * e[i]);
  }
  const double w = fmax(fabs(gl), fabs(gu));
  TriInfo t;
  t.gl = gl - 2.0 * DBL_EPSILON * w * n - 1e-300;
  t.gu = gu + 2.0 * DBL_EPSILON * w * n + 1e-300;
  t.pivmin = DBL_MIN * fmax(1.0, emax);
  t.tnorm = tn;
  return t;
}

// i-th smallest eigenvalue (0-based) by bisection on [lo, hi], to the
// absolute accuracy 2 eps ||T|| (the accuracy a backward-stable reduction to
// T provides, and all that the shifted solves of inverse iteration need)
__device__ double bisect_eig(const double* d, const double* e, int n, int i, double lo, double hi,
                             double pivmin) {
  const double atol = 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin;
  for (int it = 0; it < 256; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (hi - lo <= atol) break;
    if (sturm_count(d, e, n, mid, pivmin) <= i) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// idx-th smallest eigenvalue (0-based) by multisection: the 64 lanes of a
// wavefront evaluate 64 interior points of [lo, hi] at once, so every step
// narrows the bracket 65-fold.  Called by all lanes of the wavefront.
__device__ double multisect_eig(const double* d, const double* e, int n, int idx, double lo, double hi,
                                double pivmin) {
  const int lane = threadIdx.x & 63;
  const double atol = 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin;
  for (int it = 0; it < 48; ++it) {
    if (hi - lo <= atol) break;
    const double w = hi - lo;
    const double x = lo + w * (double)(lane + 1) / 65.0;
    const int c = sturm_count(d, e, n, x, pivmin);
    const unsigned long long m = __ballot(c <= idx);     // lanes whose point lies at or below lambda_idx
    const int nb = __popcll(m);
    const double nlo = nb > 0 ? lo + w * (double)nb / 65.0 : lo;
    const double nhi = nb < 64 ? lo + w * (double)(nb + 1) / 65.0 : hi;
    if (!(nlo < nhi)) break;
    lo = nlo;
    hi = nhi;
  }
  return 0.5 * (lo + hi);
}

// one wavefront per block
__global__ __launch_bounds__(64) void k_tri_count(TriEigArgs a, const double* thr_in, int thr_mode, double eps0,
                                                  double* thr_out, int* count, double* minmax) {
  const int b = blockIdx.x;
  const int n = a.n[b];
  if (n == 0) {
    if (threadIdx.x == 0) count[b] = 0;
    return;
  }
  const double* d = a.d + a.off[b];
  const double* e = a.e + a.off[b];
  const TriInfo t = tri_info(d, e, n);
  double thr;
  if (thr_mode == 1) {
    const double lmin = multisect_eig(d, e, n, 0, t.gl, t.gu, t.pivmin);
    const double lmax = multisect_eig(d, e, n, n - 1, t.gl, t.gu, t.pivmin);
    if (threadIdx.x == 0) {
      minmax[2 * b] = lmin;
      minmax[2 * b + 1] = lmax;
    }
    thr = eps0 * fmax(fabs(lmin), fabs(lmax));
  } else {
    thr = thr_in[b];
  }
  if (threadIdx.x == 0) {
    thr_out[b] = thr;
    count[b] = sturm_count(d, e, n, thr, t.pivmin);
  }
}

void tri_count(const TriEigArgs& a, const double* thr_in, int thr_mode, double eps0, double* thr_out, int* count,
               double* lam_minmax, hipStream_t s) {
  if (a.nb == 0) return;
  KScope kt("k_tri_count", s, 0.0, 0.0);
  hipLaunchKernelGGL(k_tri_count, dim3(a.nb), dim3(64), 0, s, a, thr_in, thr_mode, eps0, thr_out, count,
                     lam_minmax);
  AWG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// eigenvectors of T by inverse iteration, one lane per eigenvalue
// ---------------------------------------------------------------------------
constexpr int INVIT_SWEEPS = 4;
constexpr int INVIT_PF = 8;       // rows loaded ahead per block in the sweeps
constexpr int INVIT_LANES = 64;

// Modified Gram-Schmidt of vector xj (length n, rows lane, lane + 64, ...)
// against the earlier vectors XT[0..jj), twice, then normalised: the same
// operations in the same order as the loop over memory in k_tri_vecs, with xj
// held in registers and the next earlier vector's loads issued before the
// current dot product is reduced.
constexpr int MGS_REG_ROWS = 40;   // rows per lane held in registers (n <= 2560)

__device__ inline void mgs_reg(const double* __restrict__ XT, double* __restrict__ xj, int jj, int n, int lane) {
  double r[MGS_REG_ROWS], qv[MGS_REG_ROWS], qn[MGS_REG_ROWS];
#pragma unroll
  for (int t = 0; t < MGS_REG_ROWS; ++t) {
    const int i = lane + 64 * t;
    r[t] = i < n ? xj[i] : 0.0;
  }
  const int steps = 2 * jj;       // (pass, q) in order
  if (steps > 0) {
#pragma unroll
    for (int t = 0; t < MGS_REG_ROWS; ++t) {
      const int i = lane + 64 * t;
      qv[t] = i < n ? XT[i] : 0.0;
    }
  }
  for (int st = 0; st < steps; ++st) {
    if (st + 1 < steps) {
      const double* __restrict__ xq = XT + (long)((st + 1) % jj) * n;
#pragma unroll
      for (int t = 0; t < MGS_REG_ROWS; ++t) {
        const int i = lane + 64 * t;
        qn[t] = i < n ? xq[i] : 0.0;
      }
    }
    double dt = 0.0;
#pragma unroll
    for (int t = 0; t < MGS_REG_ROWS; ++t)
      if (lane + 64 * t < n) dt += qv[t] * r[t];
    dt = wave_sum(dt);
#pragma unroll
    for (int t = 0; t < MGS_REG_ROWS; ++t)
      if (lane + 64 * t < n) r[t] -= dt * qv[t];
#pragma unroll
    for (int t = 0; t < MGS_REG_ROWS; ++t) qv[t] = qn[t];
  }
  double nr = 0.0;
#pragma unroll
  for (int t = 0; t < MGS_REG_ROWS; ++t)
    if (lane + 64 * t < n) nr += r[t] * r[t];
  nr = wave_sum(nr);
  const double inr = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
#pragma unroll
  for (int t = 0; t < MGS_REG_ROWS; ++t) {
    const int i = lane + 64 * t;
    if (i < n) xj[i] = r[t] * inr;
  }
}

// Work per block (doubles): 6 arrays of n x 64, interleaved so that step i of
// all 64 lanes is one contiguous 512-byte row: u0, u1, u2 (U of the LU with
// partial pivoting), l (multipliers), pivot flags, x (iterates).
// d and e are staged in LDS when use_lds (dynamic shared memory of 2 n
// doubles): the bisection and the LU factorisations walk them sequentially.
__global__ __launch_bounds__(64) void k_tri_vecs(TriEigArgs a, const int* count, const long* lam_off, double* lam,
                                                  const MatDesc* Zs, double* work, const long* work_off,
                                                  double* resid, int* nstrict, const double* thr, int use_lds) {
  extern __shared__ double tri_lds[];
  const int b = blockIdx.x;
  const int n = a.n[b];
  const int k = count[b];
  const int lane = threadIdx.x;
  if (n == 0 || k == 0) {
    if (lane == 0 && nstrict) nstrict[b] = 0;
    return;
  }
  const double* d = a.d + a.off[b];
  const double* e = a.e + a.off[b];
  if (use_lds) {
    for (int i = lane; i < n; i += 64) {
      tri_lds[i] = d[i];
      tri_lds[n + i] = i < n - 1 ? e[i] : 0.0;
    }
    __syncthreads();
    d = tri_lds;
    e = tri_lds + n;
  }
  double* L = lam + lam_off[b];
  const MatDesc Z = Zs[b];
  const long W = INVIT_LANES;
  double* wk = work + work_off[b];
  double* __restrict__ U0 = wk;
  double* __restrict__ U1 = wk + W * n;
  double* __restrict__ U2 = wk + 2 * W * n;
  double* __restrict__ LF = wk + 3 * W * n;
  double* __restrict__ PV = wk + 4 * W * n;
  double* __restrict__ X = wk + 5 * W * n;
  double* __restrict__ XT = wk + 6 * W * n;    // the chunk with each vector contiguous (Gram-Schmidt)
  __shared__ double tile[64][65];
  const TriInfo t = tri_info(d, e, n);
  for (int j = lane; j < k; j += 64) L[j] = bisect_eig(d, e, n, j, t.gl, t.gu, t.pivmin);
  __syncthreads();
  if (lane == 0 && nstrict) {
    int c = 0;
    for (int j = 0; j < k; ++j) c += (L[j] < -thr[b]) ? 1 : 0;
    nstrict[b] = c;
  }
  const double pert = DBL_EPSILON * fmax(t.tnorm, DBL_MIN);
  for (int j0 = 0; j0 < k; j0 += 64) {
    const int jc = j0 + lane;
    const bool act = jc < k;
    const int kc = min(64, k - j0);
    const double lj = act ? L[jc] : 0.0;
    // LU of T - lj I with partial pivoting (each lane its own shift)
    if (act) {
      double cd = d[0] - lj, cs = n > 1 ? e[0] : 0.0;
      for (int i = 0; i < n - 1; ++i) {
        const double sub = e[i];
        const double nd = d[i + 1] - lj;
        const double ns = (i + 1 < n - 1) ? e[i + 1] : 0.0;
        const long o = i * W + lane;
        if (fabs(cd) >= fabs(sub)) {
          if (cd == 0.0) cd = pert;
          const double l = sub / cd;
          U0[o] = cd; U1[o] = cs; U2[o] = 0.0; LF[o] = l; PV[o] = 0.0;
          cd = nd - l * cs;
          cs = ns;
        } else {
          const double l = cd / sub;
          U0[o] = sub; U1[o] = nd; U2[o] = ns; LF[o] = l; PV[o] = 1.0;
          cd = cs - l * nd;
          cs = -l * ns;
        }
      }
      if (fabs(cd) < pert) cd = cd < 0.0 ? -pert : pert;
      U0[(n - 1) * W + lane] = cd;
      // deterministic pseudo-random start vector
      for (int i = 0; i < n; ++i) {
        unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)((jc + 1) * 40503u) ^ 0x9e3779b9u;
        h ^= h >> 16; h *= 0x7feb352du; h ^= h >> 15; h *= 0x846ca68bu; h ^= h >> 16;
        X[i * W + lane] = (double)(h & 0xffffff) / 16777216.0 - 0.5;
      }
    }
    for (int sweep = 0; sweep < INVIT_SWEEPS; ++sweep) {
      if (act) {
        // solve (T - lj I) y = x in place, then scale to unit max norm.  The
        // per-lane arrays exceed the L2, so both sweeps load INVIT_PF rows a
        // block ahead of their use (the operations and their order are those
        // of the plain row-by-row sweeps)
        double xi = X[lane];
        {
          double xb[INVIT_PF], pb[INVIT_PF], lb[INVIT_PF], xq[INVIT_PF], pq[INVIT_PF], lq[INVIT_PF];
          auto ldf = [&](int i0, double* xr, double* pr, double* lr) {
#pragma unroll
            for (int u = 0; u < INVIT_PF; ++u) {
              const int i = i0 + u;
              const bool ok = i < n - 1;
              xr[u] = ok ? X[(long)(i + 1) * W + lane] : 0.0;
              pr[u] = ok ? PV[(long)i * W + lane] : 0.0;
              lr[u] = ok ? LF[(long)i * W + lane] : 0.0;
            }
          };
          ldf(0, xb, pb, lb);
          for (int i0 = 0; i0 < n - 1; i0 += INVIT_PF) {
            if (i0 + INVIT_PF < n - 1) ldf(i0 + INVIT_PF, xq, pq, lq);
#pragma unroll
            for (int u = 0; u < INVIT_PF; ++u) {
              const int i = i0 + u;
              if (i < n - 1) {
                double xn = xb[u];
                if (pb[u] != 0.0) { const double tt = xi; xi = xn; xn = tt; }
                X[(long)i * W + lane] = xi;
                xi = xn - lb[u] * xi;
              }
            }
#pragma unroll
            for (int u = 0; u < INVIT_PF; ++u) {
              xb[u] = xq[u];
              pb[u] = pq[u];
              lb[u] = lq[u];
            }
          }
        }
        double x1 = xi / U0[(n - 1) * W + lane];
        X[(n - 1) * W + lane] = x1;
        double x2 = 0.0;
        double mx = fabs(x1);
        if (n > 1) {
          // rows n-2 down to 0 in blocks of INVIT_PF
          double xb[INVIT_PF], ab[INVIT_PF], bb[INVIT_PF], cb[INVIT_PF];
          double xq[INVIT_PF], aq[INVIT_PF], bq[INVIT_PF], cq[INVIT_PF];
          auto ldb = [&](int i0, double* xr, double* a0, double* a1, double* a2) {
#pragma unroll
            for (int u = 0; u < INVIT_PF; ++u) {
              const int i = i0 - u;
              const long o = (long)i * W + lane;
              const bool ok = i >= 0;
              xr[u] = ok ? X[o] : 0.0;
              a0[u] = ok ? U0[o] : 1.0;
              a1[u] = ok ? U1[o] : 0.0;
              a2[u] = ok ? U2[o] : 0.0;
            }
          };
          ldb(n - 2, xb, ab, bb, cb);
          for (int i0 = n - 2; i0 >= 0; i0 -= INVIT_PF) {
            if (i0 - INVIT_PF >= 0) ldb(i0 - INVIT_PF, xq, aq, bq, cq);
#pragma unroll
            for (int u = 0; u < INVIT_PF; ++u) {
              const int i = i0 - u;
              if (i >= 0) {
                const double v = (xb[u] - bb[u] * x1 - cb[u] * x2) / ab[u];
                X[(long)i * W + lane] = v;
                x2 = x1;
                x1 = v;
                mx = fmax(mx, fabs(v));
              }
            }
#pragma unroll
            for (int u = 0; u < INVIT_PF; ++u) {
              xb[u] = xq[u];
              ab[u] = aq[u];
              bb[u] = bq[u];
              cb[u] = cq[u];
            }
          }
        }
        const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
        for (int i = 0; i < n; ++i) X[i * W + lane] *= inv;
      }
      __syncthreads();
      // against the vectors of earlier chunks (already in Z), twice
      for (int pass = 0; pass < 2 && act; ++pass)
        for (int q = 0; q < j0; ++q) {
          const double* zq = Z.A + (long)q * Z.ld;
          double dt = 0.0;
          for (int i = 0; i < n; ++i) dt += zq[i] * X[i * W + lane];
          for (int i = 0; i < n; ++i) X[i * W + lane] -= dt * zq[i];
        }
      __syncthreads();
      // modified Gram-Schmidt inside the chunk, in eigenvalue order, twice, on
      // a transposed copy (vector j contiguous at XT + j n) so that the
      // wavefront's loads over rows are coalesced; 64 x 64 tiles through LDS
      for (int i0 = 0; i0 < n; i0 += 64) {
        const int ni = min(64, n - i0);
        for (int r = 0; r < ni; ++r) tile[r][lane] = X[(long)(i0 + r) * W + lane];
        __syncthreads();
        for (int jq = 0; jq < kc; ++jq)
          if (lane < ni) XT[(long)jq * n + i0 + lane] = tile[lane][jq];
        __syncthreads();
      }
      for (int jj = 0; jj < kc; ++jj) {
        double* __restrict__ xj = XT + (long)jj * n;
        if (n <= 64 * MGS_REG_ROWS) {
          mgs_reg(XT, xj, jj, n, lane);
          continue;
        }
        for (int pass = 0; pass < 2; ++pass)
          for (int q = 0; q < jj; ++q) {
            const double* __restrict__ xq = XT + (long)q * n;
            double dt = 0.0;
            for (int i = lane; i < n; i += 64) dt += xq[i] * xj[i];
            dt = wave_sum(dt);
            for (int i = lane; i < n; i += 64) xj[i] -= dt * xq[i];
          }
        double nr = 0.0;
        for (int i = lane; i < n; i += 64) nr += xj[i] * xj[i];
        nr = wave_sum(nr);
        const double inr = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
        for (int i = lane; i < n; i += 64) xj[i] *= inr;
      }
      __syncthreads();
      for (int i0 = 0; i0 < n; i0 += 64) {
        const int ni = min(64, n - i0);
        for (int jq = 0; jq < kc; ++jq)
          if (lane < ni) tile[lane][jq] = XT[(long)jq * n + i0 + lane];
        __syncthreads();
        for (int r = 0; r < ni; ++r)
          if (lane < kc) X[(long)(i0 + r) * W + lane] = tile[r][lane];
        __syncthreads();
      }
    }
    if (act) {
      // residual ||T x - lj x||_inf / ||T|| and copy out
      double rmax = 0.0;
      for (int i = 0; i < n; ++i) {
        const double xv = X[i * W + lane];
        double v = (d[i] - lj) * xv;
        if (i > 0) v += e[i - 1] * X[(i - 1) * W + lane];
        if (i < n - 1) v += e[i] * X[(i + 1) * W + lane];
        rmax = fmax(rmax, fabs(v));
        Z.A[i + (long)jc * Z.ld] = xv;
      }
      resid[lam_off[b] + jc] = rmax / fmax(t.tnorm, DBL_MIN);
    }
    __syncthreads();
  }
}

void tri_eigvecs(const TriEigArgs& a, const int* count, const long* lam_off, double* lam, const MatDesc* d_Z,
                 double* work, const long* work_off, double* resid, int* nstrict, const double* thr,
                 hipStream_t s, int maxn) {
  if (a.nb == 0) return;
  const bool lds = maxn > 0 && maxn <= 6144;
  KScope kt("k_tri_vecs", s, 0.0, 0.0);
  hipLaunchKernelGGL(k_tri_vecs, dim3(a.nb), dim3(64), lds ? sizeof(double) * 2 * maxn : 0, s, a, count, lam_off,
                     lam, d_Z, work, work_off, resid, nstrict, thr, (int)lds);
  AWG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// back-transformation Z <- H_0 H_1 ... H_{n-3} Z
// ---------------------------------------------------------------------------
constexpr int ORM_COLS = 4;     // columns of Z per workgroup (each column's sums are independent of it)
constexpr int ORM_RPT = 8;      // rows per thread held in registers (n <= 2048), else read twice

__global__ __launch_bounds__(256) void k_ormtr(const MatDesc* mats, const MatDesc* Zs, const double* tau,
                                               const long* off) {
  const MatDesc M = mats[blockIdx.y];
  const MatDesc Z = Zs[blockIdx.y];
  const int n = M.n;
  const int c0 = blockIdx.x * ORM_COLS;
  if (c0 >= Z.n || n < 3) return;
  const int nc = min(ORM_COLS, Z.n - c0);
  extern __shared__ double zs[];          // [ORM_COLS][n]
  __shared__ double red[4][ORM_COLS];
  const long o = off[blockIdx.y];
  for (int c = 0; c < nc; ++c)
    for (int i = threadIdx.x; i < n; i += 256) zs[c * n + i] = Z.A[i + (long)(c0 + c) * Z.ld];
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j = n - 3; j >= 0; --j) {
    const double tj = tau[o + j];
    if (tj == 0.0) continue;
    const double* v = M.A + (long)j * M.ld;    // v[j+1] = 1 stored explicitly
    const bool inreg = n - (j + 1) <= 256 * ORM_RPT;
    double vr[ORM_RPT];
    if (inreg) {
#pragma unroll
      for (int u = 0; u < ORM_RPT; ++u) {
        const int i = j + 1 + threadIdx.x + 256 * u;
        vr[u] = i < n ? v[i] : 0.0;
      }
    }
    double dots[ORM_COLS];
#pragma unroll
    for (int c = 0; c < ORM_COLS; ++c) dots[c] = 0.0;
    if (inreg) {
#pragma unroll
      for (int u = 0; u < ORM_RPT; ++u) {
        const int i = j + 1 + threadIdx.x + 256 * u;
        if (i < n) {
#pragma unroll
          for (int c = 0; c < ORM_COLS; ++c)
            if (c < nc) dots[c] += vr[u] * zs[c * n + i];
        }
      }
    } else {
      for (int i = j + 1 + threadIdx.x; i < n; i += 256) {
        const double vi = v[i];
#pragma unroll
        for (int c = 0; c < ORM_COLS; ++c)
          if (c < nc) dots[c] += vi * zs[c * n + i];
      }
    }
#pragma unroll
    for (int c = 0; c < ORM_COLS; ++c) {
      const double s = wave_sum(dots[c]);
      if (lane == 0) red[wid][c] = s;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < ORM_COLS; ++c) dots[c] = tj * ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c]));
    if (inreg) {
#pragma unroll
      for (int u = 0; u < ORM_RPT; ++u) {
        const int i = j + 1 + threadIdx.x + 256 * u;
        if (i < n) {
#pragma unroll
          for (int c = 0; c < ORM_COLS; ++c)
            if (c < nc) zs[c * n + i] -= dots[c] * vr[u];
        }
      }
    } else {
      for (int i = j + 1 + threadIdx.x; i < n; i += 256) {
        const double vi = v[i];
#pragma unroll
        for (int c = 0; c < ORM_COLS; ++c)
          if (c < nc) zs[c * n + i] -= dots[c] * vi;
      }
    }
    __syncthreads();
  }
  for (int c = 0; c < nc; ++c)
    for (int i = threadIdx.x; i < n; i += 256) Z.A[i + (long)(c0 + c) * Z.ld] = zs[c * n + i];
}

void ormtr_batched(const MatDesc* d_mats, const MatDesc* d_Z, const double* tau, const long* d_off,
                   const std::vector<int>& h_n, const std::vector<int>& h_k, hipStream_t s) {
  const int batch = (int)h_n.size();
  int maxn = 0, maxk = 0;
  for (size_t b = 0; b < h_n.size(); ++b) {
    maxn = h_n[b] > maxn ? h_n[b] : maxn;
    maxk = h_k[b] > maxk ? h_k[b] : maxk;
  }
  if (batch == 0 || maxk == 0 || maxn < 3) return;
  const size_t lds = (size_t)ORM_COLS * maxn * sizeof(double);
  if (lds > 150 * 1024) throw Error(-1, "ormtr: block too large for the LDS-resident back-transformation");
  KScope kt("k_ormtr", s, 0.0, 0.0);
  hipLaunchKernelGGL(k_ormtr, dim3(cdiv(maxk, ORM_COLS), batch), dim3(256), lds, s, d_mats, d_Z, tau, d_off);
  AWG_LAUNCH_CHECK();
}

}  // namespace awg
