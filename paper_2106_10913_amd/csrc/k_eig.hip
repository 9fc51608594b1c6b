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

namespace awg {

constexpr int TRD_ROWS = 64;

// Per-block work layout (doubles), offset work_off[b]:
//   v0[n] w0[n] v1[n] w1[n] p[n]   (reflector / w of the two last steps, product)
struct TrdWork {
  double* base;
  int n;
  __device__ double* v(int par) const { return base + (par ? 2 * n : 0); }
  __device__ double* w(int par) const { return base + (par ? 3 * n : n); }
  __device__ double* p() const { return base + 4 * n; }
};

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

// Step k, part 1: bring column k up to date with the previous rank-2 update
// and build the Householder reflector of its subdiagonal part.
__global__ __launch_bounds__(256) void k_trd_hh(const MatDesc* mats, int k, double* dd, double* ee,
                                                double* tau, const long* off, double* work) {
  const MatDesc M = mats[blockIdx.x];
  const int n = M.n;
  if (n == 1 && k == 0 && threadIdx.x == 0) {
    dd[off[blockIdx.x]] = M.A[0];
    tau[off[blockIdx.x]] = 0.0;
  }
  if (k > n - 2) return;
  __shared__ double sh[4];
  const long o = off[blockIdx.x];
  TrdWork W{work + 5 * o, n};
  const int par = k & 1;
  const double* vp = W.v(par ^ 1);
  const double* wp = W.w(par ^ 1);
  double* vc = W.v(par);
  double* col = M.A + (long)k * M.ld;
  const bool upd = k > 0;
  const double vk = upd ? vp[k] : 0.0, wk = upd ? wp[k] : 0.0;
  // updated column entries rows k..n-1
  double ss = 0.0;
  for (int i = k + 2 + threadIdx.x; i < n; i += 256) {
    double a = col[i];
    if (upd) a -= __dadd_rn(__dmul_rn(vp[i], wk), __dmul_rn(wp[i], vk));
    col[i] = a;
    ss += a * a;
  }
  ss = block_sum256(ss, sh);
  if (threadIdx.x == 0) {
    double dkk = col[k], alpha = col[k + 1];
    if (upd) {
      dkk -= __dadd_rn(__dmul_rn(vk, wk), __dmul_rn(wk, vk));
      alpha -= __dadd_rn(__dmul_rn(vp[k + 1], wk), __dmul_rn(wp[k + 1], vk));
    }
    dd[o + k] = dkk;
    if (k == n - 2) {
      double last = M.A[(k + 1) + (long)(k + 1) * M.ld];
      if (upd) last -= __dadd_rn(__dmul_rn(vp[k + 1], wp[k + 1]), __dmul_rn(wp[k + 1], vp[k + 1]));
      dd[o + k + 1] = last;
      ee[o + k] = alpha;
      tau[o + k] = 0.0;
      col[k + 1] = 1.0;
      sh[0] = 0.0;
    } else if (ss == 0.0) {
      ee[o + k] = alpha;
      tau[o + k] = 0.0;
      col[k + 1] = 1.0;
      sh[0] = 0.0;       // v = e1 scaled by 0: rest of v stays as the (zero) column
    } else {
      const double beta = -copysign(sqrt(alpha * alpha + ss), alpha);
      tau[o + k] = (beta - alpha) / beta;
      ee[o + k] = beta;
      col[k + 1] = 1.0;
      sh[0] = 1.0 / (alpha - beta);
    }
  }
  __syncthreads();
  if (k == n - 2) return;
  const double scale = sh[0];
  for (int i = k + 1 + threadIdx.x; i < n; i += 256) {
    double v = (i == k + 1) ? 1.0 : col[i] * scale;
    if (i > k + 1) col[i] = v;
    vc[i] = v;
  }
}

// Step k, part 2: A22 <- A22 - v_{k-1} w_{k-1}^T - w_{k-1} v_{k-1}^T on rows and
// columns k+1..n-1 (fused), then p = A22 v_k.  64 rows per workgroup, 4
// column groups; partial sums combined in LDS.
__global__ __launch_bounds__(256) void k_trd_upd(const MatDesc* mats, int k, const long* off, double* work) {
  const MatDesc M = mats[blockIdx.y];
  const int n = M.n;
  if (k > n - 3) return;
  const int i0 = k + 1 + blockIdx.x * TRD_ROWS;
  if (i0 >= n) return;
  const long o = off[blockIdx.y];
  TrdWork W{work + 5 * o, n};
  const int par = k & 1;
  const double* vp = W.v(par ^ 1);
  const double* wp = W.w(par ^ 1);
  const double* vc = W.v(par);
  const bool upd = k > 0;
  const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int i = i0 + r;
  __shared__ double part[4][TRD_ROWS];
  double acc = 0.0;
  if (i < n) {
    const double vi = upd ? vp[i] : 0.0, wi = upd ? wp[i] : 0.0;
    double* a = M.A + i;
    for (int j = k + 1 + g; j < n; j += 4) {
      double x = a[(long)j * M.ld];
      if (upd) {
        x -= __dadd_rn(__dmul_rn(vi, wp[j]), __dmul_rn(wi, vp[j]));
        a[(long)j * M.ld] = x;
      }
      acc += x * vc[j];
    }
  }
  part[g][r] = acc;
  __syncthreads();
  if (g == 0 && i < n) W.p()[i] = (part[0][r] + part[1][r]) + (part[2][r] + part[3][r]);
}

// Step k, part 3: w = tau p - (tau^2/2)(p.v) v.
__global__ __launch_bounds__(256) void k_trd_w(const MatDesc* mats, int k, const double* tau, const long* off,
                                               double* work) {
  const MatDesc M = mats[blockIdx.x];
  const int n = M.n;
  if (k > n - 3) return;
  __shared__ double sh[4];
  const long o = off[blockIdx.x];
  TrdWork W{work + 5 * o, n};
  const int par = k & 1;
  const double* vc = W.v(par);
  double* wc = W.w(par);
  const double* p = W.p();
  const double t = tau[o + k];
  double s = 0.0;
  for (int i = k + 1 + threadIdx.x; i < n; i += 256) s += p[i] * vc[i];
  s = block_sum256(s, sh);
  const double alpha = -0.5 * t * t * s;
  for (int i = k + 1 + threadIdx.x; i < n; i += 256) wc[i] = t * p[i] + alpha * vc[i];
}

void sytrd_batched(const MatDesc* d_mats, const std::vector<int>& h_n, double* d, double* e, double* tau,
                   const long* d_off, double* work, hipStream_t s) {
  const int batch = (int)h_n.size();
  int maxn = 0;
  for (int v : h_n) maxn = v > maxn ? v : maxn;
  if (batch == 0 || maxn == 0) return;
  // (1x1 blocks are copied by the k = 0 launch)
  for (int k = 0; k <= (maxn > 2 ? maxn - 2 : 0); ++k) {
    hipLaunchKernelGGL(k_trd_hh, dim3(batch), dim3(256), 0, s, d_mats, k, d, e, tau, d_off, work);
    AWG_LAUNCH_CHECK();
    if (k <= maxn - 3) {
      const int rows = maxn - k - 1;
      double tb = 0.0;
      if (ktimer_on())
        for (int nb : h_n) {
          const double r = nb - k - 1;
          if (nb - k - 3 >= 0) tb += r * r * (k > 0 ? 16.0 : 8.0);
        }
      KScope kt("k_trd_upd", s, tb, tb / 8.0 * (k > 0 ? 3.0 : 2.0));
      hipLaunchKernelGGL(k_trd_upd, dim3(cdiv(rows, TRD_ROWS), batch), dim3(256), 0, s, d_mats, k, d_off, work);
      AWG_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_trd_w, dim3(batch), dim3(256), 0, s, d_mats, k, tau, d_off, work);
      AWG_LAUNCH_CHECK();
    }
  }
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

// i-th smallest eigenvalue (0-based) by bisection on [lo, hi]
__device__ double bisect_eig(const double* d, const double* e, int n, int i, double lo, double hi,
                             double pivmin) {
  for (int it = 0; it < 256; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
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
  for (int it = 0; it < 48; ++it) {
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
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
  hipLaunchKernelGGL(k_tri_count, dim3(a.nb), dim3(64), 0, s, a, thr_in, thr_mode, eps0, thr_out, count,
                     lam_minmax);
  AWG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// eigenvectors of T by inverse iteration, one lane per eigenvalue
// ---------------------------------------------------------------------------
constexpr int INVIT_SWEEPS = 4;
constexpr int INVIT_LANES = 64;

// Work per block (doubles): 6 arrays of n x 64, interleaved so that step i of
// all 64 lanes is one contiguous 512-byte row: u0, u1, u2 (U of the LU with
// partial pivoting), l (multipliers), pivot flags, x (iterates).
__global__ __launch_bounds__(64) void k_tri_vecs(TriEigArgs a, const int* count, const long* lam_off, double* lam,
                                                  const MatDesc* Zs, double* work, const long* work_off,
                                                  double* resid, int* nstrict, const double* thr) {
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
  double* L = lam + lam_off[b];
  const MatDesc Z = Zs[b];
  const long W = INVIT_LANES;
  double* wk = work + work_off[b];
  double* U0 = wk;
  double* U1 = wk + W * n;
  double* U2 = wk + 2 * W * n;
  double* LF = wk + 3 * W * n;
  double* PV = wk + 4 * W * n;
  double* X = wk + 5 * W * n;
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
        // solve (T - lj I) y = x in place, then scale to unit max norm
        double xi = X[lane];
        for (int i = 0; i < n - 1; ++i) {
          const long o = i * W + lane;
          double xn = X[o + W];
          if (PV[o] != 0.0) { const double tt = xi; xi = xn; xn = tt; }
          X[o] = xi;
          xi = xn - LF[o] * xi;
        }
        X[(n - 1) * W + lane] = xi;
        double x1 = xi / U0[(n - 1) * W + lane];
        X[(n - 1) * W + lane] = x1;
        double x2 = 0.0;
        double mx = fabs(x1);
        for (int i = n - 2; i >= 0; --i) {
          const long o = i * W + lane;
          const double v = (X[o] - U1[o] * x1 - U2[o] * x2) / U0[o];
          X[o] = v;
          x2 = x1;
          x1 = v;
          mx = fmax(mx, fabs(v));
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
      // modified Gram-Schmidt inside the chunk, in eigenvalue order, twice;
      // the wavefront cooperates on one vector at a time
      for (int jj = 0; jj < kc; ++jj) {
        for (int pass = 0; pass < 2; ++pass)
          for (int q = 0; q < jj; ++q) {
            double dt = 0.0;
            for (int i = lane; i < n; i += 64) dt += X[i * W + q] * X[i * W + jj];
            dt = wave_sum(dt);
            for (int i = lane; i < n; i += 64) X[i * W + jj] -= dt * X[i * W + q];
            __syncthreads();
          }
        double nr = 0.0;
        for (int i = lane; i < n; i += 64) nr += X[i * W + jj] * X[i * W + jj];
        nr = wave_sum(nr);
        const double inr = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
        for (int i = lane; i < n; i += 64) X[i * W + jj] *= inr;
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
                 hipStream_t s) {
  if (a.nb == 0) return;
  hipLaunchKernelGGL(k_tri_vecs, dim3(a.nb), dim3(64), 0, s, a, count, lam_off, lam, d_Z, work, work_off, resid,
                     nstrict, thr);
  AWG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// back-transformation Z <- H_0 H_1 ... H_{n-3} Z
// ---------------------------------------------------------------------------
constexpr int ORM_COLS = 8;

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
    double dots[ORM_COLS];
#pragma unroll
    for (int c = 0; c < ORM_COLS; ++c) dots[c] = 0.0;
    for (int i = j + 1 + threadIdx.x; i < n; i += 256) {
      const double vi = v[i];
#pragma unroll
      for (int c = 0; c < ORM_COLS; ++c)
        if (c < nc) dots[c] += vi * zs[c * n + i];
    }
#pragma unroll
    for (int c = 0; c < ORM_COLS; ++c) {
      const double s = wave_sum(dots[c]);
      if (lane == 0) red[wid][c] = s;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < ORM_COLS; ++c) dots[c] = tj * ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c]));
    for (int i = j + 1 + threadIdx.x; i < n; i += 256) {
      const double vi = v[i];
#pragma unroll
      for (int c = 0; c < ORM_COLS; ++c)
        if (c < nc) zs[c * n + i] -= dots[c] * vi;
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
  hipLaunchKernelGGL(k_ormtr, dim3(cdiv(maxk, ORM_COLS), batch), dim3(256), lds, s, d_mats, d_Z, tau, d_off);
  AWG_LAUNCH_CHECK();
}

}  // namespace awg
