// Kernels of the iterative GenEO eigensolver: block subspace iteration with
// Rayleigh-Ritz on the operator T = Pi_B G M_B of every subdomain, where
// G = D^s (A^s_+)^+ D^s is a generalised inverse of M_A = (D^s)^-1 A^s_+ (D^s)^-1
// and Pi_B is the M_B-orthogonal projector that removes ker M_A = D^s V^s_-.
// For an eigenpair M_A y = lambda M_B y with lambda > 0, T y = y / lambda, so
// the GenEO modes below tau (Theorem on H^NN_hyb, Section 3.4) are the modes of
// T above 1 / tau.  Every small dense problem of one subdomain (Cholesky of
// the q x q Gram matrix, the q x q symmetric eigenproblem by cyclic Jacobi)
// runs in one wavefront in LDS.
#include <hip/hip_runtime.h>

#include "awg_common.h"
#include "awg_subspace.h"

namespace awg {

namespace {

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ double bsum256(double v, double* sh) {
  v = wsum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// out_s = diag(dw_s) V_s for the column blocks of every subdomain
__global__ void k_rows_dw(int N, const long* sub_ptr, const long* eoff, const long* coff, const double* V,
                          const double* dw, double* out) {
  const int s = blockIdx.y;
  const long ns = sub_ptr[s + 1] - sub_ptr[s];
  const long k = coff[s + 1] - coff[s];
  const long tot = ns * k;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const long i = e % ns;
    out[eoff[s] + e] = V[eoff[s] + e] * dw[sub_ptr[s] + i];
  }
}

// splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014), used as a counter-based generator
__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// X_s (n_s x q, column-major at sub_ptr[s] * q) uniform in [-1, 1), keyed by
// the global dof, the column and the seed
__global__ void k_rand_block(int N, const long* sub_ptr, const int* sub_idx, int q, uint64_t seed, double* X) {
  const int s = blockIdx.y;
  const long base = sub_ptr[s];
  const long ns = sub_ptr[s + 1] - base;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < ns * q; e += (long)gridDim.x * blockDim.x) {
    const long i = e % ns, j = e / ns;
    const uint64_t key = ((uint64_t)(uint32_t)sub_idx[base + i] << 8 | (uint64_t)j) ^ (seed * 0xD1B54A32D192ED03ull);
    const uint64_t r = splitmix64(key);
    X[base * q + e] = 2.0 * ((double)(r >> 11) * 0x1.0p-53) - 1.0;
  }
}

// Copy the first ncol[s] columns of the block at src (n_s x q, column-major)
// into columns c0.. of the column layout dst.
__global__ void k_init_cols(int N, const long* sub_ptr, int q, const double* src, const int* ncol, double* X) {
  const int s = blockIdx.y;
  const long base = sub_ptr[s];
  const long ns = sub_ptr[s + 1] - base;
  const long tot = ns * (long)ncol[s];
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x)
    X[base * q + e] = src[base * q + e];
}

constexpr int RR_MAX = SUBSPACE_MAX_BLOCK;

// Rayleigh-Ritz of one subdomain: S1 c = mu S0 c with S0 = X^T M_B X and
// S1 = (M_B X)^T T X, both q x q.  Cholesky S0 = R R^T, Jacobi on
// R^-1 S1 R^-T = W diag(mu) W^T, c = R^-T W (so c^T S0 c = I), mu descending.
// flag[s] = 1 when S0 is numerically singular.
__global__ __launch_bounds__(64) void k_rr_small(int q, const double* S0, const double* S1, double* C, double* mu,
                                                 int* flag) {
  const int s = blockIdx.x;
  const int lane = threadIdx.x;
  __shared__ double R[RR_MAX][RR_MAX + 1];
  __shared__ double A[RR_MAX][RR_MAX + 1];
  __shared__ double V[RR_MAX][RR_MAX + 1];
  __shared__ double cs[RR_MAX / 2], sn[RR_MAX / 2];
  __shared__ int pp[RR_MAX / 2], rr[RR_MAX / 2], perm[RR_MAX];
  __shared__ double mus[RR_MAX];
  __shared__ int bad;
  const double* s0 = S0 + (long)s * q * q;
  const double* s1 = S1 + (long)s * q * q;
  if (lane == 0) bad = 0;
  if (lane < q)
    for (int r = 0; r < q; ++r) {
      R[r][lane] = 0.5 * (s0[r + lane * q] + s0[lane + r * q]);
      A[r][lane] = 0.5 * (s1[r + lane * q] + s1[lane + r * q]);
      V[r][lane] = (r == lane) ? 1.0 : 0.0;
    }
  __syncthreads();
  double dmax = 0.0;
  for (int j = 0; j < q; ++j) dmax = fmax(dmax, R[j][j]);
  // Cholesky S0 = R R^T (lower, in place)
  for (int j = 0; j < q; ++j) {
    const double d = R[j][j];
    const bool ok = d > 1e-13 * dmax && dmax > 0.0;
    const double sd = ok ? sqrt(d) : 1.0;
    __syncthreads();
    if (lane == 0) {
      if (!ok) bad = 1;
      R[j][j] = sd;
    }
    if (lane > j && lane < q) R[lane][j] /= sd;
    __syncthreads();
    if (lane > j && lane < q)
      for (int l = j + 1; l <= lane; ++l) R[lane][l] -= R[lane][j] * R[l][j];
    __syncthreads();
  }
  // A <- R^-1 A (lane = column)
  if (lane < q)
    for (int r = 0; r < q; ++r) {
      double v = A[r][lane];
      for (int l = 0; l < r; ++l) v -= R[r][l] * A[l][lane];
      A[r][lane] = v / R[r][r];
    }
  __syncthreads();
  // V <- R^-1 A^T (lane = column of A^T = row of A), then A <- sym(V)
  if (lane < q)
    for (int r = 0; r < q; ++r) {
      double v = A[lane][r];
      for (int l = 0; l < r; ++l) v -= R[r][l] * V[l][lane];
      V[r][lane] = v / R[r][r];
    }
  __syncthreads();
  if (lane < q)
    for (int r = 0; r < q; ++r) A[r][lane] = 0.5 * (V[r][lane] + V[lane][r]);
  __syncthreads();
  if (lane < q)
    for (int r = 0; r < q; ++r) V[r][lane] = (r == lane) ? 1.0 : 0.0;
  __syncthreads();
  // cyclic Jacobi with round-robin (circle method) ordering of disjoint pairs;
  // rotation of Golub and Van Loan, Matrix Computations, Section 8.5
  const int qq = (q + 1) & ~1;
  const int npair = qq / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    if (lane < q)
      for (int r = 0; r < q; ++r) {
        const double v = A[r][lane] * A[r][lane];
        tot += v;
        if (r != lane) off += v;
      }
    off = wsum(off);
    tot = wsum(tot);
    if (!(off > 1e-32 * tot)) break;
    for (int t = 0; t < qq - 1; ++t) {
      if (lane < npair) {
        int a, b;
        if (lane == 0) {
          a = 0;
          b = ((qq - 2 + t) % (qq - 1)) + 1;
        } else {
          a = ((lane - 1 + t) % (qq - 1)) + 1;
          b = ((qq - 2 - lane + t) % (qq - 1)) + 1;
        }
        const int p = a < b ? a : b, r = a < b ? b : a;
        double c = 1.0, sv = 0.0;
        if (r < q) {
          const double apr = A[p][r];
          if (apr != 0.0) {
            const double th = (A[r][r] - A[p][p]) / (2.0 * apr);
            const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + tt * tt);
            sv = tt * c;
          }
        }
        pp[lane] = p;
        rr[lane] = r < q ? r : p;
        cs[lane] = c;
        sn[lane] = sv;
      }
      __syncthreads();
      if (lane < q)
        for (int i = 0; i < npair; ++i) {
          const int p = pp[i], r = rr[i];
          if (p == r) continue;
          const double c = cs[i], sv = sn[i];
          const double ap = A[p][lane], ar = A[r][lane];
          A[p][lane] = c * ap - sv * ar;
          A[r][lane] = sv * ap + c * ar;
        }
      __syncthreads();
      if (lane < q)
        for (int i = 0; i < npair; ++i) {
          const int p = pp[i], r = rr[i];
          if (p == r) continue;
          const double c = cs[i], sv = sn[i];
          const double ap = A[lane][p], ar = A[lane][r];
          A[lane][p] = c * ap - sv * ar;
          A[lane][r] = sv * ap + c * ar;
          const double vp = V[lane][p], vr = V[lane][r];
          V[lane][p] = c * vp - sv * vr;
          V[lane][r] = sv * vp + c * vr;
        }
      __syncthreads();
    }
  }
  // descending order
  if (lane < q) {
    const double me = A[lane][lane];
    int rank = 0;
    for (int j = 0; j < q; ++j) {
      const double o = A[j][j];
      rank += (o > me) || (o == me && j < lane);
    }
    perm[rank] = lane;
  }
  __syncthreads();
  if (lane < q) mus[lane] = A[perm[lane]][perm[lane]];
  __syncthreads();
  if (lane < q) {
    const int j = perm[lane];
    // c_k = R^-T w_k, w_k = V[:, j]; back substitution into column k of A
    for (int r = q - 1; r >= 0; --r) {
      double v = V[r][j];
      for (int l = r + 1; l < q; ++l) v -= R[l][r] * A[l][lane];
      A[r][lane] = v / R[r][r];
    }
  }
  __syncthreads();
  if (lane < q) {
    for (int r = 0; r < q; ++r) C[(long)s * q * q + r + (long)lane * q] = bad ? (r == lane ? 1.0 : 0.0) : A[r][lane];
    mu[(long)s * q + lane] = bad ? 0.0 : mus[lane];
  }
  if (lane == 0) flag[s] = bad;
}

// Residuals of the Ritz pairs (mu_j, z_j): ||T z_j - mu_j z_j|| / (mu_j ||z_j||),
// next block X_j = T z_j / ||T z_j||, and the per-subdomain state:
// conv[s] = 1 when every Ritz value with 1/mu < window*tau has residual <= tol
// (or, with none in that window, the leading pair has residual <= tol_far);
// nsel[s] = #{j : mu_j > 1/tau}.
__global__ __launch_bounds__(256) void k_ritz_resid(int N, const long* sub_ptr, int q, const double* Z,
                                                    const double* TZ, const double* mu, double* X, double* res,
                                                    int* conv, int* nsel, double tau, double window, double tol,
                                                    double tol_far) {
  const int s = blockIdx.x;
  __shared__ double sh[4];
  const long base = sub_ptr[s] * q;
  const long ns = sub_ptr[s + 1] - sub_ptr[s];
  for (int j = 0; j < q; ++j) {
    const double m = mu[(long)s * q + j];
    const double* z = Z + base + (long)j * ns;
    const double* t = TZ + base + (long)j * ns;
    double a = 0.0, b = 0.0, c = 0.0;
    for (long i = threadIdx.x; i < ns; i += 256) {
      const double d = t[i] - m * z[i];
      a += d * d;
      b += z[i] * z[i];
      c += t[i] * t[i];
    }
    a = bsum256(a, sh);
    b = bsum256(b, sh);
    c = bsum256(c, sh);
    const double inv = c > 0.0 ? 1.0 / sqrt(c) : 0.0;
    double* x = X + base + (long)j * ns;
    for (long i = threadIdx.x; i < ns; i += 256) x[i] = t[i] * inv;
    if (threadIdx.x == 0) res[(long)s * q + j] = (m > 0.0 && b > 0.0) ? sqrt(a) / (m * sqrt(b)) : 1e300;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1, inwin = 0, sel = 0;
    for (int j = 0; j < q; ++j) {
      const double m = mu[(long)s * q + j];
      if (m * tau > 1.0) ++sel;
      if (m * window * tau > 1.0) {
        ++inwin;
        if (!(res[(long)s * q + j] <= tol)) ok = 0;
      }
    }
    if (inwin == 0) ok = res[(long)s * q] <= tol_far;
    conv[s] = ok;
    nsel[s] = sel;
  }
}

// Y_s = [K_s | first nsel_s columns of Z_s]; lam = [0 ... 0 | 1/mu]
__global__ void k_assemble_modes(int N, const long* sub_ptr, int q, const double* K, const long* koff_e,
                                 const long* koff_c, const double* Z, const double* mu, double* Y, const long* yoff_e,
                                 const long* yoff_c, double* lam) {
  const int s = blockIdx.y;
  const long ns = sub_ptr[s + 1] - sub_ptr[s];
  const long k = koff_c[s + 1] - koff_c[s];
  const long m = yoff_c[s + 1] - yoff_c[s];
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < ns * m; e += (long)gridDim.x * blockDim.x) {
    const long i = e % ns, j = e / ns;
    Y[yoff_e[s] + e] = j < k ? K[koff_e[s] + e] : Z[sub_ptr[s] * q + (j - k) * ns + i];
  }
  if (blockIdx.x == 0)
    for (long j = threadIdx.x; j < m; j += blockDim.x)
      lam[yoff_c[s] + j] = j < k ? 0.0 : 1.0 / mu[(long)s * q + (j - k)];
}

__global__ void k_axpy_flat(long n, double a, const double* x, double* y) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    y[e] += a * x[e];
}

}  // namespace

void l_rows_dw(int N, int maxns, int maxk, const long* sub_ptr, const long* eoff, const long* coff, const double* V,
               const double* dw, double* out, hipStream_t s) {
  if (N == 0 || maxk == 0) return;
  hipLaunchKernelGGL(k_rows_dw, dim3(std::max(1u, std::min(256u, cdiv((long)maxns * maxk, 256))), N), dim3(256), 0,
                     s, N, sub_ptr, eoff, coff, V, dw, out);
  AWG_LAUNCH_CHECK();
}

void l_rand_block(int N, int maxns, const long* sub_ptr, const int* sub_idx, int q, uint64_t seed, double* X,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_rand_block, dim3(std::max(1u, std::min(256u, cdiv((long)maxns * q, 256))), N), dim3(256), 0,
                     s, N, sub_ptr, sub_idx, q, seed, X);
  AWG_LAUNCH_CHECK();
}

void l_init_cols(int N, int maxns, const long* sub_ptr, int q, const double* src, const int* ncol, double* X,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_init_cols, dim3(std::max(1u, std::min(256u, cdiv((long)maxns * q, 256))), N), dim3(256), 0,
                     s, N, sub_ptr, q, src, ncol, X);
  AWG_LAUNCH_CHECK();
}

void l_rr_small(int N, int q, const double* S0, const double* S1, double* C, double* mu, int* flag, hipStream_t s) {
  KScope kt("k_rr_small", s, 0.0, 0.0);
  hipLaunchKernelGGL(k_rr_small, dim3(N), dim3(64), 0, s, q, S0, S1, C, mu, flag);
  AWG_LAUNCH_CHECK();
}

void l_ritz_resid(int N, const long* sub_ptr, int q, const double* Z, const double* TZ, const double* mu, double* X,
                  double* res, int* conv, int* nsel, double tau, double window, double tol, double tol_far,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_ritz_resid, dim3(N), dim3(256), 0, s, N, sub_ptr, q, Z, TZ, mu, X, res, conv, nsel, tau,
                     window, tol, tol_far);
  AWG_LAUNCH_CHECK();
}

void l_assemble_modes(int N, int maxns, int maxm, const long* sub_ptr, int q, const double* K, const long* koff_e,
                      const long* koff_c, const double* Z, const double* mu, double* Y, const long* yoff_e,
                      const long* yoff_c, double* lam, hipStream_t s) {
  if (maxm == 0) return;
  hipLaunchKernelGGL(k_assemble_modes, dim3(std::max(1u, std::min(256u, cdiv((long)maxns * maxm, 256))), N),
                     dim3(256), 0, s, N, sub_ptr, q, K, koff_e, koff_c, Z, mu, Y, yoff_e, yoff_c, lam);
  AWG_LAUNCH_CHECK();
}

void l_axpy_flat(long n, double a, const double* x, double* y, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_axpy_flat, dim3(std::min(4096u, cdiv(n, 256))), dim3(256), 0, s, n, a, x, y);
  AWG_LAUNCH_CHECK();
}

}  // namespace awg
