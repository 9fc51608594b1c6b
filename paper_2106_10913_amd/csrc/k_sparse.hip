// Sparse, gather/scatter, reduction and integer set-up kernels (gfx950).
//
// Multi-column vectors are column-major n x b with leading dimension ld.
// Per-subdomain blocks ("restricted" vectors R^s X) are stored back to back:
// block s starts at sub_off[s] * b and is n_s x b with leading dimension n_s.
// The prolongation (sum_s R^sT X_s) is computed as a gather over the inverse
// map dof -> (s, local index), so every output is written by one thread and the
// sum order is fixed (no atomics, bitwise reproducible).
#include "awg_sparse.h"

namespace awg {

// ---------------------------------------------------------------------------
// integer set-up: validation, multiplicity, inverse map, M_mu, B
// ---------------------------------------------------------------------------
// err bits: 1 partition (empty/unsorted/out of range/uncovered), 2 not
// symmetric, 4 minimal overlap, 8 non-finite value, 16 malformed CSR
__global__ void k_validate_subs(int N, const long* sub_ptr, const int* sub_idx, int n, int* err) {
  const int s = blockIdx.x;
  const long a = sub_ptr[s], b = sub_ptr[s + 1];
  if (b <= a) {
    if (threadIdx.x == 0) atomicOr(err, 1);
    return;
  }
  for (long p = a + threadIdx.x; p < b; p += blockDim.x) {
    const int v = sub_idx[p];
    bool bad = v < 0 || v >= n;
    if (p + 1 < b && !(v < sub_idx[p + 1])) bad = true;
    if (bad) atomicOr(err, 1);
  }
}

__global__ void k_entry_owner(int N, const long* sub_ptr, int* ent_sub) {
  const int s = blockIdx.x;
  for (long p = sub_ptr[s] + threadIdx.x; p < sub_ptr[s + 1]; p += blockDim.x) ent_sub[p] = s;
}

__global__ void k_mult(long tot, const int* sub_idx, int* mult) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < tot) atomicAdd(&mult[sub_idx[p]], 1);
}

__global__ void k_check_cover(int n, const int* mult, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && mult[i] == 0) atomicOr(err, 1);
}

// exclusive scan of n ints into out[0..n] (out[n] = total); one workgroup
__global__ __launch_bounds__(1024) void k_scan(int n, const int* in, int* out) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int a = min(n, t * chunk), b = min(n, a + chunk);
  int s = 0;
  for (int i = a; i < b; ++i) s += in[i];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = t > 0 ? part[t - 1] : 0;
  for (int i = a; i < b; ++i) {
    out[i] = run;
    run += in[i];
  }
  if (t == 1023) out[n] = part[1023];
}

__global__ void k_fill_inv(const long* sub_ptr, const int* sub_idx, const int* inv_ptr, int* fill, int* inv_sub,
                           int* inv_loc) {
  const int s = blockIdx.x;
  const long a = sub_ptr[s];
  for (long p = a + threadIdx.x; p < sub_ptr[s + 1]; p += blockDim.x) {
    const int g = sub_idx[p];
    const int q = inv_ptr[g] + atomicAdd(&fill[g], 1);
    inv_sub[q] = s;
    inv_loc[q] = (int)(p - a);
  }
}

__global__ void k_sort_inv(int n, const int* inv_ptr, int* inv_sub, int* inv_loc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = inv_ptr[i], b = inv_ptr[i + 1];
  for (int p = a + 1; p < b; ++p) {
    const int ks = inv_sub[p], kl = inv_loc[p];
    int q = p - 1;
    while (q >= a && inv_sub[q] > ks) {
      inv_sub[q + 1] = inv_sub[q];
      inv_loc[q + 1] = inv_loc[q];
      --q;
    }
    inv_sub[q + 1] = ks;
    inv_loc[q + 1] = kl;
  }
}

// symmetry, finiteness, pair counts M_mu and B = A / M_mu
__global__ void k_pairs(int n, const int* rowptr, const int* col, const double* val, const int* inv_ptr,
                        const int* inv_sub, int* cnt, double* bval, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ia = inv_ptr[i], ib = inv_ptr[i + 1];
  int e = 0;
  for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
    const int j = col[p];
    const double v = val[p];
    if (!isfinite(v)) e |= 8;
    if (j < 0 || j >= n) { e |= 16; cnt[p] = 0; bval[p] = 0.0; continue; }
    if (p + 1 < rowptr[i + 1] && !(j < col[p + 1])) e |= 16;  // unsorted or duplicate column
    // A_ji must exist and equal A_ij
    int lo = rowptr[j], hi = rowptr[j + 1] - 1;
    bool found = false;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int c = col[mid];
      if (c == i) { found = (val[mid] == v); break; }
      if (c < i) lo = mid + 1; else hi = mid - 1;
    }
    if (!found) e |= 2;
    // number of subdomains holding both i and j (sorted merge)
    int a = ia, b = inv_ptr[j];
    const int be = inv_ptr[j + 1];
    int c = 0;
    while (a < ib && b < be) {
      const int sa = inv_sub[a], sb = inv_sub[b];
      if (sa == sb) { ++c; ++a; ++b; }
      else if (sa < sb) ++a;
      else ++b;
    }
    cnt[p] = c;
    if (c == 0) { e |= 4; bval[p] = 0.0; }
    else bval[p] = v / (double)c;
  }
  if (e) atomicOr(err, e);
}

__global__ void k_pou(long tot, const int* sub_idx, const int* mult, double* dw) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < tot) dw[p] = 1.0 / (double)mult[sub_idx[p]];
}

// dense R^s M R^sT into block s (zeroed beforehand); one workgroup per subdomain
__global__ void k_extract(const long* sub_ptr, const int* sub_idx, const int* rowptr, const int* col,
                          const double* vals, const MatDesc* mats) {
  const int s = blockIdx.x;
  const MatDesc M = mats[s];
  const long a = sub_ptr[s];
  const int ns = M.n;
  const int* idx = sub_idx + a;
  for (int l = threadIdx.x; l < ns; l += blockDim.x) {
    const int i = idx[l];
    for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      const int j = col[p];
      int lo = 0, hi = ns - 1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = idx[mid];
        if (v == j) { M.A[l + (long)mid * M.ld] = vals[p]; break; }
        if (v < j) lo = mid + 1; else hi = mid - 1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// multi-column vector kernels
// ---------------------------------------------------------------------------
// Y = alpha A X + beta Y for b columns: one thread per row and SPMM_CB
// columns, so each row's nonzeros are read once per column block.
constexpr int SPMM_CB = 8;
__global__ __launch_bounds__(256) void k_spmm(int n, const int* rowptr, const int* col, const double* val,
                                              const double* X, long ldx, double* Y, long ldy, int b, double alpha,
                                              double beta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c0 = blockIdx.y * SPMM_CB;
  const int nc = min(SPMM_CB, b - c0);
  const double* x = X + c0 * ldx;
  double acc[SPMM_CB];
#pragma unroll
  for (int c = 0; c < SPMM_CB; ++c) acc[c] = 0.0;
  const int pe = rowptr[i + 1];
  if (nc == SPMM_CB) {
    for (int p = rowptr[i]; p < pe; ++p) {
      const double v = val[p];
      const long j = col[p];
#pragma unroll
      for (int c = 0; c < SPMM_CB; ++c) acc[c] += v * x[j + c * ldx];
    }
  } else {
    for (int p = rowptr[i]; p < pe; ++p) {
      const double v = val[p];
      const long j = col[p];
      for (int c = 0; c < nc; ++c) acc[c] += v * x[j + c * ldx];
    }
  }
  double* y = Y + c0 * ldy + i;
  for (int c = 0; c < nc; ++c) y[c * ldy] = (beta == 0.0) ? alpha * acc[c] : alpha * acc[c] + beta * y[c * ldy];
}

__global__ void k_gather(long tot, const int* sub_idx, const int* ent_sub, const long* sub_ptr, const double* X,
                         long ldx, int b, const double* scale, double* Xs) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= tot) return;
  const int c = blockIdx.y;
  const int s = ent_sub[p];
  const long a = sub_ptr[s];
  const long ns = sub_ptr[s + 1] - a;
  double v = X[sub_idx[p] + c * ldx];
  if (scale) v *= scale[p];
  Xs[a * b + c * ns + (p - a)] = v;
}

__global__ void k_scatter(int n, const int* inv_ptr, const int* inv_sub, const int* inv_loc, const long* sub_ptr,
                          const double* Zs, int b, const double* scale, double* Y, long ldy, double alpha,
                          double beta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = blockIdx.y;
  double acc = 0.0;
  for (int q = inv_ptr[i]; q < inv_ptr[i + 1]; ++q) {
    const int s = inv_sub[q];
    const long a = sub_ptr[s];
    const long ns = sub_ptr[s + 1] - a;
    double v = Zs[a * b + c * ns + inv_loc[q]];
    if (scale) v *= scale[a + inv_loc[q]];
    acc += v;
  }
  double* y = Y + c * ldy + i;
  *y = (beta == 0.0) ? alpha * acc : alpha * acc + beta * *y;
}

// out[c] = sum_i X[i,c] Y[i,c] (one workgroup per column, fixed order)
__global__ __launch_bounds__(256) void k_coldot(int n, const double* X, long ldx, const double* Y, long ldy,
                                                double* out) {
  const int c = blockIdx.x;
  const double* x = X + c * ldx;
  const double* y = Y + c * ldy;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += x[i] * y[i];
  __shared__ double sh[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[c] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Y[:,c] = sa a[c] X[:,c] + sb b[c] Y[:,c]   (a or b may be null: 1)
__global__ void k_colaxpby(int n, const double* X, long ldx, const double* a, double* Y, long ldy, const double* bb,
                           double sa, double sb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = blockIdx.y;
  const double ac = (a ? a[c] : 1.0) * sa;
  const double bc = (bb ? bb[c] : 1.0) * sb;
  double* y = Y + c * ldy + i;
  *y = ac * X[c * ldx + i] + bc * *y;
}

// ---------------------------------------------------------------------------
// small dense helpers
// ---------------------------------------------------------------------------
__global__ void k_set_identity(const MatDesc* mats) {
  const MatDesc M = mats[blockIdx.y];
  const long tot = (long)M.m * M.n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e % M.m), c = (int)(e / M.m);
    M.A[r + (long)c * M.ld] = (r == c) ? 1.0 : 0.0;
  }
}

__global__ void k_copy_mat(const MatDesc* src, const MatDesc* dst) {
  const MatDesc S = src[blockIdx.y], D = dst[blockIdx.y];
  const long tot = (long)S.m * S.n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e % S.m), c = (int)(e / S.m);
    D.A[r + (long)c * D.ld] = S.A[r + (long)c * S.ld];
  }
}

// M <- diag(dl) M diag(dr) (dl/dr: per-block vectors at offsets), optional
// symmetrisation (M + M^T)/2 done by the (r >= c) thread for both entries.
__global__ void k_scale_sym(const MatDesc* mats, const long* voff, const double* dl, int inv, int symmetrize) {
  const MatDesc M = mats[blockIdx.y];
  const double* d = dl ? dl + voff[blockIdx.y] : nullptr;
  const long tot = (long)M.n * M.n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e % M.n), c = (int)(e / M.n);
    if (r < c) continue;
    double a = M.A[r + (long)c * M.ld];
    double b = M.A[c + (long)r * M.ld];
    if (symmetrize) { a = 0.5 * (a + b); b = a; }
    if (d) {
      const double f = inv ? 1.0 / (d[r] * d[c]) : d[r] * d[c];
      a *= f;
      b *= f;
    }
    M.A[r + (long)c * M.ld] = a;
    M.A[c + (long)r * M.ld] = b;
  }
}

__global__ void k_transpose_inplace(const MatDesc* mats) {
  const MatDesc M = mats[blockIdx.y];
  const long tot = (long)M.n * M.n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e % M.n), c = (int)(e / M.n);
    if (r <= c) continue;
    const double a = M.A[r + (long)c * M.ld];
    M.A[r + (long)c * M.ld] = M.A[c + (long)r * M.ld];
    M.A[c + (long)r * M.ld] = a;
  }
}

// column scaling of the n_s x k_s blocks: column c of block b is multiplied by
//   mode 0: alpha * f[c]    mode 1: alpha * |f[c]|
//   mode 2: shift[b] - f[c] mode 3: alpha / shift[b]
__global__ void k_scale_cols(const MatDesc* mats, const long* coff, const double* f, double alpha,
                             const double* shift, int mode) {
  const MatDesc M = mats[blockIdx.y];
  const double* fc = f + coff[blockIdx.y];
  const long tot = (long)M.m * M.n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e % M.m), c = (int)(e / M.m);
    double g;
    if (mode == 0) g = alpha * fc[c];
    else if (mode == 1) g = alpha * fabs(fc[c]);
    else if (mode == 2) g = shift[blockIdx.y] - fc[c];
    else g = alpha / shift[blockIdx.y];
    M.A[r + (long)c * M.ld] *= g;
  }
}

// mean of the diagonal of each block
__global__ __launch_bounds__(256) void k_diag_mean(const MatDesc* mats, double* out) {
  const MatDesc M = mats[blockIdx.x];
  double acc = 0.0;
  for (int i = threadIdx.x; i < M.n; i += 256) acc += M.A[i + (long)i * M.ld];
  __shared__ double sh[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = ((sh[0] + sh[1]) + (sh[2] + sh[3])) / (double)(M.n > 0 ? M.n : 1);
}

// Neighbour low-rank terms of M_B^s = R^s A_+ R^sT (Remark 4, Section 4.4):
// entry (a, b) of block s gets sum over t != s holding both dofs of
// sum_k V^t[a_t,k] |lam^t_k| V^t[b_t,k].  One thread per entry; entries whose
// dofs lie in s only are skipped at once.
__global__ void k_mb_neighbours(const long* sub_ptr, const int* sub_idx, const int* mult, const int* inv_ptr,
                                const int* inv_sub, const int* inv_loc, const MatDesc* mats, const double* V,
                                const long* voff, const double* lam, const long* loff) {
  const int s = blockIdx.y;
  const MatDesc M = mats[s];
  const long a0 = sub_ptr[s];
  const long tot = (long)M.n * M.n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int ra = (int)(e % M.n), cb = (int)(e / M.n);
    const int gi = sub_idx[a0 + ra], gj = sub_idx[a0 + cb];
    if (mult[gi] < 2 || mult[gj] < 2) continue;
    double acc = 0.0;
    int p = inv_ptr[gi], q = inv_ptr[gj];
    const int pe = inv_ptr[gi + 1], qe = inv_ptr[gj + 1];
    while (p < pe && q < qe) {
      const int sp = inv_sub[p], sq = inv_sub[q];
      if (sp == sq) {
        if (sp != s) {
          const int t = sp;
          const int kt = (int)(loff[t + 1] - loff[t]);
          const long nt = sub_ptr[t + 1] - sub_ptr[t];
          const double* Vt = V + voff[t];
          const double* lt = lam + loff[t];
          const int la = inv_loc[p], lb = inv_loc[q];
          for (int k = 0; k < kt; ++k) acc += Vt[la + k * nt] * fabs(lt[k]) * Vt[lb + k * nt];
        }
        ++p;
        ++q;
      } else if (sp < sq) {
        ++p;
      } else {
        ++q;
      }
    }
    M.A[ra + (long)cb * M.ld] += acc;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned grid1(long n, int bs = 256) { return cdiv(n, bs); }

void l_validate_subs(int N, const long* sub_ptr, const int* sub_idx, int n, int* err, hipStream_t s) {
  hipLaunchKernelGGL(k_validate_subs, dim3(N), dim3(256), 0, s, N, sub_ptr, sub_idx, n, err);
  AWG_LAUNCH_CHECK();
}
void l_entry_owner(int N, const long* sub_ptr, int* ent_sub, hipStream_t s) {
  hipLaunchKernelGGL(k_entry_owner, dim3(N), dim3(256), 0, s, N, sub_ptr, ent_sub);
  AWG_LAUNCH_CHECK();
}
void l_mult(long tot, const int* sub_idx, int* mult, hipStream_t s) {
  hipLaunchKernelGGL(k_mult, dim3(grid1(tot)), dim3(256), 0, s, tot, sub_idx, mult);
  AWG_LAUNCH_CHECK();
}
void l_check_cover(int n, const int* mult, int* err, hipStream_t s) {
  hipLaunchKernelGGL(k_check_cover, dim3(grid1(n)), dim3(256), 0, s, n, mult, err);
  AWG_LAUNCH_CHECK();
}
void l_scan(int n, const int* in, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, n, in, out);
  AWG_LAUNCH_CHECK();
}
void l_fill_inv(int N, const long* sub_ptr, const int* sub_idx, const int* inv_ptr, int* fill, int* inv_sub,
                int* inv_loc, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_inv, dim3(N), dim3(256), 0, s, sub_ptr, sub_idx, inv_ptr, fill, inv_sub, inv_loc);
  AWG_LAUNCH_CHECK();
}
void l_sort_inv(int n, const int* inv_ptr, int* inv_sub, int* inv_loc, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_inv, dim3(grid1(n)), dim3(256), 0, s, n, inv_ptr, inv_sub, inv_loc);
  AWG_LAUNCH_CHECK();
}
void l_pairs(int n, const int* rowptr, const int* col, const double* val, const int* inv_ptr, const int* inv_sub,
             int* cnt, double* bval, int* err, hipStream_t s) {
  hipLaunchKernelGGL(k_pairs, dim3(grid1(n)), dim3(256), 0, s, n, rowptr, col, val, inv_ptr, inv_sub, cnt, bval,
                     err);
  AWG_LAUNCH_CHECK();
}
void l_pou(long tot, const int* sub_idx, const int* mult, double* dw, hipStream_t s) {
  hipLaunchKernelGGL(k_pou, dim3(grid1(tot)), dim3(256), 0, s, tot, sub_idx, mult, dw);
  AWG_LAUNCH_CHECK();
}
void l_extract(int N, const long* sub_ptr, const int* sub_idx, const int* rowptr, const int* col,
               const double* vals, const MatDesc* mats, hipStream_t s) {
  hipLaunchKernelGGL(k_extract, dim3(N), dim3(256), 0, s, sub_ptr, sub_idx, rowptr, col, vals, mats);
  AWG_LAUNCH_CHECK();
}
void l_spmm(int n, long nnz, const int* rowptr, const int* col, const double* val, const double* X, long ldx,
            double* Y, long ldy, int b, double alpha, double beta, hipStream_t s) {
  if (n == 0 || b == 0) return;
  KScope kt("k_spmm", s,
            12.0 * nnz + 4.0 * (n + 1) + 16.0 * n * (double)b + (beta != 0.0 ? 8.0 * n * (double)b : 0.0),
            2.0 * nnz * (double)b);
  hipLaunchKernelGGL(k_spmm, dim3(grid1(n), cdiv(b, SPMM_CB)), dim3(256), 0, s, n, rowptr, col, val, X, ldx, Y, ldy, b,
                     alpha, beta);
  AWG_LAUNCH_CHECK();
}
void l_gather(long tot, const int* sub_idx, const int* ent_sub, const long* sub_ptr, const double* X, long ldx,
              int b, const double* scale, double* Xs, hipStream_t s) {
  if (tot == 0 || b == 0) return;
  KScope kt("k_gather", s, 8.0 * tot * (double)b + 8.0 * tot + 8.0 * (double)tot * b, 0.0);
  hipLaunchKernelGGL(k_gather, dim3(grid1(tot), b), dim3(256), 0, s, tot, sub_idx, ent_sub, sub_ptr, X, ldx, b,
                     scale, Xs);
  AWG_LAUNCH_CHECK();
}
void l_scatter(int n, long tot, const int* inv_ptr, const int* inv_sub, const int* inv_loc, const long* sub_ptr,
               const double* Zs, int b, const double* scale, double* Y, long ldy, double alpha, double beta,
               hipStream_t s) {
  if (n == 0 || b == 0) return;
  KScope kt("k_scatter", s, 8.0 * (double)tot * b + 8.0 * tot + 4.0 * n + 8.0 * n * (double)b * (beta != 0.0 ? 2.0 : 1.0),
            (double)tot * b);
  hipLaunchKernelGGL(k_scatter, dim3(grid1(n), b), dim3(256), 0, s, n, inv_ptr, inv_sub, inv_loc, sub_ptr, Zs, b,
                     scale, Y, ldy, alpha, beta);
  AWG_LAUNCH_CHECK();
}
void l_coldot(int n, int b, const double* X, long ldx, const double* Y, long ldy, double* out, hipStream_t s) {
  if (b == 0) return;
  hipLaunchKernelGGL(k_coldot, dim3(b), dim3(256), 0, s, n, X, ldx, Y, ldy, out);
  AWG_LAUNCH_CHECK();
}
void l_colaxpby(int n, int b, const double* X, long ldx, const double* a, double* Y, long ldy, const double* bb,
                double sa, double sb, hipStream_t s) {
  if (n == 0 || b == 0) return;
  hipLaunchKernelGGL(k_colaxpby, dim3(grid1(n), b), dim3(256), 0, s, n, X, ldx, a, Y, ldy, bb, sa, sb);
  AWG_LAUNCH_CHECK();
}
void l_set_identity(const MatDesc* mats, int batch, hipStream_t s) {
  if (!batch) return;
  hipLaunchKernelGGL(k_set_identity, dim3(256, batch), dim3(256), 0, s, mats);
  AWG_LAUNCH_CHECK();
}
void l_copy_mat(const MatDesc* src, const MatDesc* dst, int batch, hipStream_t s) {
  if (!batch) return;
  hipLaunchKernelGGL(k_copy_mat, dim3(256, batch), dim3(256), 0, s, src, dst);
  AWG_LAUNCH_CHECK();
}
void l_scale_sym(const MatDesc* mats, int batch, const long* voff, const double* d, bool inv, bool symmetrize,
                 hipStream_t s) {
  if (!batch) return;
  hipLaunchKernelGGL(k_scale_sym, dim3(256, batch), dim3(256), 0, s, mats, voff, d, (int)inv, (int)symmetrize);
  AWG_LAUNCH_CHECK();
}
void l_transpose_inplace(const MatDesc* mats, int batch, hipStream_t s) {
  if (!batch) return;
  hipLaunchKernelGGL(k_transpose_inplace, dim3(256, batch), dim3(256), 0, s, mats);
  AWG_LAUNCH_CHECK();
}
void l_scale_cols(const MatDesc* mats, int batch, const long* coff, const double* f, double alpha,
                  const double* shift, int mode, hipStream_t s) {
  if (!batch) return;
  hipLaunchKernelGGL(k_scale_cols, dim3(64, batch), dim3(256), 0, s, mats, coff, f, alpha, shift, mode);
  AWG_LAUNCH_CHECK();
}
void l_diag_mean(const MatDesc* mats, int batch, double* out, hipStream_t s) {
  if (!batch) return;
  hipLaunchKernelGGL(k_diag_mean, dim3(batch), dim3(256), 0, s, mats, out);
  AWG_LAUNCH_CHECK();
}
void l_mb_neighbours(int N, const long* sub_ptr, const int* sub_idx, const int* mult, const int* inv_ptr,
                     const int* inv_sub, const int* inv_loc, const MatDesc* mats, const double* V, const long* voff,
                     const double* lam, const long* loff, hipStream_t s) {
  if (!N) return;
  hipLaunchKernelGGL(k_mb_neighbours, dim3(512, N), dim3(256), 0, s, sub_ptr, sub_idx, mult, inv_ptr, inv_sub,
                     inv_loc, mats, V, voff, lam, loff);
  AWG_LAUNCH_CHECK();
}

}  // namespace awg
