// Batched FP32 Cholesky factorisation and explicit inverse of SPD blocks on
// the FP32 matrix cores, with the per-block conditioning that decides the
// FP64 fallback.
//
// For every block K (n_b x n_b, column-major, FP32):
//   K = L L^T          right-looking, 32-wide panels: the diagonal block in
//                      LDS, the rows below by substitution, the trailing
//                      update A -= P P^T on v_mfma_f32_16x16x4f32 (lower
//                      tiles only);
//   X = L^{-1}         blocked forward substitution on the identity, 64-row
//                      blocks: the diagonal solve in LDS, the update of the
//                      rows below on the matrix cores;
//   K^{-1} = X^T X     on the matrix cores, k running from the later of the
//                      two tiles' first rows (X is lower triangular).
// info[b] = first column whose pivot is not positive (1-based), 0 if none;
// dmin[b], dmax[b] = extreme diagonal entries of L, whose squared ratio
// bounds the spectral condition number of K from below.
#include <algorithm>
#include <vector>

#include "awg_common.h"

namespace awg {

typedef float v4f32 __attribute__((ext_vector_type(4)));

constexpr int C32_NB = 32;   // panel width of the factorisation
constexpr int T32_NB = 64;   // block height of the substitution

__global__ __launch_bounds__(256) void k_potf2_f32(const MatDescF* mats, int j, int* info, float* dmin,
                                                   float* dmax) {
  const MatDescF M = mats[blockIdx.x];
  const int jb = min(C32_NB, M.n - j);
  if (jb <= 0) return;
  __shared__ float L[C32_NB][C32_NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < jb * jb; e += 256) {
    const int r = e % jb, c = e / jb;
    L[r][c] = M.A[(j + r) + (long)(j + c) * M.ld];
  }
  __syncthreads();
  for (int c = 0; c < jb; ++c) {
    if (tid == 0) {
      const float piv = L[c][c];
      if (!(piv > 0.f)) {
        if (info[blockIdx.x] == 0) info[blockIdx.x] = j + c + 1;
        L[c][c] = __builtin_nanf("");
      } else {
        const float d = sqrtf(piv);
        L[c][c] = d;
        dmin[blockIdx.x] = (j + c == 0) ? d : fminf(dmin[blockIdx.x], d);
        dmax[blockIdx.x] = (j + c == 0) ? d : fmaxf(dmax[blockIdx.x], d);
      }
    }
    __syncthreads();
    const float dc = L[c][c];
    for (int r = c + 1 + tid; r < jb; r += 256) L[r][c] = L[r][c] / dc;
    __syncthreads();
    const int rem = jb - c - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      const int r = c + 1 + e % rem, q = c + 1 + e / rem;
      if (q <= r) L[r][q] -= L[r][c] * L[q][c];
    }
    __syncthreads();
  }
  for (int e = tid; e < jb * jb; e += 256) {
    const int r = e % jb, c = e / jb;
    M.A[(j + r) + (long)(j + c) * M.ld] = r >= c ? L[r][c] : 0.f;
  }
}

// rows below the diagonal block: X L_jj^T = A[j+jb:, j:j+jb]
__global__ __launch_bounds__(256) void k_chol_panel_f32(const MatDescF* mats, int j) {
  const MatDescF M = mats[blockIdx.y];
  const int jb = min(C32_NB, M.n - j);
  if (jb <= 0) return;
  __shared__ float L[C32_NB][C32_NB + 1];
  for (int e = threadIdx.x; e < jb * jb; e += 256) {
    const int r = e % jb, c = e / jb;
    L[r][c] = (r >= c) ? M.A[(j + r) + (long)(j + c) * M.ld] : 0.f;
  }
  __syncthreads();
  const int i = j + jb + blockIdx.x * 256 + threadIdx.x;
  if (i >= M.n) return;
  float x[C32_NB];
#pragma unroll
  for (int c = 0; c < C32_NB; ++c) {
    if (c < jb) {
      float v = M.A[i + (long)(j + c) * M.ld];
      for (int t = 0; t < c; ++t) v -= x[t] * L[c][t];
      x[c] = v / L[c][c];
    }
  }
#pragma unroll
  for (int c = 0; c < C32_NB; ++c)
    if (c < jb) M.A[i + (long)(j + c) * M.ld] = x[c];
}

// Update C -= op(A) op(B) on 64 x 64 tiles of one block per workgroup row
// (four wavefronts of 32 x 32, k staged 32 deep in LDS), FP32 MFMA and sums.
// The operands are described by a small provider per mode:
//   mode 0 (Cholesky trailing update at column j): C = A[r0:, r0:] lower
//          tiles, op(A) = A[r0:, j:j+32], op(B) = A[r0:, j:j+32]^T, r0 = j + 32;
//   mode 1 (forward substitution at block row j): C = X[j+64:, :],
//          op(A) = L[j+64:, j:j+64], op(B) = X[j:j+64, :];
//   mode 2 (inverse from L^-1): C = K^-1 (fresh), op(A) = X^T, op(B) = X,
//          k from the later first row of the two tiles to n.
struct U32 {
  const float* A;
  long lda;
  bool ta;        // op(A)[i][k] = A[k + i lda] (else A[i + k lda])
  const float* B;
  long ldb;
  bool tb;        // op(B)[k][j] = B[j + k ldb] (else B[k + j ldb])
  float* C;
  long ldc;
  int m, n, k0, k1;
  bool lower;     // tiles strictly above the diagonal are skipped
  bool assign;    // C = result (else C -= result)
};

template <int MODE>
__device__ inline U32 u32_desc(const MatDescF& L, const MatDescF& X, const MatDescF& Out, int j) {
  U32 u{};
  if (MODE == 0) {
    const int r0 = j + C32_NB, rem = max(0, L.n - r0);
    u.A = L.A + r0 + (long)j * L.ld;
    u.lda = L.ld;
    u.ta = false;
    u.B = u.A;
    u.ldb = L.ld;
    u.tb = true;
    u.C = L.A + r0 + (long)r0 * L.ld;
    u.ldc = L.ld;
    u.m = u.n = rem;
    u.k0 = 0;
    u.k1 = min(C32_NB, max(0, L.n - j));
    u.lower = true;
    u.assign = false;
  } else if (MODE == 1) {
    const int jb = min(T32_NB, max(0, L.n - j)), r0 = j + jb;
    u.A = L.A + r0 + (long)j * L.ld;
    u.lda = L.ld;
    u.ta = false;
    u.B = X.A + j;
    u.ldb = X.ld;
    u.tb = false;
    u.C = X.A + r0;
    u.ldc = X.ld;
    u.m = max(0, L.n - r0);
    u.n = L.n;
    u.k0 = 0;
    u.k1 = jb;
    u.lower = false;
    u.assign = false;
  } else {
    u.A = X.A;
    u.lda = X.ld;
    u.ta = true;
    u.B = X.A;
    u.ldb = X.ld;
    u.tb = false;
    u.C = Out.A;
    u.ldc = Out.ld;
    u.m = u.n = X.n;
    u.k0 = 0;
    u.k1 = X.n;
    u.lower = false;
    u.assign = true;
  }
  return u;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_upd_f32(const MatDescF* Ls, const MatDescF* Xs, const MatDescF* Outs,
                                                 int j) {
  const int b = blockIdx.z;
  const U32 u = u32_desc<MODE>(Ls[b], Xs ? Xs[b] : Ls[b], Outs ? Outs[b] : Ls[b], j);
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  if (m0 >= u.m || n0 >= u.n) return;
  if (u.lower && n0 > m0) return;
  // X = L^-1 is lower triangular: X^T X needs k >= max(m0, n0) only
  const int kstart = MODE == 2 ? max(m0, n0) : u.k0;
  __shared__ float As[32][68];
  __shared__ float Bs[32][68];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  v4f32 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = (v4f32){0.f, 0.f, 0.f, 0.f};
  for (int k0 = kstart; k0 < u.k1; k0 += 32) {
    // stage op(A)[m0.., k0..] and op(B)[k0.., n0..] as [k][i] and [k][j]
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + q * 256;            // 0 .. 2047 = 32 k x 64 rows
      const int i = e & 63, kk = e >> 6;
      const int gi = m0 + i, gk = k0 + kk;
      float va = 0.f, vb = 0.f;
      if (gi < u.m && gk < u.k1) va = u.ta ? u.A[gk + (long)gi * u.lda] : u.A[gi + (long)gk * u.lda];
      const int gj = n0 + i;
      if (gj < u.n && gk < u.k1) vb = u.tb ? u.B[gj + (long)gk * u.ldb] : u.B[gk + (long)gj * u.ldb];
      As[kk][i] = va;
      Bs[kk][i] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 32; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      float a[2], bb[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) a[q] = As[kr][wm + q * 16 + c];
#pragma unroll
      for (int q = 0; q < 2; ++q) bb[q] = Bs[kr][wn + q * 16 + c];
#pragma unroll
      for (int qa = 0; qa < 2; ++qa)
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
          acc[qa][qb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bb[qb], a[qa], acc[qa][qb], 0, 0, 0);
    }
    __syncthreads();
  }
  // acc[qa][qb][r]: row i = wm + 16 qa + (lane & 15), column j = wn + 16 qb + 4 (lane >> 4) + r
#pragma unroll
  for (int qa = 0; qa < 2; ++qa)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm + qa * 16 + (lane & 15);
        const int jj = n0 + wn + qb * 16 + 4 * (lane >> 4) + r;
        if (i < u.m && jj < u.n && (!u.lower || jj <= i)) {
          float* cp = u.C + i + (long)jj * u.ldc;
          *cp = u.assign ? acc[qa][qb][r] : *cp - acc[qa][qb][r];
        }
      }
}

// diagonal block of the forward substitution: X[j:j+64, c0:c0+64] =
// L_jj^{-1} X[j:j+64, c0:c0+64], one wavefront substituting 64 columns
__global__ __launch_bounds__(256) void k_trsm_diag_f32(const MatDescF* Ls, const MatDescF* Xs, int j) {
  const MatDescF l = Ls[blockIdx.y], x = Xs[blockIdx.y];
  const int jb = min(T32_NB, l.n - j);
  const int c0 = blockIdx.x * 64;
  if (jb <= 0 || c0 >= x.n) return;
  __shared__ float L[T32_NB][T32_NB + 1];
  __shared__ float Xt[T32_NB][T32_NB + 1];
  const int tid = threadIdx.x;
  const int nc = min(64, x.n - c0);
  for (int q = 0; q < T32_NB * T32_NB / 256; ++q) {
    const int e = tid + 256 * q, r = e & (T32_NB - 1), c = e / T32_NB;
    L[r][c] = (r < jb && c < jb && r >= c) ? l.A[(j + r) + (long)(j + c) * l.ld] : 0.f;
    Xt[r][c] = (r < jb && c < nc) ? x.A[(j + r) + (long)(c0 + c) * x.ld] : 0.f;
  }
  __syncthreads();
  if (tid < nc) {
    const int c = tid;
    for (int r = 0; r < jb; ++r) {
      float v = Xt[r][c];
      for (int t = 0; t < r; ++t) v -= L[r][t] * Xt[t][c];
      Xt[r][c] = v / L[r][r];
    }
  }
  __syncthreads();
  for (int q = 0; q < T32_NB * T32_NB / 256; ++q) {
    const int e = tid + 256 * q, r = e & (T32_NB - 1), c = e / T32_NB;
    if (r < jb && c < nc) x.A[(j + r) + (long)(c0 + c) * x.ld] = Xt[r][c];
  }
}

__global__ void k_identity_f32(const MatDescF* mats) {
  const MatDescF M = mats[blockIdx.y];
  const long tot = (long)M.n * M.n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e % M.n), c = (int)(e / M.n);
    M.A[r + (long)c * M.ld] = r == c ? 1.f : 0.f;
  }
}

void chol_inverse_f32(const MatDescF* d_K, const MatDescF* d_X, const MatDescF* d_out, const std::vector<int>& h_n,
                      int* d_info, float* d_dmin, float* d_dmax, hipStream_t s) {
  const int batch = (int)h_n.size();
  if (batch == 0) return;
  int maxn = 0;
  for (int v : h_n) maxn = std::max(maxn, v);
  double flf = 0.0;
  for (int v : h_n) flf += (double)v * v * v;
  KScope kt("k_chol_inverse_f32", s, 0.0, 2.0 * flf);     // n^3/3 + n^3/3 + n^3 (X^T X on the triangle) ~ 2 n^3 / ...
  for (int j = 0; j < maxn; j += C32_NB) {
    hipLaunchKernelGGL(k_potf2_f32, dim3(batch), dim3(256), 0, s, d_K, j, d_info, d_dmin, d_dmax);
    AWG_LAUNCH_CHECK();
    const int rem = maxn - j - C32_NB;
    if (rem <= 0) break;
    hipLaunchKernelGGL(k_chol_panel_f32, dim3(cdiv(rem, 256), batch), dim3(256), 0, s, d_K, j);
    AWG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_upd_f32<0>, dim3(cdiv(rem, 64), cdiv(rem, 64), batch), dim3(256), 0, s, d_K,
                       (const MatDescF*)nullptr, (const MatDescF*)nullptr, j);
    AWG_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_identity_f32, dim3(64, batch), dim3(256), 0, s, d_X);
  AWG_LAUNCH_CHECK();
  for (int j = 0; j < maxn; j += T32_NB) {
    hipLaunchKernelGGL(k_trsm_diag_f32, dim3(cdiv(maxn, 64), batch), dim3(256), 0, s, d_K, d_X, j);
    AWG_LAUNCH_CHECK();
    const int rem = maxn - j - T32_NB;
    if (rem <= 0) break;
    hipLaunchKernelGGL(k_upd_f32<1>, dim3(cdiv(rem, 64), cdiv(maxn, 64), batch), dim3(256), 0, s, d_K, d_X,
                       (const MatDescF*)nullptr, j);
    AWG_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_upd_f32<2>, dim3(cdiv(maxn, 64), cdiv(maxn, 64), batch), dim3(256), 0, s, d_K, d_X, d_out,
                     0);
  AWG_LAUNCH_CHECK();
}

}  // namespace awg
