// Batched dense kernels for variable-size column-major blocks (gfx950).
//
//  * k_gemm     : C = alpha op(A) op(B) + beta C, FP64 MFMA (v_mfma_f64_16x16x4),
//                 64x64 output tile per 256-thread workgroup, K staged in LDS.
//  * k_gemv     : memory-bound y = alpha op(A) x + beta y.
//  * potrf      : right-looking blocked Cholesky (32-wide panels): LDS panel
//                 factorisation, row-parallel panel solve, MFMA trailing update.
//  * trsm       : blocked forward / backward substitution with many right-hand
//                 sides: 64x64 diagonal solve in LDS + MFMA update of the rest.
#include <algorithm>

#include "awg_common.h"
#include "awg_tune.h"

namespace awg {

typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// descriptor providers
// ---------------------------------------------------------------------------
struct DescArray {
  const GemmDesc* d;
  __device__ GemmDesc operator()(int b) const { return d[b]; }
};

// explicit descriptors whose A operands are row gathers of X (see
// gemm_batched_gather)
struct DescGather {
  const GemmDesc* d;
  const double* X;
  const int* idx;
  const long* off;
  __device__ GemmDesc operator()(int b) const {
    GemmDesc g = d[b];
    g.A = X;
    g.acol = idx + off[b];
    return g;
  }
};

template <class DF>
struct gathers_a {
  static constexpr bool value = false;
};
template <>
struct gathers_a<DescGather> {
  static constexpr bool value = true;
};

// Gathered A operands: the workgroup copies the first ACOL_LDS column indices
// into LDS once, so the A loads of the k loop do not wait on a global index
// load (columns beyond ACOL_LDS read the index from global memory).
constexpr int ACOL_LDS = 2048;

template <class DF>
struct AcolTable {
  int* s;   // LDS table (gathered instantiations only)
  __device__ long operator()(const GemmDesc& d, int k) const {
    if (!gathers_a<DF>::value) return (long)k * d.lda;
    return (long)(k < ACOL_LDS ? s[k] : d.acol[k]) * d.lda;
  }
};

// fills the LDS table; every thread of the workgroup must call it (barrier)
template <class DF>
__device__ inline AcolTable<DF> acol_table(int* s, const GemmDesc& d) {
  if (gathers_a<DF>::value) {
    const int kn = d.k < ACOL_LDS ? d.k : ACOL_LDS;
    for (int k = threadIdx.x; k < kn; k += blockDim.x) s[k] = d.acol[k];
    __syncthreads();
  }
  return AcolTable<DF>{s};
}

// trailing update of the Cholesky panel step at column j (panel width nb):
// A[j+nb:, j+nb:] -= A[j+nb:, j:j+nb] * A[j+nb:, j:j+nb]^T
struct CholUpdate {
  const MatDesc* m;
  int j, nb;
  __device__ GemmDesc operator()(int b) const {
    MatDesc M = m[b];
    GemmDesc g;
    int r0 = j + nb;
    int rem = M.n - r0;
    if (rem < 0) rem = 0;
    g.A = M.A + r0 + (long)j * M.ld;
    g.B = g.A;
    g.C = M.A + r0 + (long)r0 * M.ld;
    g.m = rem;
    g.n = rem;
    g.k = nb;
    g.lda = g.ldb = g.ldc = M.ld;
    return g;
  }
};

// trsm update at block row j (block height nb):
//  forward : B[j+nb:, :] -= L[j+nb:, j:j+nb] * B[j:j+nb, :]
//  backward: B[0:j, :]   -= L[j:j+nb, 0:j]^T * B[j:j+nb, :]
struct TrsmUpdate {
  const MatDesc* L;
  const MatDesc* B;
  int j, nb;
  bool backward;
  __device__ GemmDesc operator()(int b) const {
    MatDesc l = L[b], x = B[b];
    GemmDesc g;
    int n = l.n;
    int jb = n - j < nb ? n - j : nb;
    g.n = x.n;
    g.ldb = x.ld;
    g.ldc = x.ld;
    g.lda = l.ld;
    if (jb <= 0) {
      g.m = 0; g.k = 0; g.A = l.A; g.B = x.A; g.C = x.A;
      return g;
    }
    if (!backward) {
      g.A = l.A + (j + jb) + (long)j * l.ld;
      g.B = x.A + j;
      g.C = x.A + (j + jb);
      g.m = n - j - jb;
      g.k = jb;
    } else {
      g.A = l.A + j;                // rows j..j+jb of L, columns 0..j; used transposed
      g.B = x.A + j;
      g.C = x.A;
      g.m = j;
      g.k = jb;
    }
    return g;
  }
};

// panel update of the blocked tridiagonalisation at panel start p0:
// A[r0:, r0:] -= X[r0:, 0:kb] Y[r0:, 0:kb]^T with r0 = p0 + kb and
// (X, Y) = (V, W) or (W, V); V and W are n x TRD_NB per block at voff/woff.
struct Syr2kUpdate {
  const MatDesc* m;
  const double* X;
  const double* Y;
  const long* off;     // per block: element offset of its n x nbw work panels
  int p0, nbw;
  __device__ GemmDesc operator()(int b) const {
    MatDesc M = m[b];
    GemmDesc g;
    int kb = M.n - 2 - p0;
    kb = kb < 0 ? 0 : (kb > nbw ? nbw : kb);
    const int r0 = p0 + kb;
    const int rem = kb > 0 ? M.n - r0 : 0;
    const long o = off[b] * (long)nbw;
    g.A = X + o + r0;
    g.B = Y + o + r0;
    g.C = M.A + r0 + (long)r0 * M.ld;
    g.m = rem;
    g.n = rem;
    g.k = kb;
    g.lda = g.ldb = M.n;
    g.ldc = M.ld;
    return g;
  }
};

// ---------------------------------------------------------------------------
// GEMM, FP64 MFMA
// ---------------------------------------------------------------------------
// MFMA f64 16x16x4 operand layout (one wavefront of 64 lanes):
//   A (16x4): lane l holds A[l % 16][l / 16]
//   B (4x16): lane l holds B[l / 16][l % 16]
//   D (16x16): lane l holds D[l/16 + 4*r][l % 16], r = 0..3 (checked on gfx950)
// The tile kernels pass the B fragment as the first operand and the A
// fragment as the second, which yields each 16 x 16 block of C transposed
// (same products, same k order): lane l then holds C[l % 16][l/16 + 4*r], so
// 16 consecutive lanes store 16 consecutive rows of the column-major C.
template <class DF, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(DF df, double alpha, double beta, int lower) {
  const GemmDesc d = df(blockIdx.z);
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  if (m0 >= d.m || n0 >= d.n) return;
  if (lower && m0 + 64 <= n0) return;
  __shared__ double As[16][66];
  __shared__ double Bs[16][66];
  __shared__ int s_acol[gathers_a<DF>::value ? ACOL_LDS : 1];
  const AcolTable<DF> a_col = acol_table<DF>(s_acol, d);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < d.k; k0 += 16) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * 256;
      int i, kk;
      if (!TA) { i = e & 63; kk = e >> 6; } else { kk = e & 15; i = e >> 4; }
      const int gi = m0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < d.m && gk < d.k) v = TA ? d.A[gk + (long)gi * d.lda] : d.A[gi + a_col(d, gk)];
      As[kk][i] = v;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * 256;
      int j, kk;
      if (!TB) { kk = e & 15; j = e >> 4; } else { j = e & 63; kk = e >> 6; }
      const int gj = n0 + j, gk = k0 + kk;
      double v = 0.0;
      if (gj < d.n && gk < d.k) v = TB ? d.B[gj + (long)gk * d.ldb] : d.B[gk + (long)gj * d.ldb];
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      const double a0 = As[kr][wm + c], a1 = As[kr][wm + 16 + c];
      const double b0 = Bs[kr][wn + c], b1 = Bs[kr][wn + 16 + c];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a1, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm + a * 16 + (lane & 15);
        const int j = n0 + wn + b * 16 + (lane >> 4) + 4 * r;
        if (i < d.m && j < d.n) {
          double* c = d.C + i + (long)j * d.ldc;
          const double v = alpha * acc[a][b][r];
          *c = (beta == 0.0) ? v : v + beta * *c;
        }
      }
}

// 128x128 output tile per workgroup (each wavefront a 64x64 quarter = 4x4
// MFMA blocks), K staged in LDS in steps of 16 with the next step's global
// loads held in registers while the current one is multiplied.
template <class DF, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm128(DF df, double alpha, double beta, int lower) {
  const GemmDesc d = df(blockIdx.z);
  const int m0 = blockIdx.x * 128, n0 = blockIdx.y * 128;
  if (m0 >= d.m || n0 >= d.n) return;
  if (lower && m0 + 128 <= n0) return;
  __shared__ double As[2][16][132];
  __shared__ double Bs[2][16][132];
  __shared__ int s_acol[gathers_a<DF>::value ? ACOL_LDS : 1];
  const AcolTable<DF> a_col = acol_table<DF>(s_acol, d);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  double ra[8], rb[8];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tid + r * 256;
      int i, kk;
      if (!TA) { i = e & 127; kk = e >> 7; } else { kk = e & 15; i = e >> 4; }
      const int gi = m0 + i, gk = k0 + kk;
      ra[r] = (gi < d.m && gk < d.k) ? (TA ? d.A[gk + (long)gi * d.lda] : d.A[gi + a_col(d, gk)]) : 0.0;
      int j, kb;
      if (!TB) { kb = e & 15; j = e >> 4; } else { j = e & 127; kb = e >> 7; }
      const int gj = n0 + j, gkb = k0 + kb;
      rb[r] = (gj < d.n && gkb < d.k) ? (TB ? d.B[gj + (long)gkb * d.ldb] : d.B[gkb + (long)gj * d.ldb]) : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tid + r * 256;
      int i, kk;
      if (!TA) { i = e & 127; kk = e >> 7; } else { kk = e & 15; i = e >> 4; }
      As[buf][kk][i] = ra[r];
      int j, kb;
      if (!TB) { kb = e & 15; j = e >> 4; } else { j = e & 127; kb = e >> 7; }
      Bs[buf][kb][j] = rb[r];
    }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < d.k; k0 += 16) {
    const bool more = k0 + 16 < d.k;
    if (more) gload(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[buf][kr][wm + q * 16 + c];
        b[q] = Bs[buf][kr][wn + q * 16 + c];
      }
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
          acc[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[qb], a[qa], acc[qa][qb], 0, 0, 0);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int qa = 0; qa < 4; ++qa)
#pragma unroll
    for (int qb = 0; qb < 4; ++qb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm + qa * 16 + (lane & 15);
        const int j = n0 + wn + qb * 16 + (lane >> 4) + 4 * r;
        if (i < d.m && j < d.n) {
          double* cp = d.C + i + (long)j * d.ldc;
          const double v = alpha * acc[qa][qb][r];
          *cp = (beta == 0.0) ? v : v + beta * *cp;
        }
      }
}

// 128x128 tiles with eight wavefronts (2 x 4, each 64 x 32): half the
// accumulators per lane of k_gemm128, so more wavefronts fit per SIMD to hide
// the global-load latency.  Same k order and MFMA as the other tile shapes
// (bit-identical results).  The MFMA takes its operands swapped and yields
// each 16 x 16 block transposed, so that 16 consecutive lanes hold 16
// consecutive rows of C and store one contiguous 128-byte segment.
template <class DF, bool TA, bool TB>
__global__ __launch_bounds__(512, 4) void k_gemm128w8(DF df, double alpha, double beta, int lower) {
  const GemmDesc d = df(blockIdx.z);
  const int m0 = blockIdx.x * 128, n0 = blockIdx.y * 128;
  if (m0 >= d.m || n0 >= d.n) return;
  if (lower && m0 + 128 <= n0) return;
  __shared__ double As[2][16][132];
  __shared__ double Bs[2][16][132];
  __shared__ int s_acol[gathers_a<DF>::value ? ACOL_LDS : 1];
  const AcolTable<DF> a_col = acol_table<DF>(s_acol, d);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 32;
  v4d acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  double ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * 512;
      int i, kk;
      if (!TA) { i = e & 127; kk = e >> 7; } else { kk = e & 15; i = e >> 4; }
      const int gi = m0 + i, gk = k0 + kk;
      ra[r] = (gi < d.m && gk < d.k) ? (TA ? d.A[gk + (long)gi * d.lda] : d.A[gi + a_col(d, gk)]) : 0.0;
      int j, kb;
      if (!TB) { kb = e & 15; j = e >> 4; } else { j = e & 127; kb = e >> 7; }
      const int gj = n0 + j, gkb = k0 + kb;
      rb[r] = (gj < d.n && gkb < d.k) ? (TB ? d.B[gj + (long)gkb * d.ldb] : d.B[gkb + (long)gj * d.ldb]) : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * 512;
      int i, kk;
      if (!TA) { i = e & 127; kk = e >> 7; } else { kk = e & 15; i = e >> 4; }
      As[buf][kk][i] = ra[r];
      int j, kb;
      if (!TB) { kb = e & 15; j = e >> 4; } else { j = e & 127; kb = e >> 7; }
      Bs[buf][kb][j] = rb[r];
    }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < d.k; k0 += 16) {
    const bool more = k0 + 16 < d.k;
    if (more) gload(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      double a[4], b[2];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = As[buf][kr][wm + q * 16 + c];
#pragma unroll
      for (int q = 0; q < 2; ++q) b[q] = Bs[buf][kr][wn + q * 16 + c];
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
          acc[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[qb], a[qa], acc[qa][qb], 0, 0, 0);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int qa = 0; qa < 4; ++qa)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm + qa * 16 + (lane & 15);
        const int j = n0 + wn + qb * 16 + (lane >> 4) + 4 * r;
        if (i < d.m && j < d.n) {
          double* cp = d.C + i + (long)j * d.ldc;
          const double v = alpha * acc[qa][qb][r];
          *cp = (beta == 0.0) ? v : v + beta * *cp;
        }
      }
}

// Skinny products (N small, untransposed operands): each wavefront computes a
// 32 x 32 output block on its own, loading its A and B operands from global
// memory straight into the MFMA register layout (no LDS, no barrier), with the
// next k step's loads in flight while the current one is multiplied and the
// gathered column indices fetched one step further ahead.  Same k order and
// MFMA as the tile kernels (bit-identical results).
template <class DF, int KB>
__global__ __launch_bounds__(256) void k_gemm_skinny(DF df, double alpha, double beta) {
  constexpr int T = KB / 4;   // groups of 4 k values per load batch
  const GemmDesc d = df(blockIdx.z);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.x * 128 + wave * 32, n0 = blockIdx.y * 32;
  if (m0 >= d.m || n0 >= d.n) return;
  const int r16 = lane & 15, kq = lane >> 4;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  // column offsets of A for the k values k0 + 4 t + kq of a batch
  auto colofs = [&](int k0, long* o) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int k = k0 + 4 * t + kq;
      o[t] = k < d.k ? (gathers_a<DF>::value ? (long)d.acol[k] * d.lda : (long)k * d.lda) : -1;
    }
  };
  auto load = [&](int k0, const long* o, double* ra, double* rb) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int k = k0 + 4 * t + kq;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int m = m0 + 16 * q + r16, n = n0 + 16 * q + r16;
        ra[2 * t + q] = (o[t] >= 0 && m < d.m) ? d.A[m + o[t]] : 0.0;
        rb[2 * t + q] = (k < d.k && n < d.n) ? d.B[k + (long)n * d.ldb] : 0.0;
      }
    }
  };
  long oc[T], on[T];
  double ca[2 * T], cb[2 * T], na[2 * T], nb[2 * T];
  colofs(0, oc);
  load(0, oc, ca, cb);
  colofs(KB, on);
  // k is taken in steps of 16 like the tile kernels; KB = 32 loads two steps at once
  const int kend = (d.k + 15) & ~15;
  for (int k0 = 0; k0 < kend; k0 += KB) {
    const bool more = k0 + KB < kend;
    if (more) {
      load(k0 + KB, on, na, nb);
      colofs(k0 + 2 * KB, on);
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      if (KB == 32 && t == 4 && k0 + 16 >= kend) break;
#pragma unroll
      for (int qa = 0; qa < 2; ++qa)
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
          acc[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[2 * t + qa], cb[2 * t + qb], acc[qa][qb], 0, 0, 0);
    }
    if (more) {
#pragma unroll
      for (int r = 0; r < 2 * T; ++r) {
        ca[r] = na[r];
        cb[r] = nb[r];
      }
    }
  }
#pragma unroll
  for (int qa = 0; qa < 2; ++qa)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + qa * 16 + kq + 4 * r;
        const int j = n0 + qb * 16 + r16;
        if (i < d.m && j < d.n) {
          double* cp = d.C + i + (long)j * d.ldc;
          const double v = alpha * acc[qa][qb][r];
          *cp = (beta == 0.0) ? v : v + beta * *cp;
        }
      }
}

// k_gemm_skinny with the 16 x 32 B panel of each k step loaded once per
// workgroup into LDS (double-buffered) instead of once per wavefront: the
// four wavefronts (128 rows of A) share it.  Same MFMA sequence per output.
template <class DF>
__global__ __launch_bounds__(256) void k_gemm_skinny_lds(DF df, double alpha, double beta) {
  const GemmDesc d = df(blockIdx.z);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, tid = threadIdx.x;
  const int m0 = blockIdx.x * 128 + wave * 32, n0 = blockIdx.y * 32;
  if (blockIdx.x * 128 >= d.m || n0 >= d.n) return;     // whole workgroup
  const bool live = m0 < d.m;                          // this wavefront has rows
  const int r16 = lane & 15, kq = lane >> 4;
  __shared__ double Bs[2][16][33];
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  auto colofs = [&](int k0, long* o) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + 4 * t + kq;
      o[t] = k < d.k ? (gathers_a<DF>::value ? (long)d.acol[k] * d.lda : (long)k * d.lda) : -1;
    }
  };
  auto loadA = [&](const long* o, double* ra) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int m = m0 + 16 * q + r16;
        ra[2 * t + q] = (live && o[t] >= 0 && m < d.m) ? d.A[m + o[t]] : 0.0;
      }
  };
  // B panel element (kb, j) of step k0: thread e = tid + 256 r, kb = e & 15, j = e >> 4
  auto loadB = [&](int k0, double* rb) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = tid + 256 * r, kb = e & 15, j = e >> 4;
      const int k = k0 + kb, n = n0 + j;
      rb[r] = (k < d.k && n < d.n) ? d.B[k + (long)n * d.ldb] : 0.0;
    }
  };
  auto storeB = [&](int buf, const double* rb) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = tid + 256 * r;
      Bs[buf][e & 15][e >> 4] = rb[r];
    }
  };
  long oc[4], on[4];
  double ca[8], na[8], rbn[2];
  colofs(0, oc);
  loadA(oc, ca);
  loadB(0, rbn);
  storeB(0, rbn);
  colofs(16, on);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < d.k; k0 += 16) {
    const bool more = k0 + 16 < d.k;
    if (more) {
      loadA(on, na);
      loadB(k0 + 16, rbn);
      colofs(k0 + 32, on);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      double cb[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) cb[q] = Bs[buf][4 * t + kq][16 * q + r16];
#pragma unroll
      for (int qa = 0; qa < 2; ++qa)
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
          acc[qa][qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[2 * t + qa], cb[qb], acc[qa][qb], 0, 0, 0);
    }
    if (more) {
      storeB(buf ^ 1, rbn);
#pragma unroll
      for (int r = 0; r < 8; ++r) ca[r] = na[r];
    }
    __syncthreads();
    buf ^= 1;
  }
  if (!live) return;
#pragma unroll
  for (int qa = 0; qa < 2; ++qa)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + qa * 16 + kq + 4 * r;
        const int j = n0 + qb * 16 + r16;
        if (i < d.m && j < d.n) {
          double* cp = d.C + i + (long)j * d.ldc;
          const double v = alpha * acc[qa][qb][r];
          *cp = (beta == 0.0) ? v : v + beta * *cp;
        }
      }
}

// ---------------------------------------------------------------------------
// mixed-precision GEMM for FP32 local operators: C (FP64) = alpha A B + beta C
// with A FP64 (rounded to FP32 when staged in LDS), B FP32, FP32 MFMA
// 16x16x4 and FP32 accumulation.  FP32 16x16x4 output layout (checked on
// gfx950): lane l holds D[4*(l/16) + r][l % 16].
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline GemmDescMix mix_desc(const GemmDescMix* descs, int z, const double* gX, const int* gidx,
                                       const long* goff) {
  GemmDescMix d = descs[z];
  if (gX) {
    d.A = gX;
    d.acol = gidx + goff[z];
  }
  return d;
}

__global__ __launch_bounds__(256) void k_gemm128_mix(const GemmDescMix* descs, double alpha, double beta,
                                                     const double* gX, const int* gidx, const long* goff) {
  const GemmDescMix d = mix_desc(descs, blockIdx.z, gX, gidx, goff);
  const int m0 = blockIdx.x * 128, n0 = blockIdx.y * 128;
  if (m0 >= d.m || n0 >= d.n) return;
  __shared__ float As[2][16][132];
  __shared__ float Bs[2][16][132];
  __shared__ int s_acol[ACOL_LDS];
  if (d.acol) {
    const int kn = d.k < ACOL_LDS ? d.k : ACOL_LDS;
    for (int k = threadIdx.x; k < kn; k += blockDim.x) s_acol[k] = d.acol[k];
    __syncthreads();
  }
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  v4f acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
  float ra[8], rb[8];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tid + r * 256;
      const int i = e & 127, kk = e >> 7;
      const int gi = m0 + i, gk = k0 + kk;
      ra[r] = (gi < d.m && gk < d.k) ? (float)d.A[gi + (d.acol ? (long)(gk < ACOL_LDS ? s_acol[gk] : d.acol[gk]) : (long)gk) * d.lda] : 0.f;
      const int kb = e & 15, j = e >> 4;
      const int gj = n0 + j, gkb = k0 + kb;
      rb[r] = (gj < d.n && gkb < d.k) ? d.B[gkb + (long)gj * d.ldb] : 0.f;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tid + r * 256;
      As[buf][e >> 7][e & 127] = ra[r];
      Bs[buf][e & 15][e >> 4] = rb[r];
    }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < d.k; k0 += 16) {
    const bool more = k0 + 16 < d.k;
    if (more) gload(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      float a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[buf][kr][wm + q * 16 + c];
        b[q] = Bs[buf][kr][wn + q * 16 + c];
      }
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
          acc[qa][qb] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[qb], a[qa], acc[qa][qb], 0, 0, 0);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int qa = 0; qa < 4; ++qa)
#pragma unroll
    for (int qb = 0; qb < 4; ++qb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm + qa * 16 + (lane & 15);
        const int j = n0 + wn + qb * 16 + 4 * (lane >> 4) + r;
        if (i < d.m && j < d.n) {
          double* cp = d.C + i + (long)j * d.ldc;
          const double v = alpha * (double)acc[qa][qb][r];
          *cp = (beta == 0.0) ? v : v + beta * *cp;
        }
      }
}

// eight-wavefront form of k_gemm128_mix (2 x 4 wavefronts of 64 x 32), same
// k order (bit-identical results)
__global__ __launch_bounds__(512, 4) void k_gemm128_mix_w8(const GemmDescMix* descs, double alpha, double beta,
                                                           const double* gX, const int* gidx, const long* goff) {
  const GemmDescMix d = mix_desc(descs, blockIdx.z, gX, gidx, goff);
  const int m0 = blockIdx.x * 128, n0 = blockIdx.y * 128;
  if (m0 >= d.m || n0 >= d.n) return;
  __shared__ float As[2][16][132];
  __shared__ float Bs[2][16][132];
  __shared__ int s_acol[ACOL_LDS];
  if (d.acol) {
    const int kn = d.k < ACOL_LDS ? d.k : ACOL_LDS;
    for (int k = threadIdx.x; k < kn; k += blockDim.x) s_acol[k] = d.acol[k];
    __syncthreads();
  }
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 32;
  v4f acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
  float ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * 512;
      const int i = e & 127, kk = e >> 7;
      const int gi = m0 + i, gk = k0 + kk;
      ra[r] = (gi < d.m && gk < d.k) ? (float)d.A[gi + (d.acol ? (long)(gk < ACOL_LDS ? s_acol[gk] : d.acol[gk]) : (long)gk) * d.lda] : 0.f;
      const int kb = e & 15, j = e >> 4;
      const int gj = n0 + j, gkb = k0 + kb;
      rb[r] = (gj < d.n && gkb < d.k) ? d.B[gkb + (long)gj * d.ldb] : 0.f;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * 512;
      As[buf][e >> 7][e & 127] = ra[r];
      Bs[buf][e & 15][e >> 4] = rb[r];
    }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < d.k; k0 += 16) {
    const bool more = k0 + 16 < d.k;
    if (more) gload(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      float a[4], b[2];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = As[buf][kr][wm + q * 16 + c];
#pragma unroll
      for (int q = 0; q < 2; ++q) b[q] = Bs[buf][kr][wn + q * 16 + c];
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
          acc[qa][qb] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[qb], a[qa], acc[qa][qb], 0, 0, 0);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int qa = 0; qa < 4; ++qa)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm + qa * 16 + (lane & 15);
        const int j = n0 + wn + qb * 16 + 4 * (lane >> 4) + r;
        if (i < d.m && j < d.n) {
          double* cp = d.C + i + (long)j * d.ldc;
          const double v = alpha * (double)acc[qa][qb][r];
          *cp = (beta == 0.0) ? v : v + beta * *cp;
        }
      }
}

void gemm_mix_batched(const GemmDescMix* d_desc, int batch, int max_m, int max_n, double alpha, double beta,
                      hipStream_t s, double flops, const double* X, const int* idx, const long* off) {
  if (batch <= 0 || max_m <= 0 || max_n <= 0) return;
  const dim3 grid(cdiv(max_m, 128), cdiv(max_n, 128), batch);
  auto run = [&](int v) {
    if (v == 1) hipLaunchKernelGGL(k_gemm128_mix_w8, grid, dim3(512), 0, s, d_desc, alpha, beta, X, idx, off);
    else hipLaunchKernelGGL(k_gemm128_mix, grid, dim3(256), 0, s, d_desc, alpha, beta, X, idx, off);
    AWG_LAUNCH_CHECK();
  };
  const std::string key = std::string(X ? "gemm_mix:Pg" : "gemm_mix:P") + ":m=" + std::to_string(max_m) +
                          ":n=" + std::to_string(max_n) + ":batch=" + std::to_string(batch);
  int v = tune_lookup(key);
  if (v < 0 && beta == 0.0) v = tune_pick(key, 2, run, s);
  if (v < 0) v = 1;
  KScope kt(v == 1 ? "k_gemm128_mix_w8:P" : "k_gemm128_mix:P", s, 0.0, flops);
  run(v);
}

// FP32 A and B (A already rounded, e.g. by l_gather_f32): 128 x 128 tiles,
// eight wavefronts of 64 x 32, k staged in LDS 32 deep (half the barriers per
// flop of the mixed kernels); same MFMA sequence per output as
// k_gemm128_mix_w8 (bit-identical to it: the k tail past K adds zero products)
__device__ __forceinline__ void gemm128_f32_w8_tile(const GemmDescF32& d, double alpha, double beta, int m0, int n0) {
  __shared__ float As[2][32][132];
  __shared__ float Bs[2][32][132];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 32;
  v4f acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
  float ra[8], rb[8];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tid + r * 512;
      const int i = e & 127, kk = e >> 7;
      const int gi = m0 + i, gk = k0 + kk;
      ra[r] = (gi < d.m && gk < d.k) ? d.A[gi + (long)gk * d.lda] : 0.f;
      const int kb = e & 31, j = e >> 5;
      const int gj = n0 + j, gkb = k0 + kb;
      rb[r] = (gj < d.n && gkb < d.k) ? d.B[gkb + (long)gj * d.ldb] : 0.f;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tid + r * 512;
      As[buf][e >> 7][e & 127] = ra[r];
      Bs[buf][e & 31][e >> 5] = rb[r];
    }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < d.k; k0 += 32) {
    const bool more = k0 + 32 < d.k;
    if (more) gload(k0 + 32);
#pragma unroll
    for (int kk = 0; kk < 32; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
      float a[4], b[2];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = As[buf][kr][wm + q * 16 + c];
#pragma unroll
      for (int q = 0; q < 2; ++q) b[q] = Bs[buf][kr][wn + q * 16 + c];
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
          acc[qa][qb] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[qb], a[qa], acc[qa][qb], 0, 0, 0);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int qa = 0; qa < 4; ++qa)
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm + qa * 16 + (lane & 15);
        const int j = n0 + wn + qb * 16 + 4 * (lane >> 4) + r;
        if (i < d.m && j < d.n) {
          double* cp = d.C + i + (long)j * d.ldc;
          const double v = alpha * (double)acc[qa][qb][r];
          *cp = (beta == 0.0) ? v : v + beta * *cp;
        }
      }
}

__global__ __launch_bounds__(512, 4) void k_gemm128_f32_w8(const GemmDescF32* descs, double alpha, double beta) {
  const GemmDescF32 d = descs[blockIdx.z];
  const int m0 = blockIdx.x * 128, n0 = blockIdx.y * 128;
  if (m0 >= d.m || n0 >= d.n) return;
  gemm128_f32_w8_tile(d, alpha, beta, m0, n0);
}

// Persistent form: a fixed grid whose workgroup w takes the tiles
// tiles[w], tiles[w + G], ... (G = gridDim.x) of a list built by
// f32_tile_list (code = batch entry << 12 | m tile << 6 | n tile, -1 =
// padding).  The same tile computation as k_gemm128_f32_w8 (bit-identical).
__global__ __launch_bounds__(512, 4) void k_gemm128_f32_w8_persist(const GemmDescF32* descs, double alpha,
                                                                   double beta, const int* tiles, int ntiles) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int code = tiles[t];
    if (code < 0) continue;
    const GemmDescF32 d = descs[code >> 12];
    __syncthreads();            // the previous tile's LDS reads are done
    gemm128_f32_w8_tile(d, alpha, beta, ((code >> 6) & 63) * 128, (code & 63) * 128);
  }
}

// Tile list of the persistent launch: the batch entries are sized by their
// work (tiles x k), sorted by it (size buckets, largest first) and dealt to
// the 8 XCDs, each to the least loaded one; each XCD's workgroups (those
// with w = x mod 8, which the hardware places on XCD x) sweep the tiles of
// the entries dealt to it, so one entry's operands are re-read through one
// XCD's L2.  Returns the grid size (0 and an empty list when a size does not
// fit the tile code); tiles (host) gets the list.
int f32_tile_list(const std::vector<int>& m, const std::vector<int>& n, const std::vector<int>& k, int wgs_per_xcd,
                  std::vector<int>& tiles) {
  constexpr int XCD = 8;
  const int batch = (int)m.size();
  tiles.clear();
  for (int b = 0; b < batch; ++b)     // the code holds 6 bits per tile index
    if (cdiv(m[b], 128) > 64 || cdiv(n[b], 128) > 64 || batch >= (1 << 19)) return 0;
  std::vector<int> order(batch);
  std::vector<double> work(batch);
  for (int b = 0; b < batch; ++b) {
    order[b] = b;
    work[b] = (double)cdiv(m[b], 128) * cdiv(n[b], 128) * std::max(1, k[b]);
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  std::vector<std::vector<int>> q(XCD);
  std::vector<double> load(XCD, 0.0);
  for (int b : order) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[x] += work[b];
    for (int tn = 0; tn < (int)cdiv(n[b], 128); ++tn)
      for (int tm = 0; tm < (int)cdiv(m[b], 128); ++tm) q[x].push_back(b << 12 | tm << 6 | tn);
  }
  size_t rounds = 0;
  for (auto& v : q) rounds = std::max(rounds, (v.size() + wgs_per_xcd - 1) / wgs_per_xcd);
  const int G = XCD * wgs_per_xcd;
  tiles.assign(rounds * G, -1);
  for (int x = 0; x < XCD; ++x)
    for (size_t i = 0; i < q[x].size(); ++i) {
      const size_t r = i / wgs_per_xcd, l = i % wgs_per_xcd;
      tiles[r * G + l * XCD + x] = q[x][i];
    }
  return G;
}

void gemm_f32_batched(const GemmDescF32* d_desc, int batch, int max_m, int max_n, double alpha, double beta,
                      hipStream_t s, double flops, const int* tiles, int ntiles, int grid) {
  if (batch <= 0 || max_m <= 0 || max_n <= 0) return;
  auto run = [&](int v) {
    if (v == 1)
      hipLaunchKernelGGL(k_gemm128_f32_w8_persist, dim3(grid), dim3(512), 0, s, d_desc, alpha, beta, tiles, ntiles);
    else
      hipLaunchKernelGGL(k_gemm128_f32_w8, dim3(cdiv(max_m, 128), cdiv(max_n, 128), batch), dim3(512), 0, s, d_desc,
                         alpha, beta);
    AWG_LAUNCH_CHECK();
  };
  int v = 0;
  if (tiles && ntiles > 0) {
    const std::string key = "gemm_f32:P:m=" + std::to_string(max_m) + ":n=" + std::to_string(max_n) +
                            ":batch=" + std::to_string(batch);
    v = tune_lookup(key);
    if (v < 0 && beta == 0.0) v = tune_pick(key, 2, run, s);
    if (v < 0) v = 0;
  }
  KScope kt(v == 1 ? "k_gemm128_f32_w8_persist:P" : "k_gemm128_f32_w8:P", s, 0.0, flops);
  run(v);
}

template <class DF>
static const char* gemm_name(bool tA, bool tB);
template <>
const char* gemm_name<DescArray>(bool tA, bool tB) {
  return tA ? (tB ? "k_gemm<DescArray,T,T>" : "k_gemm<DescArray,T,N>") : (tB ? "k_gemm<DescArray,N,T>" : "k_gemm<DescArray,N,N>");
}
template <>
const char* gemm_name<DescGather>(bool, bool tB) {
  return tB ? "k_gemm<DescGather,N,T>" : "k_gemm<DescGather,N,N>";
}
template <>
const char* gemm_name<CholUpdate>(bool, bool) { return "k_gemm<CholUpdate,N,T>"; }
template <>
const char* gemm_name<TrsmUpdate>(bool tA, bool) { return tA ? "k_gemm<TrsmUpdate,T,N>" : "k_gemm<TrsmUpdate,N,N>"; }
template <>
const char* gemm_name<Syr2kUpdate>(bool, bool) { return "k_gemm<Syr2kUpdate,N,T>"; }

// 128x128 tiles pay off for the long-k products with explicit descriptors;
// the k = 32/64 updates inside the factorisations keep 64x64 tiles unless
// default_tiles says otherwise (they accumulate into C, so they cannot be
// timed by repeated launches)
template <class DF>
static int default_tiles(int max_m) { return 0; }
template <>
int default_tiles<TrsmUpdate>(int max_m) { return max_m >= 128 ? 2 : 0; }
template <>
int default_tiles<CholUpdate>(int max_m) { return max_m >= 128 ? 2 : 0; }
template <>
int default_tiles<Syr2kUpdate>(int max_m) { return max_m >= 128 ? 2 : 0; }
template <class DF>
static bool use_big_tiles() { return false; }
template <>
bool use_big_tiles<DescArray>() { return true; }
template <>
bool use_big_tiles<DescGather>() { return true; }

template <class DF>
static void launch_tiles(DF df, int batch, int max_m, int max_n, bool tA, bool tB, double alpha, double beta,
                         bool lower, hipStream_t s, int variant) {
  if (variant >= 3 && !tA && !tB && !lower) {
    const dim3 grid(cdiv(max_m, 128), cdiv(max_n, 32), batch);
    if (variant == 3) hipLaunchKernelGGL((k_gemm_skinny<DF, 16>), grid, dim3(256), 0, s, df, alpha, beta);
    else if (variant == 4) hipLaunchKernelGGL((k_gemm_skinny<DF, 32>), grid, dim3(256), 0, s, df, alpha, beta);
    else hipLaunchKernelGGL((k_gemm_skinny_lds<DF>), grid, dim3(256), 0, s, df, alpha, beta);
    AWG_LAUNCH_CHECK();
    return;
  }
  if (variant >= 3) variant = 2;
  if (variant == 2) {
    dim3 grid(cdiv(max_m, 128), cdiv(max_n, 128), batch);
    if (!tA && !tB) hipLaunchKernelGGL((k_gemm128w8<DF, false, false>), grid, dim3(512), 0, s, df, alpha, beta, (int)lower);
    else if (tA && !tB) hipLaunchKernelGGL((k_gemm128w8<DF, true, false>), grid, dim3(512), 0, s, df, alpha, beta, (int)lower);
    else if (!tA && tB) hipLaunchKernelGGL((k_gemm128w8<DF, false, true>), grid, dim3(512), 0, s, df, alpha, beta, (int)lower);
    else hipLaunchKernelGGL((k_gemm128w8<DF, true, true>), grid, dim3(512), 0, s, df, alpha, beta, (int)lower);
    AWG_LAUNCH_CHECK();
    return;
  }
  const bool big = variant == 1;
  if (big) {
    dim3 grid(cdiv(max_m, 128), cdiv(max_n, 128), batch);
    if (!tA && !tB) hipLaunchKernelGGL((k_gemm128<DF, false, false>), grid, dim3(256), 0, s, df, alpha, beta, (int)lower);
    else if (tA && !tB) hipLaunchKernelGGL((k_gemm128<DF, true, false>), grid, dim3(256), 0, s, df, alpha, beta, (int)lower);
    else if (!tA && tB) hipLaunchKernelGGL((k_gemm128<DF, false, true>), grid, dim3(256), 0, s, df, alpha, beta, (int)lower);
    else hipLaunchKernelGGL((k_gemm128<DF, true, true>), grid, dim3(256), 0, s, df, alpha, beta, (int)lower);
    AWG_LAUNCH_CHECK();
    return;
  }
  dim3 grid(cdiv(max_m, 64), cdiv(max_n, 64), batch);
  if (!tA && !tB) hipLaunchKernelGGL((k_gemm<DF, false, false>), grid, dim3(256), 0, s, df, alpha, beta, (int)lower);
  else if (tA && !tB) hipLaunchKernelGGL((k_gemm<DF, true, false>), grid, dim3(256), 0, s, df, alpha, beta, (int)lower);
  else if (!tA && tB) hipLaunchKernelGGL((k_gemm<DF, false, true>), grid, dim3(256), 0, s, df, alpha, beta, (int)lower);
  else hipLaunchKernelGGL((k_gemm<DF, true, true>), grid, dim3(256), 0, s, df, alpha, beta, (int)lower);
  AWG_LAUNCH_CHECK();
}

// 64x64 or 128x128 output tiles.  Both kernels take the k loop in the same
// order with the same MFMA, so they give bit-identical results; for the
// explicit-descriptor products the faster one is measured per shape (tag =
// the call site) on the first call with beta = 0, otherwise 128x128 tiles
// when max_m >= 128.
template <class DF>
static void launch_gemm(DF df, int batch, int max_m, int max_n, bool tA, bool tB, double alpha, double beta,
                        bool lower, hipStream_t s, double flops = 0.0, const char* tag = nullptr) {
  if (batch <= 0 || max_m <= 0 || max_n <= 0) return;
  int variant = (use_big_tiles<DF>() && max_m >= 128) ? 1 : default_tiles<DF>(max_m);
  if (use_big_tiles<DF>() && tag) {
    const std::string key = std::string("gemm:") + tag + (gathers_a<DF>::value ? "g" : "") + (tA ? ":T" : ":N") +
                            (tB ? "T" : "N") + ":m=" +
                            std::to_string(max_m) + ":n=" + std::to_string(max_n) + ":batch=" + std::to_string(batch);
    int v = tune_lookup(key);
    // the skinny kernel is a candidate for untransposed products with N <= 64
    const int nvar = (!tA && !tB && max_n <= 64) ? 6 : 3;
    if (v < 0 && beta == 0.0 && !lower)
      v = tune_pick(key, nvar, [&](int w) { launch_tiles(df, batch, max_m, max_n, tA, tB, alpha, beta, lower, s, w); }, s);
    if (v >= 0) variant = v;
  }
  if (variant >= 3 && (tA || tB || lower)) variant = 2;
  static const char* const prefix[6] = {"k_gemm",        "k_gemm128",       "k_gemm128w8",
                                        "k_gemm_skinny", "k_gemm_skinny32", "k_gemm_skinny_lds"};
  std::string nm = std::string(prefix[variant]) + (gemm_name<DF>(tA, tB) + 6);
  if (tag) nm += std::string(":") + tag;
  KScope kt(nm.c_str(), s, 0.0, flops);
  launch_tiles(df, batch, max_m, max_n, tA, tB, alpha, beta, lower, s, variant);
}

void syr2k_panel_update(const MatDesc* d_mats, const double* V, const double* W, const long* d_off, int p0, int nbw,
                        int max_rem, int batch, hipStream_t s, double flops) {
  // only the lower triangle of the trailing matrix is read afterwards
  launch_gemm(Syr2kUpdate{d_mats, V, W, d_off, p0, nbw}, batch, max_rem, max_rem, false, true, -1.0, 1.0, true, s,
              0.25 * flops);
  launch_gemm(Syr2kUpdate{d_mats, W, V, d_off, p0, nbw}, batch, max_rem, max_rem, false, true, -1.0, 1.0, true, s,
              0.25 * flops);
}

void gemm_batched(const GemmDesc* d_desc, int batch, int max_m, int max_n, bool transA, bool transB,
                  double alpha, double beta, bool lower, hipStream_t s, double flops, const char* tag) {
  launch_gemm(DescArray{d_desc}, batch, max_m, max_n, transA, transB, alpha, beta, lower, s, flops, tag);
}

void gemm_batched_fixed(const GemmDesc* d_desc, const double* X, const int* idx, const long* off, int batch,
                        int max_m, int max_n, bool transA, bool transB, double alpha, double beta, hipStream_t s,
                        int variant) {
  if (batch <= 0 || max_m <= 0 || max_n <= 0) return;
  if (X)
    launch_tiles(DescGather{d_desc, X, idx, off}, batch, max_m, max_n, false, transB, alpha, beta, false, s, variant);
  else
    launch_tiles(DescArray{d_desc}, batch, max_m, max_n, transA, transB, alpha, beta, false, s, variant);
}

void gemm_batched_gather(const GemmDesc* d_desc, const double* X, const int* idx, const long* off, int batch,
                         int max_m, int max_n, bool transB, double alpha, double beta, hipStream_t s, double flops,
                         const char* tag) {
  launch_gemm(DescGather{d_desc, X, idx, off}, batch, max_m, max_n, false, transB, alpha, beta, false, s, flops, tag);
}

// ---------------------------------------------------------------------------
// GEMV (memory bound)
// ---------------------------------------------------------------------------
// notrans: y[i] = alpha sum_j A[i,j] x[j] + beta y[i]; 64 rows x 4 column
// groups per workgroup, partial sums combined in LDS (deterministic).
__global__ __launch_bounds__(256) void k_gemv_n(const GemmDesc* descs, double alpha, double beta) {
  const GemmDesc d = descs[blockIdx.y];
  const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + r;
  __shared__ double part[4][64];
  double acc = 0.0;
  if (i < d.m) {
    const double* a = d.A + i;
    double a0 = 0.0, a1 = 0.0;
    int j = g;
    for (; j + 4 < d.k; j += 8) {
      a0 += a[(long)j * d.lda] * d.B[j];
      a1 += a[(long)(j + 4) * d.lda] * d.B[j + 4];
    }
    for (; j < d.k; j += 4) a0 += a[(long)j * d.lda] * d.B[j];
    acc = a0 + a1;
  }
  part[g][r] = acc;
  __syncthreads();
  if (g == 0 && i < d.m) {
    const double v = alpha * ((part[0][r] + part[1][r]) + (part[2][r] + part[3][r]));
    d.C[i] = (beta == 0.0) ? v : v + beta * d.C[i];
  }
}

// trans: y[j] = alpha sum_i A[i,j] x[i] + beta y[j] with A stored k x m
// (op(A) = A^T is m x k, as for the GEMM); one wavefront per output.
__global__ __launch_bounds__(256) void k_gemv_t(const GemmDesc* descs, double alpha, double beta) {
  const GemmDesc d = descs[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= d.m) return;
  const double* a = d.A + (long)j * d.lda;
  double acc = 0.0;
  for (int i = lane; i < d.k; i += 64) acc += a[i] * d.B[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) {
    const double v = alpha * acc;
    d.C[j] = (beta == 0.0) ? v : v + beta * d.C[j];
  }
}

// notrans with few rows and a long k (single descriptor): the columns are
// split into GEMV_KSPLIT ranges whose partial sums are added in a fixed order
__global__ __launch_bounds__(256) void k_gemv_n_part(const GemmDesc* descs, double* part) {
  const GemmDesc d = descs[0];
  const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + r;
  const int ks = blockIdx.y;
  const int j0 = (int)((long)d.k * ks / GEMV_KSPLIT), j1 = (int)((long)d.k * (ks + 1) / GEMV_KSPLIT);
  __shared__ double sh[4][64];
  double acc = 0.0;
  if (i < d.m)
    for (int j = j0 + g; j < j1; j += 4) acc += d.A[i + (long)j * d.lda] * d.B[j];
  sh[g][r] = acc;
  __syncthreads();
  if (g == 0 && i < d.m) part[(long)ks * d.m + i] = (sh[0][r] + sh[1][r]) + (sh[2][r] + sh[3][r]);
}

__global__ void k_gemv_n_sum(const GemmDesc* descs, const double* part, double alpha, double beta) {
  const GemmDesc d = descs[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.m) return;
  double acc = 0.0;
  for (int ks = 0; ks < GEMV_KSPLIT; ++ks) acc += part[(long)ks * d.m + i];
  const double v = alpha * acc;
  d.C[i] = (beta == 0.0) ? v : v + beta * d.C[i];
}

void gemv_batched(const GemmDesc* d_desc, int batch, int max_m, int max_k, bool transA, double alpha,
                  double beta, hipStream_t s, double bytes, double* part) {
  if (batch <= 0) return;
  if (part && !transA && batch == 1 && max_m > 0 && max_k >= 16 * max_m) {
    KScope kt("k_gemv_n_part", s, bytes, bytes / 4.0);
    hipLaunchKernelGGL(k_gemv_n_part, dim3(cdiv(max_m, 64), GEMV_KSPLIT), dim3(256), 0, s, d_desc, part);
    AWG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gemv_n_sum, dim3(cdiv(max_m, 256)), dim3(256), 0, s, d_desc, part, alpha, beta);
    AWG_LAUNCH_CHECK();
    return;
  }
  KScope kt(transA ? "k_gemv_t" : "k_gemv_n", s, bytes, bytes / 4.0);
  if (!transA) {
    if (max_m <= 0) return;
    hipLaunchKernelGGL(k_gemv_n, dim3(cdiv(max_m, 64), batch), dim3(256), 0, s, d_desc, alpha, beta);
  } else {
    if (max_m <= 0 || max_k <= 0) return;
    hipLaunchKernelGGL(k_gemv_t, dim3(cdiv(max_m, 4), batch), dim3(256), 0, s, d_desc, alpha, beta);
  }
  AWG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Cholesky
// ---------------------------------------------------------------------------
constexpr int CHOL_NB = 32;

// factor the diagonal block A[j:j+jb, j:j+jb] in LDS
// With dropped != NULL (one matrix): a column whose Schur-complement pivot is
// <= tol times its original diagonal diag0 is numerically dependent on the
// previous ones; it is deleted (unit pivot, zero column) and flagged, so the
// factor of the kept columns is the Cholesky factor of their principal submatrix.
__global__ __launch_bounds__(256) void k_potf2(const MatDesc* mats, int j, int* info, const double* diag0,
                                               int* dropped, double tol, double* pivrel) {
  const MatDesc M = mats[blockIdx.x];
  const int jb = min(CHOL_NB, M.n - j);
  if (jb <= 0) return;
  __shared__ double L[CHOL_NB][CHOL_NB + 1];
  __shared__ int drop_c;
  const int tid = threadIdx.x;
  for (int e = tid; e < jb * jb; e += 256) {
    const int r = e % jb, c = e / jb;
    L[r][c] = M.A[(j + r) + (long)(j + c) * M.ld];
  }
  __syncthreads();
  for (int c = 0; c < jb; ++c) {
    if (tid == 0) {
      const double piv = L[c][c];
      drop_c = 0;
      if (pivrel) pivrel[j + c] = diag0[j + c] > 0.0 ? piv / diag0[j + c] : 0.0;
      if (dropped && piv == piv && !(piv > tol * diag0[j + c])) {
        dropped[j + c] = 1;
        drop_c = 1;
        L[c][c] = 1.0;
      } else if (!(piv > 0.0)) {
        if (info[blockIdx.x] == 0) info[blockIdx.x] = j + c + 1;
        L[c][c] = __builtin_nan("");
      } else {
        L[c][c] = sqrt(piv);
      }
    }
    __syncthreads();
    const double dc = L[c][c];
    for (int r = c + 1 + tid; r < jb; r += 256) L[r][c] = drop_c ? 0.0 : L[r][c] / dc;
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
    if (r >= c) M.A[(j + r) + (long)(j + c) * M.ld] = L[r][c];
  }
}

// rows below the diagonal block: X L_jj^T = A[j+jb:, j:j+jb]
__global__ __launch_bounds__(256) void k_chol_panel(const MatDesc* mats, int j, const int* dropped) {
  const MatDesc M = mats[blockIdx.y];
  const int jb = min(CHOL_NB, M.n - j);
  if (jb <= 0) return;
  __shared__ double L[CHOL_NB][CHOL_NB + 1];
  for (int e = threadIdx.x; e < jb * jb; e += 256) {
    const int r = e % jb, c = e / jb;
    L[r][c] = (r >= c) ? M.A[(j + r) + (long)(j + c) * M.ld] : 0.0;
  }
  __syncthreads();
  const int i = j + jb + blockIdx.x * 256 + threadIdx.x;
  if (i >= M.n) return;
  double x[CHOL_NB];
#pragma unroll
  for (int c = 0; c < CHOL_NB; ++c) {
    if (c < jb) {
      double v = M.A[i + (long)(j + c) * M.ld];
      for (int t = 0; t < c; ++t) v -= x[t] * L[c][t];
      x[c] = (dropped && dropped[j + c]) ? 0.0 : v / L[c][c];
    }
  }
#pragma unroll
  for (int c = 0; c < CHOL_NB; ++c)
    if (c < jb) M.A[i + (long)(j + c) * M.ld] = x[c];
}

// the blocked loop shared by potrf_batched and potrf_uniform: batch blocks,
// the largest of order maxn; sizes (host, may be NULL = every block of order
// maxn) only feed the kernel timer's flop count
static void potrf_loop(const MatDesc* d_mats, int batch, int maxn, const int* sizes, int* d_info, hipStream_t s,
                       const double* diag0, int* dropped, double tol, double* pivrel) {
  if (batch == 0) return;
  for (int j = 0; j < maxn; j += CHOL_NB) {
    hipLaunchKernelGGL(k_potf2, dim3(batch), dim3(256), 0, s, d_mats, j, d_info, diag0, dropped, tol, pivrel);
    AWG_LAUNCH_CHECK();
    const int rem = maxn - j - CHOL_NB;
    if (rem <= 0) break;
    hipLaunchKernelGGL(k_chol_panel, dim3(cdiv(rem, 256), batch), dim3(256), 0, s, d_mats, j,
                       (const int*)dropped);
    AWG_LAUNCH_CHECK();
    double fl = 0.0;
    if (ktimer_on())
      for (int b = 0; b < batch; ++b) {
        const double r = (sizes ? sizes[b] : maxn) - j - CHOL_NB;
        if (r > 0) fl += r * r * CHOL_NB;      // lower triangle of the rank-32 update
      }
    launch_gemm(CholUpdate{d_mats, j, CHOL_NB}, batch, rem, rem, false, true, -1.0, 1.0, true, s, fl);
  }
}

void potrf_batched(const MatDesc* d_mats, const std::vector<int>& h_n, int* d_info, hipStream_t s,
                   GemmDesc* /*unused*/, const double* diag0, int* dropped, double tol, double* pivrel) {
  int maxn = 0;
  for (int v : h_n) maxn = v > maxn ? v : maxn;
  potrf_loop(d_mats, (int)h_n.size(), maxn, h_n.data(), d_info, s, diag0, dropped, tol, pivrel);
}

void potrf_uniform(const MatDesc* d_mats, int batch, int n, int* d_info, hipStream_t s) {
  potrf_loop(d_mats, batch, n, nullptr, d_info, s, nullptr, nullptr, 0.0, nullptr);
}

// ---------------------------------------------------------------------------
// triangular solves with many right-hand sides
// ---------------------------------------------------------------------------
constexpr int TRSM_NB = 64;

// Solve the diagonal block: forward  X_j = L_jj^{-1} B_j
//                           backward X_j = L_jj^{-T} B_j
// one wavefront per 64 right-hand sides; L_jj and the B tile live in LDS.
// 64-row diagonal block of a blocked triangular solve for 64 right-hand
// sides: the 256 threads load L and X into LDS together (16 independent
// loads each), the first wavefront substitutes (one column per lane), and all
// threads store
__global__ __launch_bounds__(256) void k_trsm_diag(const MatDesc* Ls, const MatDesc* Bs, int j, int backward) {
  const MatDesc l = Ls[blockIdx.y], b = Bs[blockIdx.y];
  const int jb = min(TRSM_NB, l.n - j);
  const int c0 = blockIdx.x * 64;
  if (jb <= 0 || c0 >= b.n) return;
  __shared__ double L[TRSM_NB][TRSM_NB + 1];
  __shared__ double X[TRSM_NB][TRSM_NB + 1];   // X[row][col]
  const int tid = threadIdx.x;
  const int nc = min(64, b.n - c0);
#pragma unroll
  for (int q = 0; q < TRSM_NB * TRSM_NB / 256; ++q) {
    const int e = tid + 256 * q, r = e & (TRSM_NB - 1), c = e / TRSM_NB;
    L[r][c] = (r < jb && c < jb && r >= c) ? l.A[(j + r) + (long)(j + c) * l.ld] : 0.0;
    X[r][c] = (r < jb && c < nc) ? b.A[(j + r) + (long)(c0 + c) * b.ld] : 0.0;
  }
  __syncthreads();
  if (tid < nc) {
    const int c = tid;
    if (!backward) {
      for (int r = 0; r < jb; ++r) {
        double v = X[r][c];
        for (int t = 0; t < r; ++t) v -= L[r][t] * X[t][c];
        X[r][c] = v / L[r][r];
      }
    } else {
      for (int r = jb - 1; r >= 0; --r) {
        double v = X[r][c];
        for (int t = r + 1; t < jb; ++t) v -= L[t][r] * X[t][c];
        X[r][c] = v / L[r][r];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < TRSM_NB * TRSM_NB / 256; ++q) {
    const int e = tid + 256 * q, r = e & (TRSM_NB - 1), c = e / TRSM_NB;
    if (r < jb && c < nc) b.A[(j + r) + (long)(c0 + c) * b.ld] = X[r][c];
  }
}

void trsm_batched(const MatDesc* d_L, const MatDesc* d_B, const std::vector<int>& h_n,
                  const std::vector<int>& h_ncols, bool trans, hipStream_t s, GemmDesc* /*unused*/) {
  const int batch = (int)h_n.size();
  if (batch == 0) return;
  int maxn = 0, maxc = 0;
  for (size_t b = 0; b < h_n.size(); ++b) {
    maxn = h_n[b] > maxn ? h_n[b] : maxn;
    maxc = h_ncols[b] > maxc ? h_ncols[b] : maxc;
  }
  if (maxn == 0 || maxc == 0) return;
  const int nblk = cdiv(maxn, TRSM_NB);
  for (int t = 0; t < nblk; ++t) {
    const int blk = trans ? nblk - 1 - t : t;
    const int j = blk * TRSM_NB;
    hipLaunchKernelGGL(k_trsm_diag, dim3(cdiv(maxc, 64), batch), dim3(256), 0, s, d_L, d_B, j, (int)trans);
    AWG_LAUNCH_CHECK();
    const int mrows = trans ? j : maxn - j - TRSM_NB;
    double fl = 0.0;
    if (ktimer_on())
      for (size_t b = 0; b < h_n.size(); ++b) {
        const int jb = std::min(TRSM_NB, h_n[b] - j);
        if (jb <= 0) continue;
        const double m = trans ? j : h_n[b] - j - jb;
        fl += 2.0 * m * h_ncols[b] * jb;
      }
    if (mrows > 0)
      launch_gemm(TrsmUpdate{d_L, d_B, j, TRSM_NB, trans}, batch, mrows, maxc, trans, false, -1.0, 1.0, false, s,
                  fl);
  }
}

// ---------------------------------------------------------------------------
// sustained FP64 MFMA rate of the device: register-only chains of
// v_mfma_f64_16x16x4 (8 independent accumulators per wavefront, 8 wavefronts
// per SIMD on every CU), no memory traffic inside the loop
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mfma_probe(double* out, int iters, double a0, double b0) {
  v4d acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = (v4d){0.0, 0.0, 0.0, 0.0};
  const double a = a0 + threadIdx.x * 1e-9, b = b0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[(long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

double probe_mfma_f64(int iters, hipStream_t s) {
  int dev = 0, ncu = 0;
  AWG_HIP(hipGetDevice(&dev));
  AWG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = 8 * ncu, threads = 256;
  DBuf<double> out;
  out.alloc((size_t)blocks * threads);
  hipEvent_t e0, e1;
  AWG_HIP(hipEventCreate(&e0));
  AWG_HIP(hipEventCreate(&e1));
  hipLaunchKernelGGL(k_mfma_probe, dim3(blocks), dim3(threads), 0, s, out.p, 64, 1.0, 1e-3);   // warm-up
  AWG_LAUNCH_CHECK();
  double best = 0.0;
  for (int r = 0; r < 3; ++r) {
    AWG_HIP(hipEventRecord(e0, s));
    hipLaunchKernelGGL(k_mfma_probe, dim3(blocks), dim3(threads), 0, s, out.p, iters, 1.0, 1e-3);
    AWG_LAUNCH_CHECK();
    AWG_HIP(hipEventRecord(e1, s));
    AWG_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    AWG_HIP(hipEventElapsedTime(&ms, e0, e1));
    const double flops = 2.0 * 16 * 16 * 4 * 8.0 * iters * ((double)blocks * threads / 64.0);
    best = std::max(best, flops / (ms * 1e-3) / 1e12);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

}  // namespace awg
