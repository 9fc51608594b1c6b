// Warm-start network for the iterative GenEO eigensolves: a per-dof
// perceptron (tanh hidden layers) trained on GenEO modes with the
// rotation-invariant subspace loss
//     g(P) = min_C ||T - P C||_F^2 + eps ||C||_F^2,  eps = ridge * n_s,
// normalised by ||T||_F^2, whose gradient is -2 (T - P C) C^T at the minimiser
// (variable projection, Golub and Pereyra 1973).  Training runs in FP32 (tiled
// GEMMs with deterministic split-K reductions, Adam of Kingma and Ba 2015);
// inference runs as one fused BF16-MFMA kernel with FP32 accumulation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "awg.h"
#include "awg_common.h"
#include "awg_mlp.h"
#include "awg_mlp_impl.h"

using awg::cdiv;
using awg::DBuf;
using awg::Error;

namespace awg {
namespace {

// ---------------------------------------------------------------------------
// parameters
// ---------------------------------------------------------------------------
__device__ inline uint64_t mix64(uint64_t z) {   // splitmix64 finaliser (Steele, Lea, Flood 2014)
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Glorot-uniform weights U(-a, a), a = sqrt(6 / (fan_in + fan_out)); zero biases
__global__ void k_init_layer(float* W, long nw, float* b, int nb, float a, uint64_t key) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nw; e += (long)gridDim.x * blockDim.x) {
    const uint64_t r = mix64(key ^ (uint64_t)e * 0xD1B54A32D192ED03ull);
    W[e] = (float)((2.0 * ((double)(r >> 11) * 0x1.0p-53) - 1.0) * a);
  }
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nb; e += (long)gridDim.x * blockDim.x) b[e] = 0.f;
}

__device__ inline uint16_t f2bf(float x) {   // round to nearest even
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ void k_to_bf16(long n, const float* x, uint16_t* y) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    y[e] = f2bf(x[e]);
}

// ---------------------------------------------------------------------------
// FP32 GEMM (row-major): C = op(A) op(B), op(A) M x K, op(B) K x N.
// op(A)[i][k] = TA ? A[k*lda + i] : A[i*lda + k]
// op(B)[k][j] = TB ? B[j*ldb + k] : B[k*ldb + j]
// blockIdx.z splits K into chunks of klen; chunk z writes C + z * M * ldc.
// ---------------------------------------------------------------------------
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_sgemm(int M, int N, int K, const float* A, int lda, const float* B, int ldb,
                                               float* C, int ldc, int klen) {
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int kb = blockIdx.z * klen;
  const int ke = min(K, kb + klen);
  C += (long)blockIdx.z * M * ldc;
  __shared__ float As[16][68];
  __shared__ float Bs[16][68];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
  for (int k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * 256;
      int i, kk;
      if (TA) { kk = e >> 6; i = e & 63; } else { i = e >> 4; kk = e & 15; }
      const int gi = m0 + i, gk = k0 + kk;
      float v = 0.f;
      if (gi < M && gk < ke) v = TA ? A[(long)gk * lda + gi] : A[(long)gi * lda + gk];
      As[kk][i] = v;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * 256;
      int j, kk;
      if (TB) { j = e >> 4; kk = e & 15; } else { kk = e >> 6; j = e & 63; }
      const int gj = n0 + j, gk = k0 + kk;
      float v = 0.f;
      if (gj < N && gk < ke) v = TB ? B[(long)gj * ldb + gk] : B[(long)gk * ldb + gj];
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[t] = As[kk][ty * 4 + t];
        b[t] = Bs[kk][tx * 4 + t];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fmaf(a[x], b[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int i = m0 + ty * 4 + x;
    if (i >= M) continue;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int j = n0 + tx * 4 + y;
      if (j < N) C[(long)i * ldc + j] = acc[x][y];
    }
  }
}

// returns the number of K chunks (partial products written)
template <bool TA, bool TB>
int sgemm(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc, int splits,
          hipStream_t s) {
  if (M <= 0 || N <= 0) return 0;
  const int klen = std::max(16, (int)(cdiv(std::max(K, 1), splits * 16) * 16));
  const int nz = std::max(1, (int)cdiv(std::max(K, 1), klen));
  hipLaunchKernelGGL((k_sgemm<TA, TB>), dim3(cdiv(M, 64), cdiv(N, 64), nz), dim3(256), 0, s, M, N, K, A, lda, B,
                     ldb, C, ldc, klen);
  AWG_LAUNCH_CHECK();
  return nz;
}

// Z[i][j] += b[j], then tanh when act
__global__ void k_bias_act(long M, int N, float* Z, const float* b, int act) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < M * N; e += (long)gridDim.x * blockDim.x) {
    const float v = Z[e] + b[e % N];
    Z[e] = act ? tanhf(v) : v;
  }
}

// dH[i][j] *= 1 - H[i][j]^2 (derivative of tanh at its output)
__global__ void k_dtanh(long n, float* dH, const float* H) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    dH[e] *= 1.f - H[e] * H[e];
}

// out[j] = sum_i Z[i][j] in a fixed order (64 columns per block)
__global__ __launch_bounds__(256) void k_colsum(long M, int N, const float* Z, float* out) {
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), r = threadIdx.x >> 6;
  __shared__ float sh[4][64];
  float acc = 0.f;
  if (c < N)
    for (long i = r; i < M; i += 4) acc += Z[i * N + c];
  sh[r][threadIdx.x & 63] = acc;
  __syncthreads();
  if (r == 0 && c < N) out[c] = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}

// out[e] = sum_z part[z * cnt + e] in z order
__global__ void k_sum_parts(int nz, long cnt, const float* part, float* out) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (long)gridDim.x * blockDim.x) {
    float a = 0.f;
    for (int z = 0; z < nz; ++z) a += part[(long)z * cnt + e];
    out[e] = a;
  }
}

// Adam (Kingma and Ba, ICLR 2015) with bias correction
__global__ void k_adam(long n, float* w, const float* g, float* m1, float* m2, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const float gr = g[e];
    const float a = b1 * m1[e] + (1.f - b1) * gr;
    const float v = b2 * m2[e] + (1.f - b2) * gr * gr;
    m1[e] = a;
    m2[e] = v;
    w[e] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
  }
}

// Subspace loss of subdomain s (one block of 256 threads); FP64 accumulation.
// O: rows x p (row-major), T_s: n_s x m_s column-major at tgt_off[s].
// Writes dO rows of s (zero when m_s = 0) scaled by 1 / cnt and loss_s[s].
__global__ __launch_bounds__(256) void k_subspace_loss(const long* row_ptr, const long* tgt_off, const int* tgt_cols,
                                                       const float* O, int p, const float* T, double ridge,
                                                       double inv_cnt, float* dO, float* loss_s) {
  const int s = blockIdx.x;
  const long r0 = row_ptr[s], ns = row_ptr[s + 1] - r0;
  const int m = tgt_cols[s];
  const float* Ts = T + tgt_off[s];
  const int tid = threadIdx.x;
  if (m == 0) {
    for (long e = tid; e < ns * p; e += 256) dO[r0 * p + e] = 0.f;
    if (tid == 0) loss_s[s] = 0.f;
    return;
  }
  __shared__ double Pc[64][MLP_MAX_OUT + 1];
  __shared__ double Tc[64][MLP_MAX_OUT + 1];
  __shared__ double G[MLP_MAX_OUT][MLP_MAX_OUT + 1];
  __shared__ double Bm[MLP_MAX_OUT][MLP_MAX_OUT + 1];
  __shared__ double Cm[MLP_MAX_OUT][MLP_MAX_OUT + 1];
  __shared__ double red[4];
  __shared__ double tts, cc;
  const int ng = p * (p + 1) / 2, nb = p * m, npair = ng + nb + 1;
  double acc0 = 0.0, acc1 = 0.0;
  // pair t: t < ng -> G(a, b), a <= b; t < ng + nb -> Bm(a, j); else ||T||^2
  auto pair_of = [&](int t, int& kind, int& a, int& b) {
    if (t < ng) {
      kind = 0;
      int rem = t, aa = 0;
      while (rem >= p - aa) { rem -= p - aa; ++aa; }
      a = aa;
      b = aa + rem;
    } else if (t < ng + nb) {
      kind = 1;
      a = (t - ng) / m;
      b = (t - ng) % m;
    } else {
      kind = 2;
      a = b = 0;
    }
  };
  for (long c0 = 0; c0 < ns; c0 += 64) {
    const int nr = (int)min(64L, ns - c0);
    for (int e = tid; e < 64 * p; e += 256) {
      const int i = e / p, a = e % p;
      Pc[i][a] = i < nr ? (double)O[(r0 + c0 + i) * p + a] : 0.0;
    }
    for (int e = tid; e < 64 * m; e += 256) {
      const int i = e % 64, j = e / 64;
      Tc[i][j] = i < nr ? (double)Ts[c0 + i + (long)j * ns] : 0.0;
    }
    __syncthreads();
    for (int h = 0; h < 2; ++h) {
      const int t = tid + 256 * h;
      if (t >= npair) continue;
      int kind, a, b;
      pair_of(t, kind, a, b);
      double v = 0.0;
      for (int i = 0; i < nr; ++i) {
        if (kind == 0) v += Pc[i][a] * Pc[i][b];
        else if (kind == 1) v += Pc[i][a] * Tc[i][b];
        else
          for (int j = 0; j < m; ++j) v += Tc[i][j] * Tc[i][j];
      }
      if (h == 0) acc0 += v; else acc1 += v;
    }
    __syncthreads();
  }
  const double eps = ridge * (double)ns;
  for (int h = 0; h < 2; ++h) {
    const int t = tid + 256 * h;
    if (t >= npair) continue;
    int kind, a, b;
    pair_of(t, kind, a, b);
    const double v = h == 0 ? acc0 : acc1;
    if (kind == 0) {
      G[a][b] = v + (a == b ? eps : 0.0);
      G[b][a] = v + (a == b ? eps : 0.0);
    } else if (kind == 1) {
      Bm[a][b] = v;
    } else {
      tts = v;
    }
  }
  __syncthreads();
  if (tid == 0) {
    // Cholesky G = L L^T (lower, in place), then C = G^-1 Bm, ||C||^2
    for (int j = 0; j < p; ++j) {
      double d = G[j][j];
      for (int k = 0; k < j; ++k) d -= G[j][k] * G[j][k];
      d = sqrt(fmax(d, 1e-300));
      G[j][j] = d;
      for (int i = j + 1; i < p; ++i) {
        double v = G[i][j];
        for (int k = 0; k < j; ++k) v -= G[i][k] * G[j][k];
        G[i][j] = v / d;
      }
    }
    double c2 = 0.0;
    for (int j = 0; j < m; ++j) {
      double y[MLP_MAX_OUT];
      for (int i = 0; i < p; ++i) {
        double v = Bm[i][j];
        for (int k = 0; k < i; ++k) v -= G[i][k] * y[k];
        y[i] = v / G[i][i];
      }
      for (int i = p - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < p; ++k) v -= G[k][i] * Cm[k][j];
        Cm[i][j] = v / G[i][i];
        c2 += Cm[i][j] * Cm[i][j];
      }
    }
    cc = c2;
  }
  __syncthreads();
  const double tt = tts;
  const double sc = -2.0 * inv_cnt / tt;
  double rr = 0.0;
  for (long i = tid; i < ns; i += 256) {
    double Pr[MLP_MAX_OUT], Rr[MLP_MAX_OUT];
    for (int a = 0; a < p; ++a) Pr[a] = (double)O[(r0 + i) * p + a];
    for (int j = 0; j < m; ++j) {
      double v = (double)Ts[i + (long)j * ns];
      for (int a = 0; a < p; ++a) v -= Pr[a] * Cm[a][j];
      Rr[j] = v;
      rr += v * v;
    }
    for (int a = 0; a < p; ++a) {
      double v = 0.0;
      for (int j = 0; j < m; ++j) v += Rr[j] * Cm[a][j];
      dO[(r0 + i) * p + a] = (float)(sc * v);
    }
  }
  // block reduction of rr
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) rr += __shfl_xor(rr, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = rr;
  __syncthreads();
  if (tid == 0) loss_s[s] = (float)(((red[0] + red[1]) + (red[2] + red[3]) + eps * cc) / tt);
}

// ---------------------------------------------------------------------------
// fused BF16 inference: one block (4 wavefronts) per 64 rows; activations in
// LDS as bf16, weights read as bf16 (L2-resident), FP32 accumulation with
// v_mfma_f32_16x16x16_bf16.  Operand layout of that instruction for a 16x16x16
// product (checked on gfx950): lane l holds A[l%16][4*(l/16) + 0..3] and
// B[4*(l/16) + 0..3][l%16]; accumulator register r of lane l is
// D[4*(l/16) + r][l%16].
// ---------------------------------------------------------------------------
typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int INF_ROWS = 64;
constexpr int INF_LD = MLP_MAX_WIDTH + 8;   // bf16 row pitch in LDS

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// one layer: Hout (64 x N) = act(Hin (64 x K) W^T + b); K multiple of 16,
// N multiple of 16 (weights beyond dims read as zero)
__device__ void infer_layer(const uint16_t* __restrict__ Wb, const float* __restrict__ b, int Kreal, int Kpad,
                            int Nreal, int Npad, const uint16_t (*Hin)[INF_LD], uint16_t (*Hout)[INF_LD],
                            float* out, long row0, long rows, int ldo, bool last) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rt = wave;                       // row tile of this wave (16 rows)
  const int li = lane & 15, lk = (lane >> 4) * 4;
  for (int n0 = 0; n0 < Npad; n0 += 16) {
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    const int wrow = n0 + li;               // output column held by this lane's B operand
    for (int k0 = 0; k0 < Kpad; k0 += 16) {
      v4s a, bb;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[t] = (short)Hin[rt * 16 + li][k0 + lk + t];
        const int kk = k0 + lk + t;
        bb[t] = (wrow < Nreal && kk < Kreal) ? (short)Wb[(long)wrow * Kreal + kk] : (short)0;
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc, 0, 0, 0);
    }
    const int col = n0 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rt * 16 + lk + r;
      float v = acc[r] + (col < Nreal ? b[col] : 0.f);
      if (!last) {
        Hout[row][col] = col < Nreal ? f2bf(tanhf(v)) : (uint16_t)0;
      } else if (col < Nreal && row0 + row < rows) {
        out[(row0 + row) * ldo + col] = v;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_mlp_infer_bf16(long rows, const float* X, int F, int Fpad,
                                                        const uint16_t* Wb, const float* W, const long* offW,
                                                        const long* offB, const int* dims, int L, float* Y) {
  __shared__ uint16_t H0[INF_ROWS][INF_LD];
  __shared__ uint16_t H1[INF_ROWS][INF_LD];
  const long row0 = (long)blockIdx.x * INF_ROWS;
  for (int e = threadIdx.x; e < INF_ROWS * Fpad; e += 256) {
    const int i = e / Fpad, k = e % Fpad;
    const long gi = row0 + i;
    H0[i][k] = (k < F && gi < rows) ? f2bf(X[gi * F + k]) : (uint16_t)0;
  }
  __syncthreads();
  uint16_t(*hin)[INF_LD] = H0;
  uint16_t(*hout)[INF_LD] = H1;
  for (int l = 1; l <= L; ++l) {
    const int K = dims[l - 1], N = dims[l];
    const int Kpad = (l == 1) ? Fpad : ((K + 15) & ~15);
    const int Npad = (N + 15) & ~15;
    infer_layer(Wb + offW[l - 1], W + offB[l - 1], K, Kpad, N, Npad, hin, hout, Y, row0, rows, dims[L], l == L);
    __syncthreads();
    uint16_t(*t)[INF_LD] = hin;
    hin = hout;
    hout = t;
  }
}

// ---------------------------------------------------------------------------
// features of the (subdomain, local dof) rows
// ---------------------------------------------------------------------------
__device__ inline int find_local(const int* inv_ptr, const int* inv_sub, const int* inv_loc, int j, int s) {
  int lo = inv_ptr[j], hi = inv_ptr[j + 1] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int v = inv_sub[mid];
    if (v == s) return inv_loc[mid];
    if (v < s) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

__global__ void k_diag_log(int n, const int* rowptr, const int* col, const double* val, double* ld) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e)
    if (col[e] == i) d = val[e];
  ld[i] = log10(fmax(fabs(d), 1e-300));
}

// per subdomain: mean log10 A_ii, mean log10 P_ii, coordinate box; one block each
__global__ __launch_bounds__(256) void k_feat_stats(const long* sub_ptr, const int* sub_idx, const double* ldiag,
                                                    const double* P, const long* sq_off, const double* coords,
                                                    int cdim, double* st) {
  const int s = blockIdx.x;
  const long b0 = sub_ptr[s], ns = sub_ptr[s + 1] - b0;
  __shared__ double sh[256];
  double v[8];
  v[0] = 0.0;
  v[1] = 0.0;
  for (int d = 0; d < 3; ++d) {
    v[2 + 2 * d] = 1e300;
    v[3 + 2 * d] = -1e300;
  }
  for (long i = threadIdx.x; i < ns; i += 256) {
    const int g = sub_idx[b0 + i];
    v[0] += ldiag[g];
    v[1] += log10(fmax(fabs(P[sq_off[s] + i + i * ns]), 1e-300));
    for (int d = 0; d < 3 && d < cdim; ++d) {
      const double x = coords[(long)g * cdim + d];
      v[2 + 2 * d] = fmin(v[2 + 2 * d], x);
      v[3 + 2 * d] = fmax(v[3 + 2 * d], x);
    }
  }
  for (int q = 0; q < 8; ++q) {
    sh[threadIdx.x] = v[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        const double a = sh[threadIdx.x], b = sh[threadIdx.x + w];
        sh[threadIdx.x] = q < 2 ? a + b : ((q & 1) == 0 ? fmin(a, b) : fmax(a, b));
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) st[s * 8 + q] = q < 2 ? sh[0] / (double)ns : sh[0];
    __syncthreads();
  }
}

// depth: 0 for a dof with a graph neighbour outside the subdomain, else min
// over in-subdomain neighbours + 1 (capped at 4); one sweep per launch
__global__ void k_depth(int N, const long* sub_ptr, const int* sub_idx, const int* ent_sub, long tot,
                        const int* rowptr, const int* col, const int* inv_ptr, const int* inv_sub,
                        const int* inv_loc, const float* din, float* dout, int first) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= tot) return;
  const int s = ent_sub[e];
  const int g = sub_idx[e];
  float best = first ? 4.f : din[e];
  for (int k = rowptr[g]; k < rowptr[g + 1]; ++k) {
    const int j = col[k];
    if (j == g) continue;
    const int lj = find_local(inv_ptr, inv_sub, inv_loc, j, s);
    if (lj < 0) {
      best = 0.f;
      break;
    }
    if (!first) best = fminf(best, din[sub_ptr[s] + lj] + 1.f);
  }
  dout[e] = fminf(best, 4.f);
}

__global__ void k_features(long tot, const long* sub_ptr, const int* sub_idx, const int* ent_sub, const int* rowptr,
                           const int* col, const double* val, const double* ldiag, double gmean, const int* mult,
                           const double* V, const long* v_eoff, const long* v_coff, const double* P,
                           const long* sq_off, const double* coords, int cdim, const double* st, const float* depth,
                           float* out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= tot) return;
  const int s = ent_sub[e];
  const long i = e - sub_ptr[s];
  const long ns = sub_ptr[s + 1] - sub_ptr[s];
  const int g = sub_idx[e];
  const double* S = st + s * 8;
  float f[MLP_FEATURES];
  for (int d = 0; d < 3; ++d) {
    double x = 0.0;
    if (coords && d < cdim) {
      const double lo = S[2 + 2 * d], hi = S[3 + 2 * d];
      x = hi > lo ? 2.0 * (coords[(long)g * cdim + d] - lo) / (hi - lo) - 1.0 : 0.0;
    }
    f[d] = (float)x;
  }
  const double li = ldiag[g];
  f[3] = (float)((li - S[0]) * 0.25);
  f[4] = (float)((li - gmean) * 0.25);
  double mx = li, mn = li, cs = 0.0;
  int cnt = 0;
  for (int k = rowptr[g]; k < rowptr[g + 1]; ++k) {
    const int j = col[k];
    if (j == g) continue;
    mx = fmax(mx, ldiag[j]);
    mn = fmin(mn, ldiag[j]);
    cs += log10(fmax(fabs(val[k]), 1e-300));
    ++cnt;
  }
  f[5] = (float)((mx - li) * 0.25);
  f[6] = (float)((mn - li) * 0.25);
  f[7] = (float)(cnt ? (cs / cnt - li) * 0.25 : 0.0);
  f[8] = (float)(1.0 / mult[g]);
  f[9] = depth[e] * 0.25f;
  const long k = v_coff[s + 1] - v_coff[s];
  double lev = 0.0;
  const double dwi = 1.0 / mult[g];
  for (long c = 0; c < k; ++c) {
    const double v = V[v_eoff[s] + i + c * ns] * dwi;
    lev += v * v;
  }
  f[10] = (float)(k ? lev * (double)ns / (double)k : 0.0);
  f[11] = (float)((log10(fmax(fabs(P[sq_off[s] + i + i * ns]), 1e-300)) - S[1]) * 0.25);
  for (int q = 0; q < MLP_FEATURES; ++q) out[e * MLP_FEATURES + q] = f[q];
}

__global__ __launch_bounds__(256) void k_mean(int n, const double* x, double* out) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += x[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0] / (double)n;
}

__global__ void k_block_from_rows(const long* sub_ptr, int q, int p, const float* O, double* X) {
  const int s = blockIdx.x;
  const long b0 = sub_ptr[s], ns = sub_ptr[s + 1] - b0;
  __shared__ double sh[256];
  for (int j = 0; j < p; ++j) {
    double a = 0.0;
    for (long i = threadIdx.x; i < ns; i += 256) {
      const double v = O[(b0 + i) * p + j];
      a += v * v;
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    const double inv = sh[0] > 0.0 ? 1.0 / sqrt(sh[0]) : 0.0;
    __syncthreads();
    for (long i = threadIdx.x; i < ns; i += 256) X[b0 * q + (long)j * ns + i] = O[(b0 + i) * p + j] * inv;
  }
}

__global__ void k_ent_sub(int N, const long* sub_ptr, int* ent) {
  const int s = blockIdx.y;
  for (long e = sub_ptr[s] + (long)blockIdx.x * blockDim.x + threadIdx.x; e < sub_ptr[s + 1];
       e += (long)gridDim.x * blockDim.x)
    ent[e] = s;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void mlp_forward(awg_mlp& m, long rows, const float* X, float* Y, bool bf16, hipStream_t s) {
  if (rows <= 0) return;
  const int L = (int)m.dims.size() - 1;
  if (bf16) {
    if (!m.wb_valid) {
      hipLaunchKernelGGL(k_to_bf16, dim3(std::min(4096u, cdiv(m.nparams, 256))), dim3(256), 0, s, m.nparams, m.w.p,
                         m.wb.p);
      AWG_LAUNCH_CHECK();
      m.wb_valid = true;
    }
    DBuf<long> dW, dB;
    DBuf<int> dd;
    dW.upload(m.offW, s);
    dB.upload(m.offB, s);
    dd.upload(m.dims, s);
    const int F = m.dims[0];
    KScope kt("k_mlp_infer_bf16", s, 4.0 * rows * (F + m.dims[L]) + 2.0 * m.nparams, 0.0);
    hipLaunchKernelGGL(k_mlp_infer_bf16, dim3(cdiv(rows, INF_ROWS)), dim3(256), 0, s, rows, X, F, (F + 15) & ~15,
                       m.wb.p, m.w.p, dW.p, dB.p, dd.p, L, Y);
    AWG_LAUNCH_CHECK();
    AWG_HIP(hipStreamSynchronize(s));   // the descriptor buffers die here
    return;
  }
  // FP32: layer by layer through two ping-pong buffers
  DBuf<float> h0, h1;
  const int W = m.dims[1];
  h0.alloc((size_t)rows * W);
  h1.alloc((size_t)rows * W);
  const float* in = X;
  for (int l = 1; l <= L; ++l) {
    const int K = m.dims[l - 1], N = m.dims[l];
    float* out = (l == L) ? Y : ((l & 1) ? h0.p : h1.p);
    sgemm<false, true>((int)rows, N, K, in, K, m.w.p + m.offW[l - 1], K, out, N, 1, s);
    hipLaunchKernelGGL(k_bias_act, dim3(std::min(8192u, cdiv(rows * N, 256))), dim3(256), 0, s, rows, N, out,
                       m.w.p + m.offB[l - 1], (int)(l < L));
    AWG_LAUNCH_CHECK();
    in = out;
  }
  AWG_HIP(hipStreamSynchronize(s));
}

void l_mlp_features(int N, int n, int maxns, const long* sub_ptr, const int* sub_idx, const int* rowptr,
                    const int* col, const double* val, const int* inv_ptr, const int* inv_sub, const int* inv_loc,
                    const int* mult, const double* V, const long* v_eoff, const long* v_coff, const double* P,
                    const long* sq_off, const double* coords, int cdim, float* out, hipStream_t s) {
  long tot = 0;
  AWG_HIP(hipMemcpyAsync(&tot, sub_ptr + N, sizeof(long), hipMemcpyDeviceToHost, s));
  AWG_HIP(hipStreamSynchronize(s));
  DBuf<double> ldiag, st, gm;
  DBuf<int> ent;
  DBuf<float> d0, d1;
  ldiag.alloc(n);
  st.alloc((size_t)N * 8);
  gm.alloc(1);
  ent.alloc(tot);
  d0.alloc(tot);
  d1.alloc(tot);
  hipLaunchKernelGGL(k_diag_log, dim3(cdiv(n, 256)), dim3(256), 0, s, n, rowptr, col, val, ldiag.p);
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, s, n, ldiag.p, gm.p);
  hipLaunchKernelGGL(k_ent_sub, dim3(std::max(1u, std::min(64u, cdiv(maxns, 256))), N), dim3(256), 0, s, N, sub_ptr,
                     ent.p);
  hipLaunchKernelGGL(k_feat_stats, dim3(N), dim3(256), 0, s, sub_ptr, sub_idx, ldiag.p, P, sq_off, coords,
                     coords ? cdim : 0, st.p);
  AWG_LAUNCH_CHECK();
  float* a = d0.p;
  float* b = d1.p;
  for (int sweep = 0; sweep < 4; ++sweep) {
    hipLaunchKernelGGL(k_depth, dim3(cdiv(tot, 256)), dim3(256), 0, s, N, sub_ptr, sub_idx, ent.p, tot, rowptr, col,
                       inv_ptr, inv_sub, inv_loc, a, b, (int)(sweep == 0));
    AWG_LAUNCH_CHECK();
    std::swap(a, b);
  }
  double g = 0.0;
  AWG_HIP(hipMemcpyAsync(&g, gm.p, sizeof(double), hipMemcpyDeviceToHost, s));
  AWG_HIP(hipStreamSynchronize(s));
  hipLaunchKernelGGL(k_features, dim3(cdiv(tot, 256)), dim3(256), 0, s, tot, sub_ptr, sub_idx, ent.p, rowptr, col,
                     val, ldiag.p, g, mult, V, v_eoff, v_coff, P, sq_off, coords, coords ? cdim : 0, st.p, a, out);
  AWG_LAUNCH_CHECK();
  AWG_HIP(hipStreamSynchronize(s));
}

void l_block_from_rows(int N, int /*maxns*/, const long* sub_ptr, int q, int p, const float* O, double* X,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_block_from_rows, dim3(N), dim3(256), 0, s, sub_ptr, q, p, O, X);
  AWG_LAUNCH_CHECK();
}

}  // namespace awg

// ---------------------------------------------------------------------------
// C ABI (include/awg_mlp.h)
// ---------------------------------------------------------------------------
namespace {
std::string g_mlp_error = "no error";

int mlp_fail(awg_mlp* m, const Error& e) {
  if (m) m->err = e.what();
  g_mlp_error = e.what();
  return e.code;
}

void ensure_ws(awg_mlp& m, long rows) {
  if (rows <= m.ws_rows) return;
  const int L = (int)m.dims.size() - 1;
  const int W = m.dims[1];
  m.acts.alloc((size_t)rows * W * (L - 1) + (size_t)rows * m.dims[L]);
  m.dH0.alloc((size_t)rows * W);
  m.dH1.alloc((size_t)rows * W);
  m.ws_rows = rows;
}

constexpr int DW_SPLITS = 64;
}  // namespace

extern "C" {

int awg_mlp_create(awg_mlp** out, int32_t in_features, int32_t width, int32_t hidden_layers, int32_t out_channels,
                   uint64_t seed) {
  if (!out) return AWG_ERR_ARG;
  *out = nullptr;
  if (in_features < 1 || in_features > 32 || width < 16 || width > awg::MLP_MAX_WIDTH || width % 16 ||
      hidden_layers < 1 || hidden_layers > 8 || out_channels < 1 || out_channels > awg::MLP_MAX_OUT) {
    g_mlp_error = "awg_mlp_create: in_features 1..32, width 16..256 (multiple of 16), hidden_layers 1..8, "
                  "out_channels 1..16";
    return AWG_ERR_ARG;
  }
  auto* m = new awg_mlp();
  try {
    m->dims.push_back(in_features);
    for (int l = 0; l < hidden_layers; ++l) m->dims.push_back(width);
    m->dims.push_back(out_channels);
    const int L = (int)m->dims.size() - 1;
    long o = 0;
    for (int l = 1; l <= L; ++l) {
      m->offW.push_back(o);
      o += (long)m->dims[l] * m->dims[l - 1];
      m->offB.push_back(o);
      o += m->dims[l];
    }
    m->nparams = o;
    m->w.alloc(o);
    m->g.alloc(o);
    m->m1.alloc(o);
    m->m2.alloc(o);
    m->wb.alloc(o);
    m->loss_s.alloc(1);
    hipStream_t s = nullptr;
    for (int l = 1; l <= L; ++l) {
      const long nw = (long)m->dims[l] * m->dims[l - 1];
      const float a = (float)std::sqrt(6.0 / (m->dims[l] + m->dims[l - 1]));
      hipLaunchKernelGGL(awg::k_init_layer, dim3(std::min(1024u, cdiv(nw, 256))), dim3(256), 0, s,
                         m->w.p + m->offW[l - 1], nw, m->w.p + m->offB[l - 1], m->dims[l], a,
                         seed * 0x9E3779B97F4A7C15ull + (uint64_t)l);
      AWG_LAUNCH_CHECK();
    }
    m->g.zero(s);
    m->m1.zero(s);
    m->m2.zero(s);
    AWG_HIP(hipStreamSynchronize(s));
  } catch (const Error& e) {
    g_mlp_error = e.what();
    delete m;
    return e.code;
  }
  *out = m;
  return AWG_OK;
}

int64_t awg_mlp_num_params(const awg_mlp* m) { return m ? m->nparams : AWG_ERR_ARG; }

int awg_mlp_get_params(const awg_mlp* m, float* host, int64_t count) {
  if (!m || !host || count != m->nparams) return AWG_ERR_ARG;
  if (hipMemcpy(host, m->w.p, sizeof(float) * count, hipMemcpyDeviceToHost) != hipSuccess) return AWG_ERR_HIP;
  return AWG_OK;
}

int awg_mlp_get_grads(const awg_mlp* m, float* host, int64_t count) {
  if (!m || !host || count != m->nparams) return AWG_ERR_ARG;
  if (hipMemcpy(host, m->g.p, sizeof(float) * count, hipMemcpyDeviceToHost) != hipSuccess) return AWG_ERR_HIP;
  return AWG_OK;
}

int awg_mlp_set_params(awg_mlp* m, const float* host, int64_t count) {
  if (!m || !host || count != m->nparams) return AWG_ERR_ARG;
  if (hipMemcpy(m->w.p, host, sizeof(float) * count, hipMemcpyHostToDevice) != hipSuccess) return AWG_ERR_HIP;
  m->wb_valid = false;
  return AWG_OK;
}

int awg_mlp_forward(awg_mlp* m, int64_t rows, const float* X, float* Y, int32_t bf16, void* stream) {
  if (!m || rows < 0 || (rows > 0 && (!X || !Y))) return AWG_ERR_ARG;
  try {
    awg::mlp_forward(*m, rows, X, Y, bf16 != 0, (hipStream_t)stream);
  } catch (const Error& e) {
    return mlp_fail(m, e);
  }
  return AWG_OK;
}

int awg_mlp_loss_grad(awg_mlp* m, int64_t rows, const float* X, int32_t nsub, const int64_t* row_ptr,
                      const int64_t* tgt_off, const int32_t* tgt_cols, const float* T, double ridge,
                      double* loss_host, void* stream) {
  if (!m || rows <= 0 || nsub <= 0 || !X || !row_ptr || !tgt_off || !tgt_cols || !T || !(ridge >= 0.0))
    return AWG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  try {
    const int L = (int)m->dims.size() - 1;
    const int W = m->dims[1], p = m->dims[L];
    std::vector<int32_t> hc(nsub);
    std::vector<int64_t> hr(nsub + 1);
    AWG_HIP(hipMemcpyAsync(hc.data(), tgt_cols, sizeof(int32_t) * nsub, hipMemcpyDeviceToHost, s));
    AWG_HIP(hipMemcpyAsync(hr.data(), row_ptr, sizeof(int64_t) * (nsub + 1), hipMemcpyDeviceToHost, s));
    AWG_HIP(hipStreamSynchronize(s));
    if (hr[0] != 0 || hr[nsub] != rows) throw Error(AWG_ERR_ARG, "awg_mlp_loss_grad: row_ptr must run from 0 to rows");
    int cnt = 0;
    for (int t = 0; t < nsub; ++t) {
      if (hr[t + 1] < hr[t]) throw Error(AWG_ERR_ARG, "awg_mlp_loss_grad: decreasing row_ptr");
      if (hc[t] < 0 || hc[t] > awg::MLP_MAX_OUT) throw Error(AWG_ERR_ARG, "awg_mlp_loss_grad: 0..16 target columns");
      cnt += hc[t] > 0;
    }
    ensure_ws(*m, rows);
    DBuf<float> ls;
    ls.alloc(nsub);
    // forward, keeping h_1 .. h_{L-1} and the output
    std::vector<float*> h(L + 1);
    h[0] = const_cast<float*>(X);
    for (int l = 1; l <= L; ++l) h[l] = m->acts.p + (size_t)rows * W * (l - 1);
    for (int l = 1; l <= L; ++l) {
      const int K = m->dims[l - 1], N = m->dims[l];
      awg::sgemm<false, true>((int)rows, N, K, h[l - 1], K, m->w.p + m->offW[l - 1], K, h[l], N, 1, s);
      hipLaunchKernelGGL(awg::k_bias_act, dim3(std::min(8192u, cdiv(rows * N, 256))), dim3(256), 0, s, (long)rows, N,
                         h[l], m->w.p + m->offB[l - 1], (int)(l < L));
      AWG_LAUNCH_CHECK();
    }
    // loss and dL/dO
    float* d = m->dH0.p;
    hipLaunchKernelGGL(awg::k_subspace_loss, dim3(nsub), dim3(256), 0, s, row_ptr, tgt_off, tgt_cols, h[L], p, T,
                       ridge, cnt ? 1.0 / cnt : 0.0, d, ls.p);
    AWG_LAUNCH_CHECK();
    // backward
    const long maxcnt = (long)W * std::max(W, m->dims[0]);
    if ((long)m->part.n < DW_SPLITS * maxcnt) m->part.alloc(DW_SPLITS * maxcnt);
    float* dn = m->dH1.p;
    for (int l = L; l >= 1; --l) {
      const int K = m->dims[l - 1], N = m->dims[l];
      // dW_l = d^T h_{l-1}  (N x K), split over the rows
      const int nz = awg::sgemm<true, false>(N, K, (int)rows, d, N, h[l - 1], K, m->part.p, K, DW_SPLITS, s);
      hipLaunchKernelGGL(awg::k_sum_parts, dim3(std::min(1024u, cdiv((long)N * K, 256))), dim3(256), 0, s, nz,
                         (long)N * K, m->part.p, m->g.p + m->offW[l - 1]);
      hipLaunchKernelGGL(awg::k_colsum, dim3(cdiv(N, 64)), dim3(256), 0, s, (long)rows, N, d,
                         m->g.p + m->offB[l - 1]);
      AWG_LAUNCH_CHECK();
      if (l > 1) {
        // d_{l-1} = (d W_l) * (1 - h_{l-1}^2)
        awg::sgemm<false, false>((int)rows, K, N, d, N, m->w.p + m->offW[l - 1], K, dn, K, 1, s);
        hipLaunchKernelGGL(awg::k_dtanh, dim3(std::min(8192u, cdiv(rows * K, 256))), dim3(256), 0, s,
                           (long)rows * K, dn, h[l - 1]);
        AWG_LAUNCH_CHECK();
        std::swap(d, dn);
      }
    }
    if (loss_host) {
      std::vector<float> hl(nsub);
      AWG_HIP(hipMemcpyAsync(hl.data(), ls.p, sizeof(float) * nsub, hipMemcpyDeviceToHost, s));
      AWG_HIP(hipStreamSynchronize(s));
      double a = 0.0;
      for (int t = 0; t < nsub; ++t) a += hl[t];
      *loss_host = cnt ? a / cnt : 0.0;
    } else {
      AWG_HIP(hipStreamSynchronize(s));
    }
  } catch (const Error& e) {
    return mlp_fail(m, e);
  }
  return AWG_OK;
}

int awg_mlp_adam_step(awg_mlp* m, double lr, double beta1, double beta2, double eps, void* stream) {
  if (!m || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return AWG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  try {
    m->adam_t += 1;
    const float c1 = (float)(1.0 - std::pow(beta1, (double)m->adam_t));
    const float c2 = (float)(1.0 - std::pow(beta2, (double)m->adam_t));
    hipLaunchKernelGGL(awg::k_adam, dim3(std::min(4096u, cdiv(m->nparams, 256))), dim3(256), 0, s, m->nparams,
                       m->w.p, m->g.p, m->m1.p, m->m2.p, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2);
    AWG_LAUNCH_CHECK();
    AWG_HIP(hipStreamSynchronize(s));
    m->wb_valid = false;
  } catch (const Error& e) {
    return mlp_fail(m, e);
  }
  return AWG_OK;
}

const char* awg_mlp_last_error(const awg_mlp* m) { return m ? m->err.c_str() : g_mlp_error.c_str(); }

void awg_mlp_destroy(awg_mlp* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  delete m;
}

}  // extern "C"
