// Local products on split half-precision operands (FP16 matrix cores).
//
// The multi-column local product of the W solves, Os^s = Xs^s P^s summed over
// the subdomains (the H^NN term of H2, Definition of H^NN, Section 3.3), is
// the dominant dense contraction of the set-up.  Here both operands are
// scaled by powers of two (per subdomain for P^s, per column for the
// multi-vector) and split as x = hi + lo with hi = fp16(x) and
// lo = fp16(x - hi): 22 significant bits, close to FP32's 24.  The product
// takes the three terms hi.hi + hi.lo + lo.hi on the FP16 MFMA
// (v_mfma_f32_16x16x32_f16) with FP32 accumulation; the dropped lo.lo term
// is below 2^-22 of a product.  The power-of-two scalings are exact, and
// the result is scaled back and stored in FP64.
//
// Layouts (halves; one "entry" = 8 consecutive k of one row or column):
//   multi-vector operand  entry (g, i) at A + (g * m + i) * 8 (hi plane),
//                         A + plane + (g * m + i) * 8 (lo plane): the rows
//                         8g .. 8g+7 of subdomain s at column i;
//   matrix operand        entry (j, g) at B + (j * G + g) * 8 (and + plane):
//                         rows 8g .. 8g+7 of column j of P^s;
// rows past n_s hold zeros, so the k loop runs over whole groups of 8.
#include <string>

#include "awg_common.h"
#include "awg_tune.h"

namespace awg {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v4f_h3 __attribute__((ext_vector_type(4)));

// biased IEEE exponent of |x| (0 for zero and subnormals)
__device__ __forceinline__ int bexp(double x) {
  return (int)((__double_as_longlong(x) >> 52) & 0x7ff);
}

// scale exponent that maps a maximum of biased exponent e into [2^14, 2^15)
__device__ __forceinline__ int split_scale(int e) { return e ? 1023 + 14 - e : 0; }

__device__ __forceinline__ void split2(double x, _Float16& hi, _Float16& lo) {
  hi = (_Float16)x;
  lo = (_Float16)(x - (double)hi);
}

__global__ void k_fill_int(int n, int v, int* a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// emax[c] = max over the n rows of the biased exponent of X[i, c] (row-major
// n x b); every block takes a range of rows and 256 columns
__global__ __launch_bounds__(256) void k_colexp(int n, int b, const double* X, int rows_per_block, int* emax) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= b) return;
  const long r0 = (long)blockIdx.y * rows_per_block;
  const long r1 = min((long)n, r0 + rows_per_block);
  int e = 0;
  for (long r = r0; r < r1; ++r) e = max(e, bexp(X[r * b + c]));
  if (e) atomicMax(emax + c, e);
}

// split restriction: one thread per (row group, column); row group q holds
// the cnt[q] (1..8) rows sub_idx[row0[q] ..] of one subdomain, written as the
// entry (g, i) of that subdomain's operand (groups numbered consecutively
// over the subdomains, so the entry is at (q * b + i) * 8)
__global__ __launch_bounds__(256) void k_gather_h3(long ngroups, const int* row0, const int* cnt, const int* sub_idx,
                                                   const double* X, int b, const int* emax, _Float16* out,
                                                   long plane) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= ngroups * b) return;
  const long q = t / b;
  const int i = (int)(t - q * b);
  const int r0 = row0[q], nr = cnt[q];
  const int sc = split_scale(emax[i]);
  v8h hi, lo;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const double x = u < nr ? ldexp(X[(long)sub_idx[r0 + u] * b + i], sc) : 0.0;
    _Float16 h, l;
    split2(x, h, l);
    hi[u] = h;
    lo[u] = l;
  }
  *(v8h*)(out + t * 8) = hi;
  *(v8h*)(out + plane + t * 8) = lo;
}

// split local matrices: one block per subdomain; sp[s] = scale exponent of
// P^s (its largest entry mapped into [2^14, 2^15)), then the entries (j, g)
template <class T>
__global__ __launch_bounds__(256) void k_p16_build(const long* sqoff, const long* sub_ptr, const long* poff,
                                                   const T* P, _Float16* out, long plane, int* sp) {
  __shared__ int red[256];
  const int s = blockIdx.x;
  const int ns = (int)(sub_ptr[s + 1] - sub_ptr[s]);
  const int G = (ns + 7) / 8;
  const T* Ps = P + sqoff[s];
  int e = 0;
  for (long k = threadIdx.x; k < (long)ns * ns; k += 256) e = max(e, bexp((double)Ps[k]));
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  const int sc = split_scale(red[0]);
  if (threadIdx.x == 0) sp[s] = sc;
  _Float16* o = out + poff[s];
  for (long t = threadIdx.x; t < (long)ns * G; t += 256) {
    const int j = (int)(t / G), g = (int)(t - (long)j * G);
    v8h hi, lo;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = 8 * g + u;
      const double x = k < ns ? ldexp((double)Ps[k + (long)j * ns], sc) : 0.0;
      _Float16 h, l;
      split2(x, h, l);
      hi[u] = h;
      lo[u] = l;
    }
    *(v8h*)(o + t * 8) = hi;
    *(v8h*)(o + plane + t * 8) = lo;
  }
}

// C = (A B) 2^-(sx_i + sp_s) per batch entry: 128 x 128 tiles, four
// wavefronts of 64 x 64.  KG row groups (8 k each) per LDS stage: KG = 4 with
// two LDS buffers (the next stage's loads land in registers and are stored to
// the other buffer), KG = 8 with one buffer (stored after a barrier), which
// leaves twice the compute time to cover the loads' latency.  A staged entry
// row is PAD entries long, so that the KG row groups of one column written by
// consecutive lanes fall on distinct LDS banks.  Both forms issue the same
// MFMA sequence per output (bit-identical results).
template <int KG>
__global__ __launch_bounds__(256, 2) void k_gemm_h3(const GemmDescH3* descs, const int* emax, const int* sp) {
  constexpr int NBUF = KG == 4 ? 2 : 1;
  constexpr int PAD = KG == 4 ? 132 : 130;
  constexpr int NR = KG;   // 16-byte chunks per thread and operand: 2 planes x KG groups x 128 / 256
  const GemmDescH3 d = descs[blockIdx.z];
  const int m0 = blockIdx.x * 128, n0 = blockIdx.y * 128;
  if (m0 >= d.m || n0 >= d.n) return;
  __shared__ v8h As[2][NBUF][KG][PAD];   // [plane][buffer][row group][i]
  __shared__ v8h Bs[2][NBUF][KG][PAD];   // [plane][buffer][row group][j]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  v4f_h3 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (v4f_h3){0.f, 0.f, 0.f, 0.f};
  const v8h zero = (v8h){0, 0, 0, 0, 0, 0, 0, 0};
  v8h ra[NR], rb[NR];
  // chunk c = tid + 256 r, PL = 128 KG chunks per plane: A (plane c / PL,
  // group (c / 128) mod KG, i = c mod 128); B (plane c / PL, j = (c / KG) mod
  // 128, group c mod KG)
  constexpr int PL = 128 * KG;
  auto gload = [&](int g0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int c = tid + 256 * r;
      const int pl = c / PL;
      const int ga = g0 + (c / 128) % KG, i = m0 + (c & 127);
      ra[r] = (ga < d.G && i < d.m) ? *(const v8h*)(d.A + pl * d.planeA + ((long)ga * d.m + i) * 8) : zero;
      const int j = n0 + (c / KG) % 128, gb = g0 + c % KG;
      rb[r] = (gb < d.G && j < d.n) ? *(const v8h*)(d.B + pl * d.planeB + ((long)j * d.G + gb) * 8) : zero;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int c = tid + 256 * r;
      As[c / PL][buf][(c / 128) % KG][c & 127] = ra[r];
      Bs[c / PL][buf][c % KG][(c / KG) % 128] = rb[r];
    }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  const int gr = lane >> 4, li = lane & 15;
  for (int g0 = 0; g0 < d.G; g0 += KG) {
    const bool more = g0 + KG < d.G;
    if (more) gload(g0 + KG);
#pragma unroll
    for (int h = 0; h < KG / 4; ++h) {
      v8h ah[4], al[4], bh[4], bl[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ah[q] = As[0][buf][4 * h + gr][wm + q * 16 + li];
        al[q] = As[1][buf][4 * h + gr][wm + q * 16 + li];
        bh[q] = Bs[0][buf][4 * h + gr][wn + q * 16 + li];
        bl[q] = Bs[1][buf][4 * h + gr][wn + q * 16 + li];
      }
      // the two small terms first; the output rows are j (from B), columns i
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb) {
          acc[qa][qb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bl[qb], ah[qa], acc[qa][qb], 0, 0, 0);
          acc[qa][qb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bh[qb], al[qa], acc[qa][qb], 0, 0, 0);
          acc[qa][qb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bh[qb], ah[qa], acc[qa][qb], 0, 0, 0);
        }
    }
    if (NBUF == 2) {
      if (more) sstore(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    } else {
      __syncthreads();   // every wavefront is done reading the stage
      if (more) {
        sstore(0);
        __syncthreads();
      }
    }
  }
  const int sps = sp[blockIdx.z];
#pragma unroll
  for (int qa = 0; qa < 4; ++qa) {
    const int i = m0 + wm + qa * 16 + li;
    if (i >= d.m) continue;
    const int sh = -(split_scale(emax[i]) + sps);
#pragma unroll
    for (int qb = 0; qb < 4; ++qb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = n0 + wn + qb * 16 + 4 * gr + r;
        if (j < d.n) d.C[i + (long)j * d.ldc] = ldexp((double)acc[qa][qb][r], sh);
      }
  }
}

void l_colexp(int n, int b, const double* X, int* emax, hipStream_t s) {
  if (b == 0) return;
  KScope kt("k_colexp", s, 8.0 * n * (double)b, 0.0);
  hipLaunchKernelGGL(k_fill_int, dim3(cdiv(b, 256)), dim3(256), 0, s, b, 0, emax);
  AWG_LAUNCH_CHECK();
  const int cb = (int)cdiv(b, 256);
  const int rb = (int)std::max<long>(1, std::min<long>(n, 2048 / cb));
  const int rows = (int)cdiv(n, rb);
  hipLaunchKernelGGL(k_colexp, dim3(cb, cdiv(n, rows)), dim3(256), 0, s, n, b, X, rows, emax);
  AWG_LAUNCH_CHECK();
}

void l_gather_h3(long ngroups, const int* row0, const int* cnt, const int* sub_idx, const double* X, int b,
                 const int* emax, _Float16* out, long plane, hipStream_t s) {
  if (ngroups == 0 || b == 0) return;
  KScope kt("k_gather_h3", s, 0.0, 0.0);
  hipLaunchKernelGGL(k_gather_h3, dim3(cdiv(ngroups * b, 256)), dim3(256), 0, s, ngroups, row0, cnt, sub_idx, X, b,
                     emax, out, plane);
  AWG_LAUNCH_CHECK();
}

void l_p16_build(int N, const long* sqoff, const long* sub_ptr, const long* poff, const double* P, _Float16* out,
                 long plane, int* sp, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_p16_build<double>, dim3(N), dim3(256), 0, s, sqoff, sub_ptr, poff, P, out, plane, sp);
  AWG_LAUNCH_CHECK();
}
void l_p16_build(int N, const long* sqoff, const long* sub_ptr, const long* poff, const float* P, _Float16* out,
                 long plane, int* sp, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_p16_build<float>, dim3(N), dim3(256), 0, s, sqoff, sub_ptr, poff, P, out, plane, sp);
  AWG_LAUNCH_CHECK();
}

void gemm_h3_batched(const GemmDescH3* d_desc, int batch, int max_m, int max_n, const int* emax, const int* sp,
                     hipStream_t s, double flops) {
  if (batch <= 0 || max_m <= 0 || max_n <= 0) return;
  const dim3 grid(cdiv(max_m, 128), cdiv(max_n, 128), batch);
  auto run = [&](int v) {
    if (v == 1) hipLaunchKernelGGL(k_gemm_h3<8>, grid, dim3(256), 0, s, d_desc, emax, sp);
    else hipLaunchKernelGGL(k_gemm_h3<4>, grid, dim3(256), 0, s, d_desc, emax, sp);
    AWG_LAUNCH_CHECK();
  };
  const std::string key = "gemm_h3:P:m=" + std::to_string(max_m) + ":n=" + std::to_string(max_n) +
                          ":batch=" + std::to_string(batch);
  int v = tune_lookup(key);
  if (v < 0) v = tune_pick(key, 2, run, s);
  KScope kt("k_gemm_h3:P", s, 0.0, flops);
  run(v);
}

}  // namespace awg
