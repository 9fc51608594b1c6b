// Internal declarations shared by the HIP sources of libawg (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>
#include <vector>

namespace awg {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define AWG_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::awg::Error(e_ == hipErrorOutOfMemory ? -8 : -7,                          \
                         std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

#define AWG_LAUNCH_CHECK() AWG_HIP(hipGetLastError())

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

// Sum over the 256 threads of a block in a fixed order (a butterfly within
// each wavefront, whose pairwise sums are the same on every lane, then the
// four wavefront sums as (w0 + w1) + (w2 + w3)); every thread returns it.
// Every thread of the block must call it.
__device__ inline double block_sum_256(double v, double* sh4) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
// wall time (ms) spent in the device allocations and frees of DBuf,
// process-wide; the set-up reports its share per phase
extern double g_alloc_ms;
double alloc_clock_ms();

// Device memory of DBuf goes through a process-wide cache: a freed block is
// kept (after a device synchronisation, as hipFree does) and handed out again
// to a later allocation of at most its size and at least half of it, on the
// same device.  Repeated set-ups then allocate nothing from the driver, whose
// large allocations and frees took up to seconds on some calls.  The cache
// holds at most half of the device's memory (oldest blocks freed first), and
// before a new block is taken from the driver it is emptied when less than
// 16 GB would stay free for other allocators (the caller's framework, the
// runtime's queues and kernel scratch).  An allocation that fails empties the
// cache and retries; dev_cache_trim returns every cached block to the driver.
void* dev_alloc(size_t bytes);
void dev_free(void* p, size_t bytes);
size_t dev_cache_trim();

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) {
      // the wait for queued work that may still use the block is not
      // allocation time
      (void)hipDeviceSynchronize();
      const double t = alloc_clock_ms();
      dev_free(p, n * sizeof(T));
      g_alloc_ms += alloc_clock_ms() - t;
    }
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    const double t = alloc_clock_ms();
    p = (T*)dev_alloc(count * sizeof(T));
    g_alloc_ms += alloc_clock_ms() - t;
    n = count;
  }
  // keep the allocation when it holds count elements already (the W
  // solves narrow their multi-vectors without reallocating them)
  void ensure(size_t count) {
    if (p && n >= count) return;
    alloc(count);
  }
  void zero(hipStream_t s) {
    if (p) AWG_HIP(hipMemsetAsync(p, 0, n * sizeof(T), s));
  }
  void upload(const std::vector<T>& h, hipStream_t s) {
    alloc(h.size());
    if (!h.empty()) AWG_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
  std::vector<T> download(hipStream_t s, size_t count = (size_t)-1) const {
    if (count == (size_t)-1) count = n;
    std::vector<T> h(count);
    if (count) {
      AWG_HIP(hipMemcpyAsync(h.data(), p, count * sizeof(T), hipMemcpyDeviceToHost, s));
      AWG_HIP(hipStreamSynchronize(s));
    }
    return h;
  }
  operator T*() const { return p; }
};

// ---------------------------------------------------------------------------
// kernel timing (off by default): HIP events around instrumented launches,
// accumulated per kernel with the algorithmic bytes and flops of each launch
// ---------------------------------------------------------------------------
struct KScope {
  int slot = -1;
  KScope(const char* name, hipStream_t s, double bytes, double flops);
  ~KScope();
  KScope(const KScope&) = delete;
  KScope& operator=(const KScope&) = delete;
 private:
  hipStream_t s_ = nullptr;
};
void ktimer_enable(bool on);
void ktimer_capturing(bool on);
bool ktimer_on();
std::string ktimer_json(bool reset);

// ---------------------------------------------------------------------------
// batched dense descriptors (column-major blocks)
// ---------------------------------------------------------------------------
// acol (untransposed A only): when set, column k of A starts at
// A + acol[k] * lda instead of A + k * lda (a row gather fused into the load)
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  int m, n, k;
  int lda, ldb, ldc;
  const int* acol = nullptr;
};

struct GemmDescMix {     // FP64 A, FP32 B, FP64 C (FP32 local operators)
  const double* A;
  const float* B;
  double* C;
  int m, n, k;
  int lda, ldb, ldc;
  const int* acol = nullptr;
};

struct GemmDescF32 {     // FP32 A and B, FP64 C (FP32 local operators, FP32 accumulation)
  const float* A;
  const float* B;
  double* C;
  int m, n, k;
  int lda, ldb, ldc;
};

struct GemmDescH3 {      // split FP16 operands (hi and lo planes), FP64 C: C = A B of one subdomain
  const _Float16* A;     // multi-vector operand: entry (g, i) at A + (g m + i) 8, lo plane at + planeA
  const _Float16* B;     // matrix operand: entry (j, g) at B + (j G + g) 8, lo plane at + planeB
  double* C;             // C[i + j ldc]
  long planeA, planeB;
  int m, n, G, ldc;      // G = row groups of 8 (k = 8 G, zero-padded)
};

struct MatDescF {        // one square FP32 column-major block
  float* A;
  int n, ld;
};

struct MatDesc {         // one square or rectangular column-major block
  double* A;
  int m, n, ld;
  int pad;
};

// ---------------------------------------------------------------------------
// kernel launchers (implemented in k_*.hip)
// ---------------------------------------------------------------------------
// C = alpha * op(A) op(B) + beta * C for every descriptor; lower != 0 skips
// 64x64 output tiles lying strictly above the diagonal.
// flops: algorithmic flop count of the whole batch (for the kernel timer only)
// tag: name of the call site (kernel timer label suffix and autotuning key;
// tagged products choose their tile size by measurement)
void gemm_batched(const GemmDesc* d_desc, int batch, int max_m, int max_n, bool transA, bool transB,
                  double alpha, double beta, bool lower, hipStream_t s, double flops = 0.0,
                  const char* tag = nullptr);
// C = alpha A B + beta C with FP32 B (A rounded to FP32, FP32 MFMA and accumulation)
// Batched products whose untransposed A operands are row gathers of one
// row-major multi-vector X (n x lda): batch entry q reads its column k from
// row idx[off[q] + k] of X (A and acol of the descriptors are replaced).
void gemm_batched_gather(const GemmDesc* d_desc, const double* X, const int* idx, const long* off, int batch,
                         int max_m, int max_n, bool transB, double alpha, double beta, hipStream_t s, double flops,
                         const char* tag);
// sustained FP64 MFMA rate (TFLOP/s) of the current device, best of 3 timed
// launches of a register-only MFMA kernel
double probe_mfma_f64(int iters, hipStream_t s);
// one fixed launch variant (0..3) of gemm_batched (X == nullptr) or of
// gemm_batched_gather (transA must then be false)
void gemm_batched_fixed(const GemmDesc* d_desc, const double* X, const int* idx, const long* off, int batch,
                        int max_m, int max_n, bool transA, bool transB, double alpha, double beta, hipStream_t s,
                        int variant);
// C = alpha A B + beta C with FP32 A and B (FP32 MFMA and accumulation):
// the same products and k order as gemm_mix_batched on A rounded to FP32
// tiles/ntiles/grid (optional): the list of a persistent launch from
// f32_tile_list, offered to the autotuner beside the plain grid (same bits)
void gemm_f32_batched(const GemmDescF32* d_desc, int batch, int max_m, int max_n, double alpha, double beta,
                      hipStream_t s, double flops, const int* tiles = nullptr, int ntiles = 0, int grid = 0);
// tile list (host) of the persistent local-product launch for batch entries
// of sizes m x n with inner dimension k; returns its grid size
// FP32 Cholesky K = L L^T of every block of d_K (overwritten by L), X = L^-1
// in d_X and K^-1 = X^T X in d_out, all FP32 on the matrix cores; info[b] =
// first non-positive pivot column (1-based) or 0, dmin/dmax[b] = extreme
// diagonal entries of L
void chol_inverse_f32(const MatDescF* d_K, const MatDescF* d_X, const MatDescF* d_out, const std::vector<int>& h_n,
                      int* d_info, float* d_dmin, float* d_dmax, hipStream_t s);
// split-FP16 local product (three FP16 MFMA products, FP32 accumulation):
// emax (b) = per-column largest biased exponent of the multi-vector, from
// l_colexp; sp (batch) = the power-of-two scale of each matrix, from l_p16_build
void gemm_h3_batched(const GemmDescH3* d_desc, int batch, int max_m, int max_n, const int* emax, const int* sp,
                     hipStream_t s, double flops);
void l_colexp(int n, int b, const double* X, int* emax, hipStream_t s);
void l_gather_h3(long ngroups, const int* row0, const int* cnt, const int* sub_idx, const double* X, int b,
                 const int* emax, _Float16* out, long plane, hipStream_t s);
void l_p16_build(int N, const long* sqoff, const long* sub_ptr, const long* poff, const double* P, _Float16* out,
                 long plane, int* sp, hipStream_t s);
void l_p16_build(int N, const long* sqoff, const long* sub_ptr, const long* poff, const float* P, _Float16* out,
                 long plane, int* sp, hipStream_t s);
int f32_tile_list(const std::vector<int>& m, const std::vector<int>& n, const std::vector<int>& k, int wgs_per_xcd,
                  std::vector<int>& tiles);
// X, idx, off (optional): the same row gather of the A operands as in
// gemm_batched_gather
void gemm_mix_batched(const GemmDescMix* d_desc, int batch, int max_m, int max_n, double alpha, double beta,
                      hipStream_t s, double flops, const double* X = nullptr, const int* idx = nullptr,
                      const long* off = nullptr);
// y = alpha * op(A) x + beta * y per descriptor, with the GEMM convention
// (n == 1: A = matrix, B = x, C = y; op(A) is m x k).  A single long
// non-transposed product (k >= 16 m) splits k over GEMV_KSPLIT ranges when the
// caller passes `part`, a device buffer of GEMV_KSPLIT * max_m doubles owned
// by the caller's workspace (so concurrent solvers and captured graphs never
// share it).
constexpr int GEMV_KSPLIT = 64;
void gemv_batched(const GemmDesc* d_desc, int batch, int max_m, int max_k, bool transA, double alpha,
                  double beta, hipStream_t s, double bytes = 0.0, double* part = nullptr);

// Cholesky A = L L^T (lower, in place) of every block; info[b] = 0 or the
// 1-based column of the first non-positive pivot.  With dropped != NULL (a
// single block only): columns whose pivot is <= tol * diag0[c] are deleted
// (dropped[c] = 1, unit diagonal, zero column below), see k_potf2; pivrel,
// when given, receives every column's pivot / diag0[c] (the distance of the
// decision from tol).
void potrf_batched(const MatDesc* d_mats, const std::vector<int>& h_n, int* d_info, hipStream_t s,
                   GemmDesc* d_scratch_desc, const double* diag0 = nullptr, int* dropped = nullptr,
                   double tol = 0.0, double* pivrel = nullptr);
// potrf_batched for batch blocks of one order n (no host size list)
void potrf_uniform(const MatDesc* d_mats, int batch, int n, int* d_info, hipStream_t s);
// Solve L X = B (trans = false) or L^T X = B (trans = true) with the lower
// factor L of block b (n_b x n_b) and B_b (n_b x ncols_b); X overwrites B.
void trsm_batched(const MatDesc* d_L, const MatDesc* d_B, const std::vector<int>& h_n,
                  const std::vector<int>& h_ncols, bool trans, hipStream_t s, GemmDesc* d_scratch_desc);

// A[r0:, r0:] -= V W^T + W V^T for the panel at p0 of the blocked
// tridiagonalisation (two MFMA products; see k_eig.hip)
void syr2k_panel_update(const MatDesc* d_mats, const double* V, const double* W, const long* d_off, int p0, int nbw,
                        int max_rem, int batch, hipStream_t s, double flops);
// Householder tridiagonalisation of symmetric blocks (full storage,
// destroyed).  d, e, tau: per-block arrays at offsets off[b] (size n_b).
// work: TRD_WORK_PER_ROW * n_b doubles per block at off[b] * TRD_WORK_PER_ROW.
constexpr int TRD_NB = 32;
constexpr long TRD_WORK_PER_ROW = 2 * TRD_NB + 2;
void sytrd_batched(const MatDesc* d_mats, const std::vector<int>& h_n, double* d, double* e,
                   double* tau, const long* d_off, double* work, hipStream_t s);
// Eigenvalues < thr of the tridiagonal T_b: count, values and eigenvectors.
struct TriEigArgs {
  const double* d;
  const double* e;
  const long* off;        // per block: offset of d/e
  const int* n;           // per block order
  int nb;
};
// thr_mode 0: thr[b] is absolute (count lambda < thr[b]);
// thr_mode 1: thr[b] = eps0 * max|lambda| computed here, counting lambda <= thr.
void tri_count(const TriEigArgs& a, const double* thr_in, int thr_mode, double eps0, double* thr_out,
               int* count, double* lam_minmax, hipStream_t s);
// Work: 384 * n_b doubles per block at work_off[b] (see k_eig.hip).
constexpr long TRIVEC_WORK_PER_ROW = 7 * 64;
// maxn: largest block order (d and e are staged in LDS when it is <= 6144)
void tri_eigvecs(const TriEigArgs& a, const int* count, const long* lam_off, double* lam,
                 const MatDesc* d_Z, double* work, const long* work_off, double* resid,
                 int* nstrict, const double* thr, hipStream_t s, int maxn = 0);
// Z_b <- Q_b Z_b with the reflectors stored by sytrd_batched.
void ormtr_batched(const MatDesc* d_mats, const MatDesc* d_Z, const double* tau, const long* d_off,
                   const std::vector<int>& h_n, const std::vector<int>& h_k, hipStream_t s);

}  // namespace awg
