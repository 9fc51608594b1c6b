// AWG preconditioner and PCG on one MI355X: set-up pipeline, application,
// solver and the C ABI (include/awg.h).
//
// Method (Gouarin & Spillane): H = H2 + W (W^T A W)^{-1} W^T with
// H2 = Pi H^NN Pi^T + R0^T E0^{-1} R0 (Sections 3.3-3.4, 4.3).  Every step
// runs as a HIP kernel on the context's stream; the host only sequences the
// launches, sizes buffers from counts read back between phases, and tests
// convergence.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>

#include "awg.h"
#include "awg_dense.h"
#include "awg_common.h"
#include "awg_sparse.h"
#include "awg_subspace.h"
#include "awg_tune.h"
#include "awg_mlp.h"
#include "awg_mlp_impl.h"

using namespace awg;

// ---------------------------------------------------------------------------
// kernel timer
// ---------------------------------------------------------------------------
namespace awg {
namespace {
struct KRec {
  std::string name;
  hipEvent_t a, b;
  double bytes, flops;
};
struct KAcc {
  double calls = 0, ms = 0, bytes = 0, flops = 0;
};
bool g_kt_on = false;
bool g_kt_capturing = false;   // no event records while a graph is being captured
std::string g_kt_filter;       // when not empty: time only kernels whose label starts with it
std::vector<KRec> g_kt_pending;
std::vector<hipEvent_t> g_kt_pool;
std::map<std::string, KAcc> g_kt_acc;

hipEvent_t kt_event() {
  if (!g_kt_pool.empty()) {
    hipEvent_t e = g_kt_pool.back();
    g_kt_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  AWG_HIP(hipEventCreate(&e));
  return e;
}

void kt_flush() {
  for (auto& r : g_kt_pending) {
    AWG_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    AWG_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    KAcc& a = g_kt_acc[r.name];
    a.calls += 1;
    a.ms += ms;
    a.bytes += r.bytes;
    a.flops += r.flops;
    g_kt_pool.push_back(r.a);
    g_kt_pool.push_back(r.b);
  }
  g_kt_pending.clear();
}
}  // namespace

KScope::KScope(const char* name, hipStream_t s, double bytes, double flops) : s_(s) {
  if (!g_kt_on || g_kt_capturing) return;
  if (!g_kt_filter.empty() && std::strncmp(name, g_kt_filter.c_str(), g_kt_filter.size()) != 0) return;
  if (g_kt_pending.size() >= 8192) kt_flush();
  KRec r{name, kt_event(), kt_event(), bytes, flops};
  AWG_HIP(hipEventRecord(r.a, s));
  slot = (int)g_kt_pending.size();
  g_kt_pending.push_back(r);
}

KScope::~KScope() {
  if (slot >= 0) (void)hipEventRecord(g_kt_pending[slot].b, s_);
}

void ktimer_enable(bool on) { g_kt_on = on; }
void ktimer_capturing(bool on) { g_kt_capturing = on; }
bool ktimer_on() { return g_kt_on; }

std::string ktimer_json(bool reset) {
  kt_flush();
  std::ostringstream o;
  o.precision(10);
  o << "{";
  bool first = true;
  for (auto& kv : g_kt_acc) {
    o << (first ? "" : ",") << "\"" << kv.first << "\":{\"calls\":" << kv.second.calls << ",\"ms\":" << kv.second.ms
      << ",\"bytes\":" << kv.second.bytes << ",\"flops\":" << kv.second.flops << "}";
    first = false;
  }
  o << "}";
  if (reset) g_kt_acc.clear();
  return o.str();
}

double g_alloc_ms = 0.0;
double alloc_clock_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

namespace {
struct CachedBlock {
  void* p;
  size_t bytes;
  int dev;
};
std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache;   // oldest first
size_t g_cache_bytes = 0;
// device memory left to other allocators (the caller's framework, the
// runtime's queues and kernel scratch) before a new block is taken from the
// driver: the cache is emptied first when less than this would remain free
constexpr size_t CACHE_HEADROOM = size_t(16) << 30;

// frees cached blocks, oldest first, until at most keep bytes stay cached
// (the caller holds g_cache_mu)
size_t trim_locked(size_t keep) {
  size_t freed = 0, i = 0;
  if (g_cache_bytes > keep && !g_cache.empty()) (void)hipDeviceSynchronize();
  for (; i < g_cache.size() && g_cache_bytes > keep; ++i) {
    (void)hipFree(g_cache[i].p);
    g_cache_bytes -= g_cache[i].bytes;
    freed += g_cache[i].bytes;
  }
  g_cache.erase(g_cache.begin(), g_cache.begin() + i);
  return freed;
}
}  // namespace

void* dev_alloc(size_t bytes) {
  int dev = 0;
  AWG_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int best = -1;
    for (int i = 0; i < (int)g_cache.size(); ++i) {
      const CachedBlock& b = g_cache[i];
      if (b.dev == dev && b.bytes >= bytes && b.bytes / 2 <= bytes && (best < 0 || b.bytes < g_cache[best].bytes))
        best = i;
    }
    if (best >= 0) {
      void* p = g_cache[best].p;
      g_cache_bytes -= g_cache[best].bytes;
      g_cache.erase(g_cache.begin() + best);
      return p;
    }
    size_t fr = 0, tot = 0;
    if (!g_cache.empty() && hipMemGetInfo(&fr, &tot) == hipSuccess && fr < bytes + CACHE_HEADROOM)
      trim_locked(0);
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    dev_cache_trim();
    AWG_HIP(hipMalloc(&p, bytes));
  }
  return p;
}

void dev_free(void* p, size_t bytes) {
  if (!p) return;
  // queued work of any stream may still use the block
  (void)hipDeviceSynchronize();
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache.push_back(CachedBlock{p, bytes, dev});
  g_cache_bytes += bytes;
  // at most half of the device stays cached
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) == hipSuccess && g_cache_bytes > tot / 2) trim_locked(tot / 2);
}

size_t dev_cache_trim() {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  return trim_locked(0);
}
}  // namespace awg

namespace {

thread_local std::string g_setup_error = "no error";

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// per-subdomain column blocks (n_s x c_s, leading dimension n_s)
struct ColLayout {
  std::vector<int> c;        // columns per subdomain
  std::vector<long> eoff;    // element offset of block s
  std::vector<long> coff;    // offset of the columns of s in the concatenation
  long elems = 0, cols = 0;
  DBuf<long> d_eoff, d_coff;
  void build(const std::vector<int>& ns, const std::vector<int>& cs, hipStream_t s) {
    c = cs;
    eoff.assign(ns.size() + 1, 0);
    coff.assign(ns.size() + 1, 0);
    for (size_t i = 0; i < ns.size(); ++i) {
      eoff[i + 1] = eoff[i] + (long)ns[i] * cs[i];
      coff[i + 1] = coff[i] + cs[i];
    }
    elems = eoff.back();
    cols = coff.back();
    d_eoff.upload(eoff, s);
    d_coff.upload(coff, s);
  }
};

}  // namespace

// workspace for applying the operators to b columns at once; every n x b,
// sum_s n_s x b, k x b array is row-major (the b values of a row contiguous)
// relative pivot below which a basis vector of a coarse space counts as
// dependent on the previous ones (Gram matrices E0 and W^T A W)
constexpr double GRAM_DROP_TOL = 1e-10;

struct MultiWS {
  int b = 0;
  int h2mode = 0;       // AWG_H2_* applied by op_h2 on this workspace
  bool wops = false;    // local products with the W solves' operators
  DBuf<double> R, Z, T1, T2;          // n x b
  DBuf<double> Xs, Os;                // sum n_s x b (restricted rows, subdomain order)
  DBuf<double> Tk;                    // sum k_s x b
  DBuf<double> G0, G1, G2;            // n0 x b
  DBuf<double> H0, H1;                // n_minus x b
  DBuf<double> R3, H2b;               // hybrid H3: projected residual (n x b), second n_minus x b
  DBuf<GemmDesc> dWT1, dWtT1, dEW2;   // hybrid H3: W t -> T1, W^T T1 -> H0, E_W^{-1} H0 -> H2b
  DBuf<double> dotpart, dots;         // column dot products
  DBuf<double> gvpart;                // split-k partial sums of W^T r (b == 1)
  DBuf<GemmDesc> dVt, dV, dYt, dY, dP, dE0a, dE0b, dWt, dEW, dW;
  DBuf<GemmDescMix> dP32;             // FP32 local operators (b > 1)
  DBuf<float> Xs32;                   // restricted rows rounded to FP32 (b > 1, FP32 local operators)
  DBuf<GemmDescF32> dP32f;
  DBuf<GemmDesc> dCu, dCt, dAYt;      // C u0, C^T (..), (A R0^T)^T y (precomputed A_+ R0^T, b > 1)
  DBuf<int> tilesP32;                 // tile list of the persistent FP32 local product
  int ntilesP32 = 0, gridP32 = 0;
  DBuf<_Float16> Xs16;                // split-FP16 restricted rows (hi plane, then lo plane)
  long xs16_plane = 0;
  DBuf<GemmDescH3> dH3;
  DBuf<int> emax;                     // per-column largest exponent of the restricted multi-vector
  int maxk = 0, maxm = 0, maxns = 0;
  double flV = 0, flY = 0, flP = 0, flE0 = 0, flW = 0, flEW = 0;   // algorithmic flops per product
};

struct awg_ctx {
  hipStream_t s = nullptr;
  awg_options opt{};
  int n = 0, nnz = 0, N = 0;
  long sumns = 0;
  std::string err = "no error";
  // inputs (copied)
  DBuf<int> rowptr, col;
  SpmmGroups sgrp;    // row groups of the multi-column SpMM
  // multi-column A_+ and R0^T products as sparse products: [A | V_-] (V_-
  // the n x sum_s k_s prolongation of the V^s) applied to [X; |L_-| V^T R X],
  // and R0^T itself (n x n0) applied to the coarse coefficients
  DBuf<int> aug_rp, aug_col, y_rp, y_col;
  DBuf<double> aug_val, y_val;
  long aug_nnz = 0, y_nnz = 0;
  // A_+ R0^T precomputed for H2 on many columns: the extended sets
  // N(Omega^s) (support of A R^sT), AY^s = A[N_s, Omega^s] Y^s, the CSR of
  // [A R0^T | V_-] (n x (n0 + sum k_s)) and C = V_-^T R0^T (sum k_s x n0,
  // column-major), so that A_+ R0^T u = [A R0^T | V_-][u; |L_-| C u] and
  // R0 A_+ y = (A R0^T)^T y + C^T |L_-| V_-^T R y
  bool ap_ok = false;
  std::vector<long> h_extptr;
  DBuf<long> extptr;
  DBuf<int> extidx;
  ColLayout LAY;
  DBuf<double> AY, Cmat;
  DBuf<int> apv_rp, apv_col;
  DBuf<double> apv_val;
  long apv_nnz = 0;
  SpmmGroups apv_grp;
  double flAY1 = 0.0;          // 2 sum_s |N_s| m_s (flops per column of the (A R0^T)^T product)
  // their restrictions V_-^T and R0 as CSR (one-column products of the PCG)
  DBuf<int> vt_rp, vt_col, yt_rp, yt_col;
  DBuf<double> vt_val, yt_val;
  long vt_nnz = 0, yt_nnz = 0;
  SpmmGroups aug_grp, y_grp;
  DBuf<double> val;
  std::vector<long> h_subptr;
  std::vector<int> ns;
  DBuf<long> subptr;
  DBuf<int> subidx, entsub;
  // maps
  DBuf<int> mult, invptr, invsub, invloc, cnt;
  DBuf<double> bval, dw;
  // dense blocks: one "arena" holds every n_s x n_s block
  std::vector<long> sqoff;
  DBuf<long> d_sqoff;
  long sqtot = 0;
  int maxns = 0;
  // local results
  std::vector<int> ks, kstrict, ms;
  ColLayout LV, LY;
  DBuf<double> V, lamV, Y, lamY;
  DBuf<double> P;
  DBuf<float> P32;
  // split-FP16 local operators (multi-column local products): P^s scaled by
  // 2^sp_s and split into hi and lo planes of row groups of 8; the row
  // groups of the restriction (first entry into sub_idx, row count)
  DBuf<_Float16> P16;
  long p16_plane = 0;
  DBuf<int> p16_sp, h3_row0, h3_cnt;
  // the local operators of the preconditioner of the W solves when it is not
  // H2 itself (w_h2 with h2 = H^NN_hyb): P^s = (R^s A_+ R^sT)^{-1} of
  // H^AS_+ and their reduced-precision copies
  int wmode = 0;          // AWG_H2_* of the W solves
  DBuf<double> Pw;
  DBuf<float> P32w;
  DBuf<_Float16> P16w;
  DBuf<int> p16_sp_w;
  DBuf<long> p16_off;
  std::vector<long> h_p16_off, h3_gofs;
  long h3_groups = 0;
  int n0 = 0, nminus = 0;
  DBuf<double> E0inv, W, EWinv;
  MultiWS ws1;           // single-vector workspace (apply / PCG)
  DBuf<double> pcg_buf;  // x r z p q of the main PCG
  DBuf<double> scal;     // device scalars
  hipGraphExec_t pcg_graph = nullptr;   // one PCG iteration, captured on first use
  hipStream_t cap_stream = nullptr;
  int use_graph = 1;
  ~awg_ctx() {
    if (pcg_graph) (void)hipGraphExecDestroy(pcg_graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
  std::map<std::string, double> tms;
  int w_iters = 0;
  double w_iters_mean = 0.0;    // mean over the W columns of their iteration counts
  int w_compactions = 0;        // narrowings of the W solves' multi-vectors
  int w_factor_fallbacks = -1;  // subdomains of the FP32 factorisation redone in FP64 (-1: not run)
  double w_time = 0.0;
  std::vector<double> eig_resid_max;
  std::vector<int> eig_iters;   // subspace GenEO: iteration of convergence per subdomain
  int eig_fallbacks = 0;        // subdomains whose subspace result was not certified
  int eig_learned = 0;          // start block came from the network
  int n0_dropped = 0;           // dependent coarse vectors deleted from E0 (rank = n0 - n0_dropped)
  int nminus_dropped = 0;       // dependent W columns deleted from W^T A W
  // distance of the deletion decisions from the threshold (spd_inverse):
  // factor by which the threshold would have to move to change one of them
  double e0_margin = INFINITY, ew_margin = INFINITY;
  DBuf<double> ritzZ, ritzMu;   // last Ritz block (sum n_s x q) and values mu = 1/lambda
  int ritz_q = 0;
  DBuf<double> coords;          // optional node coordinates (n x cdim)
  int cdim = 0;
};

namespace {

// ---------------------------------------------------------------------------
// small device kernels used only here
// ---------------------------------------------------------------------------
// rows of the k_s x b blocks of T (V^T X) scaled by |lambda|: row r of
// block s is row coff[s] + r of the row-major concatenation
__global__ void k_scale_rows(double* T, const double* lam, long rows, int b) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * b) return;
  T[e] *= fabs(lam[e / b]);
}

// the same scaled rows written to dst (the coefficient rows appended to the
// multi-vector of a [A | V_-] product)
__global__ void k_scale_rows_to(const double* T, const double* lam, long rows, int b, double* dst) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * b) return;
  dst[e] = T[e] * fabs(lam[e / b]);
}

// G (n0 x b, row-major) = columns c0 .. c0+b-1 of the identity
__global__ void k_identity_cols(double* G, int n0, int b, int c0) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n0 * b) return;
  const int r = (int)(e / b), c = (int)(e % b);
  G[e] = (r == c0 + c) ? 1.0 : 0.0;
}

// dst[r * ldd + c0 + c] = src[r * b + c] for c < bc (row-major column block copy)
__global__ void k_copy_cols(const double* src, int b, double* dst, long ldd, long rows, int c0, int bc) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * bc) return;
  const long r = e / bc;
  const int c = (int)(e % bc);
  dst[r * ldd + c0 + c] = src[r * b + c];
}

// dst (rows x bn, row-major) = the columns perm[0 .. bn) of src (rows x bo)
__global__ void k_gather_cols(long rows, int bo, const double* src, int bn, const int* perm, double* dst) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * bn) return;
  const long r = e / bn;
  const int j = (int)(e - r * bn);
  dst[e] = src[r * bo + perm[j]];
}

// W[:, dst[j]] = X[:, pos[j]] for j < cnt (X rows x b, W rows x ldw, row-major)
__global__ void k_copy_cols_list(long rows, int b, const double* X, const int* pos, const int* dst, int cnt,
                                 double* W, long ldw) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cnt) return;
  const long r = e / cnt;
  const int j = (int)(e - r * cnt);
  W[r * ldw + dst[j]] = X[r * b + pos[j]];
}

// right-hand sides of W, row-major n x b: column gc = g0_s + j - c0 holds
// R^sT V^s[:, j] for the strictly negative pairs j < kstrict_s
__global__ void k_build_vg(const long* sub_ptr, const int* sub_idx, const double* V, const long* veoff,
                           const long* gcoff, double* Vg, int c0, int b) {
  const int s = blockIdx.y;
  const long a = sub_ptr[s], ns = sub_ptr[s + 1] - a;
  const long g0 = gcoff[s], kst = gcoff[s + 1] - g0;
  const long tot = ns * kst;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const long l = e % ns, j = e / ns;
    const long gc = g0 + j - c0;
    if (gc < 0 || gc >= b) continue;
    Vg[(long)sub_idx[a + l] * b + gc] = V[veoff[s] + l + j * ns];
  }
}

// Device-side PCG control.  sc layout: [0] rz, [1] pq, [2] alpha, [3] rz_new,
// [4] beta, [5] rr, [6] ||b||^2, [7] scratch, [8] (tol ||b||)^2, [9] done flag
// (1 converged, 2 breakdown, 3 maxit), [10] iterations, [11] maxit;
// alpha_k at sc[16 + 2k], beta_k at sc[17 + 2k].  Once done is set, alpha and
// beta are 0, so further launches leave x, r and p unchanged.
// The three scalar kernels run on one block of 256 threads: they first add
// the DOT1_BLOCKS partial sums of their dot product (fixed order) into sc[slot].
__device__ inline void sum_partials(const double* part, double* sc, int slot) {
  __shared__ double sh4[4];
  double acc = 0.0;
  for (int k = threadIdx.x; k < DOT1_BLOCKS; k += 256) acc += part[k];
  const double t = block_sum_256(acc, sh4);
  if (threadIdx.x == 0) sc[slot] = t;
}

__global__ __launch_bounds__(256) void k_pcg_alpha(double* sc, const double* part) {
  sum_partials(part, sc, 1);                  // pq
  if (threadIdx.x != 0) return;
  if (sc[9] != 0.0) { sc[2] = 0.0; return; }
  if (!(sc[1] > 0.0)) { sc[9] = 2.0; sc[2] = 0.0; return; }
  const double a = sc[0] / sc[1];
  sc[2] = a;
  sc[16 + 2 * (long)sc[10]] = a;
}

__global__ __launch_bounds__(256) void k_pcg_check(double* sc, const double* part) {
  sum_partials(part, sc, 5);                  // rr
  if (threadIdx.x != 0) return;
  if (sc[9] != 0.0) return;
  sc[10] += 1.0;
  if (sc[5] <= sc[8]) sc[9] = 1.0;
  else if (sc[10] >= sc[11]) sc[9] = 3.0;
}

__global__ __launch_bounds__(256) void k_pcg_beta(double* sc, const double* part) {
  sum_partials(part, sc, 3);                  // rz_new
  if (threadIdx.x != 0) return;
  if (sc[9] != 0.0) { sc[4] = 0.0; return; }
  const double bta = sc[3] / sc[0];
  sc[4] = bta;
  sc[0] = sc[3];
  sc[17 + 2 * ((long)sc[10] - 1)] = bta;
}

// x += alpha p, r -= alpha q, and part[blockIdx.x] = this block's share of
// r^T r (grid-stride over DOT1_BLOCKS blocks, fixed order)
__global__ __launch_bounds__(256) void k_pcg_update_xr(int n, double* x, double* r, const double* p, const double* q,
                                                       const double* sc, double* part) {
  __shared__ double sh4[4];
  const double a = sc[2];
  double acc = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    x[i] += a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  const double t = block_sum_256(acc, sh4);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k_pcg_update_p(int n, double* p, const double* z, const double* sc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[i] = z[i] + sc[4] * p[i];
}

__global__ void k_f32_from_f64(long tot, const double* a, float* b) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x)
    b[e] = (float)a[e];
}

// FP32 local solve: Os_s = P32_s Xs_s (FP32 matrix, FP64 vectors and sums)
__global__ __launch_bounds__(256) void k_gemv_f32(const float* P, const long* sqoff, const long* subptr,
                                                  const double* Xs, double* Os) {
  const int s = blockIdx.y;
  const long a = subptr[s];
  const int ns = (int)(subptr[s + 1] - a);
  const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + r;
  __shared__ double part[4][64];
  double acc = 0.0;
  if (i < ns) {
    const float* pa = P + sqoff[s] + i;
    const double* x = Xs + a;
    for (int j = g; j < ns; j += 4) acc += (double)pa[(long)j * ns] * x[j];
  }
  part[g][r] = acc;
  __syncthreads();
  if (g == 0 && i < ns) Os[a + i] = (part[0][r] + part[1][r]) + (part[2][r] + part[3][r]);
}

int errbits_to_status(int e, std::string& msg) {
  if (e & 16) { msg = "A is not a valid CSR matrix (column out of range, unsorted or duplicate)"; return AWG_ERR_ARG; }
  if (e & 1) { msg = "subdomain lists are not a partition: empty, unsorted, duplicate, out of range or not covering [0,n)"; return AWG_ERR_PARTITION; }
  if (e & 8) { msg = "A holds a NaN or Inf"; return AWG_ERR_NONFINITE; }
  if (e & 2) { msg = "A is not symmetric"; return AWG_ERR_NOT_SYMMETRIC; }
  if (e & 4) { msg = "minimal overlap assumption violated: some A_ij != 0 has no subdomain holding both i and j"; return AWG_ERR_MIN_OVERLAP; }
  return AWG_OK;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
std::vector<MatDesc> square_descs(const awg_ctx& c, double* arena) {
  std::vector<MatDesc> v(c.N);
  for (int s = 0; s < c.N; ++s) v[s] = MatDesc{arena + c.sqoff[s], c.ns[s], c.ns[s], c.ns[s], 0};
  return v;
}

std::vector<MatDesc> col_descs(const awg_ctx& c, double* base, const ColLayout& L) {
  std::vector<MatDesc> v(c.N);
  for (int s = 0; s < c.N; ++s) v[s] = MatDesc{base + L.eoff[s], c.ns[s], L.c[s], c.ns[s], 0};
  return v;
}

// Products of b row-major columns by a matrix M.  With X^T the b x k
// column-major view of a row-major k x b array X, every product of the
// method is written  Y^T = X^T op(M)  (op = identity or transpose): a GEMM
// with the column count b as its M dimension.  For b = 1 it is the GEMV
// y = op(M)^T x.
GemmDesc mk(const double* X, const double* M, int ldm, double* Y, int nout, int k, bool transM, int b) {
  if (b > 1) return GemmDesc{X, M, Y, b, nout, k, b, ldm, b};
  return GemmDesc{M, X, Y, nout, 1, k, ldm, 1, 1};
}

// flops: algorithmic flops of the whole batched product (2 m n k summed)
void bmm(const DBuf<GemmDesc>& d, int batch, int maxout, int maxk, bool transM, double alpha, double beta, int b,
         hipStream_t s, double flops, double* gemv_part = nullptr, const char* tag = nullptr) {
  if (batch == 0) return;
  if (b == 1) gemv_batched(d, batch, maxout, maxk, !transM, alpha, beta, s, 4.0 * flops, gemv_part);
  else gemm_batched(d, batch, b, maxout, false, transM, alpha, beta, false, s, flops, tag);
}

void gemm_upload(DBuf<GemmDesc>& d, const std::vector<GemmDesc>& h, hipStream_t s) { d.upload(h, s); }

// build the b-column workspace and its descriptors
void build_ws(awg_ctx& c, MultiWS& w, int b, bool wops = false) {
  // the W solves may run their own preconditioner (c.wmode) with its own
  // local operators; everything else applies H2 as chosen (c.opt.h2)
  w.wops = wops && c.wmode != c.opt.h2;
  w.h2mode = wops ? c.wmode : c.opt.h2;
  const DBuf<double>& Pl = w.wops ? c.Pw : c.P;
  const DBuf<float>& P32l = w.wops ? c.P32w : c.P32;
  const DBuf<_Float16>& P16l = w.wops ? c.P16w : c.P16;
  hipStream_t s = c.s;
  w.b = b;
  const long n = c.n;
  w.R.ensure(n * b);
  // T1 and Z are inputs of A_+ products: LV.cols extra rows hold the
  // coefficient rows of the [A | V_-] product
  w.Z.ensure((n + c.LV.cols) * b);
  w.T1.ensure((n + c.LV.cols) * b);
  w.T2.ensure(n * b);
  w.Xs.ensure(c.sumns * b);
  w.Os.ensure(c.sumns * b);
  w.Tk.ensure(std::max<long>(1, c.LV.cols) * b);
  w.G0.ensure(std::max(1, c.n0) * (long)b);
  w.G1.ensure((std::max(1, c.n0) + c.LV.cols) * (long)b);   // u0 and, below, |L_-| C u0
  w.G2.ensure(std::max(1, c.n0) * (long)b);
  w.H0.ensure(std::max(1, c.nminus) * (long)b);
  w.H1.ensure(std::max(1, c.nminus) * (long)b);
  w.dotpart.ensure(std::max<long>(std::max<long>(2L * DOT_CHUNKS_H * b, rb_part_size((int)n, b)), DOT1_BLOCKS));
  w.dots.ensure(2L * b);
  if (b == 1) w.gvpart.alloc((long)GEMV_KSPLIT * std::max(1, c.nminus));
  std::vector<GemmDesc> vt(c.N), vv(c.N), yt(c.N), yy(c.N), pp(c.N);
  w.maxk = w.maxm = w.maxns = 0;
  w.flV = w.flY = w.flP = 0;
  for (int q = 0; q < c.N; ++q) {
    const int nsq = c.ns[q];
    const long so = c.h_subptr[q] * b;
    const int kq = c.ks[q], mq = c.ms[q];
    w.flV += 2.0 * nsq * kq * b;
    w.flY += 2.0 * nsq * mq * b;
    w.flP += 2.0 * nsq * (double)nsq * b;
    w.maxk = std::max(w.maxk, kq);
    w.maxm = std::max(w.maxm, mq);
    w.maxns = std::max(w.maxns, nsq);
    const double* Vq = c.V.p + c.LV.eoff[q];
    const double* Yq = c.Y.p + c.LY.eoff[q];
    const double* xs = w.Xs.p + so;   // replaced by the rows of X in the in-place form
    // T_q = V_q^T X_q ;  O_q = V_q T_q ;  G0_q = Y_q^T X_q ;  O_q = Y_q G1_q ;  O_q = P_q X_q
    vt[q] = mk(xs, Vq, nsq, w.Tk.p + c.LV.coff[q] * b, kq, nsq, false, b);
    vv[q] = mk(w.Tk.p + c.LV.coff[q] * b, Vq, nsq, w.Os.p + so, nsq, kq, true, b);
    yt[q] = mk(xs, Yq, nsq, w.G0.p + c.LY.coff[q] * b, mq, nsq, false, b);
    yy[q] = mk(w.G1.p + c.LY.coff[q] * b, Yq, nsq, w.Os.p + so, nsq, mq, true, b);
    pp[q] = mk(xs, Pl.p + c.sqoff[q], nsq, w.Os.p + so, nsq, nsq, false, b);
  }
  gemm_upload(w.dVt, vt, s);
  gemm_upload(w.dV, vv, s);
  gemm_upload(w.dYt, yt, s);
  gemm_upload(w.dY, yy, s);
  gemm_upload(w.dP, pp, s);
  if (P32l.p && b > 1) {
    std::vector<GemmDescMix> pm(c.N);
    for (int q = 0; q < c.N; ++q) {
      const int nsq = c.ns[q];
      const long so = c.h_subptr[q] * b;
      pm[q] = GemmDescMix{w.Xs.p + so, P32l.p + c.sqoff[q], w.Os.p + so, b, nsq, nsq, b, nsq, b};
    }
    w.dP32.upload(pm, s);
    w.Xs32.ensure(c.sumns * b);
    std::vector<GemmDescF32> pf(c.N);
    for (int q = 0; q < c.N; ++q) {
      const int nsq = c.ns[q];
      const long so = c.h_subptr[q] * b;
      pf[q] = GemmDescF32{w.Xs32.p + so, P32l.p + c.sqoff[q], w.Os.p + so, b, nsq, nsq, b, nsq, b};
    }
    w.dP32f.upload(pf, s);
    // persistent, size-bucketed launch of the local product: two 512-thread
    // workgroups per CU, tiles dealt to the XCDs by subdomain
    int dev = 0, cus = 0;
    AWG_HIP(hipGetDevice(&dev));
    AWG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    std::vector<int> tl;
    w.gridP32 = f32_tile_list(std::vector<int>(c.N, b), c.ns, c.ns, std::max(1, 2 * cus / 8), tl);
    w.ntilesP32 = (int)tl.size();
    w.tilesP32.upload(tl, s);
  }
  if (P16l.p && b > 1) {
    w.xs16_plane = c.h3_groups * (long)b * 8;
    w.Xs16.ensure(2 * (size_t)w.xs16_plane);
    w.emax.ensure(b);
    std::vector<GemmDescH3> ph(c.N);
    for (int q = 0; q < c.N; ++q) {
      const int nsq = c.ns[q];
      ph[q] = GemmDescH3{w.Xs16.p + c.h3_gofs[q] * b * 8, P16l.p + c.h_p16_off[q], w.Os.p + c.h_subptr[q] * b,
                         w.xs16_plane, c.p16_plane, b, nsq, (nsq + 7) / 8, b};
    }
    w.dH3.upload(ph, s);
  }
  const int n0 = std::max(1, c.n0), nm = std::max(1, c.nminus);
  w.flE0 = 2.0 * c.n0 * (double)c.n0 * b;
  w.flW = 2.0 * c.n * (double)c.nminus * b;
  w.flEW = 2.0 * c.nminus * (double)c.nminus * b;
  // E0inv and EWinv are symmetric; W is stored row-major (n_minus values per dof)
  gemm_upload(w.dE0a, {mk(w.G0, c.E0inv, n0, w.G1, c.n0, c.n0, false, b)}, s);
  gemm_upload(w.dE0b, {mk(w.G0, c.E0inv, n0, w.G2, c.n0, c.n0, false, b)}, s);
  gemm_upload(w.dWt, {mk(w.R, c.W, nm, w.H0, c.nminus, c.n, true, b)}, s);
  gemm_upload(w.dEW, {mk(w.H0, c.EWinv, nm, w.H1, c.nminus, c.nminus, false, b)}, s);
  gemm_upload(w.dW, {mk(w.H1, c.W, nm, w.Z, c.n, c.nminus, false, b)}, s);
  if (c.ap_ok && b > 1) {
    const int nk = (int)c.LV.cols;
    gemm_upload(w.dCu, {mk(w.G1, c.Cmat, nk, w.G1.p + (long)c.n0 * b, nk, c.n0, true, b)}, s);
    gemm_upload(w.dCt, {mk(w.Tk, c.Cmat, nk, w.G0, c.n0, nk, false, b)}, s);
    std::vector<GemmDesc> ay(c.N);
    for (int q = 0; q < c.N; ++q) {
      const int ne = (int)(c.h_extptr[q + 1] - c.h_extptr[q]);
      ay[q] = mk(w.Xs, c.AY.p + c.LAY.eoff[q], ne, w.G0.p + c.LY.coff[q] * b, c.ms[q], ne, false, b);
    }
    gemm_upload(w.dAYt, ay, s);
  }
  if (c.opt.coarse2 == AWG_COARSE2_HYB && c.nminus > 0) {
    w.R3.ensure(c.n * (long)b);
    w.H2b.ensure(std::max(1, c.nminus) * (long)b);
    gemm_upload(w.dWT1, {mk(w.H1, c.W, nm, w.T1, c.n, c.nminus, false, b)}, s);
    gemm_upload(w.dWtT1, {mk(w.T1, c.W, nm, w.H0, c.nminus, c.n, true, b)}, s);
    gemm_upload(w.dEW2, {mk(w.H0, c.EWinv, nm, w.H2b, c.nminus, c.nminus, false, b)}, s);
  }
}

// Products with the restricted multi-vector R^q X (b > 1) as their A operand
// come in two forms with identical results: the restriction written out by
// l_gather and a plain batched GEMM, or the GEMM reading the rows
// sub_idx[sub_ptr[q] ..] of X in place.  In-place reads save the restricted
// block's write and re-read but scatter the GEMM's loads over all of X; the
// faster form per call site and shape is measured on the first call.
void restricted_product(awg_ctx& c, MultiWS& w, const char* tag, const double* X,
                        const std::function<void(bool fused)>& run) {
  const std::string key = std::string("restrict:") + tag + ":b=" + std::to_string(w.b) + ":sumns=" +
                          std::to_string(c.sumns) + ":N=" + std::to_string(c.N);
  int v = tune_lookup(key);
  if (v < 0) v = tune_pick(key, 2, [&](int f) {
    if (!f) l_gather(c.sumns, c.subidx, X, w.b, w.Xs, c.s);
    run(f != 0);
  }, c.s);
  if (v == 0) l_gather(c.sumns, c.subidx, X, w.b, w.Xs, c.s);
  run(v != 0);
}

// restricted product through the explicit descriptors d (A = the restricted block)
void bmm_restricted(awg_ctx& c, MultiWS& w, const DBuf<GemmDesc>& d, const double* X, int maxout, int maxk,
                    double flops, const char* tag) {
  restricted_product(c, w, tag, X, [&](bool fused) {
    if (fused)
      gemm_batched_gather(d, X, c.subidx.p, c.subptr.p, c.N, w.b, maxout, false, 1.0, 0.0, c.s, flops, tag);
    else
      gemm_batched(d, c.N, w.b, maxout, false, false, 1.0, 0.0, false, c.s, flops, tag);
  });
}

// Y = beta Y + A_- X   (A_- = sum_s R^sT V^s |L^s_-| V^sT R^s; Definition of A_-, Section 3.2)
void op_aminus(awg_ctx& c, MultiWS& w, const double* X, double* Yo, double beta) {
  const int b = w.b;
  if (c.LV.cols == 0) {
    if (beta == 0.0) AWG_HIP(hipMemsetAsync(Yo, 0, sizeof(double) * c.n * (size_t)b, c.s));
    return;
  }
  if (b > 1) {
    bmm_restricted(c, w, w.dVt, X, w.maxk, w.maxns, w.flV, "Vt");
  } else {
    l_gather(c.sumns, c.subidx, X, b, w.Xs, c.s);
    bmm(w.dVt, c.N, w.maxk, w.maxns, false, 1.0, 0.0, b, c.s, w.flV, nullptr, "Vt");
  }
  hipLaunchKernelGGL(k_scale_rows, dim3(cdiv(c.LV.cols * b, 256)), dim3(256), 0, c.s, w.Tk.p, c.lamV.p,
                     (long)c.LV.cols, b);
  AWG_LAUNCH_CHECK();
  bmm(w.dV, c.N, w.maxns, w.maxk, true, 1.0, 0.0, b, c.s, w.flV, nullptr, "V");
  l_scatter(c.n, c.sumns, c.invptr, c.invsub, c.invloc, c.subptr, w.Os, b, Yo, 1.0, beta, c.s);
}

// Y = A_+ X = A X + A_- X (item (i) of the A_+ theorem, Section 3.2).  For
// b > 1: T = V^T R X by the restricted GEMMs, its rows scaled by |L_-| and
// written below X (X has LV.cols extra rows), then one sparse product with
// [A | V_-], so the prolongation of the A_- term costs no pass of its own.
void op_aplus(awg_ctx& c, MultiWS& w, double* X, double* Yo) {
  const int b = w.b;
  if (c.aug_nnz > 0) {
    if (b > 1)
      bmm_restricted(c, w, w.dVt, X, w.maxk, w.maxns, w.flV, "Vt");
    else
      l_spmm((int)c.LV.cols, c.vt_nnz, c.vt_rp, c.vt_col, c.vt_val, X, w.Tk, 1, 1.0, 0.0, c.s);
    hipLaunchKernelGGL(k_scale_rows_to, dim3(cdiv(c.LV.cols * b, 256)), dim3(256), 0, c.s, w.Tk.p, c.lamV.p,
                       (long)c.LV.cols, b, X + c.n * (long)b);
    AWG_LAUNCH_CHECK();
    l_spmm(c.n, c.aug_nnz, c.aug_rp, c.aug_col, c.aug_val, X, Yo, b, 1.0, 0.0, c.s, &c.aug_grp, "k_spmm:A+");
    return;
  }
  l_spmm(c.n, c.nnz, c.rowptr, c.col, c.val, X, Yo, b, 1.0, 0.0, c.s, &c.sgrp);
  op_aminus(c, w, X, Yo, 1.0);
}

// G0 = R0 X  (R0^T = [R^1T Y^1 | ... | R^NT Y^N])
void op_r0(awg_ctx& c, MultiWS& w, const double* X) {
  if (w.b > 1) {
    bmm_restricted(c, w, w.dYt, X, w.maxm, w.maxns, w.flY, "Yt");
    return;
  }
  if (c.yt_nnz > 0) {
    l_spmm((int)c.LY.cols, c.yt_nnz, c.yt_rp, c.yt_col, c.yt_val, X, w.G0, 1, 1.0, 0.0, c.s);
    return;
  }
  l_gather(c.sumns, c.subidx, X, w.b, w.Xs, c.s);
  bmm(w.dYt, c.N, w.maxm, w.maxns, false, 1.0, 0.0, w.b, c.s, w.flY, nullptr, "Yt");
}

// Yo = beta Yo + alpha R0^T G1 (b > 1: a sparse product with R0^T in CSR)
void op_r0t(awg_ctx& c, MultiWS& w, double* Yo, double beta, double alpha = 1.0) {
  if (c.y_nnz > 0) {
    l_spmm(c.n, c.y_nnz, c.y_rp, c.y_col, c.y_val, w.G1, Yo, w.b, alpha, beta, c.s, &c.y_grp, "k_spmm:R0T");
    return;
  }
  bmm(w.dY, c.N, w.maxns, w.maxm, true, 1.0, 0.0, w.b, c.s, w.flY, nullptr, "Y");
  l_scatter(c.n, c.sumns, c.invptr, c.invsub, c.invloc, c.subptr, w.Os, w.b, Yo, alpha, beta, c.s);
}

// tuning key of the FP32 local product at width b
std::string p32_key(const awg_ctx& c, int b) {
  return "restrict:P32:b=" + std::to_string(b) + ":sumns=" + std::to_string(c.sumns) + ":N=" + std::to_string(c.N);
}

// Yo = sum_s R^sT P^s R^s X: H^NN X with P^s = D^s (A^s_+)^+ D^s (Definition of
// H^NN, Section 3.3), or H^AS_+ X with P^s = (R^s A_+ R^sT)^{-1} (Section 3.4);
// with add_r0t, Yo = that + R0^T G1 (the coarse prolongation added while the
// local results are scattered, for b > 1 where the one-pass kernel applies)
void op_hnn(awg_ctx& c, MultiWS& w, const double* X, double* Yo, bool f32, bool add_r0t = false) {
  if (w.b == 1) l_gather(c.sumns, c.subidx, X, w.b, w.Xs, c.s);
  if (f32 && w.b == 1) {
    KScope kt("k_gemv_f32", c.s, 4.0 * c.sqtot, 2.0 * c.sqtot);
    hipLaunchKernelGGL(k_gemv_f32, dim3(cdiv(w.maxns, 64), c.N), dim3(256), 0, c.s, c.P32.p, c.d_sqoff.p,
                       c.subptr.p, w.Xs.p, w.Os.p);
    AWG_LAUNCH_CHECK();
  } else if (f32 && w.dH3.p) {
    // split-FP16 local product: per-column exponents, split restriction,
    // three FP16 matrix-core products per tile
    l_colexp(c.n, w.b, X, w.emax, c.s);
    l_gather_h3(c.h3_groups, c.h3_row0, c.h3_cnt, c.subidx, X, w.b, w.emax, w.Xs16, w.xs16_plane, c.s);
    gemm_h3_batched(w.dH3, c.N, w.b, w.maxns, w.emax, w.wops ? c.p16_sp_w : c.p16_sp, c.s, w.flP);
  } else if (f32) {
    // FP32 local product, three forms with identical results: the restricted
    // FP64 rows written out or read in place and rounded while staged, or
    // the rows written out in FP32 (half the operand bytes) for the FP32 GEMM
    auto run = [&](int v) {
      if (v == 0) {
        l_gather(c.sumns, c.subidx, X, w.b, w.Xs, c.s);
        gemm_mix_batched(w.dP32, c.N, w.b, w.maxns, 1.0, 0.0, c.s, w.flP);
      } else if (v == 1) {
        gemm_mix_batched(w.dP32, c.N, w.b, w.maxns, 1.0, 0.0, c.s, w.flP, X, c.subidx.p, c.subptr.p);
      } else {
        l_gather_f32(c.sumns, c.subidx, X, w.b, w.Xs32, c.s);
        gemm_f32_batched(w.dP32f, c.N, w.b, w.maxns, 1.0, 0.0, c.s, w.flP, w.tilesP32, w.ntilesP32, w.gridP32);
      }
    };
    const std::string key = p32_key(c, w.b);
    int v = tune_lookup(key);
    if (v < 0) v = tune_pick(key, 3, run, c.s);
    run(v);
  } else if (w.b > 1) {
    bmm_restricted(c, w, w.dP, X, w.maxns, w.maxns, w.flP, "P");
  } else {
    bmm(w.dP, c.N, w.maxns, w.maxns, false, 1.0, 0.0, w.b, c.s, w.flP, nullptr, "P");
  }
  if (add_r0t && w.b > 1 && c.y_nnz > 0 &&
      l_scatter_prolong(c.n, c.sumns, c.invptr, c.invsub, c.invloc, c.subptr, w.Os, w.b, c.n0, c.y_nnz, c.y_rp,
                        c.y_col, c.y_val, w.G1, Yo, c.s))
    return;
  l_scatter(c.n, c.sumns, c.invptr, c.invsub, c.invloc, c.subptr, w.Os, w.b, Yo, 1.0, 0.0, c.s);
  if (add_r0t) op_r0t(c, w, Yo, 1.0);
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// H2 and H on the b columns of w.R -> w.Z
// ---------------------------------------------------------------------------
// H2 = Pi H^NN Pi^T + R0^T E0^{-1} R0 (Theorem on H^NN_hyb, Section 3.4):
//   u0 = E0^{-1} R0 r; t = r - A_+ R0^T u0; y = H^NN t;
//   v = E0^{-1} R0 A_+ y; z = y + R0^T (u0 - v)
void op_h2(awg_ctx& c, MultiWS& w, bool f32, const double* rin = nullptr) {
  const int b = w.b;
  const double* r = rin ? rin : w.R.p;
  if (c.n0 == 0) {
    op_hnn(c, w, r, w.Z, f32);
    return;
  }
  if (w.h2mode == AWG_H2_ASP_AD) {
    // H^AS_{+,ad} = H^AS_+ + R0^T E0^{-1} R0 (Theorem on H^AS_{+,hyb/ad}, Section 3.4)
    op_r0(c, w, r);                                                      // G0 = R0 r
    bmm(w.dE0a, 1, c.n0, c.n0, false, 1.0, 0.0, b, c.s, w.flE0, nullptr, "E0");         // G1 = E0^{-1} R0 r
    op_hnn(c, w, r, w.Z, f32, true);                                     // Z = H^AS_+ r + R0^T G1
    return;
  }
  op_r0(c, w, r);                                                        // G0 = R0 r
  bmm(w.dE0a, 1, c.n0, c.n0, false, 1.0, 0.0, b, c.s, w.flE0, nullptr, "E0");           // G1 = u0
  if (b > 1 && c.ap_ok) {
    // with A_+ R0^T precomputed: two coarse-sized GEMMs and one sparse
    // product with small sources in place of R0^T, A_+ and R0 on n x b blocks
    const long nk = c.LV.cols;
    const double flC = 2.0 * nk * c.n0 * b;
    double* tail = w.G1.p + (long)c.n0 * b;
    bmm(w.dCu, 1, (int)nk, c.n0, true, 1.0, 0.0, b, c.s, flC, nullptr, "Cu");         // C u0 below u0
    hipLaunchKernelGGL(k_scale_rows, dim3(cdiv(nk * b, 256)), dim3(256), 0, c.s, tail, c.lamV.p, nk, b);
    AWG_LAUNCH_CHECK();
    l_spmm(c.n, c.apv_nnz, c.apv_rp, c.apv_col, c.apv_val, w.G1, w.T2, b, 1.0, 0.0, c.s, &c.apv_grp,
           "k_spmm:AR0T");                                                             // T2 = A_+ R0^T u0
    l_colaxpby(c.n, b, r, nullptr, w.T2, nullptr, 1.0, -1.0, c.s);                    // T2 = r - T2
    op_hnn(c, w, w.T2, w.Z, f32);                                                      // Z = y
    gemm_batched_gather(w.dAYt, w.Z, c.extidx, c.extptr, c.N, b, w.maxm, false, 1.0, 0.0, c.s, c.flAY1 * b,
                        "AYt");                                                        // G0 = (A R0^T)^T y
    bmm_restricted(c, w, w.dVt, w.Z, w.maxk, w.maxns, w.flV, "Vt");                  // Tk = V^T R y
    hipLaunchKernelGGL(k_scale_rows, dim3(cdiv(nk * b, 256)), dim3(256), 0, c.s, w.Tk.p, c.lamV.p, nk, b);
    AWG_LAUNCH_CHECK();
    bmm(w.dCt, 1, c.n0, (int)nk, false, 1.0, 1.0, b, c.s, flC, nullptr, "Ct");       // G0 += C^T |L| V^T R y
    bmm(w.dE0b, 1, c.n0, c.n0, false, 1.0, 0.0, b, c.s, w.flE0, nullptr, "E0");      // G2 = v
    l_colaxpby(c.n0, b, w.G2, nullptr, w.G1, nullptr, -1.0, 1.0, c.s);               // G1 = u0 - v
    op_r0t(c, w, w.Z, 1.0);                                                            // Z += R0^T (u0 - v)
    return;
  }
  op_r0t(c, w, w.T1, 0.0);                                               // T1 = R0^T u0
  op_aplus(c, w, w.T1, w.T2);                                            // T2 = A_+ R0^T u0
  l_colaxpby(c.n, b, r, nullptr, w.T2, nullptr, 1.0, -1.0, c.s);        // T2 = r - T2
  op_hnn(c, w, w.T2, w.Z, f32);                                          // Z = y
  op_aplus(c, w, w.Z, w.T1);                                             // T1 = A_+ y
  op_r0(c, w, w.T1);                                                     // G0 = R0 A_+ y
  bmm(w.dE0b, 1, c.n0, c.n0, false, 1.0, 0.0, b, c.s, w.flE0, nullptr, "E0");           // G2 = v
  l_colaxpby(c.n0, b, w.G2, nullptr, w.G1, nullptr, -1.0, 1.0, c.s);     // G1 = u0 - v
  op_r0t(c, w, w.Z, 1.0);                                                // Z += R0^T (u0 - v)
}

// H = H3,ad = H2 + W (W^T A W)^{-1} W^T (Definition of Pi_3 and H3, Section 4.3)
// H3,hyb = Pi3 H2 Pi3^T + W E_W^{-1} W^T with Pi3 = I - W E_W^{-1} W^T A
// (Definition of Pi_3 and H3, Section 4.3): t = E_W^{-1} W^T r,
// y = H2 (r - A W t), z = y + W (t - E_W^{-1} W^T A y)
void op_h_hyb(awg_ctx& c, MultiWS& w, bool f32) {
  const int b = w.b;
  bmm(w.dWt, 1, c.nminus, c.n, true, 1.0, 0.0, b, c.s, w.flW, w.gvpart.p, "Wt");     // H0 = W^T r
  bmm(w.dEW, 1, c.nminus, c.nminus, false, 1.0, 0.0, b, c.s, w.flEW, nullptr, "EW");   // H1 = t
  bmm(w.dWT1, 1, c.n, c.nminus, false, 1.0, 0.0, b, c.s, w.flW, nullptr, "W");         // T1 = W t
  l_spmm(c.n, c.nnz, c.rowptr, c.col, c.val, w.T1, w.R3, b, 1.0, 0.0, c.s, &c.sgrp);  // R3 = A W t
  l_colaxpby(c.n, b, w.R, nullptr, w.R3, nullptr, 1.0, -1.0, c.s);                     // R3 = Pi3^T r
  op_h2(c, w, f32, w.R3);                                                              // Z = y
  l_spmm(c.n, c.nnz, c.rowptr, c.col, c.val, w.Z, w.T1, b, 1.0, 0.0, c.s, &c.sgrp);   // T1 = A y
  bmm(w.dWtT1, 1, c.nminus, c.n, true, 1.0, 0.0, b, c.s, w.flW, w.gvpart.p, "Wt");   // H0 = W^T A y
  bmm(w.dEW2, 1, c.nminus, c.nminus, false, 1.0, 0.0, b, c.s, w.flEW, nullptr, "EW");  // H2b = s
  l_colaxpby(c.nminus, b, w.H2b, nullptr, w.H1, nullptr, -1.0, 1.0, c.s);             // H1 = t - s
  bmm(w.dW, 1, c.n, c.nminus, false, 1.0, 1.0, b, c.s, w.flW, nullptr, "W");           // Z += W (t - s)
}

void op_h(awg_ctx& c, MultiWS& w, bool f32) {
  if (c.opt.coarse2 == AWG_COARSE2_HYB && c.nminus > 0) {
    op_h_hyb(c, w, f32);
    return;
  }
  op_h2(c, w, f32);
  if (c.nminus == 0) return;
  const int b = w.b;
  bmm(w.dWt, 1, c.nminus, c.n, true, 1.0, 0.0, b, c.s, w.flW, w.gvpart.p, "Wt");  // H0 = W^T r
  bmm(w.dEW, 1, c.nminus, c.nminus, false, 1.0, 0.0, b, c.s, w.flEW, nullptr, "EW");    // H1 = E_W^{-1} H0
  bmm(w.dW, 1, c.n, c.nminus, false, 1.0, 1.0, b, c.s, w.flW, nullptr, "W");           // Z += W H1
}

void sync(awg_ctx& c) { AWG_HIP(hipStreamSynchronize(c.s)); }

// compaction of the converged columns of the W solves (process-wide switch,
// for the test that compares the two)
int g_w_compaction = 1;

// wall time of a set-up phase, and (key "alloc:<phase>") the part of it
// spent in device allocations and frees
struct PhaseTimer {
  awg_ctx& c;
  std::string name;
  double t0, a0;
  PhaseTimer(awg_ctx& c_, const char* nm) : c(c_), name(nm) {
    sync(c);
    t0 = now_ms();
    a0 = g_alloc_ms;
  }
  ~PhaseTimer() {
    (void)hipStreamSynchronize(c.s);
    c.tms[name] += now_ms() - t0;
    c.tms["alloc:" + name] += g_alloc_ms - a0;
  }
};

__global__ void k_rowptr32(int n, const int64_t* rp, int* out, long nnz, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  const int64_t v = rp[i];
  if (v < 0 || v > nnz) atomicOr(err, 16);
  if (i == 0 && v != 0) atomicOr(err, 16);
  if (i == n && v != nnz) atomicOr(err, 16);
  if (i < n && rp[i + 1] < v) atomicOr(err, 16);
  out[i] = (int)v;
}

__global__ void k_fill(double* p, long n, double v) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) p[e] = v;
}

void check_info(awg_ctx& c, DBuf<int>& info, const char* what) {
  auto h = info.download(c.s);
  for (size_t s = 0; s < h.size(); ++s)
    if (h[s] != 0) {
      std::ostringstream o;
      o << what << ": Cholesky breakdown in block " << s << " at column " << h[s];
      throw Error(AWG_ERR_NOT_SPD, o.str());
    }
}

// ---------------------------------------------------------------------------
// set-up phases
// ---------------------------------------------------------------------------
// Definition of a partition, minimal overlap (Section 2.1); partition of unity
// (Section 2.2); M_mu and B (Section 3.1).
void phase_maps(awg_ctx& c, const int64_t* rowptr, const int32_t* col, const double* val, const int64_t* sub_ptr,
                const int32_t* sub_idx) {
  PhaseTimer t(c, "maps");
  hipStream_t s = c.s;
  DBuf<int> err;
  err.alloc(1);
  err.zero(s);
  c.rowptr.alloc(c.n + 1);
  hipLaunchKernelGGL(k_rowptr32, dim3(cdiv(c.n + 1, 256)), dim3(256), 0, s, c.n, rowptr, c.rowptr.p, (long)c.nnz,
                     err.p);
  AWG_LAUNCH_CHECK();
  c.col.alloc(c.nnz);
  c.val.alloc(c.nnz);
  AWG_HIP(hipMemcpyAsync(c.col.p, col, sizeof(int) * c.nnz, hipMemcpyDeviceToDevice, s));
  AWG_HIP(hipMemcpyAsync(c.val.p, val, sizeof(double) * c.nnz, hipMemcpyDeviceToDevice, s));
  c.h_subptr.resize(c.N + 1);
  AWG_HIP(hipMemcpyAsync(c.h_subptr.data(), sub_ptr, sizeof(int64_t) * (c.N + 1), hipMemcpyDeviceToHost, s));
  sync(c);
  if (c.h_subptr[0] != 0) throw Error(AWG_ERR_PARTITION, "sub_ptr[0] must be 0");
  for (int q = 0; q < c.N; ++q)
    if (c.h_subptr[q + 1] <= c.h_subptr[q]) throw Error(AWG_ERR_PARTITION, "empty subdomain or decreasing sub_ptr");
  c.sumns = c.h_subptr[c.N];
  if (c.sumns >= (1L << 31)) throw Error(AWG_ERR_ARG, "sum of subdomain sizes must be < 2^31");
  c.ns.resize(c.N);
  c.maxns = 0;
  for (int q = 0; q < c.N; ++q) {
    c.ns[q] = (int)(c.h_subptr[q + 1] - c.h_subptr[q]);
    c.maxns = std::max(c.maxns, c.ns[q]);
  }
  c.subptr.upload(c.h_subptr, s);
  c.subidx.alloc(c.sumns);
  AWG_HIP(hipMemcpyAsync(c.subidx.p, sub_idx, sizeof(int) * c.sumns, hipMemcpyDeviceToDevice, s));
  c.entsub.alloc(c.sumns);
  l_entry_owner(c.N, c.subptr, c.entsub, s);
  l_validate_subs(c.N, c.subptr, c.subidx, c.n, err, s);
  {
    int e = err.download(s)[0];
    std::string msg;
    int st = errbits_to_status(e, msg);
    if (st) throw Error(st, msg);
  }
  c.mult.alloc(c.n);
  c.mult.zero(s);
  l_mult(c.sumns, c.subidx, c.mult, s);
  l_check_cover(c.n, c.mult, err, s);
  c.invptr.alloc(c.n + 1);
  l_scan(c.n, c.mult, c.invptr, s);
  DBuf<int> fill;
  fill.alloc(c.n);
  fill.zero(s);
  c.invsub.alloc(c.sumns);
  c.invloc.alloc(c.sumns);
  l_fill_inv(c.N, c.subptr, c.subidx, c.invptr, fill, c.invsub, c.invloc, s);
  l_sort_inv(c.n, c.invptr, c.invsub, c.invloc, s);
  c.cnt.alloc(c.nnz);
  c.bval.alloc(c.nnz);
  l_pairs(c.n, c.rowptr, c.col, c.val, c.invptr, c.invsub, c.cnt, c.bval, err, s);
  c.dw.alloc(c.sumns);
  l_pou(c.sumns, c.subidx, c.mult, c.dw, s);
  int e = err.download(s)[0];
  std::string msg;
  int st = errbits_to_status(e, msg);
  if (st) throw Error(st, msg);
  c.sqoff.assign(c.N + 1, 0);
  for (int q = 0; q < c.N; ++q) c.sqoff[q + 1] = c.sqoff[q] + (long)c.ns[q] * c.ns[q];
  c.sqtot = c.sqoff[c.N];
  c.d_sqoff.upload(c.sqoff, s);
  spmm_groups_defer((int)c.n, c.nnz, c.rowptr, c.col, c.val, c.sgrp);   // on the validated pattern
}

// Batched eigenvalues below a threshold of dense symmetric blocks (destroys
// X).  Returns counts; fills lam / vectors in the layout built from them.
struct EigOut {
  std::vector<int> count, nstrict;
  double resid_max = 0.0;
};

EigOut batched_low_eigs(awg_ctx& c, DBuf<MatDesc>& dX, int thr_mode, double thr_value, ColLayout& L,
                        DBuf<double>& vecs, DBuf<double>& lam, bool want_strict) {
  hipStream_t s = c.s;
  DBuf<double> d, e, tau, work, thr, minmax;
  d.alloc(c.sumns);
  e.alloc(c.sumns);
  tau.alloc(c.sumns);
  work.alloc(std::max<long>(5, TRIVEC_WORK_PER_ROW) * c.sumns);
  thr.alloc(c.N);
  minmax.alloc(2 * c.N);
  sytrd_batched(dX, c.ns, d, e, tau, c.subptr, work, s);
  DBuf<int> nd, cnt, nst;
  nd.upload(c.ns, s);
  cnt.alloc(c.N);
  nst.alloc(c.N);
  TriEigArgs a{d, e, c.subptr, nd, c.N};
  if (thr_mode == 0) {
    hipLaunchKernelGGL(k_fill, dim3(cdiv(c.N, 256)), dim3(256), 0, s, thr.p, (long)c.N, thr_value);
    AWG_LAUNCH_CHECK();
  }
  tri_count(a, thr, thr_mode, thr_value, thr, cnt, minmax, s);
  EigOut out;
  out.count = cnt.download(s);
  L.build(c.ns, out.count, s);
  vecs.alloc(std::max<long>(1, L.elems));
  lam.alloc(std::max<long>(1, L.cols));
  DBuf<double> resid;
  resid.alloc(std::max<long>(1, L.cols));
  std::vector<long> w6(c.N);
  for (int q = 0; q < c.N; ++q) w6[q] = TRIVEC_WORK_PER_ROW * c.h_subptr[q];
  DBuf<long> dw6;
  dw6.upload(w6, s);
  auto zd = col_descs(c, vecs, L);
  DBuf<MatDesc> dZ;
  dZ.upload(zd, s);
  tri_eigvecs(a, cnt, L.d_coff, lam, dZ, work, dw6, resid, want_strict ? nst.p : nullptr, thr, s, c.maxns);
  ormtr_batched(dX, dZ, tau, c.subptr, c.ns, out.count, s);
  if (want_strict) out.nstrict = nst.download(s);
  if (L.cols) {
    auto r = resid.download(s, L.cols);
    for (double v : r) out.resid_max = std::max(out.resid_max, v);
  }
  if (!(out.resid_max <= 1e-8))
    throw Error(AWG_ERR_EIGEN, "tridiagonal inverse iteration did not converge (residual " +
                                   std::to_string(out.resid_max) + ")");
  return out;
}

// GenEO modes by block subspace iteration (kernels in k_subspace.hip).
// MB, MA: arenas holding M_B^s and M_A^s (MA is destroyed by the certificate).
// On success fills c.Y, c.LY, c.lamY, c.ms and returns 0; otherwise returns
// the number of subdomains that failed (the caller then runs the dense solver).
int geneo_subspace(awg_ctx& c, const double* MB, double* MA) {
  hipStream_t s = c.s;
  const int N = c.N, q = c.opt.eig_block;
  const double tau = c.opt.tau, window = 2.0, tol_far = 1e-2;
  const int min_it = 3;
  std::vector<long> qoff(N + 1, 0), goff(N + 1, 0), ooff(N + 1, 0), kqoff(N + 1, 0);
  int maxk = 0;
  for (int t = 0; t < N; ++t) {
    const int k = c.ks[t];
    maxk = std::max(maxk, k);
    goff[t + 1] = goff[t] + (long)k * k;
    kqoff[t + 1] = kqoff[t] + (long)k * q;
  }
  // kernel of M_A: K = D^s V^s_-, KB = M_B K, GK = K^T M_B K = L L^T
  DBuf<double> K, KB, GK;
  K.alloc(std::max<long>(1, c.LV.elems));
  KB.alloc(std::max<long>(1, c.LV.elems));
  GK.alloc(std::max<long>(1, goff[N]));
  l_rows_dw(N, c.maxns, maxk, c.subptr, c.LV.d_eoff, c.LV.d_coff, c.V, c.dw, K, s);
  std::vector<GemmDesc> g(N);
  DBuf<GemmDesc> dKB, dGK, dg1, dg2, dg3, dg4, dg3x, dg4x, dg5, dg6, dg7, dg8;
  std::vector<MatDesc> mg(N), mc(N), mcx(N);
  for (int t = 0; t < N; ++t) {
    const int n = c.ns[t], k = c.ks[t], lk = std::max(1, k);
    const long eo = c.LV.eoff[t];
    g[t] = GemmDesc{MB + c.sqoff[t], K.p + eo, KB.p + eo, n, k, n, n, n, n};
    mg[t] = MatDesc{GK.p + goff[t], k, k, lk, 0};
  }
  dKB.upload(g, s);
  double fl = 0.0;
  for (int t = 0; t < N; ++t) fl += 2.0 * c.ns[t] * (double)c.ns[t] * c.ks[t];
  if (maxk) gemm_batched(dKB, N, c.maxns, maxk, false, false, 1.0, 0.0, false, s, fl);
  for (int t = 0; t < N; ++t) {
    const int n = c.ns[t], k = c.ks[t];
    const long eo = c.LV.eoff[t];
    g[t] = GemmDesc{K.p + eo, KB.p + eo, GK.p + goff[t], k, k, n, n, n, std::max(1, k)};
  }
  dGK.upload(g, s);
  if (maxk) gemm_batched(dGK, N, maxk, maxk, true, false, 1.0, 0.0, false, s);
  DBuf<MatDesc> dmg;
  dmg.upload(mg, s);
  DBuf<int> info;
  info.alloc(N);
  info.zero(s);
  if (maxk) {
    l_scale_sym(dmg, N, nullptr, nullptr, false, true, s);
    potrf_batched(dmg, c.ks, info, s, nullptr);
    for (int v : info.download(s))
      if (v) return N;
  }
  // iterated blocks (n_s x q per subdomain at sub_ptr[s] * q)
  const long bq = c.sumns * (long)q;
  DBuf<double> X, BX, Y, Z, TZ, cK, S0, S1, Cq, mu, res;
  X.alloc(bq);
  BX.alloc(bq);
  Y.alloc(bq);
  Z.alloc(bq);
  TZ.alloc(bq);
  cK.alloc(std::max<long>(1, kqoff[N]));
  S0.alloc((long)N * q * q);
  S1.alloc((long)N * q * q);
  Cq.alloc((long)N * q * q);
  mu.alloc((long)N * q);
  res.alloc((long)N * q);
  DBuf<int> flag, conv, nsel;
  flag.alloc(N);
  conv.alloc(N);
  nsel.alloc(N);
  auto blk = [&](const DBuf<double>& b, int t) { return b.p + c.h_subptr[t] * q; };
  auto up = [&](DBuf<GemmDesc>& d, auto f) {
    for (int t = 0; t < N; ++t) g[t] = f(t, c.ns[t], c.ks[t]);
    d.upload(g, s);
  };
  up(dg1, [&](int t, int n, int) { return GemmDesc{MB + c.sqoff[t], blk(X, t), blk(BX, t), n, q, n, n, n, n}; });
  up(dg2, [&](int t, int n, int) { return GemmDesc{c.P.p + c.sqoff[t], blk(BX, t), blk(Y, t), n, q, n, n, n, n}; });
  up(dg3, [&](int t, int n, int k) {
    return GemmDesc{KB.p + c.LV.eoff[t], blk(Y, t), cK.p + kqoff[t], k, q, n, n, n, std::max(1, k)};
  });
  up(dg4, [&](int t, int n, int k) {
    return GemmDesc{K.p + c.LV.eoff[t], cK.p + kqoff[t], blk(Y, t), n, q, k, n, std::max(1, k), n};
  });
  up(dg3x, [&](int t, int n, int k) {
    return GemmDesc{KB.p + c.LV.eoff[t], blk(X, t), cK.p + kqoff[t], k, q, n, n, n, std::max(1, k)};
  });
  up(dg4x, [&](int t, int n, int k) {
    return GemmDesc{K.p + c.LV.eoff[t], cK.p + kqoff[t], blk(X, t), n, q, k, n, std::max(1, k), n};
  });
  up(dg5, [&](int t, int n, int) { return GemmDesc{blk(X, t), blk(BX, t), S0.p + (long)t * q * q, q, q, n, n, n, q}; });
  up(dg6, [&](int t, int n, int) { return GemmDesc{blk(BX, t), blk(Y, t), S1.p + (long)t * q * q, q, q, n, n, n, q}; });
  up(dg7, [&](int t, int n, int) { return GemmDesc{blk(X, t), Cq.p + (long)t * q * q, blk(Z, t), n, q, q, n, q, n}; });
  up(dg8, [&](int t, int n, int) { return GemmDesc{blk(Y, t), Cq.p + (long)t * q * q, blk(TZ, t), n, q, q, n, q, n}; });
  for (int t = 0; t < N; ++t) mc[t] = MatDesc{cK.p + kqoff[t], c.ks[t], q, std::max(1, c.ks[t]), 0};
  DBuf<MatDesc> dmc;
  dmc.upload(mc, s);
  const std::vector<int> qcols(N, q);
  double flMB = 0.0, flK = 0.0;
  for (int t = 0; t < N; ++t) {
    flMB += 2.0 * c.ns[t] * (double)c.ns[t] * q;
    flK += 2.0 * c.ns[t] * (double)c.ks[t] * q;
  }
  // Pi_B: x <- x - K GK^-1 (KB^T x)
  auto project = [&](DBuf<GemmDesc>& a, DBuf<GemmDesc>& b) {
    if (!maxk) return;
    gemm_batched(a, N, maxk, q, true, false, 1.0, 0.0, false, s, flK);
    trsm_batched(dmg, dmc, c.ks, qcols, false, s, nullptr);
    trsm_batched(dmg, dmc, c.ks, qcols, true, s, nullptr);
    gemm_batched(b, N, c.maxns, q, false, false, -1.0, 1.0, false, s, flK);
  };
  l_rand_block(N, c.maxns, c.subptr, c.subidx, q, (uint64_t)(uint32_t)c.opt.eig_seed, X, s);
  c.eig_learned = 0;
  if (c.opt.eig_init) {
    // learned start: network outputs on the per-dof features fill the first p columns
    awg_mlp& net = *const_cast<awg_mlp*>(c.opt.eig_init);
    const int p = net.dims.back();
    DBuf<float> feat, out;
    feat.alloc((size_t)c.sumns * MLP_FEATURES);
    out.alloc((size_t)c.sumns * p);
    l_mlp_features(N, c.n, c.maxns, c.subptr, c.subidx, c.rowptr, c.col, c.val, c.invptr, c.invsub, c.invloc,
                   c.mult, c.V, c.LV.d_eoff, c.LV.d_coff, c.P, c.d_sqoff, c.coords.p, c.cdim, feat, s);
    mlp_forward(net, c.sumns, feat, out, true, s);
    l_block_from_rows(N, c.maxns, c.subptr, q, p, out, X, s);
    sync(c);
    c.eig_learned = 1;
  }
  project(dg3x, dg4x);
  c.eig_iters.assign(N, -1);
  int it = 0, nconv = 0;
  std::vector<int> hconv(N, 0), hflag(N, 0);
  for (it = 1; it <= c.opt.eig_maxit; ++it) {
    gemm_batched(dg1, N, c.maxns, q, false, false, 1.0, 0.0, false, s, flMB, "eigMB");   // BX = M_B X
    gemm_batched(dg2, N, c.maxns, q, false, false, 1.0, 0.0, false, s, flMB, "eigG");    // Y = G BX
    project(dg3, dg4);                                                              // Y = Pi_B Y
    gemm_batched(dg5, N, q, q, true, false, 1.0, 0.0, false, s);                    // S0 = X^T M_B X
    gemm_batched(dg6, N, q, q, true, false, 1.0, 0.0, false, s);                    // S1 = X^T M_B T X
    l_rr_small(N, q, S0, S1, Cq, mu, flag, s);
    gemm_batched(dg7, N, c.maxns, q, false, false, 1.0, 0.0, false, s, 0.0, "eigXC");    // Z = X C
    gemm_batched(dg8, N, c.maxns, q, false, false, 1.0, 0.0, false, s, 0.0, "eigYC");    // T Z = Y C
    l_ritz_resid(N, c.subptr, q, Z, TZ, mu, X, res, conv, nsel, tau, window, c.opt.eig_tol, tol_far, s);
    AWG_HIP(hipMemcpyAsync(hconv.data(), conv.p, sizeof(int) * N, hipMemcpyDeviceToHost, s));
    sync(c);
    nconv = 0;
    for (int t = 0; t < N; ++t) {
      if (hconv[t] && c.eig_iters[t] < 0) c.eig_iters[t] = it;
      if (!hconv[t]) c.eig_iters[t] = -1;
      nconv += hconv[t] != 0;
    }
    if (it >= min_it && nconv == N) break;
  }
  hflag = flag.download(s);
  std::vector<int> hsel = nsel.download(s);
  std::swap(c.ritzZ.p, Z.p);
  std::swap(c.ritzZ.n, Z.n);
  std::swap(c.ritzMu.p, mu.p);
  std::swap(c.ritzMu.n, mu.n);
  c.ritz_q = q;
  const double* Zk = c.ritzZ.p;
  const double* muk = c.ritzMu.p;
  int fails = 0;
  std::vector<int> ms(N);
  for (int t = 0; t < N; ++t) {
    const bool bad = !hconv[t] || hflag[t] || hsel[t] >= q;
    fails += bad;
    ms[t] = c.ks[t] + std::min(hsel[t], q);
  }
  if (fails) return fails;
  c.LY.build(c.ns, ms, s);
  c.Y.alloc(std::max<long>(1, c.LY.elems));
  c.lamY.alloc(std::max<long>(1, c.LY.cols));
  int maxm = 0;
  for (int v : ms) maxm = std::max(maxm, v);
  l_assemble_modes(N, c.maxns, maxm, c.subptr, q, K, c.LV.d_eoff, c.LV.d_coff, Zk, muk, c.Y, c.LY.d_eoff,
                   c.LY.d_coff, c.lamY, s);
  // M_B-orthonormal basis of span(Y): Y <- Y L^-T with Y^T M_B Y = L L^T
  std::vector<long> moff(N + 1, 0);
  for (int t = 0; t < N; ++t) moff[t + 1] = moff[t] + (long)ms[t] * ms[t];
  DBuf<double> BY, T1, T2, G, Li;
  BY.alloc(std::max<long>(1, c.LY.elems));
  T1.alloc(std::max<long>(1, c.LY.elems));
  T2.alloc(std::max<long>(1, c.LY.elems));
  G.alloc(std::max<long>(1, moff[N]));
  Li.alloc(std::max<long>(1, moff[N]));
  std::vector<MatDesc> dgm(N), dli(N);
  for (int t = 0; t < N; ++t) {
    const int m = ms[t];
    dgm[t] = MatDesc{G.p + moff[t], m, m, std::max(1, m), 0};
    dli[t] = MatDesc{Li.p + moff[t], m, m, std::max(1, m), 0};
  }
  DBuf<MatDesc> ddg, ddl;
  ddg.upload(dgm, s);
  ddl.upload(dli, s);
  DBuf<GemmDesc> e1, e2, e3, e4, e5;
  up(e1, [&](int t, int n, int) {
    const long eo = c.LY.eoff[t];
    return GemmDesc{MB + c.sqoff[t], c.Y.p + eo, BY.p + eo, n, ms[t], n, n, n, n};
  });
  up(e2, [&](int t, int n, int) {
    const long eo = c.LY.eoff[t];
    return GemmDesc{c.Y.p + eo, BY.p + eo, G.p + moff[t], ms[t], ms[t], n, n, n, std::max(1, ms[t])};
  });
  up(e3, [&](int t, int n, int) {
    const long eo = c.LY.eoff[t];
    return GemmDesc{c.Y.p + eo, Li.p + moff[t], T1.p + eo, n, ms[t], ms[t], n, std::max(1, ms[t]), n};
  });
  up(e4, [&](int t, int n, int) {
    const long eo = c.LY.eoff[t];
    return GemmDesc{BY.p + eo, Li.p + moff[t], T2.p + eo, n, ms[t], ms[t], n, std::max(1, ms[t]), n};
  });
  double flY = 0.0;
  for (int t = 0; t < N; ++t) flY += 2.0 * c.ns[t] * (double)c.ns[t] * ms[t];
  gemm_batched(e1, N, c.maxns, maxm, false, false, 1.0, 0.0, false, s, flY);
  gemm_batched(e2, N, maxm, maxm, true, false, 1.0, 0.0, false, s);
  l_scale_sym(ddg, N, nullptr, nullptr, false, true, s);
  info.zero(s);
  potrf_batched(ddg, ms, info, s, nullptr);
  for (int v : info.download(s))
    if (v) return N;
  l_set_identity(ddl, N, s);
  trsm_batched(ddg, ddl, ms, ms, false, s, nullptr);                  // Li = L^-1
  gemm_batched(e3, N, c.maxns, maxm, false, true, 1.0, 0.0, false, s);  // Y L^-T
  gemm_batched(e4, N, c.maxns, maxm, false, true, 1.0, 0.0, false, s);  // M_B Y L^-T
  std::swap(c.Y.p, T1.p);
  std::swap(c.Y.n, T1.n);
  std::swap(BY.p, T2.p);
  std::swap(BY.n, T2.n);
  // certificate: M_A - tau' M_B + (M_B Y)(M_B Y)^T is spd, so at most m_s
  // eigenvalues of the pencil lie below tau' = tau (1 - 1e-10); the m_s Ritz
  // values below tau bound as many eigenvalues from above
  l_axpy_flat(c.sqtot, -tau * (1.0 - 1e-10), MB, MA, s);
  up(e5, [&](int t, int n, int) {
    const long eo = c.LY.eoff[t];
    return GemmDesc{BY.p + eo, BY.p + eo, MA + c.sqoff[t], n, n, ms[t], n, n, n};
  });
  gemm_batched(e5, N, c.maxns, c.maxns, false, true, 1.0, 1.0, true, s, flY);
  DBuf<MatDesc> dma;
  dma.upload(square_descs(c, MA), s);
  info.zero(s);
  potrf_batched(dma, c.ns, info, s, nullptr);
  auto hi = info.download(s);
  for (int t = 0; t < N; ++t) fails += hi[t] != 0;
  if (fails) return fails;
  c.ms = ms;
  c.n0 = (int)c.LY.cols;
  c.eig_resid_max.push_back(0.0);
  {
    auto r = res.download(s);
    double mx = 0.0;
    for (int t = 0; t < N; ++t)
      for (int j = 0; j < ms[t] - c.ks[t]; ++j) mx = std::max(mx, r[(long)t * q + j]);
    c.eig_resid_max.back() = mx;
  }
  return 0;
}

// reduced-precision copies of the local operators P^s: FP32 (one-column
// products and the FP32 local product) and, for AWG_LOCAL_F16X3, the split
// FP16 planes with their row groups
void build_reduced_local(awg_ctx& c, const DBuf<double>& P, DBuf<float>& P32, DBuf<_Float16>& P16,
                         DBuf<int>& sp) {
  hipStream_t s = c.s;
  P32.alloc(c.sqtot);
  hipLaunchKernelGGL(k_f32_from_f64, dim3(4096), dim3(256), 0, s, (long)c.sqtot, P.p, P32.p);
  AWG_LAUNCH_CHECK();
  if (c.opt.local_prec != AWG_LOCAL_F16X3) return;
  std::vector<int> row0, cnt;
  c.h3_gofs.assign(c.N + 1, 0);
  c.h_p16_off.assign(c.N + 1, 0);
  for (int q = 0; q < c.N; ++q) {
    const int nsq = c.ns[q], G = (nsq + 7) / 8;
    for (int g = 0; g < G; ++g) {
      row0.push_back((int)(c.h_subptr[q] + 8 * g));
      cnt.push_back(std::min(8, nsq - 8 * g));
    }
    c.h3_gofs[q + 1] = c.h3_gofs[q] + G;
    c.h_p16_off[q + 1] = c.h_p16_off[q] + (long)nsq * G * 8;
  }
  c.h3_groups = c.h3_gofs[c.N];
  c.h3_row0.upload(row0, s);
  c.h3_cnt.upload(cnt, s);
  c.p16_plane = c.h_p16_off[c.N];
  c.p16_off.upload(c.h_p16_off, s);
  P16.alloc(2 * (size_t)c.p16_plane);
  sp.alloc(c.N);
  l_p16_build(c.N, c.d_sqoff, c.subptr, c.p16_off, P, P16, c.p16_plane, sp, s);
  sync(c);   // the host row-group lists end here
}
void build_reduced_local(awg_ctx& c) { build_reduced_local(c, c.P, c.P32, c.P16, c.p16_sp); }

// B^s, its non-positive eigenpairs (splitting of B^s, Section 3.2), the local
// factor and P^s = D^s (A^s_+)^+ D^s, the GenEO coarse vectors Y^s
// (Theorem on H^NN_hyb, Section 3.4).
void phase_local(awg_ctx& c) {
  hipStream_t s = c.s;
  DBuf<double> X1, X2, X3;
  X1.alloc(c.sqtot);
  X2.alloc(c.sqtot);
  X3.alloc(c.sqtot);
  DBuf<MatDesc> d1, d2, d3;
  d1.upload(square_descs(c, X1), s);
  d2.upload(square_descs(c, X2), s);
  d3.upload(square_descs(c, X3), s);
  DBuf<int> info;
  info.alloc(c.N);
  {
    PhaseTimer t(c, "local_split");
    X1.zero(s);
    l_extract(c.N, c.subptr, c.subidx, c.rowptr, c.col, c.bval, d1, s);          // B^s
    l_copy_mat(d1, d2, c.N, s);
    EigOut eo = batched_low_eigs(c, d2, 1, c.opt.zero_tol, c.LV, c.V, c.lamV, true);
    c.ks = eo.count;
    c.kstrict = eo.nstrict;
    c.eig_resid_max.push_back(eo.resid_max);
  }
  DBuf<double> cs, U;
  cs.alloc(c.N);
  U.alloc(std::max<long>(1, c.LV.elems));
  auto vdesc = col_descs(c, c.V, c.LV);
  auto udesc = col_descs(c, U, c.LV);
  DBuf<MatDesc> dV, dU;
  dV.upload(vdesc, s);
  dU.upload(udesc, s);
  std::vector<GemmDesc> g(c.N);
  DBuf<GemmDesc> dg;
  int maxk = 0;
  for (int q = 0; q < c.N; ++q) maxk = std::max(maxk, c.ks[q]);
  auto lowrank_into = [&](double* arena, double alpha) {
    // arena_s += alpha * U_s V_s^T
    for (int q = 0; q < c.N; ++q)
      g[q] = GemmDesc{U.p + c.LV.eoff[q], c.V.p + c.LV.eoff[q], arena + c.sqoff[q], c.ns[q], c.ns[q], c.ks[q],
                      c.ns[q], c.ns[q], c.ns[q]};
    dg.upload(g, s);
    double fl = 0.0;
    for (int q = 0; q < c.N; ++q) fl += 2.0 * c.ns[q] * (double)c.ns[q] * c.ks[q];
    if (maxk > 0) gemm_batched(dg, c.N, c.maxns, c.maxns, false, true, alpha, 1.0, false, s, fl);
  };
  // the AS forms of H2 need D^s (A^s_+)^+ D^s only in the subspace GenEO
  // solver (it applies the inverse of M_A^s with it)
  const bool asp = c.opt.h2 == AWG_H2_ASP_HYB || c.opt.h2 == AWG_H2_ASP_AD;
  const bool ash = c.opt.h2 == AWG_H2_AS_HYB;   // dense GenEO solver only
  const bool nn_formed = (!asp && !ash) || c.opt.geneo_solver == AWG_GENEO_SUBSPACE;
  if (nn_formed) {
    PhaseTimer t(c, "local_factor");
    // K^s = B^s + V_-(c_s - L_-)V_-^T (spd), c_s = mean diag B^s
    l_diag_mean(d1, c.N, cs, s);
    if (c.LV.elems) AWG_HIP(hipMemcpyAsync(U.p, c.V.p, sizeof(double) * c.LV.elems, hipMemcpyDeviceToDevice, s));
    l_scale_cols(dU, c.N, c.LV.d_coff, c.lamV, 1.0, cs, 2, s);
    l_copy_mat(d1, d3, c.N, s);
    lowrank_into(X3, 1.0);
    info.zero(s);
    potrf_batched(d3, c.ns, info, s, nullptr);
    check_info(c, info, "local factor K^s");
    // K^{-1} = L^{-T} L^{-1}
    l_set_identity(d2, c.N, s);
    trsm_batched(d3, d2, c.ns, c.ns, false, s, nullptr);
    trsm_batched(d3, d2, c.ns, c.ns, true, s, nullptr);
    // (A^s_+)^+ = K^{-1} - c_s^{-1} V_- V_-^T, then D^s (.) D^s
    if (c.LV.elems) AWG_HIP(hipMemcpyAsync(U.p, c.V.p, sizeof(double) * c.LV.elems, hipMemcpyDeviceToDevice, s));
    l_scale_cols(dU, c.N, c.LV.d_coff, c.lamV, 1.0, cs, 3, s);
    lowrank_into(X2, -1.0);
    l_scale_sym(d2, c.N, c.subptr, c.dw, false, true, s);
    std::swap(c.P.p, X2.p);   // d2 now addresses c.P
    std::swap(c.P.n, X2.n);
    if (c.opt.local_prec != AWG_LOCAL_F64 && !asp) build_reduced_local(c);
  }
  // M_A = D^{-1} A^s_+ D^{-1} (in X3) and M_B (in X1), with
  // A^s_+ = B^s + V_- |L_-| V_-^T and
  // M_B = R^s A R^sT + sum_t R^s R^tT V^t |L^t| V^tT R^t R^sT
  auto build_pencil = [&]() {
    if (c.LV.elems) AWG_HIP(hipMemcpyAsync(U.p, c.V.p, sizeof(double) * c.LV.elems, hipMemcpyDeviceToDevice, s));
    l_scale_cols(dU, c.N, c.LV.d_coff, c.lamV, 1.0, nullptr, 1, s);             // U = V_- |L_-|
    X3.zero(s);
    l_extract(c.N, c.subptr, c.subidx, c.rowptr, c.col, c.bval, d3, s);          // B^s
    lowrank_into(X3, 1.0);
    l_scale_sym(d3, c.N, c.subptr, c.dw, true, true, s);
    X1.zero(s);
    l_extract(c.N, c.subptr, c.subidx, c.rowptr, c.col, c.val, d1, s);
    lowrank_into(X1, 1.0);
    l_mb_neighbours(c.N, c.subptr, c.subidx, c.mult, c.invptr, c.invsub, c.invloc, d1, c.V, c.LV.d_eoff, c.lamV,
                    c.LV.d_coff, s);
    l_scale_sym(d1, c.N, nullptr, nullptr, false, true, s);
  };
  // every eigenpair of the pencil below tau by Cholesky M_B = L L^T and the
  // tridiagonal eigensolver on L^-1 M_A L^-T
  auto dense_geneo = [&]() {
    info.zero(s);
    potrf_batched(d1, c.ns, info, s, nullptr);
    check_info(c, info, "GenEO M_B^s");
    trsm_batched(d1, d3, c.ns, c.ns, false, s, nullptr);
    l_transpose_inplace(d3, c.N, s);
    trsm_batched(d1, d3, c.ns, c.ns, false, s, nullptr);
    l_scale_sym(d3, c.N, nullptr, nullptr, false, true, s);
    EigOut eo = batched_low_eigs(c, d3, 0, c.opt.tau, c.LY, c.Y, c.lamY, false);
    c.ms = eo.count;
    c.eig_resid_max.push_back(eo.resid_max);
    // Y = L^{-T} Z
    DBuf<MatDesc> dY;
    dY.upload(col_descs(c, c.Y, c.LY), s);
    trsm_batched(d1, dY, c.ns, c.ms, true, s, nullptr);
    c.n0 = (int)c.LY.cols;
  };
  // H^AS_hyb(tau_sharp, tau_flat), tau_sharp = tau, tau_flat = 1/tau (Theorem
  // on H^AS_hyb, Section 3.4): local operators (R^s A R^sT)^{-1} and the
  // coarse space of two pencils per subdomain, Y_L(tau, D^-1 A^s_+ D^-1,
  // R^s A R^sT) followed by Y_L(tau, R^s A R^sT, R^s A_+ R^sT)
  if (ash) {
    PhaseTimer t(c, "geneo");
    build_pencil();                                                               // X3 = M_A, X1 = M_B
    DBuf<double> X4;
    X4.alloc(c.sqtot);
    DBuf<MatDesc> d4;
    d4.upload(square_descs(c, X4), s);
    X2.zero(s);
    l_extract(c.N, c.subptr, c.subidx, c.rowptr, c.col, c.val, d2, s);           // R^s A R^sT
    l_scale_sym(d2, c.N, nullptr, nullptr, false, true, s);
    l_copy_mat(d2, d4, c.N, s);
    // Y_L(tau, G, F) with F = L L^T: eigenvectors Z of L^-1 G L^-T below tau,
    // Y = L^-T Z (F and G destroyed: F holds L)
    auto pencil = [&](DBuf<MatDesc>& G, DBuf<MatDesc>& F, ColLayout& L, DBuf<double>& Y, DBuf<double>& lam,
                      const char* what) {
      info.zero(s);
      potrf_batched(F, c.ns, info, s, nullptr);
      check_info(c, info, what);
      trsm_batched(F, G, c.ns, c.ns, false, s, nullptr);
      l_transpose_inplace(G, c.N, s);
      trsm_batched(F, G, c.ns, c.ns, false, s, nullptr);
      l_scale_sym(G, c.N, nullptr, nullptr, false, true, s);
      EigOut eo = batched_low_eigs(c, G, 0, c.opt.tau, L, Y, lam, false);
      c.eig_resid_max.push_back(eo.resid_max);
      DBuf<MatDesc> dY;
      dY.upload(col_descs(c, Y, L), s);
      trsm_batched(F, dY, c.ns, eo.count, true, s, nullptr);
      return eo.count;
    };
    ColLayout L1, L2;
    DBuf<double> Y1, Y2, lam1, lam2;
    const std::vector<int> m2 = pencil(d4, d1, L2, Y2, lam2, "GenEO M_B^s");                // (R A R^T, M_B)
    const std::vector<int> m1 = pencil(d3, d2, L1, Y1, lam1, "local block R^s A R^sT");      // (M_A, R A R^T)
    std::vector<int> ms(c.N);
    for (int q = 0; q < c.N; ++q) ms[q] = m1[q] + m2[q];
    c.LY.build(c.ns, ms, s);
    c.Y.alloc(std::max<long>(1, c.LY.elems));
    c.lamY.alloc(std::max<long>(1, c.LY.cols));
    for (int q = 0; q < c.N; ++q) {
      const long n1 = (long)c.ns[q] * m1[q], n2 = (long)c.ns[q] * m2[q];
      if (n1) {
        AWG_HIP(hipMemcpyAsync(c.Y.p + c.LY.eoff[q], Y1.p + L1.eoff[q], sizeof(double) * n1,
                               hipMemcpyDeviceToDevice, s));
        AWG_HIP(hipMemcpyAsync(c.lamY.p + c.LY.coff[q], lam1.p + L1.coff[q], sizeof(double) * m1[q],
                               hipMemcpyDeviceToDevice, s));
      }
      if (n2) {
        AWG_HIP(hipMemcpyAsync(c.Y.p + c.LY.eoff[q] + n1, Y2.p + L2.eoff[q], sizeof(double) * n2,
                               hipMemcpyDeviceToDevice, s));
        AWG_HIP(hipMemcpyAsync(c.lamY.p + c.LY.coff[q] + m1[q], lam2.p + L2.coff[q], sizeof(double) * m2[q],
                               hipMemcpyDeviceToDevice, s));
      }
    }
    c.ms = ms;
    c.n0 = (int)c.LY.cols;
    // P^s = (R^s A R^sT)^{-1} from the factor in d2, into X1 (its factor of M_B is spent)
    l_set_identity(d1, c.N, s);
    trsm_batched(d2, d1, c.ns, c.ns, false, s, nullptr);
    trsm_batched(d2, d1, c.ns, c.ns, true, s, nullptr);
    l_scale_sym(d1, c.N, nullptr, nullptr, false, true, s);
    sync(c);   // the host-side layouts and Y1, Y2 end with this scope
    std::swap(c.P.p, X1.p);
    std::swap(c.P.n, X1.n);
    if (c.opt.local_prec != AWG_LOCAL_F64) build_reduced_local(c);
    return;
  }
  bool mb_factored = false;   // d1 holds the Cholesky factor of M_B^s (dense solver), else M_B^s
  {
    PhaseTimer t(c, "geneo");
    build_pencil();
    c.eig_fallbacks = 0;
    if (c.opt.geneo_solver == AWG_GENEO_SUBSPACE) {
      c.eig_fallbacks = geneo_subspace(c, X1, X3);
      if (c.eig_fallbacks) {
        build_pencil();
        dense_geneo();
        mb_factored = true;
      }
    } else {
      dense_geneo();
      mb_factored = true;
    }
  }
  if (asp) {
    // local operators of H^AS_+: P^s = (R^s A_+ R^sT)^{-1} = (M_B^s)^{-1}
    // (one-level preconditioners for A_+, Section 3.3), from the factor the
    // GenEO solve left in d1 or a new one
    PhaseTimer t(c, "local_factor");
    if (!mb_factored) {
      info.zero(s);
      potrf_batched(d1, c.ns, info, s, nullptr);
      check_info(c, info, "H^AS_+ local block M_B^s");
    }
    l_set_identity(d2, c.N, s);
    trsm_batched(d1, d2, c.ns, c.ns, false, s, nullptr);
    trsm_batched(d1, d2, c.ns, c.ns, true, s, nullptr);
    l_scale_sym(d2, c.N, nullptr, nullptr, false, true, s);
    if (!nn_formed) {   // d2 still addresses X2
      std::swap(c.P.p, X2.p);
      std::swap(c.P.n, X2.n);
    }
    if (c.opt.local_prec != AWG_LOCAL_F64) build_reduced_local(c);
  }
  if (c.wmode != c.opt.h2 && c.opt.local_prec != AWG_LOCAL_F64 && !mb_factored) {
    // the W solves' H^AS_+ operators in the reduced-precision forms, M_B^s
    // intact in d1: FP32 Cholesky and inverse on the matrix cores, FP64 for
    // the subdomains whose FP32 factor fails or whose pivots show a
    // conditioning beyond FP32 (max/min diagonal of L squared > 2^18)
    PhaseTimer t(c, "local_factor");
    DBuf<float> K32, X32;
    K32.alloc(c.sqtot);
    X32.alloc(c.sqtot);
    c.P32w.alloc(c.sqtot);
    hipLaunchKernelGGL(k_f32_from_f64, dim3(4096), dim3(256), 0, s, (long)c.sqtot, X1.p, K32.p);
    AWG_LAUNCH_CHECK();
    auto fdescs = [&](float* base) {
      std::vector<MatDescF> v(c.N);
      for (int q = 0; q < c.N; ++q) v[q] = MatDescF{base + c.sqoff[q], c.ns[q], c.ns[q]};
      return v;
    };
    DBuf<MatDescF> dK, dX, dO;
    dK.upload(fdescs(K32.p), s);
    dX.upload(fdescs(X32.p), s);
    dO.upload(fdescs(c.P32w.p), s);
    DBuf<float> dmin, dmax;
    dmin.alloc(c.N);
    dmax.alloc(c.N);
    info.zero(s);
    chol_inverse_f32(dK, dX, dO, c.ns, info, dmin, dmax, s);
    const std::vector<int> hinfo = info.download(s);
    const std::vector<float> hmin = dmin.download(s), hmax = dmax.download(s);
    std::vector<int> fb;
    for (int q = 0; q < c.N; ++q) {
      const double ratio = hmin[q] > 0.f ? (double)hmax[q] / hmin[q] : 1e300;
      if (hinfo[q] != 0 || !(ratio * ratio <= 262144.0)) fb.push_back(q);
    }
    c.w_factor_fallbacks = (int)fb.size();
    if (!fb.empty()) {
      std::vector<MatDesc> sm(fb.size()), so(fb.size());
      std::vector<int> sn(fb.size());
      for (size_t t = 0; t < fb.size(); ++t) {
        const int q = fb[t];
        sm[t] = MatDesc{X1.p + c.sqoff[q], c.ns[q], c.ns[q], c.ns[q], 0};
        so[t] = MatDesc{X3.p + c.sqoff[q], c.ns[q], c.ns[q], c.ns[q], 0};
        sn[t] = c.ns[q];
      }
      DBuf<MatDesc> dsm, dso;
      dsm.upload(sm, s);
      dso.upload(so, s);
      DBuf<int> finfo;
      finfo.alloc(fb.size());
      finfo.zero(s);
      potrf_batched(dsm, sn, finfo, s, nullptr);
      check_info(c, finfo, "H^AS_+ local block M_B^s");
      l_set_identity(dso, (int)fb.size(), s);
      trsm_batched(dsm, dso, sn, sn, false, s, nullptr);
      trsm_batched(dsm, dso, sn, sn, true, s, nullptr);
      l_scale_sym(dso, (int)fb.size(), nullptr, nullptr, false, true, s);
      for (int q : fb)
        hipLaunchKernelGGL(k_f32_from_f64, dim3(256), dim3(256), 0, s, (long)c.ns[q] * c.ns[q], X3.p + c.sqoff[q],
                           c.P32w.p + c.sqoff[q]);
      AWG_LAUNCH_CHECK();
    }
    if (c.opt.local_prec == AWG_LOCAL_F16X3) {
      c.P16w.alloc(2 * (size_t)c.p16_plane);
      c.p16_sp_w.alloc(c.N);
      l_p16_build(c.N, c.d_sqoff, c.subptr, c.p16_off, (const float*)c.P32w.p, c.P16w, c.p16_plane, c.p16_sp_w, s);
    }
    sync(c);
  } else if (c.wmode != c.opt.h2) {
    // the W solves' H^AS_+ operators beside H^NN: P^s_w = (M_B^s)^{-1} from the
    // factor the dense GenEO solve left in d1, or a new one of M_B^s
    PhaseTimer t(c, "local_factor");
    if (!mb_factored) {
      info.zero(s);
      potrf_batched(d1, c.ns, info, s, nullptr);
      check_info(c, info, "H^AS_+ local block M_B^s");
    }
    c.Pw.alloc(c.sqtot);
    DBuf<MatDesc> dw;
    dw.upload(square_descs(c, c.Pw), s);
    l_set_identity(dw, c.N, s);
    trsm_batched(d1, dw, c.ns, c.ns, false, s, nullptr);
    trsm_batched(d1, dw, c.ns, c.ns, true, s, nullptr);
    l_scale_sym(dw, c.N, nullptr, nullptr, false, true, s);
    if (c.opt.local_prec != AWG_LOCAL_F64) build_reduced_local(c, c.Pw, c.P32w, c.P16w, c.p16_sp_w);
    sync(c);
  }
}

__global__ void k_get_diag(const double* M, int n, double* d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = M[i + (long)i * n];
}

// rows of deleted columns of the factor: zero left of the diagonal
__global__ void k_zero_dropped_rows(double* L, int n, const int* dropped) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int r = (int)(e % n), c = (int)(e / n);
  if (c < r && dropped[r]) L[e] = 0.0;
}

// rows and columns of deleted indices of the inverse
__global__ void k_zero_dropped_rc(double* M, int n, const int* dropped) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int r = (int)(e % n), c = (int)(e / n);
  if (dropped[r] || dropped[c]) M[e] = 0.0;
}

// Pseudo-inverse of a dense symmetric positive semi-definite Gram matrix M
// (n x n, destroyed) of a possibly dependent basis: Cholesky with deletion of
// every column whose pivot is <= 1e-10 times its diagonal (its basis vector
// lies in the span of the previous ones to that relative accuracy), inverse
// of the kept principal submatrix, zero rows and columns for the deleted
// ones.  Applied as X E^+ X^T this is the projection onto the span.  Returns
// the number of deleted columns.
int spd_inverse(awg_ctx& c, double* M, int n, DBuf<double>& Minv, const char* what, double* margin = nullptr) {
  hipStream_t s = c.s;
  Minv.alloc((long)n * n);
  DBuf<MatDesc> dm, di;
  dm.upload({MatDesc{M, n, n, n, 0}}, s);
  di.upload({MatDesc{Minv.p, n, n, n, 0}}, s);
  l_scale_sym(dm, 1, nullptr, nullptr, false, true, s);
  DBuf<double> d0, pv;
  DBuf<int> info, drop;
  d0.alloc(n);
  pv.alloc(n);
  drop.alloc(n);
  drop.zero(s);
  hipLaunchKernelGGL(k_get_diag, dim3(cdiv(n, 256)), dim3(256), 0, s, M, n, d0.p);
  AWG_LAUNCH_CHECK();
  info.alloc(1);
  info.zero(s);
  potrf_batched(dm, {n}, info, s, nullptr, d0, drop, GRAM_DROP_TOL, pv.p);
  check_info(c, info, what);
  const unsigned g = cdiv((long)n * n, 256);
  hipLaunchKernelGGL(k_zero_dropped_rows, dim3(g), dim3(256), 0, s, M, n, drop.p);
  AWG_LAUNCH_CHECK();
  l_set_identity(di, 1, s);
  trsm_batched(dm, di, {n}, {n}, false, s, nullptr);
  trsm_batched(dm, di, {n}, {n}, true, s, nullptr);
  l_scale_sym(di, 1, nullptr, nullptr, false, true, s);
  hipLaunchKernelGGL(k_zero_dropped_rc, dim3(g), dim3(256), 0, s, Minv.p, n, drop.p);
  AWG_LAUNCH_CHECK();
  int nd = 0;
  const std::vector<int> hd = drop.download(s);
  const std::vector<double> hp = pv.download(s);
  double m = INFINITY;
  for (int k = 0; k < n; ++k) {
    nd += hd[k];
    if (!hd[k]) m = std::min(m, hp[k] / GRAM_DROP_TOL);
    else if (hp[k] > 0.0) m = std::min(m, GRAM_DROP_TOL / hp[k]);
  }
  if (margin) *margin = m;
  return nd;
}

// Jacobi scale of a Gram matrix; a vanishing (or, by rounding, negative)
// diagonal entry keeps scale 1, so its zero row and column stay zero and the
// direction is deflated or deleted instead of producing Inf / NaN
__global__ void k_sqrt_diag(const double* M, int n, double* d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double v = M[i + (long)i * n];
    d[i] = v > 0.0 ? sqrt(v) : 1.0;
  }
}

// Pseudo-inverse of a Gram matrix E (n x n, destroyed) of a basis whose
// dependence its Cholesky pivots do not reveal (a combination of many
// columns, each far from the span of the previous ones): with the Jacobi
// scaling Es = S^-1 E S^-1 (unit diagonal) and the eigenvectors Z of Es with
// eigenvalue below 1e-10, E^+ = S^-1 ((Es + Z Z^T)^-1 - Z Z^T) S^-1 (the
// inverse on the complement of the near-null combinations, zero on them;
// the inverse itself by spd_inverse).  Returns the number of deflated and
// deleted directions.
int deflated_inverse(awg_ctx& c, double* E, int n, DBuf<double>& Einv, const char* what, double* margin = nullptr) {
  hipStream_t s = c.s;
  constexpr int KMAX = 64;
  DBuf<double> sc, Et, lam, Z;
  sc.alloc(n);
  hipLaunchKernelGGL(k_sqrt_diag, dim3(cdiv(n, 256)), dim3(256), 0, s, E, n, sc.p);
  AWG_LAUNCH_CHECK();
  DBuf<long> off0;
  off0.upload({0L}, s);
  DBuf<MatDesc> dm;
  dm.upload({MatDesc{E, n, n, n, 0}}, s);
  l_scale_sym(dm, 1, off0, sc, true, true, s);                              // Es
  Et.alloc((long)n * n);
  AWG_HIP(hipMemcpyAsync(Et.p, E, sizeof(double) * n * n, hipMemcpyDeviceToDevice, s));
  lam.alloc(KMAX);
  Z.alloc((long)n * KMAX);
  int32_t k = 0;
  const int rc = awg_dense_low_eigs(1, n, Et.p, n, 0, 1e-10, KMAX, &k, lam.p, Z.p, 0, s);
  if (rc == AWG_ERR_ARG)
    throw Error(AWG_ERR_NOT_SPD, std::string(what) + ": more near-null directions than the deflation keeps (64)");
  if (rc != AWG_OK)
    throw Error(rc, std::string(what) + ": the low-eigenpair solve of the scaled matrix failed (status " +
                        std::to_string(rc) + ")");
  DBuf<GemmDesc> dg;
  if (k > 0) {
    dg.upload({GemmDesc{Z.p, Z.p, E, n, n, k, n, n, n}}, s);
    gemm_batched(dg, 1, n, n, false, true, 1.0, 1.0, false, s, 2.0 * n * (double)n * k);   // Es + Z Z^T
  }
  const int nd = spd_inverse(c, E, n, Einv, what, margin);
  if (k > 0) {
    dg.upload({GemmDesc{Z.p, Z.p, Einv.p, n, n, k, n, n, n}}, s);
    gemm_batched(dg, 1, n, n, false, true, -1.0, 1.0, false, s, 2.0 * n * (double)n * k);  // - Z Z^T
  }
  DBuf<MatDesc> di;
  di.upload({MatDesc{Einv.p, n, n, n, 0}}, s);
  l_scale_sym(di, 1, off0, sc, true, true, s);                              // S^-1 (.) S^-1
  sync(c);
  return nd + k;
}

// number of columns per pass: at most cap (even), balanced over the passes and
// rounded up to even (16-byte rows for the vectorised gather / scatter); the
// columns past the total are kept at zero
int balanced_chunk(int total, int cap) {
  const int passes = (total + cap - 1) / cap;
  const int b = (total + passes - 1) / passes;
  return std::min(cap, b + (b & 1));
}

// CSR forms of [A | V_-] and R0^T for the multi-column products (built once
// V^s and Y^s are known)
void build_prolongations(awg_ctx& c) {
  hipStream_t s = c.s;
  if (c.LV.cols > 0) {
    c.aug_nnz = l_aug_csr((int)c.n, c.rowptr, c.col, c.val, c.invptr, c.invsub, c.invloc, c.subptr, c.LV.d_eoff,
                          c.LV.d_coff, c.V, (int)c.n, c.aug_rp, c.aug_col, c.aug_val, s);
    spmm_groups_defer((int)c.n, c.aug_nnz, c.aug_rp, c.aug_col, c.aug_val, c.aug_grp);
    c.vt_nnz = l_aug_csr_t(c.N, c.LV.cols, c.subptr, c.subidx, c.LV.d_eoff, c.LV.d_coff, c.V, c.vt_rp, c.vt_col,
                           c.vt_val, s);
  }
  if (c.n0 > 0) {
    c.y_nnz = l_aug_csr((int)c.n, nullptr, nullptr, nullptr, c.invptr, c.invsub, c.invloc, c.subptr, c.LY.d_eoff,
                        c.LY.d_coff, c.Y, 0, c.y_rp, c.y_col, c.y_val, s);
    spmm_groups_defer((int)c.n, c.y_nnz, c.y_rp, c.y_col, c.y_val, c.y_grp);
    c.yt_nnz = l_aug_csr_t(c.N, c.LY.cols, c.subptr, c.subidx, c.LY.d_eoff, c.LY.d_coff, c.Y, c.yt_rp, c.yt_col,
                           c.yt_val, s);
  }
  // A_+ R0^T for H2 on many columns (the bitsets of the extended sets take
  // N n / 8 bytes while they are built)
  c.ap_ok = false;
  if (c.n0 > 0 && c.LV.cols > 0 && (double)c.N * (double)c.n / 8.0 <= 1.0e9) {
    const int n = (int)c.n;
    const long next = l_ext_sets(c.N, n, c.subptr, c.subidx, c.rowptr, c.col, c.h_extptr, c.extptr, c.extidx, s);
    std::vector<int> ne(c.N);
    c.flAY1 = 0.0;
    for (int t = 0; t < c.N; ++t) {
      ne[t] = (int)(c.h_extptr[t + 1] - c.h_extptr[t]);
      c.flAY1 += 2.0 * ne[t] * c.ms[t];
    }
    c.LAY.build(ne, c.ms, s);
    c.AY.alloc(std::max<long>(1, c.LAY.elems));
    l_ext_ay(c.N, c.extptr, c.extidx, c.subptr, c.subidx, c.rowptr, c.col, c.val, c.Y, c.LY.d_eoff, c.LY.d_coff,
             c.LAY.d_eoff, c.AY, s);
    // inverse map of the extended sets, the CSR of A R0^T, then [A R0^T | V_-]
    DBuf<int> em, einvptr, einvsub, einvloc, fill;
    em.alloc(n);
    em.zero(s);
    l_mult(next, c.extidx, em, s);
    einvptr.alloc(n + 1);
    l_scan(n, em, einvptr, s);
    fill.alloc(n);
    fill.zero(s);
    einvsub.alloc(std::max(1L, next));
    einvloc.alloc(std::max(1L, next));
    l_fill_inv(c.N, c.extptr, c.extidx, einvptr, fill, einvsub, einvloc, s);
    l_sort_inv(n, einvptr, einvsub, einvloc, s);
    DBuf<int> arp, acol;
    DBuf<double> aval;
    l_aug_csr(n, nullptr, nullptr, nullptr, einvptr, einvsub, einvloc, c.extptr, c.LAY.d_eoff, c.LAY.d_coff, c.AY, 0,
              arp, acol, aval, s);
    c.apv_nnz = l_aug_csr(n, arp, acol, aval, c.invptr, c.invsub, c.invloc, c.subptr, c.LV.d_eoff, c.LV.d_coff, c.V,
                          c.n0, c.apv_rp, c.apv_col, c.apv_val, s);
    spmm_groups_defer(n, c.apv_nnz, c.apv_rp, c.apv_col, c.apv_val, c.apv_grp);
    // C = V_-^T R0^T: the rows of R0 (CSR of its transpose) applied to the dense
    // V_-, i.e. R0 V_- (n0 x sum k_s row-major) = C column-major
    // (in slabs of at most 256 columns of V_-)
    const long nk = c.LV.cols, cw = std::min<long>(nk, 256);
    DBuf<double> Vd, Cs;
    Vd.alloc((size_t)n * cw);
    Cs.alloc((size_t)c.n0 * cw);
    c.Cmat.alloc((size_t)c.n0 * nk);
    for (long c0 = 0; c0 < nk; c0 += cw) {
      const long w = std::min(cw, nk - c0);
      AWG_HIP(hipMemsetAsync(Vd.p, 0, sizeof(double) * n * (size_t)w, s));
      l_lowrank_dense(n, c.invptr, c.invsub, c.invloc, c.subptr, c.LV.d_eoff, c.LV.d_coff, c.V, c0, w, Vd, s);
      l_spmm(c.n0, c.yt_nnz, c.yt_rp, c.yt_col, c.yt_val, Vd, Cs, (int)w, 1.0, 0.0, s);
      AWG_HIP(hipMemcpy2DAsync(c.Cmat.p + c0, sizeof(double) * nk, Cs.p, sizeof(double) * w, sizeof(double) * w,
                               c.n0, hipMemcpyDeviceToDevice, s));
    }
    sync(c);
    c.ap_ok = true;
  }
}

// E0 = R0 A_+ R0^T and its inverse (Theorem on H^NN_hyb, Section 3.4)
void phase_coarse0(awg_ctx& c) {
  PhaseTimer t(c, "coarse0");
  build_prolongations(c);
  if (c.n0 == 0) return;
  hipStream_t s = c.s;
  const int b = balanced_chunk(c.n0, 2048);
  MultiWS w;
  build_ws(c, w, b);
  DBuf<double> E0;
  E0.alloc((long)c.n0 * c.n0);
  for (int c0 = 0; c0 < c.n0; c0 += b) {
    const int bc = std::min(b, c.n0 - c0);
    hipLaunchKernelGGL(k_identity_cols, dim3(cdiv((long)c.n0 * b, 256)), dim3(256), 0, s, w.G1.p, c.n0, b, c0);
    AWG_LAUNCH_CHECK();
    op_r0t(c, w, w.T1, 0.0);          // R0^T e_j
    op_aplus(c, w, w.T1, w.T2);       // A_+ R0^T e_j
    op_r0(c, w, w.T2);                // R0 A_+ R0^T e_j  -> G0 (n0 x b)
    // E0 is symmetric: row r of G0 holds E0[r, c0 + c]; store as column-major E0 rows
    hipLaunchKernelGGL(k_copy_cols, dim3(cdiv((long)c.n0 * bc, 256)), dim3(256), 0, s, w.G0.p, b, E0.p,
                       (long)c.n0, (long)c.n0, c0, bc);
    AWG_LAUNCH_CHECK();
  }
  // the two-pencil basis of H^AS_hyb can be dependent across subdomains in a
  // way no pivot shows; the other coarse spaces keep the pivoted deletion
  c.n0_dropped = c.opt.h2 == AWG_H2_AS_HYB
                     ? deflated_inverse(c, E0, c.n0, c.E0inv, "coarse matrix E0", &c.e0_margin)
                     : spd_inverse(c, E0, c.n0, c.E0inv, "coarse matrix E0", &c.e0_margin);
}

// W = A_+^{-1} [R^1T V^1_- | ... ] (strictly negative pairs; Remark 1 and 2,
// Section 4.4) by PCG on A_+ preconditioned with H2, all columns side by
// side, each with its own recurrence and stopping test.  W is stored
// row-major: the n_minus values of a dof are contiguous.
void phase_W(awg_ctx& c) {
  PhaseTimer t(c, "second_coarse_W");
  c.nminus = 0;
  for (int q = 0; q < c.N; ++q) c.nminus += c.kstrict[q];
  if (c.nminus == 0) return;
  hipStream_t s = c.s;
  std::vector<long> gcoff(c.N + 1, 0);
  for (int q = 0; q < c.N; ++q) gcoff[q + 1] = gcoff[q] + c.kstrict[q];
  DBuf<long> dgcoff;
  dgcoff.upload(gcoff, s);
  c.W.alloc((long)c.n * c.nminus);
  const int b0 = balanced_chunk(c.nminus, 2048);
  MultiWS w;
  build_ws(c, w, b0, true);
  DBuf<double> X, Pm, Q, Zold, tmp;
  DBuf<double> alpha_d;
  alpha_d.alloc(b0);
  const bool f32 = c.opt.local_prec != AWG_LOCAL_F64;
  int itmax = 0;
  double colits = 0.0;
  // the multi-vectors at the current width b (columns compacted as they converge)
  // (allocated once at the full width; narrower widths reuse them)
  auto alloc_vectors = [&](int b) {
    X.ensure((long)c.n * b);
    Pm.ensure(((long)c.n + c.LV.cols) * b);     // input of A_+ products (coefficient rows below)
    Q.ensure((long)c.n * b);
    // Zold takes turns with the workspace's Z (same size), so it needs the
    // coefficient rows below the n rows that op_aplus may write into Z
    if (f32) Zold.ensure(((long)c.n + c.LV.cols) * b);
    tmp.ensure(((long)c.n + c.LV.cols) * b);    // target of the column compaction
  };
  alloc_vectors(b0);
  DBuf<int> dpos, ddst;
  // write the columns pos[] of X (width b) into W at the original columns dst[]
  auto write_cols = [&](int b, const std::vector<int>& pos, const std::vector<int>& dst) {
    if (pos.empty()) return;
    dpos.upload(pos, s);
    ddst.upload(dst, s);
    hipLaunchKernelGGL(k_copy_cols_list, dim3(cdiv((long)c.n * pos.size(), 256)), dim3(256), 0, s, (long)c.n, b,
                       X.p, dpos.p, ddst.p, (int)pos.size(), c.W.p, (long)c.nminus);
    AWG_LAUNCH_CHECK();
    sync(c);   // pos / dst are host vectors of the caller
  };
  for (int c0 = 0; c0 < c.nminus; c0 += b0) {
    const int bc = std::min(b0, c.nminus - c0);
    int b = b0;
    if (w.b != b0) {
      build_ws(c, w, b0, true);
      alloc_vectors(b0);
    }
    double* dots = w.dots.p;
    // colid[j]: the W column held at position j (-1: padding)
    std::vector<int> colid(b);
    for (int j = 0; j < b; ++j) colid[j] = j < bc ? c0 + j : -1;
    auto coldot = [&](const double* A, const double* B) {
      l_coldot(c.n, b, A, B, w.dotpart, dots, s);
      std::vector<double> h(b);
      AWG_HIP(hipMemcpyAsync(h.data(), dots, sizeof(double) * b, hipMemcpyDeviceToHost, s));
      AWG_HIP(hipStreamSynchronize(s));
      return h;
    };
    std::vector<double> bn(b), rz(b), alpha(b), beta(b);
    std::vector<char> active(b);
    w.R.zero(s);
    hipLaunchKernelGGL(k_build_vg, dim3(64, c.N), dim3(256), 0, s, c.subptr.p, c.subidx.p, c.V.p, c.LV.d_eoff.p,
                       dgcoff.p, w.R.p, c0, b);
    AWG_LAUNCH_CHECK();
    auto h = coldot(w.R, w.R);
    for (int j = 0; j < b; ++j) {
      bn[j] = std::sqrt(h[j]);
      active[j] = (j < bc && bn[j] > 0.0) ? 1 : 0;
    }
    X.zero(s);
    op_h2(c, w, f32);
    AWG_HIP(hipMemcpyAsync(Pm.p, w.Z.p, sizeof(double) * c.n * b, hipMemcpyDeviceToDevice, s));
    h = coldot(w.R, w.Z);
    for (int j = 0; j < b; ++j) rz[j] = h[j];
    if (f32) {
      std::swap(w.Z.p, Zold.p);   // Zold = Z
      std::swap(w.Z.n, Zold.n);
    }
    int it = 0;
    for (; it < c.opt.w_maxit; ++it) {
      op_aplus(c, w, Pm, Q);
      h = coldot(Pm, Q);
      for (int j = 0; j < b; ++j) {
        if (active[j] && !(h[j] > 0.0)) throw Error(AWG_ERR_NOT_SPD, "PCG with A_+ met p^T A_+ p <= 0");
        alpha[j] = active[j] ? rz[j] / h[j] : 0.0;
      }
      AWG_HIP(hipMemcpyAsync(alpha_d.p, alpha.data(), sizeof(double) * b, hipMemcpyHostToDevice, s));
      // X += alpha P, R -= alpha Q and the new ||R_j||^2 in one pass
      l_multi_update_xr(c.n, b, alpha_d, Pm, X, Q, w.R, w.dotpart, dots, s);
      AWG_HIP(hipMemcpyAsync(h.data(), dots, sizeof(double) * b, hipMemcpyDeviceToHost, s));
      AWG_HIP(hipStreamSynchronize(s));
      int nact = 0;
      for (int j = 0; j < b; ++j) {
        if (active[j] && std::sqrt(h[j]) <= c.opt.w_rtol * bn[j]) {
          active[j] = 0;
          colits += it + 1;
        }
        nact += active[j];
      }
      if (nact == 0) { ++it; break; }
      // compaction: once a quarter of the width (at least 128 columns) has
      // converged, the converged columns are written to W and the active ones
      // moved to the front of narrower multi-vectors.  Every kernel computes
      // each column independently of the others and of its position, so the
      // iterates are those of the full width, bit for bit.
      const int bnew = nact + (nact & 1);   // even widths keep the 16-byte paths
      if (g_w_compaction && b - bnew >= std::max(128, b / 4)) {
        std::vector<int> pos, dst, perm;
        for (int j = 0; j < b; ++j) {
          if (active[j]) perm.push_back(j);
          else if (colid[j] >= 0) { pos.push_back(j); dst.push_back(colid[j]); }
        }
        write_cols(b, pos, dst);
        for (int j = 0; (int)perm.size() < bnew; ++j)   // padding: an inactive position
          if (!active[j]) perm.push_back(j);
        DBuf<int> dperm;
        dperm.upload(perm, s);
        // each multi-vector is gathered into the spare buffer, which then
        // takes its place (every buffer keeps its full-width allocation)
        auto gather = [&](DBuf<double>& A) {
          if (tmp.n < A.n) tmp.alloc(A.n);
          hipLaunchKernelGGL(k_gather_cols, dim3(cdiv((long)c.n * bnew, 256)), dim3(256), 0, s, (long)c.n, b, A.p,
                             bnew, dperm.p, tmp.p);
          AWG_LAUNCH_CHECK();
          std::swap(A.p, tmp.p);
          std::swap(A.n, tmp.n);
        };
        gather(Pm);   // the largest first: the spare buffer then fits every other one
        gather(X);
        gather(w.R);
        if (f32) gather(Zold);
        sync(c);
        build_ws(c, w, bnew, true);   // descriptors at the new width; R and the buffers are kept
        dots = w.dots.p;
        std::vector<int> cid(bnew), act(bnew);
        std::vector<double> bn2(bnew), rz2(bnew);
        for (int j = 0; j < bnew; ++j) {
          const int o = perm[j];
          const bool pad = j >= nact;
          cid[j] = pad ? -1 : colid[o];
          act[j] = pad ? 0 : 1;
          bn2[j] = bn[o];
          rz2[j] = rz[o];
        }
        colid.swap(cid);
        bn.swap(bn2);
        rz.swap(rz2);
        active.assign(act.begin(), act.end());
        b = bnew;
        ++c.w_compactions;
        alpha.assign(b, 0.0);
        beta.assign(b, 0.0);
        h.assign(b, 0.0);
      }
      op_h2(c, w, f32);
      // r^T z and, for the FP32 local operators, r^T z_old (flexible
      // Polak-Ribiere beta) in one pass over R
      l_coldot2(c.n, b, w.R, w.Z, f32 ? Zold.p : nullptr, w.dotpart, dots, dots + b, s);
      std::vector<double> h2((f32 ? 2 : 1) * (size_t)b);
      AWG_HIP(hipMemcpyAsync(h2.data(), dots, sizeof(double) * h2.size(), hipMemcpyDeviceToHost, s));
      AWG_HIP(hipStreamSynchronize(s));
      for (int j = 0; j < b; ++j) {
        const double num = f32 ? h2[j] - h2[b + j] : h2[j];
        beta[j] = active[j] ? num / rz[j] : 0.0;
        if (active[j]) rz[j] = h2[j];
      }
      AWG_HIP(hipMemcpyAsync(alpha_d.p, beta.data(), sizeof(double) * b, hipMemcpyHostToDevice, s));
      l_multi_update_p(c.n, b, w.Z, Pm, alpha_d, nullptr, s);   // P = Z + beta P
      if (f32) {
        // this Z is the next iteration's Zold: the two buffers trade places
        // (no descriptor of the W solves' operators holds the address of Z)
        std::swap(w.Z.p, Zold.p);
        std::swap(w.Z.n, Zold.n);
      }
      sync(c);   // the host buffer of beta is reused next iteration
    }
    itmax = std::max(itmax, it);
    for (int j = 0; j < b; ++j)
      if (active[j]) throw Error(AWG_ERR_NOT_SPD, "PCG with A_+ for W did not converge within w_maxit");
    std::vector<int> pos, dst;
    for (int j = 0; j < b; ++j)
      if (colid[j] >= 0) {
        pos.push_back(j);
        dst.push_back(colid[j]);
      }
    write_cols(b, pos, dst);
  }
  c.w_iters = itmax;
  c.w_iters_mean = colits / std::max(1, c.nminus);
}

// E_W = W^T A W and its inverse (Definition of H3,ad, Section 4.3)
// capacitance C = diag(1 / L) - (D + D^T) / 2, D = W^T V_- (n_minus x n_minus)
__global__ void k_capacitance(int m, const double* D, const double* L, double* C) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)m * m) return;
  const int i = (int)(e % m), j = (int)(e / m);
  const double sym = 0.5 * (D[i + (long)j * m] + D[j + (long)i * m]);
  C[e] = (i == j ? 1.0 / L[i] : 0.0) - sym;
}

// C = L_-^{-1} - V_-^T W of H3,inex (Theorem on the AWG preconditioner with
// inexact coarse space, Section 4.2) and its inverse (kept in EWinv, applied
// like E_W^{-1}); L_- = |strictly negative eigenvalues| of the columns of V_-
void phase_capacitance(awg_ctx& c) {
  hipStream_t s = c.s;
  const int nm = c.nminus;
  std::vector<long> gcoff(c.N + 1, 0);
  for (int q = 0; q < c.N; ++q) gcoff[q + 1] = gcoff[q] + c.kstrict[q];
  // D[:, gcoff[q] + j] = sum_k W[sub_idx[k], :] V^q[k, j]  (restricted rows of W read in place)
  DBuf<double> D, C, L;
  D.alloc((long)nm * nm);
  C.alloc((long)nm * nm);
  std::vector<GemmDesc> h(c.N);
  int maxk = 0;
  double fl = 0.0;
  for (int q = 0; q < c.N; ++q) {
    h[q] = GemmDesc{nullptr, c.V.p + c.LV.eoff[q], D.p + gcoff[q] * nm, nm, c.kstrict[q], c.ns[q], nm, c.ns[q], nm};
    maxk = std::max(maxk, c.kstrict[q]);
    fl += 2.0 * nm * (double)c.kstrict[q] * c.ns[q];
  }
  DBuf<GemmDesc> dg;
  dg.upload(h, s);
  gemm_batched_gather(dg, c.W, c.subidx.p, c.subptr.p, c.N, nm, maxk, false, 1.0, 0.0, s, fl, "VgW");
  // |lambda| of the strictly negative eigenpairs (the first kstrict of each subdomain)
  const std::vector<double> lam = c.lamV.download(s);
  std::vector<double> hl;
  hl.reserve(nm);
  for (int q = 0; q < c.N; ++q)
    for (int j = 0; j < c.kstrict[q]; ++j) hl.push_back(std::fabs(lam[c.LV.coff[q] + j]));
  L.upload(hl, s);
  hipLaunchKernelGGL(k_capacitance, dim3(cdiv((long)nm * nm, 256)), dim3(256), 0, s, nm, D.p, L.p, C.p);
  AWG_LAUNCH_CHECK();
  c.nminus_dropped = spd_inverse(c, C, nm, c.EWinv, "capacitance matrix L^-1 - V^T W", &c.ew_margin);
}

// out[i] = sum over q < parts of part[q * len + i], in the order of q
__global__ void k_sum_parts(long len, int parts, const double* part, double* out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double acc = 0.0;
  for (int q = 0; q < parts; ++q) acc += part[(long)q * len + i];
  out[i] = acc;
}

void phase_EW(awg_ctx& c) {
  PhaseTimer t(c, "second_coarse_EW");
  if (c.nminus == 0) return;
  if (c.opt.coarse2 == AWG_COARSE2_INEX) {
    phase_capacitance(c);
    return;
  }
  hipStream_t s = c.s;
  DBuf<double> AW, EW;
  AW.alloc((long)c.n * c.nminus);
  EW.alloc((long)c.nminus * c.nminus);
  // A W, once per set-up: without the row groups, whose construction would
  // cost more than the one product gains from them
  l_spmm(c.n, c.nnz, c.rowptr, c.col, c.val, c.W.p, AW.p, c.nminus, 1.0, 0.0, s, nullptr, "k_spmm:AW");
  // E_W = W^T (A W): column-major views W_rm (n_minus x n) and AW_rm -> W_rm AW_rm^T,
  // the long k = n split into KS ranges (batch entries writing partial
  // products, summed in a fixed order) so that the launch fills the device
  const int KS = (int)std::max<long>(1, std::min<long>(16, c.n / 4096));
  const long nm2 = (long)c.nminus * c.nminus;
  DBuf<double> part;
  part.alloc(nm2 * KS);
  std::vector<GemmDesc> hg(KS);
  for (int q = 0; q < KS; ++q) {
    const long k0 = (long)c.n * q / KS, k1 = (long)c.n * (q + 1) / KS;
    hg[q] = GemmDesc{c.W.p + k0 * c.nminus, AW.p + k0 * c.nminus, part.p + q * nm2, c.nminus, c.nminus,
                     (int)(k1 - k0), c.nminus, c.nminus, c.nminus};
  }
  DBuf<GemmDesc> g;
  g.upload(hg, s);
  gemm_batched(g, KS, c.nminus, c.nminus, false, true, 1.0, 0.0, false, s, 2.0 * c.n * (double)c.nminus * c.nminus,
               "EW");
  hipLaunchKernelGGL(k_sum_parts, dim3(cdiv(nm2, 256)), dim3(256), 0, s, nm2, KS, part.p, EW.p);
  AWG_LAUNCH_CHECK();
  c.nminus_dropped = spd_inverse(c, EW, c.nminus, c.EWinv, "second coarse matrix W^T A W", &c.ew_margin);
}

void do_setup(awg_ctx& c, const int64_t* rowptr, const int32_t* col, const double* val, const int64_t* sub_ptr,
              const int32_t* sub_idx) {
  const double t0 = now_ms();
  phase_maps(c, rowptr, col, val, sub_ptr, sub_idx);
  phase_local(c);
  phase_coarse0(c);
  {
    // the W solves and the main solves use H2 / H with the workspace below
  }
  phase_W(c);
  phase_EW(c);
  {
    PhaseTimer t(c, "workspace");
    build_ws(c, c.ws1, 1);
    c.pcg_buf.alloc(3L * c.n);
  }
  sync(c);
  c.tms["total"] = now_ms() - t0;
}

// host-side symmetric tridiagonal extremes (Lanczos estimate from the PCG
// coefficients; diagnostics only)
void lanczos_extremes(const std::vector<double>& al, const std::vector<double>& be, double& lmin, double& lmax) {
  const int k = (int)al.size();
  if (k == 0) { lmin = lmax = NAN; return; }
  std::vector<double> d(k), e(k > 1 ? k - 1 : 1, 0.0);
  for (int j = 0; j < k; ++j) {
    d[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j + 1 < k) e[j] = std::sqrt(std::max(0.0, be[j])) / al[j];
  }
  auto count = [&](double x) {
    int cnum = 0;
    double q = d[0] - x;
    if (q == 0.0) q = -1e-300;
    if (q < 0) ++cnum;
    for (int i = 1; i < k; ++i) {
      q = d[i] - x - e[i - 1] * e[i - 1] / q;
      if (q == 0.0) q = -1e-300;
      if (q < 0) ++cnum;
    }
    return cnum;
  };
  double gl = 1e300, gu = -1e300;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(e[i]) : 0.0);
    gl = std::min(gl, d[i] - r);
    gu = std::max(gu, d[i] + r);
  }
  auto bis = [&](int idx) {
    double lo = gl, hi = gu;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (count(mid) <= idx) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
  };
  lmin = bis(0);
  lmax = bis(k - 1);
}

// one PCG iteration (device-side control; see k_pcg_alpha)
void pcg_iteration(awg_ctx& c, bool f32) {
  MultiWS& w = c.ws1;
  const int n = c.n;
  hipStream_t s = c.s;
  double* xx = c.pcg_buf.p;
  double* p = xx + n;
  double* q = p + n;
  double* sc = c.scal.p;
  const unsigned g = cdiv(n, 256);
  double* part = w.dotpart.p;      // DOT1_BLOCKS partial sums, reused by the three dot products
  l_spmv_dot(n, c.nnz, c.rowptr, c.col, c.val, p, q, part, s);                    // q = A p, parts of p^T q
  hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(256), 0, s, sc, part);
  {
    KScope kt("k_pcg_update_xr", s, 48.0 * n, 6.0 * n);
    hipLaunchKernelGGL(k_pcg_update_xr, dim3(DOT1_BLOCKS), dim3(256), 0, s, n, xx, w.R.p, p, q, sc, part);
  }
  hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(256), 0, s, sc, part);
  op_h(c, w, f32);
  l_dot1_part(n, w.R, w.Z, part, s);                                               // parts of r^T z
  hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(256), 0, s, sc, part);
  hipLaunchKernelGGL(k_pcg_update_p, dim3(g), dim3(256), 0, s, n, p, w.Z.p, sc);
  AWG_LAUNCH_CHECK();
}

constexpr int PCG_HIST = 4096;     // capacity of the alpha/beta history
constexpr int PCG_AHEAD = 4;       // iterations launched between two host checks
constexpr int PCG_MAX_RESTARTS = 5;

int do_pcg(awg_ctx& c, const double* b, double* x, double tol, int maxit, awg_pcg_info* info) {
  hipStream_t s = c.s;
  MultiWS& w = c.ws1;
  const bool f32 = c.opt.local_prec != AWG_LOCAL_F64;
  const int n = c.n;
  maxit = std::min(maxit, PCG_HIST - 1);
  double* xx = c.pcg_buf.p;
  double* p = xx + n;
  double* q = p + n;
  if (!c.scal.p) c.scal.alloc(16 + 2 * (size_t)PCG_HIST + 2);
  double* sc = c.scal.p;
  AWG_HIP(hipMemsetAsync(sc, 0, sizeof(double) * 16, s));
  AWG_HIP(hipMemcpyAsync(w.R.p, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  AWG_HIP(hipMemsetAsync(xx, 0, sizeof(double) * n, s));
  l_coldot(n, 1, w.R, w.R, w.dotpart, sc + 6, s);
  double h6;
  AWG_HIP(hipMemcpyAsync(&h6, sc + 6, sizeof(double), hipMemcpyDeviceToHost, s));
  sync(c);
  const double bn = std::sqrt(h6);
  awg_pcg_info inf{};
  int status = AWG_OK;
  int it = 0;
  int first_seg = -1;     // iterations of the first segment (Lanczos estimates)
  if (bn == 0.0 || maxit <= 0) {
    inf.converged = bn == 0.0;
    inf.rel_res = bn == 0.0 ? 0.0 : 1.0;
    inf.rel_res_true = inf.rel_res;
    AWG_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    sync(c);
  } else {
    const double ctl[4] = {tol * tol * h6, 0.0, 0.0, (double)maxit};
    AWG_HIP(hipMemcpyAsync(sc + 8, ctl, sizeof(ctl), hipMemcpyHostToDevice, s));
    op_h(c, w, f32);
    AWG_HIP(hipMemcpyAsync(p, w.Z.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    l_coldot(n, 1, w.R, w.Z, w.dotpart, sc + 0, s);
    if (c.use_graph && !c.pcg_graph) {
      // capture one iteration on a private stream (default priority)
      if (!c.cap_stream) AWG_HIP(hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
      sync(c);
      hipStream_t user = c.s;
      c.s = c.cap_stream;
      ktimer_capturing(true);
      hipGraph_t graph = nullptr;
      try {
        AWG_HIP(hipStreamBeginCapture(c.s, hipStreamCaptureModeThreadLocal));
        pcg_iteration(c, f32);
        AWG_HIP(hipStreamEndCapture(c.s, &graph));
        AWG_HIP(hipGraphInstantiate(&c.pcg_graph, graph, nullptr, nullptr, 0));
        (void)hipGraphDestroy(graph);
      } catch (...) {
        hipGraph_t g2 = nullptr;
        (void)hipStreamEndCapture(c.s, &g2);
        if (g2) (void)hipGraphDestroy(g2);
        if (graph) (void)hipGraphDestroy(graph);
        c.pcg_graph = nullptr;
        c.use_graph = 0;                  // fall back to eager launches of the same kernels
        (void)hipGetLastError();
      }
      ktimer_capturing(false);
      c.s = user;
    }
    double hs[12];
    for (;;) {
      for (;;) {
        for (int k = 0; k < PCG_AHEAD; ++k) {
          if (c.pcg_graph) {
            KScope kt("graph:pcg_iteration", s, 0.0, 0.0);
            AWG_HIP(hipGraphLaunch(c.pcg_graph, s));
          } else {
            pcg_iteration(c, f32);
          }
        }
        AWG_HIP(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, s));
        sync(c);
        if (hs[9] != 0.0) break;
      }
      it = (int)hs[10];
      if (first_seg < 0) first_seg = it;
      inf.rel_res = std::sqrt(hs[5]) / bn;
      if (hs[9] == 2.0) {
        status = AWG_ERR_NOT_SPD;
        c.err = "PCG breakdown: p^T A p <= 0 (A or H not spd)";
        break;
      }
      // true residual q = b - A x, evaluated in compensated arithmetic (the
      // FP64 evaluation error eps sum_j |A_ij x_j| can exceed tol ||b|| on
      // ill-conditioned systems)
      l_resid_dd(n, c.nnz, c.rowptr, c.col, c.val, xx, b, q, s);
      l_coldot(n, 1, q, q, w.dotpart, sc + 7, s);
      double h7;
      AWG_HIP(hipMemcpyAsync(&h7, sc + 7, sizeof(double), hipMemcpyDeviceToHost, s));
      sync(c);
      inf.rel_res_true = std::sqrt(h7) / bn;
      inf.converged = hs[9] == 1.0 && inf.rel_res_true <= tol;
      if (hs[9] != 1.0 || inf.converged || inf.restarts >= PCG_MAX_RESTARTS) break;
      // the recursive residual met tol but the true one did not (finite
      // precision drift): restart the recurrence from the true residual
      ++inf.restarts;
      AWG_HIP(hipMemcpyAsync(w.R.p, q, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      op_h(c, w, f32);
      AWG_HIP(hipMemcpyAsync(p, w.Z.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      l_coldot(n, 1, w.R, w.Z, w.dotpart, sc + 0, s);
      const double zero = 0.0;
      AWG_HIP(hipMemcpyAsync(sc + 9, &zero, sizeof(double), hipMemcpyHostToDevice, s));
      sync(c);
    }
    if (status == AWG_OK) {
      AWG_HIP(hipMemcpyAsync(x, xx, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      const int nh = std::max(first_seg, 1);
      std::vector<double> hist(16 + 2 * (size_t)nh + 2);
      AWG_HIP(hipMemcpyAsync(hist.data(), sc, sizeof(double) * hist.size(), hipMemcpyDeviceToHost, s));
      sync(c);
      std::vector<double> al, be;
      for (int j = 0; j < first_seg; ++j) al.push_back(hist[16 + 2 * j]);
      for (int j = 0; j + 1 < first_seg; ++j) be.push_back(hist[17 + 2 * j]);
      lanczos_extremes(al, be, inf.lmin_est, inf.lmax_est);
    }
  }
  inf.iters = it;
  inf.iters_first = first_seg < 0 ? it : first_seg;
  if (status == AWG_OK && !inf.converged) status = AWG_NOT_CONVERGED;
  if (info) *info = inf;
  return status;
}

std::string stats_json(const awg_ctx& c) {
  std::ostringstream o;
  o.precision(17);
  auto arr = [&](const char* k, const std::vector<int>& v) {
    o << "\"" << k << "\":[";
    for (size_t i = 0; i < v.size(); ++i) o << (i ? "," : "") << v[i];
    o << "]";
  };
  o << "{\"n\":" << c.n << ",\"nnz\":" << c.nnz << ",\"N\":" << c.N << ",\"sum_ns\":" << c.sumns
    << ",\"n_minus\":" << c.nminus << ",\"n0\":" << c.n0 << ",\"w_iters\":" << c.w_iters << ",\"w_iters_mean\":" << c.w_iters_mean << ",\"w_compactions\":" << c.w_compactions << ",\"w_factor_fallbacks\":" << c.w_factor_fallbacks
    << ",\"local_prec\":" << c.opt.local_prec << ",\"tau\":" << c.opt.tau << ",";
  arr("k_s", c.ks);
  o << ",";
  arr("kstrict_s", c.kstrict);
  o << ",";
  arr("m_s", c.ms);
  o << ",\"coarse2\":" << c.opt.coarse2 << ",\"h2\":" << c.opt.h2 << ",\"w_h2\":" << c.wmode;
  o << ",\"geneo_solver\":" << c.opt.geneo_solver << ",\"eig_fallbacks\":" << c.eig_fallbacks
    << ",\"eig_learned\":" << c.eig_learned << ",\"eig_block\":" << c.opt.eig_block
    << ",\"n0_dropped\":" << c.n0_dropped << ",\"nminus_dropped\":" << c.nminus_dropped;
  // JSON has no infinity: a margin without any decision near the threshold is written as 1e300
  o << ",\"e0_margin\":" << std::min(c.e0_margin, 1e300) << ",\"ew_margin\":" << std::min(c.ew_margin, 1e300) << ",";
  arr("eig_iters", c.eig_iters);
  o << ",\"eig_resid_max\":[";
  for (size_t i = 0; i < c.eig_resid_max.size(); ++i) o << (i ? "," : "") << c.eig_resid_max[i];
  o << "],\"ms\":{";
  bool first = true;
  for (auto& kv : c.tms) {
    o << (first ? "" : ",") << "\"" << kv.first << "\":" << kv.second;
    first = false;
  }
  o << "}}";
  return o.str();
}

int fail(awg_ctx* c, const Error& e) {
  if (c) c->err = e.what();
  return e.code;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void awg_default_options(awg_options* opt) {
  if (!opt) return;
  opt->tau = 0.1;
  opt->zero_tol = 1e-12;
  opt->w_rtol = 1e-10;
  opt->w_maxit = 500;
  opt->local_prec = AWG_LOCAL_F64;
  opt->stream = nullptr;
  opt->geneo_solver = AWG_GENEO_DENSE;
  opt->eig_block = 16;
  opt->eig_maxit = 200;
  opt->eig_seed = 0;
  opt->eig_tol = 1e-10;
  opt->eig_init = nullptr;
  opt->coords = nullptr;
  opt->coord_dim = 0;
  opt->coarse2 = AWG_COARSE2_AD;
  opt->h2 = AWG_H2_NN_HYB;
  opt->w_h2 = AWG_H2_ASP_AD;
}

int awg_setup(awg_ctx** out, int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col, const double* val,
              int32_t nsub, const int64_t* sub_ptr, const int32_t* sub_idx, const awg_options* opt) {
  if (!out) {
    g_setup_error = "awg_setup: out is NULL";
    return AWG_ERR_ARG;
  }
  *out = nullptr;
  awg_options o;
  awg_default_options(&o);
  if (opt) o = *opt;
  if (n <= 0 || n >= (1L << 31) || nnz <= 0 || nnz >= (1L << 31) || nsub <= 0 || !rowptr || !col || !val ||
      !sub_ptr || !sub_idx) {
    g_setup_error = "awg_setup: invalid sizes or NULL pointer";
    return AWG_ERR_ARG;
  }
  if (!(o.tau > 0.0 && o.tau < 1.0)) {
    g_setup_error = "awg_setup: tau must lie in (0, 1)";
    return AWG_ERR_ARG;
  }
  if (!(o.zero_tol >= 0.0) || !(o.w_rtol > 0.0) || o.w_maxit <= 0 ||
      (o.local_prec != AWG_LOCAL_F64 && o.local_prec != AWG_LOCAL_F32 && o.local_prec != AWG_LOCAL_F16X3) ||
      (o.geneo_solver != AWG_GENEO_DENSE && o.geneo_solver != AWG_GENEO_SUBSPACE) || o.eig_block < 1 ||
      o.eig_block > SUBSPACE_MAX_BLOCK || o.eig_maxit < 1 || !(o.eig_tol > 0.0) ||
      (o.coords && (o.coord_dim < 1 || o.coord_dim > 3)) ||
      (o.coarse2 != AWG_COARSE2_AD && o.coarse2 != AWG_COARSE2_INEX && o.coarse2 != AWG_COARSE2_HYB) ||
      (o.h2 != AWG_H2_NN_HYB && o.h2 != AWG_H2_ASP_HYB && o.h2 != AWG_H2_ASP_AD && o.h2 != AWG_H2_AS_HYB) ||
      (o.w_h2 != AWG_H2_NN_HYB && o.w_h2 != AWG_H2_ASP_HYB && o.w_h2 != AWG_H2_ASP_AD) ||
      (o.h2 == AWG_H2_AS_HYB && o.geneo_solver != AWG_GENEO_DENSE)) {
    g_setup_error = "awg_setup: invalid option value";
    return AWG_ERR_ARG;
  }
  if (o.eig_init && (o.eig_init->dims.front() != MLP_FEATURES || o.eig_init->dims.back() > o.eig_block)) {
    g_setup_error = "awg_setup: eig_init needs in_features = AWG_MLP_FEATURES and out_channels <= eig_block";
    return AWG_ERR_ARG;
  }
  awg_ctx* c = new (std::nothrow) awg_ctx();
  if (!c) {
    g_setup_error = "awg_setup: host allocation failed";
    return AWG_ERR_OOM;
  }
  c->opt = o;
  c->wmode = o.h2 == AWG_H2_NN_HYB ? o.w_h2 : o.h2;
  c->s = (hipStream_t)o.stream;
  c->n = (int)n;
  c->nnz = (int)nnz;
  c->N = nsub;
  try {
    if (o.coords) {
      c->cdim = o.coord_dim;
      c->coords.alloc((size_t)n * o.coord_dim);
      AWG_HIP(hipMemcpyAsync(c->coords.p, o.coords, sizeof(double) * n * o.coord_dim, hipMemcpyDeviceToDevice, c->s));
    }
    do_setup(*c, rowptr, col, val, sub_ptr, sub_idx);
  } catch (const Error& e) {
    g_setup_error = e.what();
    (void)hipStreamSynchronize(c->s);
    delete c;
    return e.code;
  } catch (const std::exception& e) {
    g_setup_error = e.what();
    (void)hipStreamSynchronize(c->s);
    delete c;
    return AWG_ERR_HIP;
  }
  *out = c;
  return AWG_OK;
}

int awg_apply(awg_ctx* c, const double* r, double* z) {
  if (!c || !r || !z) return AWG_ERR_ARG;
  try {
    AWG_HIP(hipMemcpyAsync(c->ws1.R.p, r, sizeof(double) * c->n, hipMemcpyDeviceToDevice, c->s));
    op_h(*c, c->ws1, c->opt.local_prec != AWG_LOCAL_F64);
    AWG_HIP(hipMemcpyAsync(z, c->ws1.Z.p, sizeof(double) * c->n, hipMemcpyDeviceToDevice, c->s));
  } catch (const Error& e) {
    return fail(c, e);
  }
  return AWG_OK;
}

int awg_pcg(awg_ctx* c, const double* b, double* x, double tol, int32_t maxit, awg_pcg_info* info) {
  if (!c || !b || !x || !(tol > 0.0) || maxit <= 0) {
    if (c) c->err = "awg_pcg: invalid argument";
    return AWG_ERR_ARG;
  }
  try {
    return do_pcg(*c, b, x, tol, maxit, info);
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int64_t awg_stats(const awg_ctx* c, char* buf, size_t cap) {
  if (!c) return AWG_ERR_ARG;
  const std::string js = stats_json(*c);
  if (buf && cap) {
    const size_t k = std::min(cap - 1, js.size());
    std::memcpy(buf, js.data(), k);
    buf[k] = '\0';
  }
  return (int64_t)js.size();
}

int64_t awg_export(const awg_ctx* c, const char* name, void* buf, size_t cap) {
  if (!c || !name) return AWG_ERR_ARG;
  const void* src = nullptr;
  size_t bytes = 0;
  const std::string nm(name);
  if (nm == "neg_eigs") { src = c->lamV.p; bytes = sizeof(double) * c->LV.cols; }
  else if (nm == "geneo_eigs") { src = c->lamY.p; bytes = sizeof(double) * c->LY.cols; }
  else if (nm == "mult") { src = c->mult.p; bytes = sizeof(int) * c->n; }
  else if (nm == "pair_count") { src = c->cnt.p; bytes = sizeof(int) * c->nnz; }
  else if (nm == "V_minus") { src = c->V.p; bytes = sizeof(double) * c->LV.elems; }
  else if (nm == "Y") { src = c->Y.p; bytes = sizeof(double) * c->LY.elems; }
  else if (nm == "P_local") { src = c->P.p; bytes = sizeof(double) * c->sqtot; }
  else if (nm == "W") { src = c->W.p; bytes = sizeof(double) * c->n * c->nminus; }
  else if (nm == "ritz_vectors") { src = c->ritzZ.p; bytes = sizeof(double) * c->sumns * c->ritz_q; }
  else if (nm == "ritz_values") { src = c->ritzMu.p; bytes = sizeof(double) * c->N * c->ritz_q; }
  else if (nm == "mlp_features") {
    bytes = sizeof(float) * c->sumns * MLP_FEATURES;
    if (buf && cap && bytes) {
      try {
        DBuf<float> f;
        f.alloc((size_t)c->sumns * MLP_FEATURES);
        l_mlp_features(c->N, c->n, c->maxns, c->subptr, c->subidx, c->rowptr, c->col, c->val, c->invptr, c->invsub,
                       c->invloc, c->mult, c->V, c->LV.d_eoff, c->LV.d_coff, c->P, c->d_sqoff, c->coords.p, c->cdim,
                       f, c->s);
        AWG_HIP(hipMemcpyAsync(buf, f.p, std::min(cap, bytes), hipMemcpyDeviceToHost, c->s));
        AWG_HIP(hipStreamSynchronize(c->s));
      } catch (const Error& e) {
        return e.code;
      }
    }
    return (int64_t)bytes;
  }
  else return AWG_ERR_ARG;
  if (buf && cap && bytes) {
    if (hipMemcpyAsync(buf, src, std::min(cap, bytes), hipMemcpyDeviceToHost, c->s) != hipSuccess ||
        hipStreamSynchronize(c->s) != hipSuccess)
      return AWG_ERR_HIP;
  }
  return (int64_t)bytes;
}

const char* awg_last_error(const awg_ctx* c) { return c ? c->err.c_str() : g_setup_error.c_str(); }

int awg_free_cached_memory(uint64_t* bytes_out) {
  const size_t b = dev_cache_trim();
  if (bytes_out) *bytes_out = (uint64_t)b;
  return AWG_OK;
}

int awg_w_compaction(int32_t enable) {
  g_w_compaction = enable != 0;
  return AWG_OK;
}

int awg_pcg_graph(awg_ctx* c, int32_t enable) {
  if (!c) return AWG_ERR_ARG;
  c->use_graph = enable ? 1 : 0;
  return AWG_OK;
}

int awg_kernel_timing_filter(const char* prefix) {
  awg::g_kt_filter = prefix ? prefix : "";
  return AWG_OK;
}

int awg_kernel_timing(int32_t enable) {
  try {
    if (!enable) awg::ktimer_json(false);   // drain pending records
  } catch (const Error& e) {
    return e.code;
  }
  awg::ktimer_enable(enable != 0);
  return AWG_OK;
}

int64_t awg_kernel_times(char* buf, size_t cap, int32_t reset) {
  std::string js;
  try {
    js = awg::ktimer_json(reset != 0);
  } catch (const Error& e) {
    return e.code;
  }
  if (buf && cap) {
    const size_t k = std::min(cap - 1, js.size());
    std::memcpy(buf, js.data(), k);
    buf[k] = '\0';
  }
  return (int64_t)js.size();
}

void awg_destroy(awg_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->s);
  delete c;
}

}  // extern "C"
