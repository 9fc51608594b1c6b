// C ABI of the batched dense building blocks (include/awg_dense.h).
#include <algorithm>
#include <cstring>
#include <mutex>

#include "awg.h"
#include "awg_common.h"
#include "awg_dense.h"
#include "awg_sparse.h"
#include "awg_tune.h"

using namespace awg;

namespace {

std::vector<MatDesc> uniform(double* A, int batch, int m, int n, int ld, long stride) {
  std::vector<MatDesc> v(batch);
  for (int b = 0; b < batch; ++b) v[b] = MatDesc{A + b * stride, m, n, ld, 0};
  return v;
}

template <class F>
int guarded(hipStream_t s, F&& f) {
  try {
    f();
    AWG_HIP(hipStreamSynchronize(s));
  } catch (const Error& e) {
    (void)hipStreamSynchronize(s);
    return e.code;
  }
  return AWG_OK;
}

__global__ void k_rowptr_to32(int n, const int64_t* in, int* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) out[i] = (int)in[i];
}

// ---------------------------------------------------------------------------
// awg_dense_potrf_noalloc: the block descriptors and the info array of one
// call live in `scratch`, a static device array of this library (one copy
// per device, held until the process ends).  In host code `scratch` names a
// host-side stand-in, never the device memory: every host use goes through
// the device address that hipGetSymbolAddress returns, cached per device.
// ---------------------------------------------------------------------------
constexpr int NOALLOC_MAX_BATCH = AWG_NOALLOC_MAX_BATCH;
constexpr size_t NOALLOC_DESC_BYTES = sizeof(MatDesc) * NOALLOC_MAX_BATCH;
constexpr size_t NOALLOC_BYTES = NOALLOC_DESC_BYTES + sizeof(int) * NOALLOC_MAX_BATCH;
static_assert(sizeof(MatDesc) == 24, "scratch size stated in awg_dense.h");
static_assert(NOALLOC_DESC_BYTES % 256 == 0, "info array must start 256-byte aligned");

__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[MAX_DEVICES] = {};

// device address of `scratch` on the current device (looked up once per device)
unsigned char* scratch_on_current_device() {
  int dev = 0;
  AWG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) throw Error(AWG_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    AWG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(AWG_ERR_HIP, "hipGetSymbolAddress returned a null address");
    g_scratch_ptr[dev] = (unsigned char*)p;
  }
  return g_scratch_ptr[dev];
}

// descriptors of a uniform batch, and a cleared info array (the array keeps
// the previous call's values)
__global__ void k_uniform_desc(MatDesc* d, int* info, double* A, int batch, int n, int lda, long stride) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) {
    d[b] = MatDesc{A + b * stride, n, n, lda, 0};
    info[b] = 0;
  }
}

}  // namespace

namespace awg {
void spmm_variant(int v, int n, const int* rowptr, const int* col, const double* val, const double* X, double* Y,
                  int b, double alpha, double beta, hipStream_t s, const SpmmGroups* grp);
}

extern "C" {

int awg_dense_gemm(int32_t batch, int32_t m, int32_t n, int32_t k, int32_t transA, int32_t transB, double alpha,
                   const double* A, int32_t lda, int64_t strideA, const double* B, int32_t ldb, int64_t strideB,
                   double beta, double* C, int32_t ldc, int64_t strideC, void* stream) {
  if (batch <= 0 || m < 0 || n < 0 || k < 0 || !A || !B || !C) return AWG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    std::vector<GemmDesc> h(batch);
    for (int b = 0; b < batch; ++b)
      h[b] = GemmDesc{A + b * strideA, B + b * strideB, C + b * strideC, m, n, k, lda, ldb, ldc};
    DBuf<GemmDesc> d;
    d.upload(h, s);
    gemm_batched(d, batch, m, n, transA != 0, transB != 0, alpha, beta, false, s, 0.0, "dense");
    AWG_HIP(hipStreamSynchronize(s));
  });
}

int awg_dense_gemm_ex(int32_t batch, int32_t m, int32_t n, int32_t k, int32_t transA, int32_t transB,
                      double alpha, const double* A, int32_t lda, int64_t strideA, const int32_t* arows,
                      const double* B, int32_t ldb, int64_t strideB, double beta, double* C, int32_t ldc,
                      int64_t strideC, int32_t variant, void* stream) {
  if (batch <= 0 || m < 0 || n < 0 || k < 0 || !A || !B || !C || variant < -1 || variant > 5 ||
      (arows && transA))
    return AWG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    std::vector<GemmDesc> h(batch);
    std::vector<long> off(batch);
    for (int b = 0; b < batch; ++b) {
      h[b] = GemmDesc{A + (arows ? 0 : b * strideA), B + b * strideB, C + b * strideC, m, n, k, lda, ldb, ldc};
      off[b] = (long)b * k;
    }
    DBuf<GemmDesc> d;
    d.upload(h, s);
    DBuf<long> doff;
    doff.upload(off, s);
    if (variant < 0 && arows)
      gemm_batched_gather(d, A, arows, doff, batch, m, n, transB != 0, alpha, beta, s, 0.0, "dense_gather");
    else if (variant < 0)
      gemm_batched(d, batch, m, n, transA != 0, transB != 0, alpha, beta, false, s, 0.0, "dense");
    else
      gemm_batched_fixed(d, arows ? A : nullptr, arows, doff, batch, m, n, transA != 0, transB != 0, alpha, beta, s,
                         variant);
    AWG_HIP(hipStreamSynchronize(s));
  });
}

int awg_dense_local_product_f16x3(int32_t batch, const int32_t* n_host, int32_t ncols, const double* X,
                                  const double* P, double* Y, void* stream) {
  if (batch <= 0 || ncols <= 0 || !n_host || !X || !P || !Y) return AWG_ERR_ARG;
  for (int e = 0; e < batch; ++e)
    if (n_host[e] <= 0) return AWG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    const int b = ncols;
    std::vector<long> subptr(batch + 1, 0), sqoff(batch + 1, 0), poff(batch + 1, 0), gofs(batch + 1, 0);
    std::vector<int> row0, cnt;
    int maxn = 0;
    for (int e = 0; e < batch; ++e) {
      const int ne = n_host[e], G = (ne + 7) / 8;
      for (int g = 0; g < G; ++g) {
        row0.push_back((int)(subptr[e] + 8 * g));
        cnt.push_back(std::min(8, ne - 8 * g));
      }
      subptr[e + 1] = subptr[e] + ne;
      sqoff[e + 1] = sqoff[e] + (long)ne * ne;
      poff[e + 1] = poff[e] + (long)ne * G * 8;
      gofs[e + 1] = gofs[e] + G;
      maxn = std::max(maxn, ne);
    }
    const long rows = subptr[batch], groups = gofs[batch];
    std::vector<int> ident(rows);
    for (long r = 0; r < rows; ++r) ident[r] = (int)r;
    DBuf<long> dsub, dsq, dpo;
    DBuf<int> drow0, dcnt, didx, emax, sp;
    dsub.upload(subptr, s);
    dsq.upload(sqoff, s);
    dpo.upload(poff, s);
    drow0.upload(row0, s);
    dcnt.upload(cnt, s);
    didx.upload(ident, s);
    emax.alloc(b);
    sp.alloc(batch);
    DBuf<_Float16> X16, P16;
    const long xplane = groups * (long)b * 8, pplane = poff[batch];
    X16.alloc(2 * (size_t)xplane);
    P16.alloc(2 * (size_t)pplane);
    l_colexp((int)rows, b, X, emax, s);
    l_gather_h3(groups, drow0, dcnt, didx, X, b, emax, X16, xplane, s);
    l_p16_build(batch, dsq, dsub, dpo, P, P16, pplane, sp, s);
    std::vector<GemmDescH3> h(batch);
    double fl = 0.0;
    for (int e = 0; e < batch; ++e) {
      const int ne = n_host[e];
      h[e] = GemmDescH3{X16.p + gofs[e] * b * 8, P16.p + poff[e], Y + subptr[e] * b, xplane, pplane, b, ne,
                        (ne + 7) / 8, b};
      fl += 2.0 * ne * (double)ne * b;
    }
    DBuf<GemmDescH3> d;
    d.upload(h, s);
    gemm_h3_batched(d, batch, b, maxn, emax, sp, s, fl);
    AWG_HIP(hipStreamSynchronize(s));
  });
}

int awg_dense_potrf(int32_t batch, int32_t n, double* A, int32_t lda, int64_t strideA, int32_t* info_host,
                    void* stream) {
  if (batch <= 0 || n <= 0 || lda < n || !A) return AWG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  bool bad = false;
  int rc = guarded(s, [&] {
    DBuf<MatDesc> d;
    d.upload(uniform(A, batch, n, n, lda, strideA), s);
    DBuf<int> info;
    info.alloc(batch);
    info.zero(s);
    potrf_batched(d, std::vector<int>(batch, n), info, s, nullptr);
    auto h = info.download(s);
    for (int b = 0; b < batch; ++b) {
      if (info_host) info_host[b] = h[b];
      bad |= h[b] != 0;
    }
  });
  return rc ? rc : (bad ? AWG_ERR_NOT_SPD : AWG_OK);
}

__global__ void k_abi_f32_from_f64(long tot, const double* a, float* b) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x)
    b[e] = (float)a[e];
}
__global__ void k_abi_f64_from_f32(long tot, const float* a, double* b) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x)
    b[e] = (double)a[e];
}

int awg_dense_spd_inverse_f32(int32_t batch, const int32_t* n_host, const double* A, double* Ainv,
                              int32_t* info_host, float* pivot_ratio_host, void* stream) {
  if (batch <= 0 || !n_host || !A || !Ainv) return AWG_ERR_ARG;
  for (int b = 0; b < batch; ++b)
    if (n_host[b] <= 0) return AWG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  bool bad = false;
  int rc = guarded(s, [&] {
    std::vector<long> off(batch + 1, 0);
    std::vector<int> ns(n_host, n_host + batch);
    for (int b = 0; b < batch; ++b) off[b + 1] = off[b] + (long)ns[b] * ns[b];
    const long tot = off[batch];
    DBuf<float> K, X, O;
    K.alloc(tot);
    X.alloc(tot);
    O.alloc(tot);
    hipLaunchKernelGGL(k_abi_f32_from_f64, dim3(1024), dim3(256), 0, s, tot, A, K.p);
    AWG_LAUNCH_CHECK();
    auto descs = [&](float* base) {
      std::vector<MatDescF> v(batch);
      for (int b = 0; b < batch; ++b) v[b] = MatDescF{base + off[b], ns[b], ns[b]};
      return v;
    };
    DBuf<MatDescF> dK, dX, dO;
    dK.upload(descs(K.p), s);
    dX.upload(descs(X.p), s);
    dO.upload(descs(O.p), s);
    DBuf<int> info;
    info.alloc(batch);
    info.zero(s);
    DBuf<float> dmin, dmax;
    dmin.alloc(batch);
    dmax.alloc(batch);
    chol_inverse_f32(dK, dX, dO, ns, info, dmin, dmax, s);
    hipLaunchKernelGGL(k_abi_f64_from_f32, dim3(1024), dim3(256), 0, s, tot, O.p, Ainv);
    AWG_LAUNCH_CHECK();
    const auto hi = info.download(s);
    const auto lo = dmin.download(s), hiv = dmax.download(s);
    for (int b = 0; b < batch; ++b) {
      if (info_host) info_host[b] = hi[b];
      if (pivot_ratio_host) pivot_ratio_host[b] = lo[b] > 0.f ? hiv[b] / lo[b] : 0.f;
      bad |= hi[b] != 0;
    }
  });
  return rc ? rc : (bad ? AWG_ERR_NOT_SPD : AWG_OK);
}

int awg_dense_potrf_noalloc(int32_t batch, int32_t n, double* A, int32_t lda, int64_t strideA,
                            int32_t* info_host, void* stream) {
  if (batch <= 0 || batch > NOALLOC_MAX_BATCH || n <= 0 || lda < n || !A) return AWG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  bool bad = false;
  int rc = guarded(s, [&] {
    unsigned char* base = scratch_on_current_device();
    MatDesc* d = (MatDesc*)base;
    int* info = (int*)(base + NOALLOC_DESC_BYTES);
    hipLaunchKernelGGL(k_uniform_desc, dim3(cdiv(batch, 256)), dim3(256), 0, s, d, info, A, batch, n, lda,
                       (long)strideA);
    AWG_LAUNCH_CHECK();
    potrf_uniform(d, batch, n, info, s);
    if (info_host) {
      AWG_HIP(hipMemcpyAsync(info_host, info, sizeof(int32_t) * batch, hipMemcpyDeviceToHost, s));
      AWG_HIP(hipStreamSynchronize(s));
      for (int b = 0; b < batch; ++b) bad |= info_host[b] != 0;
    } else {
      // only the failure flag of the whole batch is needed: read the entries
      // in chunks through a small host array
      int32_t chunk[256];
      for (int b0 = 0; b0 < batch; b0 += 256) {
        const int m = std::min(256, batch - b0);
        AWG_HIP(hipMemcpyAsync(chunk, info + b0, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
        AWG_HIP(hipStreamSynchronize(s));
        for (int b = 0; b < m; ++b) bad |= chunk[b] != 0;
      }
    }
  });
  return rc ? rc : (bad ? AWG_ERR_NOT_SPD : AWG_OK);
}

int awg_dense_trsm(int32_t batch, int32_t n, int32_t nrhs, int32_t trans, const double* L, int32_t ldl,
                   int64_t strideL, double* B, int32_t ldb, int64_t strideB, void* stream) {
  if (batch <= 0 || n <= 0 || nrhs < 0 || ldl < n || ldb < n || !L || !B) return AWG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    DBuf<MatDesc> dl, db;
    dl.upload(uniform(const_cast<double*>(L), batch, n, n, ldl, strideL), s);
    db.upload(uniform(B, batch, n, nrhs, ldb, strideB), s);
    trsm_batched(dl, db, std::vector<int>(batch, n), std::vector<int>(batch, nrhs), trans != 0, s, nullptr);
  });
}

int awg_dense_low_eigs(int32_t batch, int32_t n, double* A, int32_t lda, int64_t strideA, double thr,
                       int32_t max_k, int32_t* count_host, double* lam, double* Z, int64_t strideZ, void* stream) {
  if (batch <= 0 || n <= 0 || lda < n || max_k < 0 || !A || !count_host) return AWG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  bool over = false;
  int rc = guarded(s, [&] {
    DBuf<MatDesc> dA;
    dA.upload(uniform(A, batch, n, n, lda, strideA), s);
    std::vector<int> hn(batch, n);
    std::vector<long> off(batch + 1);
    for (int b = 0; b <= batch; ++b) off[b] = (long)b * n;
    DBuf<long> doff, w6;
    doff.upload(off, s);
    std::vector<long> o6(batch);
    for (int b = 0; b < batch; ++b) o6[b] = TRIVEC_WORK_PER_ROW * b * n;
    w6.upload(o6, s);
    DBuf<double> d, e, tau, work, thrv, mm;
    d.alloc((long)batch * n);
    e.alloc((long)batch * n);
    tau.alloc((long)batch * n);
    work.alloc(TRIVEC_WORK_PER_ROW * batch * n);
    thrv.alloc(batch);
    mm.alloc(2 * batch);
    std::vector<double> ht(batch, thr);
    thrv.upload(ht, s);
    sytrd_batched(dA, hn, d, e, tau, doff, work, s);
    DBuf<int> nd, cnt;
    nd.upload(hn, s);
    cnt.alloc(batch);
    TriEigArgs a{d, e, doff, nd, batch};
    tri_count(a, thrv, 0, 0.0, thrv, cnt, mm, s);
    auto hc = cnt.download(s);
    std::vector<int> kk(batch);
    for (int b = 0; b < batch; ++b) {
      count_host[b] = hc[b];
      kk[b] = std::min(hc[b], max_k);
      over |= hc[b] > max_k;
    }
    cnt.upload(kk, s);
    std::vector<long> loff(batch + 1);
    for (int b = 0; b <= batch; ++b) loff[b] = (long)b * max_k;
    DBuf<long> dlo;
    dlo.upload(loff, s);
    DBuf<MatDesc> dZ;
    std::vector<MatDesc> zd(batch);
    for (int b = 0; b < batch; ++b) zd[b] = MatDesc{Z + b * strideZ, n, kk[b], n, 0};
    dZ.upload(zd, s);
    DBuf<double> resid;
    resid.alloc(std::max(1L, (long)batch * max_k));
    if (max_k > 0 && lam && Z) {
      tri_eigvecs(a, cnt, dlo, lam, dZ, work, w6, resid, nullptr, thrv, s, n);
      ormtr_batched(dA, dZ, tau, doff, hn, kk, s);
    }
  });
  return rc ? rc : (over ? AWG_ERR_ARG : AWG_OK);
}

int awg_csr_spmm(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col, const double* val,
                 const double* X, double* Y, int32_t b, double alpha, double beta, int32_t variant, void* stream) {
  if (n <= 0 || nnz < 0 || nnz >= (1LL << 31) || b <= 0 || variant < -1 || variant > 10 || !rowptr ||
      (nnz && (!col || !val)) || !X || !Y)
    return AWG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] {
    DBuf<int> rp;
    rp.alloc(n + 1);
    hipLaunchKernelGGL(k_rowptr_to32, dim3(cdiv(n + 1, 256)), dim3(256), 0, s, n, rowptr, rp.p);
    AWG_LAUNCH_CHECK();
    SpmmGroups grp;
    spmm_groups(n, nnz, rp, col, val, grp, s);
    if (variant < 0)
      l_spmm(n, nnz, rp, col, val, X, Y, b, alpha, beta, s, &grp);
    else
      spmm_variant(variant, n, rp, col, val, X, Y, b, alpha, beta, s, &grp);
    AWG_HIP(hipStreamSynchronize(s));
  });
}

int awg_probe_mfma_f64(int32_t iters, double* tflops, void* stream) {
  if (iters <= 0 || !tflops) return AWG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  return guarded(s, [&] { *tflops = probe_mfma_f64(iters, s); });
}

int awg_autotune(int32_t enable) {
  tune_enable(enable != 0);
  return AWG_OK;
}

int64_t awg_tune_report(char* buf, size_t cap) {
  const std::string js = tune_json();
  if (buf && cap) {
    const size_t k = std::min(cap - 1, js.size());
    std::memcpy(buf, js.data(), k);
    buf[k] = '\0';
  }
  return (int64_t)js.size();
}

}  // extern "C"
