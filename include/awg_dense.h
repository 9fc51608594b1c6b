/*
 * awg_dense.h -- batched dense building blocks of libawg (gfx950).
 *
 * The AWG set-up (Gouarin & Spillane, Sections 3.2-3.4 and 4.3) reduces to
 * four dense operations on many independent blocks: products (trailing
 * updates, Gram and projection products), Cholesky factorisations (local
 * K^s, M_B^s, coarse matrices), triangular solves with many right-hand sides
 * (explicit inverses, the Cholesky reduction of the GenEO pencil), and
 * eigenpairs below a threshold of symmetric blocks (the non-positive part of
 * B^s, the GenEO modes below tau).  These entry points expose them for
 * uniform batches, as used by the library internally with variable sizes.
 *
 * Conventions: float64, column-major blocks, block b of X starts at
 * X + b * strideX; all arrays are DEVICE pointers unless marked host; work is
 * ordered on `stream` (hipStream_t, NULL = default) and the call returns
 * after it completes.  Return AWG_OK (0) or a negative awg_status.
 */
#ifndef AWG_DENSE_H
#define AWG_DENSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* C_b = alpha op(A_b) op(B_b) + beta C_b;  op(A_b) is m x k, op(B_b) is k x n. */
int awg_dense_gemm(int32_t batch, int32_t m, int32_t n, int32_t k, int32_t transA, int32_t transB,
                   double alpha, const double* A, int32_t lda, int64_t strideA, const double* B,
                   int32_t ldb, int64_t strideB, double beta, double* C, int32_t ldc, int64_t strideC,
                   void* stream);

/* awg_dense_gemm with a chosen launch variant and an optional row gather of
 * the A operands (the form the multi-column products of the W solves use).
 * variant: -1 = autotuned (measured on the first call with beta = 0 for this
 * shape), 0 = 64x64 tiles, 1 = 128x128 tiles with 4 wavefronts, 2 = 128x128
 * tiles with 8 wavefronts, 3 and 4 = 32x32 blocks per wavefront without LDS
 * with 16 or 32 k values per load batch, 5 = the same blocks with the B panel
 * shared by the workgroup through LDS (3..5 only for transA = transB = 0;
 * otherwise variant 2 runs).  Every variant returns bit-identical results.
 * arows: NULL, or a device array of batch x k int32 (requires transA = 0):
 * column j of A_b is then A + arows[b k + j] * lda (strideA is ignored), i.e.
 * row arows[b k + j] of a row-major matrix with lda columns; the caller
 * guarantees that every index addresses memory inside A.
 * Returns AWG_ERR_ARG for negative sizes, null pointers, a variant outside
 * -1..5, or arows with transA = 1. */
int awg_dense_gemm_ex(int32_t batch, int32_t m, int32_t n, int32_t k, int32_t transA, int32_t transB,
                      double alpha, const double* A, int32_t lda, int64_t strideA, const int32_t* arows,
                      const double* B, int32_t ldb, int64_t strideB, double beta, double* C, int32_t ldc,
                      int64_t strideC, int32_t variant, void* stream);

/* Split-FP16 local products Y_b = P_b^T X_b for batch entries of n_b x n_b
 * matrices P_b (column-major, concatenated) and n_b x ncols row-major blocks
 * X_b (concatenated, so X is (sum n_b) x ncols row-major; Y likewise): the
 * multi-column local product of the W solves (the H^NN term of H2,
 * Definition of H^NN, Section 3.3) in the AWG_LOCAL_F16X3 arithmetic.  Each
 * P_b is scaled by a power of two, each column of X by a power of two (from
 * the largest magnitude of that column over all of X), both are split into
 * hi = fp16(v) and lo = fp16(v - hi), and hi.hi + hi.lo + lo.hi are summed on
 * the FP16 matrix cores in FP32, then scaled back into FP64.  n_host: host
 * array of the batch sizes; X, P, Y device.  Returns AWG_ERR_ARG for
 * batch <= 0, ncols <= 0, a size n_b <= 0 or null pointers. */
int awg_dense_local_product_f16x3(int32_t batch, const int32_t* n_host, int32_t ncols, const double* X,
                                  const double* P, double* Y, void* stream);

/* FP32 inverse of SPD blocks on the FP32 matrix cores (the local factors of
 * the W solves' H^AS_+ operators in the reduced-precision forms, one-level
 * preconditioners for A_+, Section 3.3): A_b rounded to FP32, A_b = L L^T,
 * X = L^{-1} by blocked substitution, A_b^{-1} = X^T X, returned in FP64.
 * A and Ainv: device, the n_b x n_b column-major blocks concatenated; n_host:
 * host sizes.  info_host[b] (host, optional) = 0 or the 1-based column of the
 * first non-positive FP32 pivot; pivot_ratio_host[b] (host, optional) = max /
 * min diagonal entry of L (its square bounds the condition number from
 * below).  Returns AWG_ERR_NOT_SPD if any block failed, AWG_ERR_ARG for
 * batch <= 0, a size <= 0 or null pointers. */
int awg_dense_spd_inverse_f32(int32_t batch, const int32_t* n_host, const double* A, double* Ainv,
                              int32_t* info_host, float* pivot_ratio_host, void* stream);

/* In-place lower Cholesky A_b = L_b L_b^T (upper triangle left unspecified).
 * info_host[b] (host, batch entries) = 0 or the 1-based column of the first
 * non-positive pivot; returns AWG_ERR_NOT_SPD if any block failed. */
int awg_dense_potrf(int32_t batch, int32_t n, double* A, int32_t lda, int64_t strideA, int32_t* info_host,
                    void* stream);

/* awg_dense_potrf for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): it calls no hipMalloc, hipFree or allocating library routine.
 * The block descriptors and the info array live in a static device array of
 * the library (4096 x 28 bytes, 112 KiB, one copy per device, held until the
 * process ends), so batch <= AWG_NOALLOC_MAX_BATCH; a larger batch returns
 * AWG_ERR_ARG before any work.  Otherwise the same arguments, factors (bit
 * for bit), info_host (may be NULL) and return values as awg_dense_potrf.
 * The array belongs to the current device (stream must be on it) and keeps
 * the last call's contents; calls that overlap on one device (several host
 * threads or streams) share it and race, so the caller serialises them. */
#define AWG_NOALLOC_MAX_BATCH 4096
int awg_dense_potrf_noalloc(int32_t batch, int32_t n, double* A, int32_t lda, int64_t strideA,
                            int32_t* info_host, void* stream);

/* B_b <- L_b^{-1} B_b (trans = 0) or L_b^{-T} B_b (trans = 1), L_b lower n x n,
 * B_b n x nrhs. */
int awg_dense_trsm(int32_t batch, int32_t n, int32_t nrhs, int32_t trans, const double* L, int32_t ldl,
                   int64_t strideL, double* B, int32_t ldb, int64_t strideB, void* stream);

/* Eigenpairs of the symmetric blocks A_b (destroyed) with eigenvalue < thr,
 * ascending: count_host[b] (host) receives their number; the first
 * min(count, max_k) eigenvalues go to lam[b * max_k ...] and the orthonormal
 * eigenvectors to Z + b * strideZ (n x max_k, leading dimension n).  Returns
 * AWG_ERR_ARG if some count exceeds max_k (counts are still reported). */
int awg_dense_low_eigs(int32_t batch, int32_t n, double* A, int32_t lda, int64_t strideA, double thr,
                       int32_t max_k, int32_t* count_host, double* lam, double* Z, int64_t strideZ,
                       void* stream);

/* Y = alpha A X + beta Y for a CSR matrix A (n x n, 0-based, rowptr int64 with
 * nnz < 2^31) and row-major n x b blocks X, Y (the multi-column product of the
 * W solves).  variant: -1 = the autotuned launch variant for this shape
 * (measured on the first call with beta = 0), 0..10 = a fixed variant (5..10
 * need an even b and 16-byte aligned X and Y, else they run variant 1; 9, 10
 * process groups of up to 4 consecutive rows on the union of their column
 * patterns and run variant 5 when grouping would not cut the row count by a
 * quarter); every variant returns bit-identical results for finite X. */
int awg_csr_spmm(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col, const double* val,
                 const double* X, double* Y, int32_t b, double alpha, double beta, int32_t variant, void* stream);

/* Sustained FP64 matrix-core rate of the device in TFLOP/s (*tflops, host):
 * best of three timed launches of a kernel that runs `iters` rounds of eight
 * independent v_mfma_f64_16x16x4 accumulations per wavefront, eight
 * wavefronts per SIMD on every CU, with no memory traffic in the loop (the
 * practical ceiling of the FP64 GEMMs, beside the published peak).  Returns
 * AWG_ERR_ARG for iters <= 0 or a null tflops. */
int awg_probe_mfma_f64(int32_t iters, double* tflops, void* stream);

/* Autotuner of launch variants: enable (default) or disable measurement
 * (disabled: variant 0 everywhere).  Choices persist as JSON lines in the file
 * named by the environment variable AWG_TUNE_CACHE when it is set. */
int awg_autotune(int32_t enable);
/* JSON object {key: {"variant": v, "us": [time per variant]}} of this
 * process's choices into buf (host, cap bytes, NUL-terminated); returns the
 * full length. */
int64_t awg_tune_report(char* buf, size_t cap);

#ifdef __cplusplus
}
#endif
#endif /* AWG_DENSE_H */
