/*
 * awg.h -- C ABI of the MI355X (gfx950) AWG-PCG library.
 *
 * Solves a sparse symmetric positive definite system A x = b with the
 * preconditioned conjugate gradient method, preconditioned by the additive
 * Algebraic-Woodbury-GenEO preconditioner of Gouarin & Spillane, "Fully
 * algebraic domain decomposition preconditioners with adaptive spectral
 * bounds":
 *
 *     H = H2 + W (W^T A W)^{-1} W^T             (Definition of Pi_3 and H3, Section 4.3)
 *     H2 = Pi H^NN Pi^T + R0^T E0^{-1} R0        (Theorem on H^NN_hyb(tau), Section 3.4)
 *     H^NN = sum_s R^sT D^s (A^s_+)^+ D^s R^s     (Definition of H^NN, Section 3.3)
 *
 * built only from A and the subdomain index sets (Sections 2 and 3.1-3.2).
 *
 * Conventions for every entry point
 *   - All array arguments are DEVICE pointers (HIP device memory of the
 *     current device) unless stated otherwise; indices are 0-based; A is
 *     given in CSR with BOTH triangles stored.
 *   - Work is stream-ordered on the stream given in awg_options.stream
 *     (NULL = the default stream).  awg_setup and awg_pcg synchronise that
 *     stream before returning; awg_apply does not.
 *   - The caller owns every buffer it passes; the library copies what it
 *     keeps during awg_setup, so inputs may be freed when it returns.  The
 *     library owns its internal buffers until awg_destroy.
 *   - Return value: AWG_OK (0), a positive warning, or a negative error.
 *     No exception crosses the ABI.  On error, output buffers are left
 *     untouched and awg_last_error() describes the failure.
 *   - A context is used by one host thread / one stream at a time.
 */
#ifndef AWG_H
#define AWG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct awg_ctx awg_ctx;

typedef enum {
  AWG_OK = 0,
  AWG_NOT_CONVERGED = 1,        /* awg_pcg hit maxit; x holds the last iterate */
  AWG_ERR_ARG = -1,             /* invalid scalar argument or NULL pointer */
  AWG_ERR_NOT_SYMMETRIC = -2,   /* A_ij != A_ji for some stored entry */
  AWG_ERR_PARTITION = -3,       /* subdomain list empty / unsorted / duplicate /
                                   out of range, or the lists do not cover [0,n)
                                   (Definition of a partition, Section 2.1) */
  AWG_ERR_MIN_OVERLAP = -4,     /* some A_ij != 0 has no subdomain holding both
                                   i and j (Assumption of minimal overlap, Section 2.1) */
  AWG_ERR_NOT_SPD = -5,         /* a Cholesky factorisation broke down (local
                                   K^s, M_B^s, E0 or W^T A W) or PCG met p^T A p <= 0 */
  AWG_ERR_EIGEN = -6,           /* a local eigensolve failed its residual check */
  AWG_ERR_HIP = -7,             /* a HIP runtime call failed */
  AWG_ERR_OOM = -8,             /* device allocation failed */
  AWG_ERR_NONFINITE = -9        /* NaN or Inf in A */
} awg_status;

/* storage and arithmetic of the local solves P^s (the H^NN term):
 *   AWG_LOCAL_F64    FP64 throughout;
 *   AWG_LOCAL_F32    P^s rounded to FP32, FP32 products and sums;
 *   AWG_LOCAL_F16X3  as AWG_LOCAL_F32 for one-column products; the
 *                    multi-column local products of the W solves split both
 *                    operands into two FP16 parts after a power-of-two scaling
 *                    (per subdomain for P^s, per column for the vectors) and
 *                    take three FP16 matrix-core products with FP32 sums
 *                    (about 2^-21 relative error per product term) */
enum { AWG_LOCAL_F64 = 0, AWG_LOCAL_F32 = 1, AWG_LOCAL_F16X3 = 2 };
enum { AWG_GENEO_DENSE = 0, AWG_GENEO_SUBSPACE = 1 };
/* second-coarse-space preconditioner H (Section 4), all with the same
 * W = A_+^{-1} V_-:
 *   AWG_COARSE2_AD   H3,ad   = H2 + W (W^T A W)^{-1} W^T (Definition of Pi_3 and H3)
 *   AWG_COARSE2_INEX H3,inex = H2 + W C^{-1} W^T, C = L_-^{-1} - V_-^T W
 *                    (Theorem on the AWG preconditioner with inexact coarse space)
 *   AWG_COARSE2_HYB  H3,hyb  = Pi3 H2 Pi3^T + W (W^T A W)^{-1} W^T,
 *                    Pi3 = I - W (W^T A W)^{-1} W^T A (Definition of Pi_3 and H3) */
enum { AWG_COARSE2_AD = 0, AWG_COARSE2_INEX = 1, AWG_COARSE2_HYB = 2 };
/* two-level preconditioner H2 for A_+ inside H (Section 3.4), all on the same
 * GenEO coarse space R0 (the pencil (D^-1 A^s_+ D^-1, R^s A_+ R^sT) below tau,
 * which is V0_{AS,+}(tau_flat) with tau_flat = 1/tau):
 *   AWG_H2_NN_HYB  H^NN_hyb(tau) = Pi H^NN Pi^T + R0^T E0^{-1} R0,
 *                  H^NN = sum_s R^sT D^s (A^s_+)^+ D^s R^s
 *                  (Theorem on H^NN_hyb); spectrum of H2 A_+ in [1, N(A_+)/tau]
 *   AWG_H2_ASP_HYB H^AS_{+,hyb}(1/tau) = Pi H^AS_+ Pi^T + R0^T E0^{-1} R0,
 *                  H^AS_+ = sum_s R^sT (R^s A_+ R^sT)^{-1} R^s
 *                  (Theorem on H^AS_{+,hyb/ad}); spectrum in [tau, N(A_+)]
 *   AWG_H2_ASP_AD  H^AS_{+,ad}(1/tau) = H^AS_+ + R0^T E0^{-1} R0 (same theorem);
 *                  spectrum in [tau / (1 + 2 N(A_+)), N(A_+) + 1]
 * and one on a coarse space of its own:
 *   AWG_H2_AS_HYB  H^AS_hyb(tau, 1/tau) = Pi H^AS Pi^T + R0^T E0^{-1} R0,
 *                  H^AS = sum_s R^sT (R^s A R^sT)^{-1} R^s, R0 from two pencils
 *                  per subdomain: (D^-1 A^s_+ D^-1, R^s A R^sT) below tau, then
 *                  (R^s A R^sT, R^s A_+ R^sT) below tau (Theorem on H^AS_hyb);
 *                  spectrum in [tau, N(A_+)/tau]; needs AWG_GENEO_DENSE.  Its
 *                  E0^+ deflates the eigenvectors of the Jacobi-scaled E0 below
 *                  1e-10 (the union of two pencils' vectors can be dependent
 *                  across subdomains); at most 64 such directions, else
 *                  AWG_ERR_NOT_SPD */
enum { AWG_H2_NN_HYB = 0, AWG_H2_ASP_HYB = 1, AWG_H2_ASP_AD = 2, AWG_H2_AS_HYB = 3 };

typedef struct {
  double tau;          /* GenEO threshold of H^NN_hyb(tau), tau_flat = 1/tau for the
                          AS forms; 0 < tau < 1 (Theorems, Section 3.4) */
  double zero_tol;     /* eps0: an eigenvalue lambda of B^s is non-positive when
                          lambda <= eps0 * max|lambda(B^s)|; default 1e-12 */
  double w_rtol;       /* relative residual tolerance of the PCG solves with A_+
                          that build W (Remark 2, Section 4.4); default 1e-10,
                          the value of the paper's experiments (Section 5) */
  int32_t w_maxit;     /* iteration cap of those solves; default 500 */
  int32_t local_prec;  /* AWG_LOCAL_F64 (default), AWG_LOCAL_F32 or
                          AWG_LOCAL_F16X3: storage and arithmetic of the
                          per-iteration local solves */
  void* stream;        /* hipStream_t; NULL = default stream */
  int32_t geneo_solver;  /* AWG_GENEO_DENSE (default): every GenEO pencil is
                            reduced to tridiagonal form and solved exactly;
                            AWG_GENEO_SUBSPACE: block subspace iteration with
                            Rayleigh-Ritz on the pencil restricted to the
                            complement of its known kernel D^s V^s_-, accepted
                            per subdomain only when every selected Ritz pair
                            meets eig_tol and a Cholesky factorisation
                            certifies that no other eigenvalue lies below
                            tau (1 - 1e-10); otherwise the dense solver runs */
  int32_t eig_block;     /* iterated columns besides the kernel, 1..64; default 16 */
  int32_t eig_maxit;     /* iteration cap of the subspace solver; default 200 */
  int32_t eig_seed;      /* seed of the random start block; default 0 */
  double eig_tol;        /* relative Ritz residual required of every Ritz value
                            below 2 tau; default 1e-10 */
  const struct awg_mlp* eig_init;  /* learned start (awg_mlp.h): the network's
                            outputs on the per-dof features fill the first
                            out_channels columns of the start block (the rest
                            stays random); needs in_features = AWG_MLP_FEATURES
                            and out_channels <= eig_block.  NULL (default):
                            random start.  Not owned; used during awg_setup only */
  const double* coords;  /* optional node coordinates of every dof, device,
                            n x coord_dim row-major (features 0-2); NULL (default) */
  int32_t coord_dim;     /* 1..3 when coords is given */
  int32_t coarse2;       /* AWG_COARSE2_AD (default), AWG_COARSE2_INEX or AWG_COARSE2_HYB */
  int32_t h2;            /* AWG_H2_NN_HYB (default), AWG_H2_ASP_HYB, AWG_H2_ASP_AD or AWG_H2_AS_HYB */
  int32_t w_h2;          /* preconditioner of the PCG solves with A_+ that build
                            W (Remark 2, Section 4.4) when h2 = AWG_H2_NN_HYB:
                            AWG_H2_ASP_AD (default), AWG_H2_ASP_HYB or
                            AWG_H2_NN_HYB (H2 itself).  Any SPD preconditioner
                            of A_+ gives the same W to w_rtol; H^AS_+,ad(1/tau)
                            (Theorem on H^AS_+,hyb/ad, Section 3.4) shares R0
                            and E0 with H^NN_hyb(tau) and costs one coarse solve
                            and one local pass per application.  With any other
                            h2 the W solves use h2 itself. */
} awg_options;

/* Fill every field of *opt with the defaults above (tau = 0.1).  Host pointer. */
void awg_default_options(awg_options* opt);

/* Build the preconditioner (every setup step runs on the GPU).
 *   n, nnz         order of A and number of stored entries (nnz < 2^31)
 *   rowptr[n+1]    int64 CSR row pointers            (device)
 *   col[nnz]       int32 column indices, sorted per row (device)
 *   val[nnz]       float64 values                      (device)
 *   nsub           number N of subdomains (>= 1)
 *   sub_ptr[N+1]   int64 offsets of each index list in sub_idx (device)
 *   sub_idx[..]    int32 dof indices, sorted and unique per subdomain (device)
 *   opt            host pointer to options (NULL = defaults)
 * On success *out receives a new context.  On failure *out is set to NULL
 * and awg_last_error(NULL) explains the failure. */
int awg_setup(awg_ctx** out, int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col,
              const double* val, int32_t nsub, const int64_t* sub_ptr, const int32_t* sub_idx,
              const awg_options* opt);

/* z = H r for device vectors of length n (r and z must not alias). */
int awg_apply(awg_ctx* ctx, const double* r, double* z);

typedef struct {
  int32_t iters;          /* number of products A p performed */
  int32_t converged;      /* 1 if ||r_k||/||b|| <= tol was reached */
  double rel_res;         /* recursively updated ||r_k|| / ||b|| */
  double rel_res_true;    /* ||b - A x_k|| / ||b|| recomputed at the end */
  double lmin_est;        /* extreme Ritz values of HA from the PCG coefficients */
  double lmax_est;        /* (of the first run of the recurrence) */
  int32_t restarts;       /* restarts from the true residual (see awg_pcg) */
  int32_t iters_first;    /* iterations of the first run of the recurrence
                             (the coefficients of lmin_est, lmax_est) */
} awg_pcg_info;

/* PCG (Saad, Section 9.2) from x0 = 0 with the AWG preconditioner; stops at
 * the first k with ||r_k||_2 / ||b||_2 <= tol on the recursive residual.
 * b, x: device vectors of length n.  info: host pointer (may be NULL).
 * maxit > 4095 is treated as 4095 (size of the coefficient history).
 * When the recursive residual meets tol but the true residual b - A x does
 * not (finite-precision drift on ill-conditioned A), the recurrence restarts
 * from the true residual (at most 5 times, iterations keep counting);
 * converged = 1 requires both residuals <= tol. */
int awg_pcg(awg_ctx* ctx, const double* b, double* x, double tol, int32_t maxit,
            awg_pcg_info* info);

/* awg_pcg runs each iteration as one captured HIP graph (default, enable != 0)
 * or as eager launches of the same kernels (enable = 0).  Convergence is
 * decided on the device; the host checks it every few iterations, and
 * iterations launched after convergence leave x unchanged. */
int awg_pcg_graph(awg_ctx* ctx, int32_t enable);

/* The multi-column PCG that builds W (Remark 2, Section 4.4) moves its
 * active columns to narrower multi-vectors as columns converge (default,
 * enable != 0); every column is computed independently of the others and of
 * its position, so W is the same bit for bit either way.  Process-wide;
 * applies to setups started afterwards.  Returns 0. */
int awg_w_compaction(int32_t enable);

/* Device memory released by the library (awg_destroy, the work buffers of a
 * set-up) is kept in a process-wide cache and reused by later allocations of
 * a similar size on the same device, so repeated set-ups allocate nothing
 * from the driver.  This call returns every cached block to the driver
 * (the device is synchronised first) and stores the number of bytes freed in
 * *bytes_out when it is not NULL.  Returns 0. */
int awg_free_cached_memory(uint64_t* bytes_out);

/* JSON description of the setup (n, N, n_minus, n0, per-subdomain counts,
 * per-phase times in ms).  buf: host buffer of cap bytes.  Returns the
 * number of bytes needed (excluding the terminator) or a negative error. */
int64_t awg_stats(const awg_ctx* ctx, char* buf, size_t cap);

/* Copy a named internal array to HOST memory (tests and diagnostics).
 *   "neg_eigs"   float64 [sum_s k_s]  non-positive eigenvalues of each B^s, ascending per s
 *   "geneo_eigs" float64 [sum_s m_s]  selected GenEO eigenvalues, ascending per s (for
 *                                     AWG_H2_AS_HYB: those of the first pencil, then of the second)
 *   "mult"       int32   [n]          multiplicity of each dof
 *   "pair_count" int32   [nnz]        M_mu on the pattern of A (CSR order)
 *   "V_minus"    float64 [sum_s n_s k_s] non-positive eigenvectors of each B^s
 *                                     (n_s x k_s column-major blocks, in subdomain order)
 *   "Y"          float64 [sum_s n_s m_s] GenEO coarse vectors Y^s (same layout)
 *   "P_local"    float64 [sum_s n_s^2] local operators of H2 (n_s x n_s blocks):
 *                                     D^s (A^s_+)^+ D^s, (R^s A_+ R^sT)^{-1} for the AS_+ forms,
 *                                     (R^s A R^sT)^{-1} for AWG_H2_AS_HYB
 *   "W"          float64 [n * n_minus] second coarse basis W = A_+^-1 V_- as computed
 *                                     (PCG to w_rtol), row-major: W[i * n_minus + j]
 * Returns the number of bytes of the array (copying min(cap, size)), or a
 * negative error for an unknown name. */
int64_t awg_export(const awg_ctx* ctx, const char* name, void* host_buf, size_t cap);

/* Message of the last error on this context, or of the last failed
 * awg_setup when ctx is NULL.  Never returns NULL. */
const char* awg_last_error(const awg_ctx* ctx);

/* Kernel timing for performance reports: when enabled, HIP events are
 * recorded on the launching stream around the main kernels of every
 * context, and per-kernel launch counts, elapsed milliseconds and the
 * algorithmic bytes / flops of each launch are accumulated.  Off by default
 * (it adds one event pair per launch). */
/* Restrict the timing to kernels whose label starts with prefix (NULL or ""
 * = every instrumented kernel); per-launch events cost a few microseconds, so
 * a benchmark times only the kernel it reports. */
int awg_kernel_timing_filter(const char* prefix);
int awg_kernel_timing(int32_t enable);

/* JSON {"kernel": {"calls", "ms", "bytes", "flops"}, ...} of the accumulated
 * kernel times (synchronises the pending events).  buf: host buffer of cap
 * bytes; reset != 0 clears the accumulators.  Returns the bytes needed or a
 * negative error. */
int64_t awg_kernel_times(char* buf, size_t cap, int32_t reset);

/* Free every device buffer of the context.  NULL is ignored. */
void awg_destroy(awg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* AWG_H */
