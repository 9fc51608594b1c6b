// Launchers of the iterative GenEO eigensolver kernels (k_subspace.hip).
// Blocks of subdomain s are column-major: a q-column block at sub_ptr[s] * q
// (leading dimension n_s); column layouts (K, Y) at their element offsets.
#pragma once
#include "awg_common.h"

namespace awg {
constexpr int SUBSPACE_MAX_BLOCK = 64;   // largest iterated block (one wavefront per subdomain)

void l_rows_dw(int N, int maxns, int maxk, const long* sub_ptr, const long* eoff, const long* coff, const double* V,
               const double* dw, double* out, hipStream_t s);
void l_rand_block(int N, int maxns, const long* sub_ptr, const int* sub_idx, int q, uint64_t seed, double* X,
                  hipStream_t s);
void l_init_cols(int N, int maxns, const long* sub_ptr, int q, const double* src, const int* ncol, double* X,
                 hipStream_t s);
void l_rr_small(int N, int q, const double* S0, const double* S1, double* C, double* mu, int* flag, hipStream_t s);
void l_ritz_resid(int N, const long* sub_ptr, int q, const double* Z, const double* TZ, const double* mu, double* X,
                  double* res, int* conv, int* nsel, double tau, double window, double tol, double tol_far,
                  hipStream_t s);
void l_assemble_modes(int N, int maxns, int maxm, const long* sub_ptr, int q, const double* K, const long* koff_e,
                      const long* koff_c, const double* Z, const double* mu, double* Y, const long* yoff_e,
                      const long* yoff_c, double* lam, hipStream_t s);
void l_axpy_flat(long n, double a, const double* x, double* y, hipStream_t s);
}  // namespace awg
