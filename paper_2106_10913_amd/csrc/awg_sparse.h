// Launchers of the sparse / vector / set-up kernels (k_sparse.hip).
#pragma once
#include "awg_common.h"

namespace awg {
void l_validate_subs(int N, const long* sub_ptr, const int* sub_idx, int n, int* err, hipStream_t s);
void l_entry_owner(int N, const long* sub_ptr, int* ent_sub, hipStream_t s);
void l_mult(long tot, const int* sub_idx, int* mult, hipStream_t s);
void l_check_cover(int n, const int* mult, int* err, hipStream_t s);
void l_scan(int n, const int* in, int* out, hipStream_t s);
void l_fill_inv(int N, const long* sub_ptr, const int* sub_idx, const int* inv_ptr, int* fill, int* inv_sub,
                int* inv_loc, hipStream_t s);
void l_sort_inv(int n, const int* inv_ptr, int* inv_sub, int* inv_loc, hipStream_t s);
void l_pairs(int n, const int* rowptr, const int* col, const double* val, const int* inv_ptr, const int* inv_sub,
             int* cnt, double* bval, int* err, hipStream_t s);
void l_pou(long tot, const int* sub_idx, const int* mult, double* dw, hipStream_t s);
void l_extract(int N, const long* sub_ptr, const int* sub_idx, const int* rowptr, const int* col,
               const double* vals, const MatDesc* mats, hipStream_t s);
// Groups of up to 4 consecutive rows stored over the union of their column
// patterns (zeros where a row has no entry), for the grouped SpMM kernel
struct SpmmGroups {
  // pattern to build the groups from when they are first needed (the host
  // analysis of every row costs tens of ms on large matrices and is skipped
  // when the autotuner's choice for a shape is already another variant)
  bool pending = false;
  int n = 0;
  long nnz = 0;
  const int* rowptr = nullptr;
  const int* col = nullptr;
  const double* val = nullptr;
  int ng = 0;
  DBuf<int> start;     // first row of each group, n at the end
  DBuf<int> uptr;      // offsets of the union patterns in ucol (ng + 1)
  DBuf<int> ucol;      // union column indices, ascending per group
  DBuf<long> voff;     // offset of each group's G x |U| value block in gval
  DBuf<double> gval;   // values, row g of a group at voff + g |U|
};
// multi-column vectors are row-major (b contiguous values per row); grp
// (optional): row groups from spmm_groups, offered to the autotuner
// (the CSR may have more columns than rows: X then has one row per column);
// label: name under which the kernel timer records the launch
void l_spmm(int n, long nnz, const int* rowptr, const int* col, const double* val, const double* X, double* Y, int b,
            double alpha, double beta, hipStream_t s, const SpmmGroups* grp = nullptr, const char* label = nullptr);
// builds the groups of a validated CSR pattern (columns sorted per row): a
// group grows while its union pattern stays within 1.4 times its longest
// row; returns the number of groups, or 0 (g left empty) when grouping would
// not cut the row count by a quarter
int spmm_groups(int n, long nnz, const int* rowptr, const int* col, const double* val, SpmmGroups& g,
                hipStream_t s);
// defer spmm_groups on this pattern until a product needs the groups
void spmm_groups_defer(int n, long nnz, const int* rowptr, const int* col, const double* val, SpmmGroups& g);
void l_gather(long tot, const int* sub_idx, const double* X, int b, double* Xs, hipStream_t s);
// the same rows rounded to FP32 (the operand of the FP32 local products)
void l_gather_f32(long tot, const int* sub_idx, const double* X, int b, float* Xs, hipStream_t s);
void l_scatter(int n, long tot, const int* inv_ptr, const int* inv_sub, const int* inv_loc, const long* sub_ptr,
               const double* Zs, int b, double* Y, double alpha, double beta, hipStream_t s);
// Y = (scatter of Zs) + A G for a CSR matrix A (n x m) and G (m x b) in one
// pass (b > 1); false, with nothing launched, where its 16-byte paths do not
// apply (odd b or unaligned buffers): the caller then runs the two steps
bool l_scatter_prolong(int n, long tot, const int* inv_ptr, const int* inv_sub, const int* inv_loc,
                       const long* sub_ptr, const double* Zs, int b, int m, long nnz, const int* rowptr, const int* col,
                       const double* val, const double* G, double* Y, hipStream_t s);
// part: max(DOT_CHUNKS_H * b, DOT1_BLOCKS) scratch doubles
constexpr int DOT_CHUNKS_H = 256;
constexpr int DOT1_BLOCKS = 2048;  // blocks (and partial sums) of the one-column kernels
void l_coldot(int n, int b, const double* X, const double* Y, double* part, double* out, hipStream_t s);
// one column: q = A p with part[k] = the k-th of DOT1_BLOCKS partial sums of p^T q
void l_spmv_dot(int n, long nnz, const int* rowptr, const int* col, const double* val, const double* p, double* q,
                double* part, hipStream_t s);
// CSR (arp, acol, aval) of [A | L] (rowptr != NULL: columns of L shifted by
// n) or of L alone: L the n x sum_s k_s prolongation of the per-subdomain
// n_s x k_s column-major blocks B + eoff[s] (k_s = coff[s+1] - coff[s]),
// column coff[s] + j = R^sT B^s e_j; returns its number of entries
long l_aug_csr(int n, const int* rowptr, const int* col, const double* val, const int* inv_ptr, const int* inv_sub,
               const int* inv_loc, const long* sub_ptr, const long* eoff, const long* coff, const double* B,
               int colbase, DBuf<int>& arp, DBuf<int>& acol, DBuf<double>& aval, hipStream_t s);
// extended index sets N(Omega^s) = {i : A_ij != 0 for some j in Omega^s},
// ascending, concatenated (h_ext_ptr: host copy of the offsets); returns their total size
long l_ext_sets(int N, int n, const long* sub_ptr, const int* sub_idx, const int* rowptr, const int* col,
                std::vector<long>& h_ext_ptr, DBuf<long>& ext_ptr, DBuf<int>& ext_idx, hipStream_t s);
// AY^s = A[N(Omega^s), Omega^s] Y^s, |N_s| x m_s column-major blocks at AY + ay_eoff[s]
void l_ext_ay(int N, const long* ext_ptr, const int* ext_idx, const long* sub_ptr, const int* sub_idx,
              const int* rowptr, const int* col, const double* val, const double* Y, const long* y_eoff,
              const long* y_coff, const long* ay_eoff, double* AY, hipStream_t s);
// D (n x ld row-major, zero on entry) = columns c0 .. c0 + ld - 1 of the
// dense prolongation of the blocks B + eoff[s]
void l_lowrank_dense(int n, const int* inv_ptr, const int* inv_sub, const int* inv_loc, const long* sub_ptr,
                     const long* eoff, const long* coff, const double* B, long c0, long ld, double* D,
                     hipStream_t s);
// CSR (rp, tcol, tval) of L^T (ncols = sum_s k_s rows, n columns) for the
// same prolongation; returns its number of entries
long l_aug_csr_t(int N, long ncols, const long* sub_ptr, const int* sub_idx, const long* eoff, const long* coff,
                 const double* B, DBuf<int>& rp, DBuf<int>& tcol, DBuf<double>& tval, hipStream_t s);
// r = b - A x in compensated (double-double) arithmetic, rounded once to FP64
void l_resid_dd(int n, long nnz, const int* rowptr, const int* col, const double* val, const double* x,
                const double* b, double* r, hipStream_t s);
// one column: part[k] = the k-th of DOT1_BLOCKS partial sums of x^T y
void l_dot1_part(int n, const double* x, const double* y, double* part, hipStream_t s);
void l_colaxpby(long rows, int b, const double* X, const double* a, double* Y, const double* bb, double sa, double sb,
                hipStream_t s);
// scratch doubles that l_multi_update_xr and l_coldot2 need in part
long rb_part_size(int n, int b);
// multi-column PCG steps in single passes (part: rb_part_size(n, b) doubles):
// X += a P, R -= a Q and rr = column norms^2 of the new R
void l_multi_update_xr(int n, int b, const double* a, const double* P, double* X, const double* Q, double* R,
                       double* part, double* rr, hipStream_t s);
// out1 = column dots X^T Y1, out2 = X^T Y2 (Y2 may be NULL) reading X once
void l_coldot2(int n, int b, const double* X, const double* Y1, const double* Y2, double* part, double* out1,
               double* out2, hipStream_t s);
// P = Z + beta P, and Zold = Z when Zold != NULL
void l_multi_update_p(long rows, int b, const double* Z, double* P, const double* beta, double* Zold, hipStream_t s);
void l_set_identity(const MatDesc* mats, int batch, hipStream_t s);
void l_copy_mat(const MatDesc* src, const MatDesc* dst, int batch, hipStream_t s);
void l_scale_sym(const MatDesc* mats, int batch, const long* voff, const double* d, bool inv, bool symmetrize,
                 hipStream_t s);
void l_transpose_inplace(const MatDesc* mats, int batch, hipStream_t s);
void l_scale_cols(const MatDesc* mats, int batch, const long* coff, const double* f, double alpha,
                  const double* shift, int mode, hipStream_t s);
void l_diag_mean(const MatDesc* mats, int batch, double* out, hipStream_t s);
void l_mb_neighbours(int N, const long* sub_ptr, const int* sub_idx, const int* mult, const int* inv_ptr,
                     const int* inv_sub, const int* inv_loc, const MatDesc* mats, const double* V, const long* voff,
                     const double* lam, const long* loff, hipStream_t s);
}  // namespace awg
