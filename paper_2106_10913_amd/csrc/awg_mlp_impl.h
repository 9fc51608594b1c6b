// Internal view of the warm-start network (k_mlp.hip) for the set-up code.
#pragma once
#include <string>
#include <vector>

#include "awg_common.h"

// Per-dof perceptron: layer sizes dims[0] = F inputs, dims[1..L-1] = width,
// dims[L] = p outputs; W_l row-major (dims[l] x dims[l-1]) followed by b_l in
// one FP32 parameter vector.
struct awg_mlp {
  std::vector<int> dims;
  std::vector<long> offW, offB;
  long nparams = 0;
  awg::DBuf<float> w, g, m1, m2;       // parameters, gradient, Adam moments
  awg::DBuf<uint16_t> wb;              // bf16 copy of w (inference)
  bool wb_valid = false;
  long adam_t = 0;
  awg::DBuf<float> acts, dH0, dH1, part, loss_s;   // training workspace
  long ws_rows = 0;
  std::string err = "no error";
};

namespace awg {
constexpr int MLP_FEATURES = 12;      // per-dof features computed by l_mlp_features
constexpr int MLP_MAX_OUT = 16;       // outputs (and target columns) per row
constexpr int MLP_MAX_WIDTH = 256;

// Y (rows x p, row-major) = network(X (rows x F, row-major)); bf16: fused
// BF16-MFMA kernel with FP32 accumulation, else FP32 layer by layer.
void mlp_forward(awg_mlp& m, long rows, const float* X, float* Y, bool bf16, hipStream_t s);

// Features of every (subdomain, local dof) row, in sub_ptr order
// (Sigma n_s x MLP_FEATURES, row-major FP32).  coords: n x cdim node
// coordinates of every dof or NULL.
void l_mlp_features(int N, int n, int maxns, const long* sub_ptr, const int* sub_idx, const int* rowptr,
                    const int* col, const double* val, const int* inv_ptr, const int* inv_sub, const int* inv_loc,
                    const int* mult, const double* V, const long* v_eoff, const long* v_coff, const double* P,
                    const long* sq_off, const double* coords, int cdim, float* out, hipStream_t s);

// Column-major iterated blocks X_s (n_s x q at sub_ptr[s] * q): columns 0..p-1
// from the rows of O (Sigma n_s x p, row-major), normalised to unit length.
void l_block_from_rows(int N, int maxns, const long* sub_ptr, int q, int p, const float* O, double* X,
                       hipStream_t s);
}  // namespace awg
