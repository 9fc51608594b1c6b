/* Warm-start network for the subspace GenEO eigensolver (C ABI).
 *
 * The network is not part of the paper.  It predicts, for every dof of every
 * subdomain, p values whose columns start the block subspace iteration that
 * finds the GenEO modes of the subdomain (Theorem on H^NN_hyb, Section 3.4);
 * the eigensolver refines the block to the same residuals and certificate as
 * from a random start, so the selected modes do not depend on the network.
 *
 * Network: a perceptron applied to each row x (in_features values):
 *   h_0 = x;  h_l = tanh(h_{l-1} W_l^T + b_l) for the hidden layers (width);
 *   output = h_L W_{L+1}^T + b_{L+1}  (out_channels values).
 * Parameters: one FP32 vector holding W_1 (row-major, out x in), b_1, W_2, b_2,
 * ...; Glorot-uniform initial weights from a counter-based generator, zero
 * biases.
 *
 * Training loss for a batch of subdomains s with predicted block P_s (its
 * rows of the output, n_s x out_channels) and target modes T_s (n_s x m_s):
 *   L = mean over {s : m_s > 0} of
 *       min_C (||T_s - P_s C||_F^2 + eps_s ||C||_F^2) / ||T_s||_F^2,
 *   eps_s = ridge * n_s,
 * invariant under rotations of P_s and of T_s.
 *
 * All pointers named X, Y, T, row_ptr, tgt_off, tgt_cols are device pointers;
 * host buffers are named host.  Functions return awg_status codes (awg.h). */
#ifndef AWG_MLP_H
#define AWG_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct awg_mlp awg_mlp;

/* Per-dof input features the solver computes for a learned start (row order:
 * subdomain by subdomain, local dofs in list order):
 *   0-2  node coordinates scaled to [-1, 1] over the subdomain's bounding box
 *        (0 when no coordinates are given);
 *   3    (log10 A_ii - mean over the subdomain of log10 A_jj) / 4;
 *   4    (log10 A_ii - mean over all dofs of log10 A_jj) / 4;
 *   5, 6 (max, min over the graph neighbours j of log10 A_jj - log10 A_ii) / 4;
 *   7    (mean over the neighbours of log10 |A_ij| - log10 A_ii) / 4;
 *   8    D^s_ii = 1 / multiplicity;
 *   9    graph distance to the outside of the subdomain, capped at 4, / 4;
 *   10   n_s / k_s * sum_j (D^s V^s_-)_ij^2 (kernel leverage; 0 when k_s = 0);
 *   11   (log10 P_ii - mean over the subdomain of log10 P_jj) / 4 with
 *        P = D^s (A^s_+)^+ D^s. */
#define AWG_MLP_FEATURES 12

/* in_features 1..32, width 16..256 (multiple of 16), hidden_layers 1..8,
 * out_channels 1..16.  *out receives the handle (NULL on error). */
int awg_mlp_create(awg_mlp** out, int32_t in_features, int32_t width, int32_t hidden_layers,
                   int32_t out_channels, uint64_t seed);
int64_t awg_mlp_num_params(const awg_mlp* m);
/* Copy the FP32 parameter vector (count = awg_mlp_num_params) to / from host memory. */
int awg_mlp_get_params(const awg_mlp* m, float* host, int64_t count);
int awg_mlp_set_params(awg_mlp* m, const float* host, int64_t count);

/* Y (rows x out_channels, row-major FP32) = network(X (rows x in_features,
 * row-major FP32)).  bf16 != 0: fused BF16 matrix-core kernel with FP32
 * accumulation (weights rounded to BF16); else FP32 throughout.  Synchronous. */
int awg_mlp_forward(awg_mlp* m, int64_t rows, const float* X, float* Y, int32_t bf16, void* stream);

/* FP32 forward and backward pass over rows = row_ptr[nsub] rows of X grouped
 * into nsub subdomains (row_ptr: nsub + 1 offsets from 0).  Subdomain s has
 * tgt_cols[s] (0..16) target columns, column-major n_s x m_s at
 * T + tgt_off[s].  Stores the gradient of L in the model; *loss_host (may be
 * NULL) receives L.  Synchronous. */
int awg_mlp_loss_grad(awg_mlp* m, int64_t rows, const float* X, int32_t nsub, const int64_t* row_ptr,
                      const int64_t* tgt_off, const int32_t* tgt_cols, const float* T, double ridge,
                      double* loss_host, void* stream);
/* Copy the last gradient (count = awg_mlp_num_params) to host memory. */
int awg_mlp_get_grads(const awg_mlp* m, float* host, int64_t count);

/* One Adam step (Kingma and Ba, 2015) with the stored gradient. */
int awg_mlp_adam_step(awg_mlp* m, double lr, double beta1, double beta2, double eps, void* stream);

/* Message of the last failure of m (m = NULL: of the last failed create). */
const char* awg_mlp_last_error(const awg_mlp* m);
void awg_mlp_destroy(awg_mlp* m);

#ifdef __cplusplus
}
#endif
#endif
