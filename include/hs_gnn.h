/*
 * hs_gnn -- C ABI of the hardness surrogate: a small edge message-passing
 * network that ranks proposed coupler mutations of the instance search
 * (Algorithm 1, Sec. II.A, proposes one mutation per step; the surrogate
 * screens several and parallel tempering scores the survivors).  The network
 * has no counterpart in the paper; its definition is:
 *
 *   graph of an instance on Chimera C_L (Appendix A, Fig. 8):
 *     node v = site 8 (L r + c) + 4 u + k, features (r/L, c/L, u, k/3, live)
 *     coupler q = (i, j), i < j, canonical order, features
 *       (J_q / 7, intra-cell, inter-cell along u = 0, inter-cell along u = 1)
 *       (J_q = 0 when q touches a missing site)
 *     directed edges 2q (i -> j) and 2q + 1 (j -> i)
 *   h0_v = W_en x_v + b_en,  m0_e = W_ee f_q(e) + b_ee
 *   three layers (width 64):
 *     m_e <- relu(W_m [h_src(e); h_dst(e); m_e] + b_m)
 *     h_v <- relu(W_h [h_v; sum of m_e over edges e into v] + b_h)
 *   y_hat = w_out . mean over live v of h_v + b_out      (predicts ln TTS)
 *   loss = mean over graphs with a finite label of (y_hat - label)^2
 *          (gnn_train_step_ranked adds child-against-parent differences)
 *
 * Parameters: one float32 vector of gnn_param_count() entries, blocks in the
 * order W_en [64][5], b_en, W_ee [64][4], b_ee, then per layer W_m [64][192],
 * b_m, W_h [64][128], b_h, then w_out [64], b_out [1] (row-major).
 * Precision: the matrix products run on bfloat16 operands (states, message
 * sums, W_m, W_h, and pre-activation gradients, rounded to nearest even) with
 * float32 accumulation (MFMA); biases, embeddings, readout, reductions,
 * master weights and Adam stay float32.
 *
 * Memory: every device pointer is the caller's and must stay valid until the
 * stream has finished; the library allocates no device memory.  Errors are
 * HS_* codes of hardspin.h with a thread-local message (hs_last_error).
 */
#ifndef HS_GNN_H
#define HS_GNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Number of float32 parameters (62593). */
int gnn_param_count(void);

/* A batch of graphs of the same size L (host memory, read during the call):
 *   live  n_graphs x N bytes (N = 8 L^2), 1 = working site; NULL = all live
 *   J     n_graphs x (24 L^2 - 8 L) couplings in canonical order */
typedef struct hs_gnn_batch {
    int32_t n_graphs;
    int32_t L;
    const uint8_t *live;
    const int8_t *J;
} hs_gnn_batch;

/* Device workspace bytes for n_graphs graphs of side L. */
int gnn_workspace_bytes(int32_t n_graphs, int32_t L, size_t *bytes);

/* Builds the node / edge features and the edge lists of the batch on the
 * host and copies them into the workspace on `stream` (synchronises the
 * stream).  Every graph needs at least one live site.  The workspace then
 * serves gnn_forward / gnn_train_step calls with the same (n_graphs, L). */
int gnn_prepare(const hs_gnn_batch *b, void *workspace, size_t workspace_bytes, void *stream);

/* y_hat (device float [n_graphs]) for the prepared batch.  Asynchronous. */
int gnn_forward(const float *params, int32_t n_graphs, int32_t L, void *workspace,
                size_t workspace_bytes, float *y_hat, void *stream);

/* Adam (Kingma and Ba) state: m, v device float [param_count]; step counts
 * from 1 and is used for the bias correction. */
typedef struct hs_adam {
    float lr, beta1, beta2, eps;
    int64_t step;
    float *m;
    float *v;
} hs_adam;

/* One training step on the prepared batch: forward, loss (device float [1]),
 * gradient of the loss with respect to every parameter (device float
 * [param_count], overwritten), y_hat (device float [n_graphs]) and, if adam
 * is not NULL, one Adam update of params in place.  labels: device float
 * [n_graphs]; non-finite labels are left out of the loss.  Asynchronous. */
int gnn_train_step(float *params, int32_t n_graphs, int32_t L, const float *labels, void *workspace,
                   size_t workspace_bytes, float *y_hat, float *loss, float *grad,
                   const hs_adam *adam, void *stream);

/* gnn_train_step with the ranked loss, for ranking proposed mutations
 * against the instance they were made from (the screen of the instance
 * search, Algorithm 1, Sec. II.A, orders a parent's one-coupler children):
 *   loss = mean over pairs of ((y_hat_g - y_hat_p) - (label_g - label_p))^2
 *          + w_abs * (the loss of gnn_train_step)
 * where graph g pairs with p = ref[g] when 0 <= p < n_graphs, p != g and
 * both labels are finite.  ref: device int32 [n_graphs] (-1 = no parent).
 * With common random numbers for a parent and its children the pair
 * differences carry far less noise than the labels.  w_abs >= 0.
 * HS_EINVAL for a NULL ref or a negative or non-finite w_abs; otherwise as
 * gnn_train_step.  Asynchronous. */
int gnn_train_step_ranked(float *params, int32_t n_graphs, int32_t L, const float *labels, const int32_t *ref,
                          float w_abs, void *workspace, size_t workspace_bytes, float *y_hat, float *loss,
                          float *grad, const hs_adam *adam, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HS_GNN_H */
