/* C ABI of the surrogate network used to pick model parameters.
 *
 * The lattice Boltzmann model of include/lbm.h is tuned by (T/T_c, kappa,
 * epsilon): Section IV shows that kappa sets the surface tension while the
 * density ratio stays put, and the mechanical-stability condition Eq. (16)
 * ties the coexistence densities to epsilon and the EOS.  The library learns
 * the map (T/T_c, kappa, epsilon) -> (rho_l, rho_v, sigma) from runs of the
 * solver itself with a small multilayer perceptron, trained and evaluated by
 * the kernels behind this header:
 *
 *   h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = W3 h2 + b3,
 *   x in R^3, h1, h2 in R^64, y in R^3, all FP32.
 *
 * Parameters are one FP32 vector of LBM_MLP_PARAMS values, row-major
 * matrices (out x in) in the order W1[64][3], b1[64], W2[64][64], b2[64],
 * W3[3][64], b3[3].  Loss over a batch with per-entry weights m (0 masks a
 * missing target): L = sum m_ik (y_ik - t_ik)^2 / (2 sum m_ik).  Training is
 * full-batch Adam (Kingma & Ba 2015, Algorithm 1, bias-corrected moments).
 * Scaling of inputs and targets is the caller's.
 *
 * Conventions as in lbm.h: the caller owns the device workspace (>= 256-byte
 * aligned, at least lbm_mlp_workspace_bytes) and every array; x, t, m, y are
 * DEVICE pointers to row-major [n][3] FP32 arrays; params and grad are HOST
 * arrays of LBM_MLP_PARAMS floats.  Work is enqueued on the given stream;
 * calls that return host data synchronise it.  Errors return a status and
 * leave a message for lbm_last_error(); an lbm_mlp is used by one thread at a
 * time.
 */
#ifndef LBM_MLP_H
#define LBM_MLP_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_MLP_IN 3
#define LBM_MLP_HIDDEN 64
#define LBM_MLP_OUT 3
#define LBM_MLP_PARAMS 4611
#define LBM_MLP_MAX_BATCH 1048576

typedef struct lbm_mlp lbm_mlp;

/* Device workspace for batches of up to max_batch samples (0 if max_batch is
 * outside [1, LBM_MLP_MAX_BATCH]). */
size_t lbm_mlp_workspace_bytes(int32_t max_batch);

/* Creates a network with the given initial parameters (host, required: the
 * caller draws them) and zero Adam moments.  stream: hipStream_t or NULL. */
lbm_status lbm_mlp_create(int32_t max_batch, const float *params, void *workspace, size_t workspace_bytes,
                          void *stream, lbm_mlp **out);

/* Replaces the parameters and resets the Adam moments and step count. */
lbm_status lbm_mlp_set_params(lbm_mlp *net, const float *params);

/* Copies the parameters to the host; synchronises. */
lbm_status lbm_mlp_get_params(lbm_mlp *net, float *params);

/* Inference: y = f(x) for n samples (0 <= n <= max_batch); asynchronous. */
lbm_status lbm_mlp_forward(lbm_mlp *net, const float *x, int32_t n, float *y);

/* Loss and its gradient with respect to the parameters at the current
 * parameters (no update).  grad may be NULL.  EINVAL if every weight is 0.
 * Synchronises. */
lbm_status lbm_mlp_loss_grad(lbm_mlp *net, const float *x, const float *t, const float *m, int32_t n,
                             double *loss, float *grad);

/* `steps` full-batch Adam steps (learning rate lr, decay rates beta1 and
 * beta2 in [0, 1), eps > 0); the step count carries over between calls.
 * last_loss (nullable) receives the loss before the final update.
 * Synchronises. */
lbm_status lbm_mlp_train(lbm_mlp *net, const float *x, const float *t, const float *m, int32_t n,
                         int32_t steps, float lr, float beta1, float beta2, float eps, double *last_loss);

/* Adam steps taken so far. */
int64_t lbm_mlp_steps_taken(const lbm_mlp *net);

void lbm_mlp_destroy(lbm_mlp *net);

#ifdef __cplusplus
}
#endif

#endif /* LBM_MLP_H */
