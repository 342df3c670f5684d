/*
 * pdipm_mlp.h - learned warm start of the interior-point solver: a ReLU
 * multilayer perceptron that maps the parameters theta of a parametric
 * problem to a start point (x, lambda), trained and evaluated on the GPU.
 *
 * The paper has no learned warm start; this is the warm-start form of the
 * parametric-QP benchmark.  The network (layer sizes dims[0..L]) is
 *   h_0 = theta, h_l = relu(W_l h_{l-1} + b_l) for l < L, z = W_L h_{L-1} + b_L,
 *   x_hat = x_scale * sigmoid(z[0..n_x)), lambda_hat = softplus(z[n_x..dims[L])),
 * trained on the loss
 *   x_weight mean (sigmoid(z_x) - x / x_scale)^2 + mean (log(softplus(z_l) + 1e-6) - log(lambda + 1e-6))^2
 * (means over batch rows and the x or lambda outputs) with Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias correction).
 *
 * Precision: parameters have FP32 master copies and BF16 working copies;
 * every matrix product takes BF16 operands with FP32 accumulation (MFMA);
 * activations are stored in BF16, the output pre-activation, the loss and
 * all gradients in FP32.  Sums are taken in a fixed order (results are
 * deterministic).
 *
 * Conventions as in pdipm.h: status codes PDIPM_*, the caller owns the
 * device workspace and the stream, no exceptions cross the ABI, a handle is
 * not thread-safe.  Parameter arrays on the host are FP32, layer by layer:
 * W_1 (dims[1] x dims[0], row-major), b_1 (dims[1]), W_2, b_2, ...
 * Device inputs are row-major batches: theta (B x dims[0]) FP32, targets
 * (B x dims[L]) FP32 holding the raw x and lambda.
 */
#ifndef PDIPM_MLP_H
#define PDIPM_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "pdipm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlp_handle mlp_handle;

/* n_layers >= 1 linear layers, dims[0..n_layers] (each >= 1), the first n_x
 * outputs are x (0 <= n_x <= dims[n_layers]) in (0, x_scale), x_weight > 0
 * weighs the x term of the loss, max_batch >= 1 rows per call.
 * Errors: PDIPM_ERR_INVALID_ARG (message in mlp_last_error(NULL)). */
int mlp_create(int32_t n_layers, const int32_t* dims, int32_t n_x, double x_scale, double x_weight,
               int32_t max_batch, mlp_handle** out);
int mlp_num_params(mlp_handle* h, int64_t* count);
int mlp_workspace_query(mlp_handle* h, size_t* bytes);
/* Device workspace (caller-owned, 256-byte aligned, >= queried bytes). */
int mlp_set_workspace(mlp_handle* h, void* d_workspace, size_t bytes);
int mlp_set_stream(mlp_handle* h, void* hip_stream);
/* Host FP32 parameters in; resets the optimiser state. */
int mlp_set_params(mlp_handle* h, const float* h_params);
int mlp_get_params(mlp_handle* h, float* h_params);
/* d_out (B x dims[L], FP32) = transformed outputs (x_hat, lambda_hat). */
int mlp_forward(mlp_handle* h, const float* d_theta, float* d_out, int32_t B);
/* Loss (host, may be NULL) and, if h_grads is not NULL, the FP32 gradients
 * in the parameter layout, without updating the parameters. */
int mlp_gradients(mlp_handle* h, const float* d_theta, const float* d_target, int32_t B, float* h_loss,
                  float* h_grads);
/* One Adam step on the batch; h_loss (may be NULL) receives the loss before
 * the step (reading it synchronises the stream). */
int mlp_train_step(mlp_handle* h, const float* d_theta, const float* d_target, int32_t B, float lr,
                   float* h_loss);
/* Algorithmic work of the matrix products of one forward (or one training)
 * pass over B rows, in flops (2 per multiply-add). */
double mlp_flops(mlp_handle* h, int32_t B, int32_t training);
const char* mlp_last_error(const mlp_handle* h);
void mlp_destroy(mlp_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* PDIPM_MLP_H */
