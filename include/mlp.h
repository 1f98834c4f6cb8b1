/*
 * mlp.h -- C ABI of the proposal network in libmodal.so: a multilayer
 * perceptron dims[0] -> dims[1] -> ... -> dims[L], ReLU between layers and a
 * linear output, trained by the library's own kernels (BF16 MFMA GEMMs with
 * FP32 accumulation, FP32 master weights, Adam).
 *
 * It maps spectral features of a target sound to initial physical
 * parameters for gradient fitting (paper: Sec. 5 names a more structured
 * initialisation as the remedy for the sensitivity of physical-parameter
 * fits to their starting point; Sec. 4.3 reports that sensitivity).
 *
 * Conventions as in modal.h: status codes (MODAL_*), streams as void*,
 * device pointers are HIP device memory.  Parameters are laid out layer by
 * layer as W_l [dims[l+1]][dims[l]] (row-major) followed by b_l [dims[l+1]].
 */
#ifndef MLP_H
#define MLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlp_ctx mlp_ctx;

/* Allocates parameters (zeroed), gradients, Adam moments and activation
 * buffers for batches of up to max_batch rows.  dims has n_layers + 1 entries
 * in 1..65536.  Errors: EINVAL, ENOMEM, EHIP. */
int mlp_init(mlp_ctx **out, int32_t n_layers, const int32_t *dims, int32_t max_batch, void *stream);

/* Number of parameters (all W and b). */
int mlp_n_params(const mlp_ctx *c, int64_t *n);

/* Copies parameters from host memory [n_params] and clears the Adam moments. */
int mlp_set_params(mlp_ctx *c, const float *host, void *stream);

/* Copies parameters (which = 0) or the last gradients (which = 1) to host. */
int mlp_get(mlp_ctx *c, int32_t which, float *host, void *stream);

/* y [B][dims[L]] = network(x [B][dims[0]]), device buffers, B <= max_batch.
 * Keeps the activations for mlp_backward. */
int mlp_forward(mlp_ctx *c, const float *x, int32_t B, float *y, void *stream);

/* Gradients of sum_b dy[b] . y[b] with respect to every parameter for the
 * batch of the last mlp_forward (dy device [B][dims[L]]); overwrites the
 * stored gradients.  ESTATE without a forward pass. */
int mlp_backward(mlp_ctx *c, const float *dy, void *stream);

/* One Adam step (Kingma & Ba, bias-corrected, step number t >= 1) on the
 * stored gradients. */
int mlp_adam_step(mlp_ctx *c, float lr, float beta1, float beta2, float eps, int32_t t, void *stream);

/* One training step of the mean squared error on a batch drawn by index:
 * x_b = X[idx[b]] (rows of dims[0] floats), z_b = Z[idx[b]] (rows of
 * dims[L] floats), b < B <= max_batch; forward, gradient of
 * L = sum_b |y_b - z_b|^2 / (B dims[L]), backward and one Adam step (as
 * mlp_adam_step with step number t), all on `stream` without host
 * synchronisation; adds L to *loss_acc (device float) unless loss_acc is
 * NULL.  X, Z, idx (int64, each in range; not checked) and loss_acc are
 * device memory.  Leaves the batch's activations and gradients as
 * mlp_forward and mlp_backward would.  Errors: EINVAL, EHIP. */
int mlp_train_step(mlp_ctx *c, const float *X, const float *Z, const int64_t *idx, int32_t B, float lr,
                   float beta1, float beta2, float eps, int32_t t, float *loss_acc, void *stream);

/* n_steps training steps as mlp_train_step, step st on the rows
 * order[st B .. st B + B) (int64, device, in range; not checked), with the
 * learning rate lr and Adam step numbers continuing the context's own count
 * (0 after mlp_init or mlp_set_params; the first step of the first epoch is
 * step 1).  The first call with a given (X, Z, order, n_steps, B, beta1,
 * beta2, eps, loss_acc) records the epoch as a HIP graph; later calls with
 * the same pointers replay it, reading lr and the step count from device
 * memory, so the caller refills order in place between epochs.  No host
 * synchronisation.  Errors: EINVAL, EHIP. */
int mlp_train_epoch(mlp_ctx *c, const float *X, const float *Z, const int64_t *order, int32_t n_steps,
                    int32_t B, float lr, float beta1, float beta2, float eps, float *loss_acc, void *stream);

void mlp_destroy(mlp_ctx *c);
const char *mlp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MLP_H */
