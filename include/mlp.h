/*
 * mlp.h - C ABI of the surrogate network's HIP kernels (gfx950).
 *
 * A 3 -> 64 -> 64 -> 1 multilayer perceptron with tanh hidden units, FP32,
 * mapping (G^a, G^r, log shear rate) of a lattice Boltzmann run to its mean
 * wall shear stress.  It is trained on points produced by batched lattice
 * runs (lbb_* in lb.h) and proposes where to refine a flow curve; the lattice
 * runs remain the reference for its error.
 *
 * Inputs are standardised inside the kernels, x' = (x - in_mean)/in_std, and
 * the network's output is read on the standardised scale
 * y' = (y - out_mean)/out_std.  Loss: mean squared error on y'.  Training:
 * full-batch Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 *
 * Parameter vector layout (MLP_NPARAM floats): W1 (64 x 3 row-major), b1 (64),
 * W2 (64 x 64 row-major, W2[j*64 + k] feeds unit j from unit k), b2 (64),
 * W3 (64), b3 (1).
 *
 * Conventions follow lb.h: lb_status return codes, lb_last_error() for the
 * message, caller-owned device state of mlp_state_bytes(max_rows) bytes
 * (256-byte aligned), all work on the stream given at init; functions that
 * take or return host arrays synchronise.
 */
#ifndef MLP_H
#define MLP_H

#include <stddef.h>
#include <stdint.h>

#include "lb.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MLP_NPARAM 4481

typedef struct mlp_handle mlp_handle;

/* Device bytes for a network that trains / infers on up to max_rows rows. */
lb_status mlp_state_bytes(int32_t max_rows, size_t* bytes);
lb_status mlp_init(void* dev_state, size_t bytes, int32_t max_rows, void* hip_stream, mlp_handle** out);

/* Host float arrays of MLP_NPARAM values.  mlp_set_params also resets Adam. */
lb_status mlp_set_params(mlp_handle* h, const float* theta);
lb_status mlp_get_params(mlp_handle* h, float* theta);

/* Standardisation constants (in_std and out_std > 0). */
lb_status mlp_set_norm(mlp_handle* h, const float in_mean[3], const float in_std[3], float out_mean,
                       float out_std);

/* Uploads n <= max_rows training rows: X host (n, 3) row-major, y host (n). */
lb_status mlp_set_data(mlp_handle* h, const float* X, const float* y, int32_t n);

/* Loss on the uploaded data and its gradient (grad: host MLP_NPARAM or NULL). */
lb_status mlp_loss_grad(mlp_handle* h, float* loss, float* grad);

/* iters full-batch Adam steps at learning rate lr on the uploaded data;
 * *loss (may be NULL) receives the loss before the last step. */
lb_status mlp_train(mlp_handle* h, int32_t iters, float lr, float* loss);

/* Predictions on the original scale for n <= max_rows host rows X (n, 3). */
lb_status mlp_infer(mlp_handle* h, const float* X, int32_t n, float* y);

lb_status mlp_destroy(mlp_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* MLP_H */
