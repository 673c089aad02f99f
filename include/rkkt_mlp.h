/*
 * Learned interior-point warm start: the multilayer perceptron that maps a
 * scenario's loads to a primal-dual start point, and its training step.
 *
 * The paper solves every load scenario of the same grid, so solutions of
 * nearby scenarios are close (case-study section); the perceptron learns that
 * map.  Network: layers of sizes sizes[0] -> ... -> sizes[n_layers], GELU
 * (erf form, g(a) = a Phi(a)) after every layer but the last; loss
 * 1/(2B) sum_b ||y_b - t_b||^2 over a batch of B rows.
 *
 * Precision: FP32 master parameters and Adam moments; every product runs on
 * BF16 copies of its operands (weights, activations, output gradients) with
 * FP32 accumulation; pre-activations, losses and gradients are FP32.
 *
 * Parameter layout (FP32, device): for every layer l in order, W_l as
 * [fan_in][fan_out] row-major (a layer is A W_l + b_l for a row-major batch
 * A [B][fan_in]), then b_l [fan_out].  Gradients use the same layout.
 *
 * All device pointers are caller-owned FP32 arrays.  Calls are ordered on
 * `stream`, allocate nothing (rkkt_mlp_create allocates all workspace for
 * up to batch_max rows) and never synchronise; a handle is used by one stream
 * at a time.  Errors: 0 OK, -1 bad argument (batch > batch_max, null
 * pointer), -2 HIP error, -6 out of memory (create); message in
 * rkkt_mlp_last_error.
 */
#ifndef RKKT_MLP_H
#define RKKT_MLP_H

#include <hip/hip_runtime.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rkkt_mlp rkkt_mlp;

/* sizes[0 .. n_layers]: input width, hidden widths, output width. */
int rkkt_mlp_create(const int* sizes, int n_layers, int batch_max, rkkt_mlp** out);
int rkkt_mlp_destroy(rkkt_mlp* m);
const char* rkkt_mlp_last_error(const rkkt_mlp* m);

/* Number of FP32 parameters (sum over layers of fan_in fan_out + fan_out). */
long long rkkt_mlp_n_params(const rkkt_mlp* m);

/* Load the master parameters (and refresh the BF16 copies); zeroes the Adam
 * moments and the step count. */
int rkkt_mlp_set_params(rkkt_mlp* m, const float* params, hipStream_t stream);
int rkkt_mlp_get_params(const rkkt_mlp* m, float* params, hipStream_t stream);

/* y [batch][out] = network(x [batch][in]). */
int rkkt_mlp_forward(rkkt_mlp* m, const float* x, int batch, float* y, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the same
 * y [batch][out] = network(x [batch][in]) as rkkt_mlp_forward, with the
 * input and hidden activations in a static 8 MiB device workspace of the
 * library instead of the handle's buffers, so batch is limited by that
 * workspace (not by batch_max): sum over layers l < n_layers of batch
 * rounded-up-to-8(sizes[l]) BF16 values, each layer's region rounded up to
 * 256 bytes, must fit in 8 MiB (2416 rows for 198 -> 512 -> 512 -> 512 -> 896);
 * a larger batch returns -1 with the limit in the message.  Allocates
 * nothing, frees nothing, does not synchronise.  Every call on a GPU shares
 * that GPU's workspace, which keeps the last call's contents: calls that
 * overlap on one GPU (two streams, two threads) race and must be ordered by
 * the caller.  The handle is only read (its parameters). */
int rkkt_mlp_forward_static(const rkkt_mlp* m, const float* x, int batch, float* y, hipStream_t stream);

/* Loss (loss[0], device) and its gradient with respect to every parameter
 * (grads [n_params], parameter layout; may be NULL) at the current
 * parameters, for targets t [batch][out]. */
int rkkt_mlp_gradients(rkkt_mlp* m, const float* x, const float* t, int batch, float* grads,
                       float* loss, hipStream_t stream);

/* One Adam step (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrected) on the master parameters with learning rate lr, after
 * rkkt_mlp_gradients; loss[0] gets the batch loss before the step. */
int rkkt_mlp_train_step(rkkt_mlp* m, const float* x, const float* t, int batch, float lr,
                        float* loss, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif
