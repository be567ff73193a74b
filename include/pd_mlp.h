/*
 * pd_mlp.h -- C ABI of the surrogate network for the RVE bulk response.
 *
 * A multilayer perceptron maps the 6 Voigt components of macroscopic strain to
 * the 6 Voigt components of bulk stress and the damage fraction of a
 * representative volume of a grain aggregate.  The paper's convergence study
 * of aggregate size (Sec. 7.5: the normalised top-wall force converges as the
 * number of grains grows) points at such a representative volume; the
 * training data come from the simulator in pd.h.
 *
 * Network: layers dims[0] -> dims[1] -> ... -> dims[n-1]; every hidden layer is
 * Z = X W + b followed by GELU(z) = z Phi(z) with the exact erf, the last layer
 * is linear.  Matrix products run on BF16 matrix cores with FP32 accumulation;
 * master weights, biases, activations kept for backward and Adam state are FP32.
 *
 * Parameters are exchanged as one FP32 vector in the order
 * [W_1 (dims[0] x dims[1], row-major), b_1, W_2, b_2, ...].
 * Loss: mean over samples and outputs of (Y_hat - Y)^2.
 *
 * Ownership and errors follow pd.h: caller pointers are read during the call
 * only; x, y (and y_hat) are device pointers to row-major FP32 [batch][dim]
 * arrays; every call returns a status (PD_OK, PD_ERR_*), details in
 * pdm_last_error.  All work runs on the stream given at creation.
 */
#ifndef PD_MLP_H
#define PD_MLP_H

#include <stdint.h>

#include "pd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdm_net pdm_net;

/* Create a network; n_dims >= 2, every dim in [1, 1024]; max_batch bounds the
   batch of pdm_train_step / pdm_gradients (workspace is sized for it).
   alloc/free_fn: the caller's device allocator (for example PyTorch's caching
   allocator), used for every device buffer of the network; both NULL for
   hipMalloc/hipFree, one NULL without the other is PD_ERR_INVALID.
   stream: hipStream_t (not the legacy null stream) or NULL for an owned one. */
pd_status pdm_create(pdm_net** out, const int32_t* dims, int32_t n_dims, int64_t max_batch,
                     pd_alloc_fn alloc, pd_free_fn free_fn, void* alloc_user, void* stream);
int64_t pdm_param_count(const pdm_net* net);
/* Load parameters (host FP32 vector of pdm_param_count entries); resets Adam. */
pd_status pdm_set_params(pdm_net* net, const float* params, int64_t n);
pd_status pdm_get_params(pdm_net* net, float* params, int64_t n);
/* Adam hyper-parameters (defaults 0.9, 0.999, 1e-8, 0): the update is
   p -= lr (m_hat / (sqrt(v_hat) + eps) + weight_decay p), decay decoupled from
   the gradient moments. */
pd_status pdm_set_adam(pdm_net* net, float beta1, float beta2, float eps, float weight_decay);
/* Inference: y[batch][dims[n-1]] = net(x[batch][dims[0]]); any batch size
   (processed in chunks of max_batch).  Matrix products use gfx950's
   16 x 16 x 32 BF16 matrix-core instruction.  For dims {din <= 16, 256, 256, 256,
   dout <= 16} a fused path runs by default: two kernels with a weight matrix
   resident in LDS, the first hidden pair's activations kept in registers and
   only the second hidden layer's BF16 activations stored between them; its
   operands are rounded to BF16 where the layer-by-layer path rounds them. */
pd_status pdm_forward(pdm_net* net, const float* x, int64_t batch, float* y);
/* Choose the inference path: fused != 0 selects the fused kernels (error
   PD_ERR_UNSUPPORTED when the dims or the device do not allow them), 0 the
   layer-by-layer kernels used for training. */
pd_status pdm_set_inference(pdm_net* net, int32_t fused);
/* Loss and gradient (host vector of pdm_param_count entries) of the mean
   squared error, without updating the parameters. */
pd_status pdm_gradients(pdm_net* net, const float* x, const float* y, int64_t batch, float* loss,
                        float* grad);
/* One Adam step on the mean squared error of the batch; loss (host) may be NULL. */
pd_status pdm_train_step(pdm_net* net, const float* x, const float* y, int64_t batch, float lr,
                         float* loss);
void pdm_destroy(pdm_net* net);
const char* pdm_last_error(const pdm_net* net);

#ifdef __cplusplus
}
#endif
#endif
