/*
 * librpca -- learned warm start for streaming Split-SPCP windows.
 *
 * The paper starts every solve from a randomized SVD (Sec. 4.2) and, for
 * streaming video, from nothing better; consecutive windows of one video
 * share most of their low-rank part (Sec. 5.4).  This part of the library
 * proposes the starting factors of a window from cheap statistics of it:
 *
 *   features  x = [ temporal mean of the factor-f average-pooled frames,
 *                   temporal standard deviation of the same,
 *                   mean of every frame ]                      (d_in values)
 *   network   y = relu(x W1 + b1) W2 + b2                      (2-layer MLP)
 *             y = [ U_low (mu x k, row-major) | V (nv x k, row-major) ]
 *   start     U = nearest-neighbour upsampling of U_low to full resolution,
 *             V as predicted; rpca_solve then runs from (U, V).
 *
 * Training pairs come from the solver itself: for a solved window with
 * factors (U*, V*) the target is the pooled low-rank part
 * T = pool(U*) V*^T (mu x nv), and the loss of a batch of B windows is
 *
 *   loss = (1/B) sum_b || U_low_b V_b^T - T_b ||_F^2 ,
 *
 * which depends on the factors only through their product, the one thing
 * the problem determines (Theorem 1: (U, V) are fixed only up to an
 * orthogonal k x k rotation).  Targets are passed as their factors
 * TU = pool(U*) (mu x k) and TV = V* (nv x k).
 *
 * Parameters are FP32 master weights; the GEMMs run on FP32 MFMA with FP32
 * accumulation; Adam (Kingma & Ba, with bias correction) updates them.
 *
 * Conventions are those of rpca.h: device pointers on the network's device,
 * row-major FP32 matrices, calls asynchronous on `stream`, argument checks
 * before any HIP call, 0 = success and < 0 = error (RPCA_EINVAL, RPCA_ENOMEM,
 * RPCA_EHIP).
 */
#ifndef RPCA_WARM_H
#define RPCA_WARM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rpca_mlp rpca_mlp;

enum rpca_mlp_tensor {
  RPCA_MLP_W1 = 0,  /* d_in x d_h, row-major */
  RPCA_MLP_B1 = 1,  /* d_h */
  RPCA_MLP_W2 = 2,  /* d_h x d_out, row-major, d_out = (mu + nv) * k */
  RPCA_MLP_B2 = 3   /* d_out */
};

/* Create a network.  d_in, d_h, mu, nv, k > 0; max_batch in [1, 4096] bounds
 * `batch` in every later call (workspace is sized for it).  Weights are drawn
 * from N(0, 2/fan_in) (He initialisation) with a SplitMix64 / Box-Muller
 * stream seeded by `seed`; biases and Adam moments start at zero.
 * On success *out owns device memory until rpca_mlp_destroy. */
int rpca_mlp_create(int32_t d_in, int32_t d_h, int32_t mu, int32_t nv, int32_t k,
                    int32_t max_batch, uint64_t seed, rpca_mlp** out);

/* Device pointer and element count of a parameter tensor (`which` from
 * rpca_mlp_tensor).  The storage belongs to the network; callers may read
 * and overwrite it (for checkpoints or tests) between calls. */
int rpca_mlp_param(rpca_mlp* net, int32_t which, float** ptr, int64_t* count);

/* Same for the gradient buffers filled by rpca_mlp_loss_grad. */
int rpca_mlp_grad(rpca_mlp* net, int32_t which, float** ptr, int64_t* count);

/* Forward pass.  x: device, batch x d_in; y: device, batch x d_out. */
int rpca_mlp_forward(rpca_mlp* net, const float* x, int32_t batch, float* y, void* stream);

/* Loss and gradients of all four tensors for one batch.
 * x: device batch x d_in; TU: device batch x mu x k; TV: device batch x nv x k;
 * loss: device, one double (the batch loss defined above). */
int rpca_mlp_loss_grad(rpca_mlp* net, const float* x, const float* TU, const float* TV,
                       int32_t batch, double* loss, void* stream);

/* One Adam step on every tensor from the current gradient buffers
 * (step counter kept by the network, starting at 1). lr > 0,
 * 0 <= beta1, beta2 < 1, eps > 0. */
int rpca_mlp_adam_step(rpca_mlp* net, float lr, float beta1, float beta2, float eps, void* stream);

/* rpca_mlp_loss_grad followed by rpca_mlp_adam_step. */
int rpca_mlp_train_step(rpca_mlp* net, const float* x, const float* TU, const float* TV,
                        int32_t batch, float lr, double* loss, void* stream);

void rpca_mlp_destroy(rpca_mlp* net);

/* Window statistics of one window of frames.  X: device, column-major
 * (width*height) x frames, pixel index y*width + x, leading dimension
 * width*height (point it at the window's first frame).  factor divides width
 * and height.  feat (device) receives d_in = 2*(width/factor)*(height/factor)
 * + frames values, laid out as in the feature definition above (pooled blocks
 * in row-major block order; the standard deviation is the population one).
 * shift/scale: device arrays of d_in values or both NULL; when given,
 * feat = (raw - shift) * scale. */
int rpca_window_features(const float* X, int64_t width, int64_t height, int32_t frames,
                         int32_t factor, const float* shift, const float* scale, float* feat,
                         void* stream);

/* Average-pool the pixel rows of A ((width*height) x c, row-major, device)
 * over factor x factor blocks: out is (width/factor * height/factor) x c. */
int rpca_pool_rows(const float* A, int64_t width, int64_t height, int32_t factor, int32_t c,
                   float* out, void* stream);

/* Nearest-neighbour upsampling, the inverse layout of rpca_pool_rows:
 * A_low ((width/factor)*(height/factor) x c) -> out ((width*height) x c). */
int rpca_upsample_rows(const float* A_low, int64_t width, int64_t height, int32_t factor,
                       int32_t c, float* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RPCA_WARM_H */
