/*
 * bfc_mlp.h -- dense layers of the warm-start network (libbfc.so).
 *
 * A small fully connected network proposes starting cores for a completion
 * in place of the initial guess of Sec. 5.2 (low-rank completion followed by
 * Alg. "Randomized_LR_to_Butterfly"), which stays the fallback.  The paper
 * defines no network: these calls are standard dense layers,
 *     Y = act(X W + b),   act = identity (0) or ReLU (1),
 * trained in FP32 with ADAM (the update of Alg. "ADAM_Update" on real
 * parameters) and run for inference with BF16 inputs and FP32 accumulation.
 * The loss gradient with respect to the proposed cores comes from
 * bfc_loss_gradient (bfc.h).
 *
 * Conventions: every matrix is row-major and dense; X is m x k, W is k x n,
 * b has n entries, Y and dY are m x n.  Pointers are DEVICE pointers owned by
 * the caller; BF16 values are stored as uint16 (the upper half of the FP32
 * pattern).  All calls are asynchronous on hip_stream (NULL: the default
 * stream) and return BFC_EINVAL, with bfc_last_error() set, for negative
 * sizes, an unknown activation or a NULL pointer that the sizes require.
 */
#ifndef BFC_MLP_H
#define BFC_MLP_H

#include <stdint.h>

#include "bfc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Y = act(X W + b); b may be NULL (no bias).  FP32 throughout.
 * Products with few 64 x 64 output tiles over a long reduction (k >= 2048)
 * are split over k into partial tiles summed in a fixed order, in a
 * workspace kept per GPU for the life of the process (first use allocates
 * it); calls on one stream are ordered, calls that overlap on different
 * streams of one GPU are not supported.  The same holds for the two
 * products of bfc_mlp_backward. */
bfc_status bfc_mlp_forward(int64_t m, int64_t k, int64_t n, const float* X, const float* W,
                           const float* b, int32_t act, float* Y, void* hip_stream);

/*
 * Backward pass of bfc_mlp_forward for the loss gradient dY = dLoss/dY:
 * dZ = dY * act'(Z) (for ReLU: where Y > 0, with Y the forward output),
 * dW = X^T dZ (k x n), db = column sums of dZ (n), dX = dZ W^T (m x k).
 * dX, dW and db may each be NULL (not computed); outputs are overwritten.
 */
bfc_status bfc_mlp_backward(int64_t m, int64_t k, int64_t n, const float* X, const float* W,
                            const float* Y, const float* dY, int32_t act, float* dX, float* dW,
                            float* db, void* hip_stream);

/*
 * Inference: Y = act(Xh Wh + b) with BF16 Xh (m x k) and Wh (k x n), FP32
 * products and sums, FP32 bias.  Writes Y (FP32) and/or Yh (BF16, rounded
 * to nearest even) when not NULL; at least one is required.
 */
bfc_status bfc_mlp_forward_bf16(int64_t m, int64_t k, int64_t n, const uint16_t* Xh,
                                const uint16_t* Wh, const float* b, int32_t act, float* Y,
                                uint16_t* Yh, void* hip_stream);

/* dst[i] = src[i] rounded to BF16 (nearest even), count values. */
bfc_status bfc_mlp_to_bf16(int64_t count, const float* src, uint16_t* dst, void* hip_stream);

/*
 * One ADAM step (t >= 1) on count FP32 parameters:
 * m <- beta1 m + (1 - beta1) g, v <- beta2 v + (1 - beta2) g^2,
 * p <- p - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
 * BFC_EINVAL unless lr > 0, 0 <= beta1, beta2 < 1, eps >= 0.
 */
bfc_status bfc_mlp_adam(int64_t count, float* params, const float* grads, float* m, float* v,
                        int32_t t, float lr, float beta1, float beta2, float eps,
                        void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* BFC_MLP_H */
