/*
 * hdc_mlp -- the HIP kernels of the parameter predictor (a small multilayer
 * perceptron classifier; classification rather than regression for the
 * discrete parameter choice, section 6.3).  Training and inference both run
 * in these kernels; the host only sequences the calls.
 *
 * All arrays are DEVICE pointers to float32 (labels int32), row-major,
 * owned by the caller.  A layer's weights W are (out x in), its bias b is
 * (out).  Calls enqueue on `stream` and do not synchronise.  Results are
 * deterministic (no atomics).  Errors: HDC_ERR_INVALID_ARG for NULL
 * required pointers or non-positive sizes, HDC_ERR_HIP for launch failures.
 */
#ifndef HDC_MLP_H
#define HDC_MLP_H

#include <stdint.h>

#include "hdc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Y = X W^T + b (B x out), then relu if `relu` is nonzero. */
hdc_status hdc_mlp_linear_forward(const float* X, const float* W, const float* b, float* Y, int64_t B, int64_t in,
                                  int64_t out, int relu, hipStream_t stream);

/* Gradients of a linear layer from dY (B x out): dW = dY^T X (out x in),
 * db = column sums of dY (out), and dX = dY W (B x in) unless dX is NULL. */
hdc_status hdc_mlp_linear_backward(const float* X, const float* W, const float* dY, float* dX, float* dW, float* db,
                                   int64_t B, int64_t in, int64_t out, hipStream_t stream);

/* dA *= (A > 0) elementwise over n values (A is the relu output). */
hdc_status hdc_mlp_relu_backward(float* dA, const float* A, int64_t n, hipStream_t stream);

/* Row softmax of Z (B x K) into P.  If labels y is non-NULL: dZ = (P - onehot(y)) / B
 * (if dZ is non-NULL) and *loss = mean_i -log P[i, y_i] (if loss is non-NULL; a
 * device float). */
hdc_status hdc_mlp_softmax_xent(const float* Z, const int32_t* y, float* P, float* dZ, float* loss, int64_t B,
                                int64_t K, hipStream_t stream);

/* As hdc_mlp_softmax_xent with target distributions T (B x K, rows summing to 1)
 * instead of labels: dZ = (P - T) / B and *loss = mean_i -sum_k T[i,k] log P[i,k]. */
hdc_status hdc_mlp_softmax_xent_soft(const float* Z, const float* T, float* P, float* dZ, float* loss, int64_t B,
                                     int64_t K, hipStream_t stream);

/* One Adam step over n parameters with step count t >= 1 (bias-corrected). */
hdc_status hdc_mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                        float eps, int64_t t, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HDC_MLP_H */
