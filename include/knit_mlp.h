/*
 * libknit: kernels of the learned energy sampler (a small MLP that proposes
 * where to place energy points so that the transmission's resonances and
 * channel steps are resolved; the transport path evaluates every proposed
 * point).
 *
 * Network: Linear layers with BF16 weights and activations and FP32
 * accumulation, GELU between layers, softmax output over energy bins,
 * cross-entropy loss against a target density, AdamW on FP32 master weights.
 * The entry points are the building blocks of one training step and of
 * inference; the caller sequences them over the layers.
 *
 * Conventions (as in knit.h): every array pointer is a device pointer owned
 * by the caller; calls are asynchronous on `stream` (a hipStream_t, NULL for
 * the default stream) and allocate nothing.  BF16 values are stored as
 * uint16_t bit patterns; float -> BF16 rounds to nearest, ties to even.
 * Return codes are the KNIT_OK / KNIT_E_* codes of knit.h.
 */
#ifndef KNIT_MLP_H
#define KNIT_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * C[m][n] = beta * C[m][n] + sum_k A(m, k) * B(n, k) + bias[n]
 * for m < M, n < N, with A(m, k) = A[m * sam + k * sak] and
 * B(n, k) = B[n * sbn + k * sbk] (BF16), products summed in FP32 on the
 * matrix cores (v_mfma_f32_16x16x16bf16_1k).  C is FP32 with row stride ldc;
 * bias may be NULL.  The strides let one kernel serve X W^T (forward),
 * dZ W (input gradient) and dZ^T X (weight gradient).
 */
int knit_mlp_gemm(int32_t M, int32_t N, int32_t K, const uint16_t *A, int64_t sam, int64_t sak,
                  const uint16_t *B, int64_t sbn, int64_t sbk, const float *bias, float beta, float *C,
                  int64_t ldc, void *stream);

/* Y[i] = bf16(gelu(Z[i])), gelu(x) = x erfc(-x / sqrt 2) / 2; n elements.  With
 * gelu = 0 it is a plain rounding cast (inputs of the first layer). */
int knit_mlp_act_fwd(int64_t n, const float *Z, uint16_t *Y, int32_t gelu, void *stream);

/* dZ[i] = bf16(dY[i] * gelu'(Z[i])); n elements. */
int knit_mlp_gelu_bwd(int64_t n, const float *dY, const float *Z, uint16_t *dZ, void *stream);

/*
 * Row-wise softmax cross-entropy for B rows of C logits:
 *   p = softmax(logits[b]),  loss[b] = -sum_c q[b][c] log p[c],
 *   dlogits[b][c] = bf16((p[c] - q[b][c]) * scale)
 * (scale = 1/B for the mean loss).  q rows are probability vectors.  probs
 * (FP32 [B][C]) receives p and may be NULL; dlogits may be NULL (inference).
 */
int knit_mlp_softmax_xent(int32_t B, int32_t C, const float *logits, const float *q, float scale,
                          float *loss, float *probs, uint16_t *dlogits, void *stream);

/* out[n] = sum_r X[r][n] for X BF16 [R][N] (bias gradients). */
int knit_mlp_colsum(int32_t R, int32_t N, const uint16_t *X, float *out, void *stream);

/*
 * AdamW step t (1-based) on n FP32 master parameters:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2
 *   w = w - lr (m / (1-b1^t) / (sqrt(v / (1-b2^t)) + eps) + wd w)
 * then w16 = bf16(w) (the copy the forward pass uses; may be NULL).
 */
int knit_mlp_adamw(int64_t n, float *w, uint16_t *w16, const float *g, float *m, float *v, float lr,
                   float b1, float b2, float eps, float wd, int32_t t, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KNIT_MLP_H */
