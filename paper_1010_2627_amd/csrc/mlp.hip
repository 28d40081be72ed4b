// Kernels of the learned energy sampler: BF16 matrix-core GEMM with FP32
// accumulation, GELU, softmax cross-entropy, bias gradients and AdamW.
// Declared in include/knit_mlp.h.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/knit.h"
#include "../../include/knit_mlp.h"

namespace knit {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bf16, round to nearest, ties to even; NaN stays NaN
__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int GEMM_THREADS = 256;   // 4 waves, a 32 x 32 block of 16 x 16 wave tiles

// Operand layout of v_mfma_f32_16x16x16bf16_1k for lane l: A holds
// A[l % 16][4 (l / 16) + j], B holds B[4 (l / 16) + j][l % 16] (j = 0..3);
// the accumulator holds D[4 (l / 16) + j][l % 16].
__global__ void __launch_bounds__(GEMM_THREADS) mlp_gemm_kernel(int M, int N, int K, const uint16_t *A, int64_t sam,
                                                                int64_t sak, const uint16_t *B, int64_t sbn,
                                                                int64_t sbk, const float *bias, float beta, float *C,
                                                                int64_t ldc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tiles_n = (N + 31) / 32;
  const int m0 = (blockIdx.x / tiles_n) * 32 + (wave >> 1) * 16;
  const int n0 = (blockIdx.x % tiles_n) * 32 + (wave & 1) * 16;
  const int r = lane & 15, kq = 4 * (lane >> 4);
  const int am = m0 + r, bn = n0 + r;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + kq + j;
      a[j] = (short)((am < M && k < K) ? A[(int64_t)am * sam + (int64_t)k * sak] : 0);
      b[j] = (short)((bn < N && k < K) ? B[(int64_t)bn * sbn + (int64_t)k * sbk] : 0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  const int n = n0 + r;
  if (n >= N) return;
  const float bn_add = bias ? bias[n] : 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int m = m0 + kq + j;
    if (m >= M) continue;
    float *c = C + (int64_t)m * ldc + n;
    *c = (beta != 0.f ? beta * *c : 0.f) + acc[j] + bn_add;
  }
}

// Phi(x) = erfc(-x / sqrt 2) / 2 keeps full relative accuracy in the left tail,
// where 1 + erf(x / sqrt 2) cancels
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * erfcf(-x * 0.70710678118654752f); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * erfcf(-x * 0.70710678118654752f) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

__global__ void mlp_act_fwd_kernel(int64_t n, const float *Z, uint16_t *Y, int use_gelu) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Y[i] = to_bf16(use_gelu ? gelu(Z[i]) : Z[i]);
}

__global__ void mlp_gelu_bwd_kernel(int64_t n, const float *dY, const float *Z, uint16_t *dZ) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dZ[i] = to_bf16(dY[i] * gelu_grad(Z[i]));
}

// one workgroup per row
constexpr int XENT_THREADS = 256;
__global__ void __launch_bounds__(XENT_THREADS) mlp_softmax_xent_kernel(int C, const float *logits, const float *q,
                                                                        float scale, float *loss, float *probs,
                                                                        uint16_t *dlogits) {
  __shared__ float red[XENT_THREADS / 64];
  const int b = blockIdx.x, tid = threadIdx.x;
  const float *z = logits + (int64_t)b * C;
  const float *qb = q ? q + (int64_t)b * C : nullptr;
  auto block_reduce = [&](float v, bool is_max) {
    for (int off = 32; off > 0; off >>= 1) {
      const float o = __shfl_xor(v, off, 64);
      v = is_max ? fmaxf(v, o) : v + o;
    }
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    float r = red[0];
    for (int w = 1; w < XENT_THREADS / 64; ++w) r = is_max ? fmaxf(r, red[w]) : r + red[w];
    return r;
  };
  float mx = -INFINITY;
  for (int c = tid; c < C; c += XENT_THREADS) mx = fmaxf(mx, z[c]);
  mx = block_reduce(mx, true);
  float s = 0.f;
  for (int c = tid; c < C; c += XENT_THREADS) s += expf(z[c] - mx);
  s = block_reduce(s, false);
  const float lse = mx + logf(s);
  float l = 0.f;
  for (int c = tid; c < C; c += XENT_THREADS) {
    const float p = expf(z[c] - lse);
    const float qc = qb ? qb[c] : 0.f;
    l -= qc * (z[c] - lse);
    if (probs) probs[(int64_t)b * C + c] = p;
    if (dlogits) dlogits[(int64_t)b * C + c] = to_bf16((p - qc) * scale);
  }
  l = block_reduce(l, false);
  if (tid == 0 && loss) loss[b] = l;
}

__global__ void mlp_colsum_kernel(int R, int N, const uint16_t *X, float *out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int r = 0; r < R; ++r) s += from_bf16(X[(int64_t)r * N + n]);
  out[n] = s;
}

__global__ void mlp_adamw_kernel(int64_t n, float *w, uint16_t *w16, const float *g, float *m, float *v, float lr,
                                 float b1, float b2, float eps, float wd, float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * w[i]);
    w[i] = wi;
    if (w16) w16[i] = to_bf16(wi);
  }
}

int elementwise_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

int done(hipError_t e) { return e == hipSuccess ? KNIT_OK : KNIT_E_DEVICE; }

}  // namespace

}  // namespace knit

using namespace knit;

extern "C" {

int knit_mlp_gemm(int32_t M, int32_t N, int32_t K, const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B,
                  int64_t sbn, int64_t sbk, const float *bias, float beta, float *C, int64_t ldc, void *stream) {
  if (M < 0 || N < 0 || K < 0) return KNIT_E_ARG;
  if (M == 0 || N == 0) return KNIT_OK;
  if (!C || ldc < N) return KNIT_E_ARG;
  if (K > 0 && (!A || !B)) return KNIT_E_ARG;
  const int tiles = ((M + 31) / 32) * ((N + 31) / 32);
  hipLaunchKernelGGL(mlp_gemm_kernel, dim3(tiles), dim3(GEMM_THREADS), 0, (hipStream_t)stream, M, N, K, A, sam, sak,
                     B, sbn, sbk, bias, beta, C, ldc);
  return done(hipGetLastError());
}

int knit_mlp_act_fwd(int64_t n, const float *Z, uint16_t *Y, int32_t gelu, void *stream) {
  if (n < 0) return KNIT_E_ARG;
  if (n == 0) return KNIT_OK;
  if (!Z || !Y) return KNIT_E_ARG;
  hipLaunchKernelGGL(mlp_act_fwd_kernel, dim3(elementwise_grid(n)), dim3(256), 0, (hipStream_t)stream, n, Z, Y,
                     (int)gelu);
  return done(hipGetLastError());
}

int knit_mlp_gelu_bwd(int64_t n, const float *dY, const float *Z, uint16_t *dZ, void *stream) {
  if (n < 0) return KNIT_E_ARG;
  if (n == 0) return KNIT_OK;
  if (!dY || !Z || !dZ) return KNIT_E_ARG;
  hipLaunchKernelGGL(mlp_gelu_bwd_kernel, dim3(elementwise_grid(n)), dim3(256), 0, (hipStream_t)stream, n, dY, Z,
                     dZ);
  return done(hipGetLastError());
}

int knit_mlp_softmax_xent(int32_t B, int32_t C, const float *logits, const float *q, float scale, float *loss,
                          float *probs, uint16_t *dlogits, void *stream) {
  if (B < 0 || C < 0) return KNIT_E_ARG;
  if (B == 0 || C == 0) return KNIT_OK;
  if (!logits) return KNIT_E_ARG;
  if ((loss || dlogits) && !q) return KNIT_E_ARG;
  hipLaunchKernelGGL(mlp_softmax_xent_kernel, dim3(B), dim3(XENT_THREADS), 0, (hipStream_t)stream, (int)C, logits, q,
                     scale, loss, probs, dlogits);
  return done(hipGetLastError());
}

int knit_mlp_colsum(int32_t R, int32_t N, const uint16_t *X, float *out, void *stream) {
  if (R < 0 || N < 0) return KNIT_E_ARG;
  if (N == 0) return KNIT_OK;
  if (!out || (R > 0 && !X)) return KNIT_E_ARG;
  hipLaunchKernelGGL(mlp_colsum_kernel, dim3((N + 255) / 256), dim3(256), 0, (hipStream_t)stream, (int)R, (int)N, X,
                     out);
  return done(hipGetLastError());
}

int knit_mlp_adamw(int64_t n, float *w, uint16_t *w16, const float *g, float *m, float *v, float lr, float b1,
                   float b2, float eps, float wd, int32_t t, void *stream) {
  if (n < 0 || t < 1) return KNIT_E_ARG;
  if (!(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f) || !(lr >= 0.f) || !(wd >= 0.f))
    return KNIT_E_ARG;
  if (n == 0) return KNIT_OK;
  if (!w || !g || !m || !v) return KNIT_E_ARG;
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(mlp_adamw_kernel, dim3(elementwise_grid(n)), dim3(256), 0, (hipStream_t)stream, n, w, w16, g,
                     m, v, lr, b1, b2, eps, wd, c1, c2);
  return done(hipGetLastError());
}

}  // extern "C"
