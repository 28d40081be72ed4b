// Workgroup-level dense linear algebra on matrices in global memory, generic
// over the real type (float, double, dd).  One workgroup owns one matrix; all
// routines must be called by every thread of the workgroup.
#pragma once

#include "knit_num.h"

namespace knit {

constexpr int WG = 256;       // threads per workgroup of the generic kernels
constexpr int WAVE = 64;

// keep (v, i) if it beats the running best: larger value, lower index on ties
__device__ __forceinline__ void argmax_merge(double &v, int &i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// Workgroup argmax; every thread contributes (v, i) and receives the winner.
// sv/si: LDS scratch of WG / WAVE entries.
__device__ __forceinline__ void wg_argmax(double &v, int &i, double *sv, int *si) {
  for (int off = WAVE / 2; off > 0; off >>= 1) {
    double v2 = __shfl_xor(v, off, WAVE);
    int i2 = __shfl_xor(i, off, WAVE);
    argmax_merge(v, i, v2, i2);
  }
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  if (lane == 0) {
    sv[w] = v;
    si[w] = i;
  }
  __syncthreads();
  v = sv[0];
  i = si[0];
  for (int k = 1; k < (int)(blockDim.x / WAVE); ++k) argmax_merge(v, i, sv[k], si[k]);
  __syncthreads();
}

// Workgroup max of a non-negative value (NaN propagates as +inf).
__device__ __forceinline__ double wg_max(double v, double *sv) {
  if (v != v) v = INFINITY;
  for (int off = WAVE / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  if (lane == 0) sv[w] = v;
  __syncthreads();
  v = sv[0];
  for (int k = 1; k < (int)(blockDim.x / WAVE); ++k) v = fmax(v, sv[k]);
  __syncthreads();
  return v;
}

// In-place Gauss-Jordan inversion with partial pivoting of the leading Mp x Mp
// block A of X (row-major, leading dimension ld), also eliminating the
// Rtot - Mp extra rows B below it, which never serve as pivots.  On return
// the leading block holds (P A)^{-1} and the extra rows hold -B (P A)^{-1},
// where P is the row permutation of the pivoting; q[0..Mp) receives P as
// "original row index at each position" (caller maps columns back).
// Pivot: largest |re|+|im| among the rows not yet used, lowest row on ties.
// Returns the status bits (singular / non-finite pivot) to every thread.
// LDS scratch: q[Mp], colj[Rtot], prow[Mp], sv/si[WG/WAVE].
template <class R>
__device__ int wg_gauss_jordan(cpx<R> *X, int ld, int Mp, int Rtot, int *q, cpx<R> *colj,
                               cpx<R> *prow, double *sv, int *si) {
  const int tid = threadIdx.x, nt = blockDim.x;
  int flags = 0;
  for (int i = tid; i < Mp; i += nt) q[i] = i;
  __syncthreads();
  for (int j = 0; j < Mp; ++j) {
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int r = j + tid; r < Mp; r += nt) argmax_merge(bv, bi, c_abs1(X[(int64_t)r * ld + j]), r);
    wg_argmax(bv, bi, sv, si);
    int p = (bi >= j && bi < Mp) ? bi : j;
    if (!(bv > 0.0)) flags |= (bv == 0.0) ? 1 : 4;
    if (!isfinite(bv)) flags |= 4;
    if (p != j) {
      for (int c = tid; c < Mp; c += nt) {
        cpx<R> t = X[(int64_t)j * ld + c];
        X[(int64_t)j * ld + c] = X[(int64_t)p * ld + c];
        X[(int64_t)p * ld + c] = t;
      }
      if (tid == 0) {
        int t = q[j];
        q[j] = q[p];
        q[p] = t;
      }
    }
    __syncthreads();
    const cpx<R> d = c_inv(X[(int64_t)j * ld + j]);
    for (int c = tid; c < Mp; c += nt) prow[c] = (c == j) ? d : c_mul(X[(int64_t)j * ld + c], d);
    for (int r = tid; r < Rtot; r += nt) colj[r] = X[(int64_t)r * ld + j];
    __syncthreads();
    for (int c = tid; c < Mp; c += nt) X[(int64_t)j * ld + c] = prow[c];
    // eliminate column j from every other row: X[r][c] = [c != j] X[r][c] - colj[r] * prow[c]
    const int64_t total = (int64_t)Rtot * Mp;
    for (int64_t e = tid; e < total; e += nt) {
      const int r = (int)(e / Mp), c = (int)(e % Mp);
      if (r == j) continue;
      cpx<R> x = (c == j) ? c_zero<R>() : X[(int64_t)r * ld + c];
      X[(int64_t)r * ld + c] = c_fms(colj[r], prow[c], x);
    }
    __syncthreads();
  }
  return flags;
}

// pinv[q[i]] = i : column b of A^{-1} is column pinv[b] of (P A)^{-1}.
__device__ __forceinline__ void wg_invert_perm(const int *q, int *pinv, int Mp) {
  for (int i = threadIdx.x; i < Mp; i += blockDim.x) pinv[q[i]] = i;
  __syncthreads();
}

// C[M x N] (=|+=) A[M x K] * B[K x N]; all row-major complex<R> with leading
// dimensions; LDS-tiled, 32 x 32 output tiles, 16-deep K panels.
// lds must hold 2 * 32 * 16 complex<R>.
template <class R>
__device__ void wg_gemm(cpx<R> *C, int ldc, const cpx<R> *A, int lda, const cpx<R> *B, int ldb,
                        int M, int N, int K, bool accumulate, cpx<R> *lds) {
  constexpr int TM = 32, TN = 32, TK = 16;
  cpx<R> *As = lds;             // [TM][TK]
  cpx<R> *Bs = lds + TM * TK;   // [TK][TN]
  const int tid = threadIdx.x;
  const int tr = tid / 16, tc = tid % 16;   // 16 x 16 threads, 2 x 2 outputs each
  for (int i0 = 0; i0 < M; i0 += TM) {
    for (int j0 = 0; j0 < N; j0 += TN) {
      cpx<R> acc[2][2];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = c_zero<R>();
      for (int k0 = 0; k0 < K; k0 += TK) {
        for (int e = tid; e < TM * TK; e += blockDim.x) {
          int r = e / TK, k = e % TK;
          As[e] = (i0 + r < M && k0 + k < K) ? A[(int64_t)(i0 + r) * lda + k0 + k] : c_zero<R>();
        }
        for (int e = tid; e < TK * TN; e += blockDim.x) {
          int k = e / TN, c = e % TN;
          Bs[e] = (k0 + k < K && j0 + c < N) ? B[(int64_t)(k0 + k) * ldb + j0 + c] : c_zero<R>();
        }
        __syncthreads();
        if (tid < 256) {
          for (int k = 0; k < TK; ++k) {
            cpx<R> a0 = As[(tr * 2 + 0) * TK + k], a1 = As[(tr * 2 + 1) * TK + k];
            cpx<R> b0 = Bs[k * TN + tc * 2 + 0], b1 = Bs[k * TN + tc * 2 + 1];
            acc[0][0] = c_fma(a0, b0, acc[0][0]);
            acc[0][1] = c_fma(a0, b1, acc[0][1]);
            acc[1][0] = c_fma(a1, b0, acc[1][0]);
            acc[1][1] = c_fma(a1, b1, acc[1][1]);
          }
        }
        __syncthreads();
      }
      if (tid < 256) {
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            int r = i0 + tr * 2 + a, c = j0 + tc * 2 + b;
            if (r < M && c < N) {
              cpx<R> v = acc[a][b];
              if (accumulate) v = c_add(C[(int64_t)r * ldc + c], v);
              C[(int64_t)r * ldc + c] = v;
            }
          }
      }
    }
  }
  __syncthreads();
}

}  // namespace knit
