// Complex matrix tiles on the CDNA matrix cores (MFMA), wave64.
//
// A complex product C += A B is carried as four real MFMA products
// (Re C += Re A Re B - Im A Im B, Im C += Re A Im B + Im A Re B).
// One wave owns a (16 NBLK) x (16 NBLK) complex output tile, i.e. NBLK x NBLK
// blocks of the 16 x 16 x 4 MFMA shape (f64: v_mfma_f64_16x16x4f64, f32:
// v_mfma_f32_16x16x4f32).  Operand lane layout of that shape, for lane l:
//   A operand: element (row l % 16, k l / 16) of the 16 x 4 slice
//   B operand: element (k l / 16, col l % 16) of the 4 x 16 slice
//   accumulator item e, column l % 16, row:
//     f32: 4 (l / 16) + e          f64: 4 e + l / 16
// (both measured on gfx950 with a lane-layout probe).
#pragma once

#include "knit_num.h"

namespace knit {

template <class R> struct Mfma;

template <> struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int e) { return 4 * e + (l >> 4); }
};

template <> struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int e) { return 4 * (l >> 4) + e; }
};

// (16 NBLK) x (16 NBLK) complex accumulator of one wave
template <class R, int NBLK = 2>
struct CTile {
  typename Mfma<R>::acc_t re[NBLK][NBLK], im[NBLK][NBLK];
  __device__ __forceinline__ void zero() {
    for (int i = 0; i < NBLK; ++i)
      for (int j = 0; j < NBLK; ++j)
        for (int e = 0; e < 4; ++e) {
          re[i][j][e] = R(0);
          im[i][j][e] = R(0);
        }
  }
};

template <class R, class T>
__device__ __forceinline__ cpx<R> cvt(cpx<T> v) {
  return {(R)v.re, (R)v.im};
}
template <class R>
__device__ __forceinline__ cpx<R> cvt(cpx<dd> v) {
  return {(R)(v.re.hi + v.re.lo), (R)(v.im.hi + v.im.lo)};
}

// acc += a * b for one k-slice of 4: a[bi] is this lane's A operand of row block bi,
// b[bj] its B operand of column block bj.
template <class R, int NBLK>
__device__ __forceinline__ void ctile_mma(CTile<R, NBLK> &t, const cpx<R> a[NBLK], const cpx<R> b[NBLK]) {
  using M = Mfma<R>;
#pragma unroll
  for (int i = 0; i < NBLK; ++i)
#pragma unroll
    for (int j = 0; j < NBLK; ++j) {
      t.re[i][j] = M::mma(a[i].re, b[j].re, t.re[i][j]);
      t.re[i][j] = M::mma(-a[i].im, b[j].im, t.re[i][j]);
      t.im[i][j] = M::mma(a[i].re, b[j].im, t.im[i][j]);
      t.im[i][j] = M::mma(a[i].im, b[j].re, t.im[i][j]);
    }
}

// (16 NBR) x (16 NBC) complex accumulator of one wave (rectangular tiles)
template <class R, int NBR, int NBC>
struct CTileRC {
  typename Mfma<R>::acc_t re[NBR][NBC], im[NBR][NBC];
};

// acc += a * b for one k-slice of 4, rectangular: a[NBR] row blocks, b[NBC] column blocks.
template <class R, int NBR, int NBC>
__device__ __forceinline__ void ctile_mma_rc(CTileRC<R, NBR, NBC> &t, const cpx<R> a[NBR], const cpx<R> b[NBC]) {
  using M = Mfma<R>;
#pragma unroll
  for (int i = 0; i < NBR; ++i)
#pragma unroll
    for (int j = 0; j < NBC; ++j) {
      t.re[i][j] = M::mma(a[i].re, b[j].re, t.re[i][j]);
      t.re[i][j] = M::mma(-a[i].im, b[j].im, t.re[i][j]);
      t.im[i][j] = M::mma(a[i].re, b[j].im, t.im[i][j]);
      t.im[i][j] = M::mma(a[i].im, b[j].re, t.im[i][j]);
    }
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Visit the rectangular tile's elements held by this lane (as ctile_for_each).
template <class R, int NBR, int NBC, class F>
__device__ __forceinline__ void ctile_for_each_rc(CTileRC<R, NBR, NBC> &t, F f) {
  const int l = lane_id();
#pragma unroll
  for (int i = 0; i < NBR; ++i)
#pragma unroll
    for (int j = 0; j < NBC; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        R re = t.re[i][j][e], im = t.im[i][j][e];
        f(16 * i + Mfma<R>::row(l, e), 16 * j + (l & 15), re, im);
        t.re[i][j][e] = re;
        t.im[i][j][e] = im;
      }
}

// Load this lane's A operands of rows [r0, r0 + 16 NBLK), k-slice [k, k+4) of a
// row-major complex matrix (any element type, converted to R).
template <class R, int NBLK, class T>
__device__ __forceinline__ void ld_a(cpx<R> a[NBLK], const cpx<T> *A, int64_t lda, int r0, int k) {
  const int l = lane_id();
#pragma unroll
  for (int i = 0; i < NBLK; ++i) a[i] = cvt<R>(A[(int64_t)(r0 + 16 * i + (l & 15)) * lda + k + (l >> 4)]);
}
template <class R, int NBLK, class T>
__device__ __forceinline__ void ld_b(cpx<R> b[NBLK], const cpx<T> *B, int64_t ldb, int k, int c0) {
  const int l = lane_id();
#pragma unroll
  for (int j = 0; j < NBLK; ++j) b[j] = cvt<R>(B[(int64_t)(k + (l >> 4)) * ldb + c0 + 16 * j + (l & 15)]);
}

// Visit the tile's elements held by this lane: f(row, col, re&, im&) with
// row/col relative to the tile origin; f may modify the values.
template <class R, int NBLK, class F>
__device__ __forceinline__ void ctile_for_each(CTile<R, NBLK> &t, F f) {
  const int l = lane_id();
#pragma unroll
  for (int i = 0; i < NBLK; ++i)
#pragma unroll
    for (int j = 0; j < NBLK; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        R re = t.re[i][j][e], im = t.im[i][j][e];
        f(16 * i + Mfma<R>::row(l, e), 16 * j + (l & 15), re, im);
        t.re[i][j][e] = re;
        t.im[i][j][e] = im;
      }
}

// C tile (at r0, c0) += A[r0.., 0..K) * B[0..K, c0..) ; K multiple of 4.
template <class R, int NBLK, class TA, class TB>
__device__ __forceinline__ void ctile_gemm(CTile<R, NBLK> &t, const cpx<TA> *A, int64_t lda, int r0,
                                           const cpx<TB> *B, int64_t ldb, int c0, int K) {
  cpx<R> a[NBLK], b[NBLK];
  for (int k = 0; k < K; k += 4) {
    ld_a<R, NBLK>(a, A, lda, r0, k);
    ld_b<R, NBLK>(b, B, ldb, k, c0);
    ctile_mma<R, NBLK>(t, a, b);
  }
}

// Workgroup GEMM on MFMA: for every 32 x 32 output tile (rows < Mr, cols < Nc,
// both multiples of 32), acc = A * B (K multiple of 4) then epi(row, col, acc_re, acc_im).
template <class R, class TA, class TB, class Epi>
__device__ void wg_gemm_mfma(int Mr, int Nc, int K, const cpx<TA> *A, int64_t lda, const cpx<TB> *B,
                             int64_t ldb, Epi epi) {
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int tr = Mr / 32, tc = Nc / 32;
  for (int t = wave; t < tr * tc; t += nwaves) {
    const int r0 = (t / tc) * 32, c0 = (t % tc) * 32;
    CTile<R, 2> acc;
    acc.zero();
    ctile_gemm<R, 2>(acc, A, lda, r0, B, ldb, c0, K);
    ctile_for_each<R, 2>(acc, [&](int i, int j, R &re, R &im) { epi(r0 + i, c0 + j, re, im); });
  }
}

}  // namespace knit
