// Slice-level helpers shared by the sweep and LDOS kernels: assembling
// A_n = E - H0 - D_n - Sigma terms - V g_{n-1} V^+ and the block-monomial
// gathers with the inter-slice hopping V.
#pragma once

#include "knit_internal.h"
#include "knit_wg.h"

namespace knit {

template <class R>
__device__ __forceinline__ cpx<R> to_r(cpx<double> v) {
  return {r_from<R>(v.re), r_from<R>(v.im)};
}

// vblk[sa][oa][ii]
__device__ __forceinline__ cpx<double> vblk_at(const StripDev &s, int sa, int oa, int ii) {
  const int no = s.norb;
  return ld_z(s.vblk + ((int64_t)sa * no + oa) * no + ii);
}

// Writes A_n into X ([M][M], ld M).  gprev = g_{n-1} in natural column order
// (ignored when first).  first/last select the Sigma_L / Sigma_R terms.
template <class R>
__device__ void form_slice_matrix(cpx<R> *X, const StripDev &s, double E, const knit_z *D,
                                  const knit_z *sL, const knit_z *sR, bool first, bool last,
                                  const cpx<R> *gprev) {
  const int M = s.M, no = s.norb;
  const int64_t mm = (int64_t)M * M;
  for (int64_t i = threadIdx.x; i < mm; i += blockDim.x) {
    const int a = (int)(i / M), b = (int)(i % M);
    const int sa = a / no, oa = a % no, sb = b / no, ob = b % no;
    cpx<double> h = ld_z(s.H0 + i);
    if (sa == sb) {
      cpx<double> d = ld_z(D + ((int64_t)sa * no + oa) * no + ob);
      h.re += d.re;
      h.im += d.im;
    }
    if (first) {
      cpx<double> x = ld_z(sL + i);
      h.re += x.re;
      h.im += x.im;
    }
    if (last) {
      cpx<double> x = ld_z(sR + i);
      h.re += x.re;
      h.im += x.im;
    }
    cpx<R> x = to_r<R>(cpx<double>{(a == b ? E : 0.0) - h.re, -h.im});
    if (!first) {
      const int ca = s.vcol[sa], cb = s.vcol[sb];
      if (ca >= 0 && cb >= 0) {
        cpx<R> acc = c_zero<R>();
        for (int ii = 0; ii < no; ++ii) {
          cpx<R> va = to_r<R>(vblk_at(s, sa, oa, ii));
          cpx<R> inner = c_zero<R>();
          for (int jj = 0; jj < no; ++jj) {
            cpx<R> vb = c_conj(to_r<R>(vblk_at(s, sb, ob, jj)));
            inner = c_fma(gprev[(int64_t)(ca * no + ii) * M + cb * no + jj], vb, inner);
          }
          acc = c_fma(va, inner, acc);
        }
        x = c_sub(x, acc);
      }
    }
    X[i] = x;
  }
}

// Y = Gm V^+  (column gather): Y[a][b] = sum_j Gm[a][vcol[sb]*no + j] conj(vblk[sb][ob][j])
template <class R>
__device__ void right_mul_vdag(cpx<R> *Y, const cpx<R> *Gm, const StripDev &s, int rows, bool negate) {
  const int M = s.M, no = s.norb;
  const int64_t tot = (int64_t)rows * M;
  for (int64_t i = threadIdx.x; i < tot; i += blockDim.x) {
    const int a = (int)(i / M), b = (int)(i % M);
    const int sb = b / no, ob = b % no, cb = s.vcol[sb];
    cpx<R> acc = c_zero<R>();
    if (cb >= 0)
      for (int jj = 0; jj < no; ++jj) {
        cpx<R> vb = c_conj(to_r<R>(vblk_at(s, sb, ob, jj)));
        acc = c_fma(Gm[(int64_t)a * M + cb * no + jj], vb, acc);
      }
    Y[i] = negate ? c_neg(acc) : acc;
  }
}

// Y = V Gm  (row gather): Y[a][b] = sum_i vblk[sa][oa][i] Gm[vcol[sa]*no + i][b];
// if rowperm != nullptr, output row k holds row rowperm[k] of V Gm.
template <class R>
__device__ void left_mul_v(cpx<R> *Y, const cpx<R> *Gm, const StripDev &s, const int *rowperm) {
  const int M = s.M, no = s.norb;
  const int64_t mm = (int64_t)M * M;
  for (int64_t i = threadIdx.x; i < mm; i += blockDim.x) {
    const int k = (int)(i / M), b = (int)(i % M);
    const int a = rowperm ? rowperm[k] : k;
    const int sa = a / no, oa = a % no, ca = s.vcol[sa];
    cpx<R> acc = c_zero<R>();
    if (ca >= 0)
      for (int ii = 0; ii < no; ++ii)
        acc = c_fma(to_r<R>(vblk_at(s, sa, oa, ii)), Gm[(int64_t)(ca * no + ii) * M + b], acc);
    Y[i] = acc;
  }
}

}  // namespace knit
