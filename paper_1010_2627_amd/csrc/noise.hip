// Transmission eigenvalues and shot noise (section 2.1 item (a): conductance
// and shot noise from the Green function between the leads), FP64.
//
// From the projected propagator P = C_L^+ G_1N (rows up to the rank r_L of
// Gamma_L = C_L C_L^+) and Gamma_R = C_R C_R^+:
//   t~ = P C_R                      (r_L x r_R)
// is the transmission amplitude matrix up to unitary factors on both sides
// (t = Gamma_R^{1/2} G_N1 Gamma_L^{1/2} and t~ share their singular values:
// C_L = Gamma_L^{1/2} U_L, C_R = Gamma_R^{1/2} U_R with U isometries, and
// G_1N, G_N1 carry the same transmission by current conservation), so the
// transmission eigenvalues T_n are the eigenvalues of the smaller of
// tau = t~^+ t~ and t~ t~^+ (n = min(r_L, r_R) of them), and
//   T = Tr tau,   F = sum T_n (1 - T_n) / sum T_n = (Tr tau - ||tau||_F^2) / Tr tau.
//
// One workgroup per problem (persistent over a grid-stride of problems):
//   1. t~ and tau by LDS-tiled complex products into the workgroup's slab;
//   2. Householder reduction of tau to real symmetric tridiagonal form
//      (d_k, e_k = |subdiagonal|), matrix-vector product and rank-2 update of
//      the trailing block per step, Householder vectors in LDS;
//   3. every eigenvalue by bisection on the Sturm sequence of the tridiagonal
//      matrix, one eigenvalue per thread (accurate to a few units of
//      rounding of ||tau||).

#include "knit_internal.h"
#include "knit_wg.h"

namespace knit {

namespace {

using Z = cpx<double>;
constexpr int NMAX = KNIT_MAX_M;   // largest tau dimension (LDS vectors)

__device__ __forceinline__ double wg_sum(double v, double *sv) {
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) sv[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < (int)(blockDim.x / WAVE); ++k) s += sv[k];
  __syncthreads();
  return s;
}

// C[a][c] = sum_k op(A)[a][k] op(B)[k][c] for a < ra, c < rc, k < K, with
// op(A)[a][k] = AH ? conj(A[k][a]) : A[a][k] and op(B)[k][c] = BH ? conj(B[c][k]) : B[k][c].
// 32 x 32 output tiles, 16-deep k tiles staged in LDS, a 2 x 2 block per thread.
template <bool AH, bool BH>
__device__ void wg_zgemm(int ra, int rc, int K, const Z *A, int64_t lda, const Z *B, int64_t ldb, Z *C,
                         int64_t ldc, Z *As, Z *Bs) {
  constexpr int TT = 32, TK = 16;
  const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
  for (int a0 = 0; a0 < ra; a0 += TT)
    for (int c0 = 0; c0 < rc; c0 += TT) {
      Z x[2][2];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) x[i][j] = Z{0.0, 0.0};
      for (int k0 = 0; k0 < K; k0 += TK) {
        for (int e = tid; e < TT * TK; e += blockDim.x) {
          const int r = e / TK, k = e % TK;
          Z av = {0.0, 0.0};
          if (a0 + r < ra && k0 + k < K)
            av = AH ? c_conj(A[(int64_t)(k0 + k) * lda + a0 + r]) : A[(int64_t)(a0 + r) * lda + k0 + k];
          As[e] = av;
          const int k2 = e / TT, c = e % TT;
          Z bv = {0.0, 0.0};
          if (k0 + k2 < K && c0 + c < rc)
            bv = BH ? c_conj(B[(int64_t)(c0 + c) * ldb + k0 + k2]) : B[(int64_t)(k0 + k2) * ldb + c0 + c];
          Bs[e] = bv;
        }
        __syncthreads();
        for (int k = 0; k < TK; ++k) {
          const Z a0v = As[(tr * 2) * TK + k], a1v = As[(tr * 2 + 1) * TK + k];
          const Z b0v = Bs[k * TT + tc * 2], b1v = Bs[k * TT + tc * 2 + 1];
          x[0][0] = c_fma(a0v, b0v, x[0][0]);
          x[0][1] = c_fma(a0v, b1v, x[0][1]);
          x[1][0] = c_fma(a1v, b0v, x[1][0]);
          x[1][1] = c_fma(a1v, b1v, x[1][1]);
        }
        __syncthreads();
      }
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          const int a = a0 + tr * 2 + i, c = c0 + tc * 2 + j;
          if (a < ra && c < rc) C[(int64_t)a * ldc + c] = x[i][j];
        }
    }
  __syncthreads();
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix (d, e),
// e2[i] = e[i]^2, from the signs of its LDL^T pivots (Sturm count).
__device__ int sturm_count(const double *d, const double *e2, int n, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

__global__ void __launch_bounds__(WG) transmission_eigs_kernel(StripTable tab, const knit_problem *probs, int P,
                                                               const knit_z *CR, const knit_z *G1Np, int ld,
                                                               double *tn, int32_t *nch, double *T, double *fano,
                                                               char *ws, int64_t slab_elems) {
  __shared__ Z As[32 * 16], Bs[16 * 32];
  __shared__ Z vv[NMAX], pp[NMAX];
  __shared__ double dd[NMAX], ee2[NMAX];
  __shared__ double sv[WG / WAVE];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nw = nt / WAVE, wave = tid / WAVE, lane = tid % WAVE;
  Z *Tt = reinterpret_cast<Z *>(ws) + (int64_t)blockIdx.x * 2 * slab_elems;   // t~, leading dimension M
  Z *Tau = Tt + slab_elems;                                                    // tau, leading dimension n
  for (int p = blockIdx.x; p < P; p += gridDim.x) {
    const knit_problem pr = probs[p];
    const int M = tab.s[pr.strip].M;
    const Z *Pm = reinterpret_cast<const Z *>(G1Np + pr.out_off);
    const Z *Cm = reinterpret_cast<const Z *>(CR + pr.sigma_off);
    // rows of P and columns of C_R up to the last nonzero one
    double lr = 0.0, lc = 0.0;
    for (int64_t i = tid; i < (int64_t)M * M; i += nt) {
      const Z a = Pm[i], c = Cm[i];
      if (a.re != 0.0 || a.im != 0.0) lr = fmax(lr, (double)(i / M + 1));
      if (c.re != 0.0 || c.im != 0.0) lc = fmax(lc, (double)(i % M + 1));
    }
    const int rl = (int)wg_max(lr, sv), rr = (int)wg_max(lc, sv);
    const int n = rl < rr ? rl : rr;
    // t~ = P C_R, then tau on the smaller side
    wg_zgemm<false, false>(rl, rr, M, Pm, M, Cm, M, Tt, M, As, Bs);
    if (rr <= rl) wg_zgemm<true, false>(n, n, rl, Tt, M, Tt, M, Tau, n, As, Bs);    // t~^+ t~
    else wg_zgemm<false, true>(n, n, rr, Tt, M, Tt, M, Tau, n, As, Bs);             // t~ t~^+
    // Tr tau and ||tau||_F^2 (the Fano factor without eigenvalues)
    double tr = 0.0, f2 = 0.0;
    for (int64_t i = tid; i < (int64_t)n * n; i += nt) {
      const Z x = Tau[i];
      f2 += x.re * x.re + x.im * x.im;
      if (i / n == i % n) tr += x.re;
    }
    tr = wg_sum(tr, sv);
    f2 = wg_sum(f2, sv);
    // Householder reduction to tridiagonal form: step k reflects rows/columns
    // k+1..n-1 so that column k below the subdiagonal vanishes
    for (int k = 0; k + 2 < n; ++k) {
      const int m = n - k - 1;
      Z *A = Tau + (int64_t)(k + 1) * n + (k + 1);           // trailing block, leading dimension n
      double tail = 0.0;
      for (int i = tid; i < m; i += nt) {
        const Z x = Tau[(int64_t)(k + 1 + i) * n + k];
        vv[i] = x;
        if (i > 0) tail += x.re * x.re + x.im * x.im;
      }
      tail = wg_sum(tail, sv);                                 // barrier: vv complete
      const Z x0 = vv[0];
      const double ax0 = sqrt(x0.re * x0.re + x0.im * x0.im);
      const double xn = sqrt(tail + ax0 * ax0);
      if (tid == 0) {
        dd[k] = Tau[(int64_t)k * n + k].re;
        ee2[k] = xn * xn;
      }
      if (!(tail > 0.0)) {                                     // already reduced (or NaN: propagates via d)
        __syncthreads();                                       // every thread has read vv[0]
        continue;
      }
      const Z ph = ax0 > 0.0 ? Z{x0.re / ax0, x0.im / ax0} : Z{1.0, 0.0};
      const double beta = 1.0 / (xn * (xn + ax0));
      __syncthreads();
      if (tid == 0) vv[0] = Z{x0.re + ph.re * xn, x0.im + ph.im * xn};
      __syncthreads();
      // p = beta A v, one row per wave step, lanes across the row
      for (int i = wave; i < m; i += nw) {
        Z acc = {0.0, 0.0};
        for (int j = lane; j < m; j += WAVE) acc = c_fma(A[(int64_t)i * n + j], vv[j], acc);
        for (int off = WAVE / 2; off > 0; off >>= 1) {
          acc.re += __shfl_xor(acc.re, off, WAVE);
          acc.im += __shfl_xor(acc.im, off, WAVE);
        }
        if (lane == 0) pp[i] = Z{beta * acc.re, beta * acc.im};
      }
      __syncthreads();
      // w = p - (beta / 2) (v^+ p) v   (v^+ A v is real for Hermitian A)
      double vp = 0.0;
      for (int i = tid; i < m; i += nt) vp += vv[i].re * pp[i].re + vv[i].im * pp[i].im;
      const double K = 0.5 * beta * wg_sum(vp, sv);
      for (int i = tid; i < m; i += nt) pp[i] = Z{pp[i].re - K * vv[i].re, pp[i].im - K * vv[i].im};
      __syncthreads();
      // A -= v w^+ + w v^+
      for (int64_t idx = tid; idx < (int64_t)m * m; idx += nt) {
        const int i = (int)(idx / m), j = (int)(idx % m);
        const Z a = A[(int64_t)i * n + j];
        const Z u = c_add(c_mul(vv[i], c_conj(pp[j])), c_mul(pp[i], c_conj(vv[j])));
        A[(int64_t)i * n + j] = c_sub(a, u);
      }
      __syncthreads();
    }
    if (n >= 2 && tid == 0) {
      dd[n - 2] = Tau[(int64_t)(n - 2) * n + (n - 2)].re;
      dd[n - 1] = Tau[(int64_t)(n - 1) * n + (n - 1)].re;
      const Z s = Tau[(int64_t)(n - 1) * n + (n - 2)];
      ee2[n - 2] = s.re * s.re + s.im * s.im;
    } else if (n == 1 && tid == 0) {
      dd[0] = Tau[0].re;
    }
    __syncthreads();
    // eigenvalues by bisection on the Sturm count, one per thread; ascending
    // index j goes to position n - 1 - j (descending output)
    double lo = 0.0, hi = 0.0, emax = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = (i > 0 ? sqrt(ee2[i - 1]) : 0.0) + (i + 1 < n ? sqrt(ee2[i]) : 0.0);
      lo = i == 0 ? dd[i] - r : fmin(lo, dd[i] - r);
      hi = i == 0 ? dd[i] + r : fmax(hi, dd[i] + r);
      if (i + 1 < n) emax = fmax(emax, ee2[i]);
    }
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax) * 4.0;
    double *out = tn + (int64_t)p * ld;
    for (int j = tid; j < n; j += nt) {
      double a = lo - 1e-300, b = hi + 1e-300;
      for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (a + b);
        if (!(mid > a && mid < b)) break;                      // interval at rounding resolution
        if (sturm_count(dd, ee2, n, mid, pivmin) > j) b = mid;
        else a = mid;
      }
      out[n - 1 - j] = 0.5 * (a + b);
    }
    for (int j = n + tid; j < ld; j += nt) out[j] = 0.0;
    if (tid == 0) {
      if (nch) nch[p] = n;
      if (T) T[p] = tr;
      if (fano) fano[p] = tr > 0.0 ? (tr - f2) / tr : __builtin_nan("");
    }
    __syncthreads();
  }
}

}  // namespace

size_t transmission_eigs_workspace(int Mmax, int P) {
  const int grid = P < 512 ? P : 512;
  return (size_t)grid * 2 * (size_t)Mmax * Mmax * sizeof(Z);
}

hipError_t launch_transmission_eigs(const StripTable &tab, const knit_problem *probs, int P, int Mmax,
                                    const knit_z *CR, const knit_z *G1Np, int ld, double *tn, int32_t *nch,
                                    double *T, double *fano, void *ws, hipStream_t stream) {
  const int grid = P < 512 ? P : 512;
  hipLaunchKernelGGL(transmission_eigs_kernel, dim3(grid), dim3(WG), 0, stream, tab, probs, P, CR, G1Np, ld, tn, nch,
                     T, fano, reinterpret_cast<char *>(ws), (int64_t)Mmax * Mmax);
  return hipGetLastError();
}

}  // namespace knit
