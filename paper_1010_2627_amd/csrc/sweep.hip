// Slice recursive Green function sweep, generic workgroup-per-problem version.
//
// Basic recursive Green function algorithm (section 1): start at the left
// lead and add the slices of the strip one by one until the right lead.
// Per problem, for n = 1..L (slice index n-1 in the code):
//   A_n  = E - H0 - D_n - [n=1] Sigma_L - [n=L] Sigma_R - [n>1] V g_{n-1} V^+
//   B_n  = -G_{1,n-1} V^+                                   (n > 1)
// The stacked matrix X = [A_n; B_n] is reduced in place by Gauss-Jordan
// elimination with partial pivoting among the rows of A_n; that leaves
// g_n = A_n^{-1} on top and -B_n A_n^{-1} = G_{1,n-1} V^+ g_n = G_1n below,
// so the propagator rides along in the same elimination.  Optionally
// G_n1 = g_n V G_{n-1,1} is carried too (for the T_RL check).
//
// V is block-monomial (each site bonds to at most one site of the previous
// slice), so V g V^+ and G V^+ are gathers with norb x norb blocks.

#include "knit_internal.h"
#include "knit_slice.h"

namespace knit {

namespace {

template <class R>
struct SweepSlab {
  cpx<R> *X;    // [2M][M]
  cpx<R> *g;    // [M][M] g_{n} (columns in natural order)
  cpx<R> *G1;   // [M][M] G_{1n}
  cpx<R> *N1a;  // [M][M] G_{n1}
  cpx<R> *N1b;  // [M][M] scratch for V G_{n-1,1} with permuted rows
};

template <class R>
__global__ void __launch_bounds__(WG) sweep_kernel(StripTable tab, const knit_problem *probs, int P,
                                                   const knit_z *onsite, const knit_z *sigmaL,
                                                   const knit_z *sigmaR, knit_z *G1N, knit_z *GN1,
                                                   knit_z *GNN, int32_t *pstatus, char *ws,
                                                   size_t slab_bytes, int Mmax) {
  using C = cpx<R>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int tid = threadIdx.x, nt = blockDim.x;
  int *q = reinterpret_cast<int *>(lds_raw);
  int *pinv = q + Mmax;
  double *sv = reinterpret_cast<double *>(pinv + Mmax);
  int *si = reinterpret_cast<int *>(sv + WG / WAVE);
  C *colj = reinterpret_cast<C *>(si + WG / WAVE + 8);
  colj = reinterpret_cast<C *>((reinterpret_cast<uintptr_t>(colj) + 15) & ~uintptr_t(15));
  C *prow = colj + 2 * Mmax;
  C *gemm_lds = colj;

  const int64_t MM = (int64_t)Mmax * Mmax;
  char *slab = ws + (size_t)blockIdx.x * slab_bytes;
  SweepSlab<R> S;
  S.X = reinterpret_cast<C *>(slab);
  S.g = S.X + 2 * MM;
  S.G1 = S.g + MM;
  S.N1a = S.G1 + MM;
  S.N1b = S.N1a + MM;
  const bool want_n1 = GN1 != nullptr;
  const double qnan = __builtin_nan("");

  for (int p = blockIdx.x; p < P; p += gridDim.x) {
    const knit_problem pr = probs[p];
    const StripDev s = tab.s[pr.strip];
    const int M = s.M, no = s.norb, L = pr.L;
    const int64_t mm = (int64_t)M * M;
    const knit_z *sL = sigmaL + pr.sigma_off;
    const knit_z *sR = sigmaR + pr.sigma_off;
    int flags = 0;
    for (int n = 0; n < L; ++n) {
      const knit_z *D = onsite + pr.onsite_off + (int64_t)n * M * no;   // [W][no][no]
      // ---- form A_n (top) and B_n = -G_{1,n-1} V^+ (bottom)
      form_slice_matrix<R>(S.X, s, pr.E, D, sL, sR, n == 0, n == L - 1, S.g);
      if (n > 0) right_mul_vdag<R>(S.X + mm, S.G1, s, M, true);
      __syncthreads();
      const int Rtot = n > 0 ? 2 * M : M;
      flags |= wg_gauss_jordan<R>(S.X, M, M, Rtot, q, colj, prow, sv, si);
      wg_invert_perm(q, pinv, M);
      // ---- G_n1 = g_n V G_{n-1,1}: rows of V G_{n-1,1} permuted by q, times (P A)^{-1}
      if (want_n1 && n > 0) {
        left_mul_v<R>(S.N1b, S.N1a, s, q);
        __syncthreads();
        wg_gemm<R>(S.N1a, M, S.X, M, S.N1b, M, M, M, M, false, gemm_lds);
      }
      // ---- unpermute columns: g_n and G_1n
      for (int64_t i = tid; i < mm; i += nt) {
        const int a = (int)(i / M), b = (int)(i % M);
        S.g[i] = S.X[(int64_t)a * M + pinv[b]];
        if (n > 0) S.G1[i] = S.X[mm + (int64_t)a * M + pinv[b]];
      }
      __syncthreads();
      if (n == 0) {
        for (int64_t i = tid; i < mm; i += nt) {
          S.G1[i] = S.g[i];
          if (want_n1) S.N1a[i] = S.g[i];
        }
        __syncthreads();
      }
    }
    // ---- outputs
    double bad = 0.0;
    for (int64_t i = tid; i < mm; i += nt) {
      C v = S.G1[i];
      bad = fmax(bad, c_abs1(v));
      if (GNN) bad = fmax(bad, c_abs1(S.g[i]));
      if (want_n1) bad = fmax(bad, c_abs1(S.N1a[i]));
    }
    bad = wg_max(bad, sv);
    if (!isfinite(bad)) flags |= KNIT_P_NONFINITE;
    const bool kill = (flags & (KNIT_P_SINGULAR | KNIT_P_NONFINITE)) != 0;
    for (int64_t i = tid; i < mm; i += nt) {
      cpx<double> v = {r_to_double(S.G1[i].re), r_to_double(S.G1[i].im)};
      if (kill) v = {qnan, qnan};
      st_z(G1N + pr.out_off + i, v);
      if (GNN) {
        cpx<double> w = {r_to_double(S.g[i].re), r_to_double(S.g[i].im)};
        if (kill) w = {qnan, qnan};
        st_z(GNN + pr.out_off + i, w);
      }
      if (want_n1) {
        cpx<double> w = {r_to_double(S.N1a[i].re), r_to_double(S.N1a[i].im)};
        if (kill) w = {qnan, qnan};
        st_z(GN1 + pr.out_off + i, w);
      }
    }
    if (tid == 0) pstatus[p] = flags;
    __syncthreads();
  }
}

size_t sweep_lds_bytes(int Mmax, int precision) {
  const size_t cs = precision == KNIT_FP64 ? sizeof(cpx<double>) : sizeof(cpx<float>);
  size_t b = 2 * (size_t)Mmax * sizeof(int) + 8 + (WG / WAVE) * (sizeof(double) + sizeof(int)) + 32 + 16;
  size_t gj = 3 * (size_t)Mmax * cs;
  size_t gm = 2 * 32 * 16 * cs;
  return b + (gj > gm ? gj : gm);
}

}  // namespace

size_t sweep_slab_bytes(int Mmax, int precision) {
  const size_t cs = precision == KNIT_FP64 ? sizeof(cpx<double>) : sizeof(cpx<float>);
  size_t b = 6 * (size_t)Mmax * Mmax * cs;
  return (b + 255) & ~size_t(255);
}

int sweep_grid(int P) { return P < 1024 ? P : 1024; }

hipError_t launch_sweep(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                        const knit_z *sigmaL, const knit_z *sigmaR, int precision, knit_z *G1N,
                        knit_z *GN1, knit_z *GNN, int32_t *pstatus, void *ws, size_t slab_bytes,
                        int Mmax, hipStream_t stream) {
  const size_t lds = sweep_lds_bytes(Mmax, precision);
  const int grid = sweep_grid(P);
  char *w = reinterpret_cast<char *>(ws);
  if (precision == KNIT_FP64) {
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void *)sweep_kernel<double>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(sweep_kernel<double>, dim3(grid), dim3(WG), lds, stream, tab, probs, P, onsite,
                       sigmaL, sigmaR, G1N, GN1, GNN, pstatus, w, slab_bytes, Mmax);
  } else {
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void *)sweep_kernel<float>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(sweep_kernel<float>, dim3(grid), dim3(WG), lds, stream, tab, probs, P, onsite,
                       sigmaL, sigmaR, G1N, GN1, GNN, pstatus, w, slab_bytes, Mmax);
  }
  return hipGetLastError();
}

}  // namespace knit
