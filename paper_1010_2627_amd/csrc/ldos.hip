// Local density of states on every slice: forward sweep with checkpoints,
// then the reverse ("sewing", section 5.3-D) sweep
//   G_LL = g_L,   G_nn = g_n + (g_n V^+) G_{n+1,n+1} (V g_n),
// LDOS_n[i] = -Im (G_nn)_ii / pi  (the on-site Green function of
// section 7.1-D, getG_retarded).  The forward pass keeps g_{ks-1} for every
// segment start ks (stride s, the analogue of the paper's saving level); the
// reverse pass recomputes the g_n of one segment at a time from its
// checkpoint, so memory is (L/s + s + 4) M^2 per problem.

#include "knit_internal.h"
#include "knit_slice.h"

namespace knit {

namespace {

template <class R>
__global__ void __launch_bounds__(WG) ldos_kernel(StripTable tab, const knit_problem *probs, int P,
                                                  const knit_z *onsite, const knit_z *sigmaL,
                                                  const knit_z *sigmaR, int stride_req, double *ldos,
                                                  int32_t *pstatus, char *ws, size_t slab_bytes,
                                                  int Mmax, int Lmax) {
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
  C *X = reinterpret_cast<C *>(slab);   // [M][M] work matrix
  C *Gnn = X + MM;                      // G_{n+1,n+1} / G_nn
  C *U = Gnn + MM;                      // g_n V^+
  C *Wm = U + MM;                       // V g_n, then temporaries
  C *T1 = Wm + MM;
  C *seg = T1 + MM;                     // [stride][M][M] g_n of the current segment
  const int smax = stride_req;          // host passes the resolved stride
  C *cps = seg + (int64_t)(smax < 2 ? 2 : smax) * MM;   // checkpoints [ceil(Lmax/s)][M][M]
  const double qnan = __builtin_nan("");
  const double inv_pi = 0.318309886183790671537767526745;

  for (int p = blockIdx.x; p < P; p += gridDim.x) {
    const knit_problem pr = probs[p];
    const StripDev s = tab.s[pr.strip];
    const int M = s.M, no = s.norb, L = pr.L;
    const int64_t mm = (int64_t)M * M;
    const int st = smax;
    const int nseg = (L + st - 1) / st;
    const knit_z *sL = sigmaL + pr.sigma_off, *sR = sigmaR + pr.sigma_off;
    int flags = 0;

    // one slice of the forward recursion: g_n from gprev (natural order) into dst
    auto step = [&](int n, const C *gprev, C *dst) {
      const knit_z *D = onsite + pr.onsite_off + (int64_t)n * M * no;
      form_slice_matrix<R>(X, s, pr.E, D, sL, sR, n == 0, n == L - 1, gprev);
      __syncthreads();
      flags |= wg_gauss_jordan<R>(X, M, M, M, q, colj, prow, sv, si);
      wg_invert_perm(q, pinv, M);
      for (int64_t i = tid; i < mm; i += nt) {
        const int a = (int)(i / M), b = (int)(i % M);
        dst[i] = X[(int64_t)a * M + pinv[b]];
      }
      __syncthreads();
    };

    // forward pass: checkpoint k holds g_{k*st - 1} (k >= 1)
    {
      C *cur = seg, *prev = seg + mm;   // ping-pong inside the segment buffer (st >= 2 or extra)
      for (int n = 0; n < L; ++n) {
        step(n, prev, cur);
        if ((n + 1) % st == 0 && (n + 1) < L) {
          C *cp = cps + (int64_t)((n + 1) / st) * MM;
          for (int64_t i = tid; i < mm; i += nt) cp[i] = cur[i];
          __syncthreads();
        }
        C *t = cur;
        cur = prev;
        prev = t;
      }
    }
    // reverse pass, one segment at a time
    double *out = ldos + pr.ldos_off;
    for (int k = nseg - 1; k >= 0; --k) {
      const int n0 = k * st, n1 = min(L, n0 + st);
      for (int n = n0; n < n1; ++n) {
        const C *gprev = (n == n0) ? (k > 0 ? cps + (int64_t)k * MM : nullptr) : seg + (int64_t)(n - n0 - 1) * MM;
        step(n, gprev, seg + (int64_t)(n - n0) * MM);
      }
      for (int n = n1 - 1; n >= n0; --n) {
        const C *g = seg + (int64_t)(n - n0) * MM;
        if (n == L - 1) {
          for (int64_t i = tid; i < mm; i += nt) Gnn[i] = g[i];
          __syncthreads();
        } else {
          // G_nn = g + U Gnn W with U = g V^+, W = V g
          right_mul_vdag<R>(U, g, s, M, false);
          left_mul_v<R>(Wm, g, s, nullptr);
          __syncthreads();
          wg_gemm<R>(T1, M, U, M, Gnn, M, M, M, M, false, gemm_lds);
          for (int64_t i = tid; i < mm; i += nt) Gnn[i] = g[i];
          __syncthreads();
          wg_gemm<R>(Gnn, M, T1, M, Wm, M, M, M, M, true, gemm_lds);
        }
        for (int i = tid; i < M; i += nt) {
          C d = Gnn[(int64_t)i * M + i];
          double v = -r_to_double(d.im) * inv_pi;
          out[(int64_t)n * M + i] = v;
        }
        __syncthreads();
      }
    }
    // non-finite check over the outputs
    double bad = 0.0;
    for (int64_t i = tid; i < (int64_t)L * M; i += nt) bad = fmax(bad, fabs(out[i]));
    bad = wg_max(bad, sv);
    if (!isfinite(bad)) flags |= KNIT_P_NONFINITE;
    if (flags & (KNIT_P_SINGULAR | KNIT_P_NONFINITE))
      for (int64_t i = tid; i < (int64_t)L * M; i += nt) out[i] = qnan;
    if (tid == 0) pstatus[p] = flags;
    __syncthreads();
  }
}

size_t ldos_lds_bytes(int Mmax, int precision) {
  const size_t cs = precision == KNIT_FP64 ? sizeof(cpx<double>) : sizeof(cpx<float>);
  size_t b = 2 * (size_t)Mmax * sizeof(int) + 8 + (WG / WAVE) * (sizeof(double) + sizeof(int)) + 32 + 16;
  size_t gj = 3 * (size_t)Mmax * cs;
  size_t gm = 2 * 32 * 16 * cs;
  return b + (gj > gm ? gj : gm);
}

}  // namespace

size_t ldos_slab_bytes(int Mmax, int Lmax, int stride, int precision) {
  const size_t cs = precision == KNIT_FP64 ? sizeof(cpx<double>) : sizeof(cpx<float>);
  const int segs = (Lmax + stride - 1) / stride;
  const int segbuf = stride < 2 ? 2 : stride;
  size_t b = (size_t)(5 + segbuf + segs) * Mmax * Mmax * cs;
  return (b + 255) & ~size_t(255);
}

hipError_t launch_ldos(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                       const knit_z *sigmaL, const knit_z *sigmaR, int precision, int stride,
                       double *ldos, int32_t *pstatus, void *ws, size_t slab_bytes, int Mmax,
                       hipStream_t stream) {
  const size_t lds = ldos_lds_bytes(Mmax, precision);
  const int grid = P < 1024 ? P : 1024;
  char *w = reinterpret_cast<char *>(ws);
  if (precision == KNIT_FP64) {
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void *)ldos_kernel<double>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(ldos_kernel<double>, dim3(grid), dim3(WG), lds, stream, tab, probs, P, onsite,
                       sigmaL, sigmaR, stride, ldos, pstatus, w, slab_bytes, Mmax, 0);
  } else {
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void *)ldos_kernel<float>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(ldos_kernel<float>, dim3(grid), dim3(WG), lds, stream, tab, probs, P, onsite,
                       sigmaL, sigmaR, stride, ldos, pstatus, w, slab_bytes, Mmax, 0);
  }
  return hipGetLastError();
}

}  // namespace knit
