// Lead self-energy by decimation, in double-double arithmetic.
//
// The leads are integrated out into self-energies on the interface slices
// (section 2.3).  A lead is the clean slice (H0, V) repeated without end
// (section 5.3-B).  Its surface Green function g solves
//   g = (z - h - alpha g beta)^{-1},   z = E + i eta,
// with alpha = V, beta = V^+ for the left lead (surface slice 0, bulk towards
// -x, H_{0,-1} = V) and alpha = V^+, beta = V for the right lead.  The
// renormalisation-group doubling of Lopez Sancho, Lopez Sancho and Rubio
// (J. Phys. F 15, 851 (1985)) halves the number of layers per step:
//   g_k    = (z - eps_k)^{-1}
//   eps_s <- eps_s + a g_k b
//   eps   <- eps + a g_k b + b g_k a
//   a     <- a g_k a,   b <- b g_k b
// until the decimated couplings a, b vanish, and g = (z - eps_s)^{-1}.
//
// Why double-double: the propagating modes of the lead have Bloch factors of
// modulus one, which the doubling squares k times; a relative rounding error
// delta in them grows like 2^k delta while eta must be tiny (the bias of the
// result is of order eta / velocity), and k ~ log2(1/eta).  In FP64 the error
// floor is about sqrt(eps_64) ~ 1e-8, far above the 1e-10 the transmission
// must meet; with ~106-bit arithmetic the same iteration reaches eta = 1e-13
// with rounding far below it.
//
// One workgroup per energy; all matrices live in this energy's workspace.

#include "knit_internal.h"
#include "knit_wg.h"

namespace knit {

namespace {

constexpr int NBUF = 13;   // eps_s, eps, a, b, a2, b2, X, ga, gb, t1, t2, Vf, Vb

__global__ void __launch_bounds__(WG) decimation_kernel(StripDev s, int side, const double *E, int nE,
                                                        double eta, double tol, int max_iter,
                                                        knit_z *sigma, int32_t *iters,
                                                        int32_t *pstatus, char *ws,
                                                        size_t per_energy) {
  using C = cpx<dd>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int e = blockIdx.x;
  if (e >= nE) return;
  const int M = s.M;
  const int64_t MM = (int64_t)M * M;
  const int tid = threadIdx.x, nt = blockDim.x;

  C *base = reinterpret_cast<C *>(ws + (size_t)e * per_energy);
  C *eps_s = base + 0 * MM, *eps = base + 1 * MM, *a = base + 2 * MM, *b = base + 3 * MM;
  C *a2 = base + 4 * MM, *b2 = base + 5 * MM, *X = base + 6 * MM, *ga = base + 7 * MM;
  C *gb = base + 8 * MM, *t1 = base + 9 * MM, *t2 = base + 10 * MM;
  C *Vf = base + 11 * MM;   // alpha as seen from the system: V (left) or V^+ (right)
  C *Vb = base + 12 * MM;   // beta: V^+ (left) or V (right)

  // LDS: GJ scratch and GEMM scratch share one region
  int *q = reinterpret_cast<int *>(lds_raw);
  int *pinv = q + M;
  double *sv = reinterpret_cast<double *>(pinv + M);
  int *si = reinterpret_cast<int *>(sv + WG / WAVE);
  C *colj = reinterpret_cast<C *>(si + WG / WAVE + 8);
  colj = reinterpret_cast<C *>((reinterpret_cast<uintptr_t>(colj) + 15) & ~uintptr_t(15));
  C *prow = colj + M;
  C *gemm_lds = colj;       // 2*32*16 entries, used only outside the GJ

  const double Ez = E[e];
  const C z = {dd{Ez, 0.0}, dd{eta, 0.0}};
  double scale = 1.0;
  for (int64_t i = tid; i < MM; i += nt) {
    const int r = (int)(i / M), c = (int)(i % M);
    cpx<double> h = ld_z(s.H0 + i);
    eps_s[i] = eps[i] = C{dd{h.re, 0.0}, dd{h.im, 0.0}};
    cpx<double> v = strip_V(s, r, c);                 // V[r][c]
    cpx<double> vt = strip_V(s, c, r);                // V[c][r] -> (V^+)[r][c] = conj(vt)
    C Vrc = {dd{v.re, 0.0}, dd{v.im, 0.0}};
    C Vdrc = {dd{vt.re, 0.0}, dd{-vt.im, 0.0}};
    scale = fmax(scale, fmax(fabs(h.re) + fabs(h.im), fabs(v.re) + fabs(v.im)));
    if (side == 0) {
      a[i] = Vrc;
      b[i] = Vdrc;
      Vf[i] = Vrc;
      Vb[i] = Vdrc;
    } else {
      a[i] = Vdrc;
      b[i] = Vrc;
      Vf[i] = Vdrc;
      Vb[i] = Vrc;
    }
  }
  scale = wg_max(scale, sv);
  __syncthreads();

  int flags = 0, it = 0;
  bool converged = false;
  for (it = 1; it <= max_iter; ++it) {
    for (int64_t i = tid; i < MM; i += nt) {
      const int r = (int)(i / M), c = (int)(i % M);
      C x = c_neg(eps[i]);
      if (r == c) x = c_add(x, z);
      X[i] = x;
    }
    __syncthreads();
    flags |= wg_gauss_jordan<dd>(X, M, M, M, q, colj, prow, sv, si);
    wg_invert_perm(q, pinv, M);
    // g = X[:, pinv] -> store in t1 (free at this point)
    for (int64_t i = tid; i < MM; i += nt) {
      const int r = (int)(i / M), c = (int)(i % M);
      t1[i] = X[(int64_t)r * M + pinv[c]];
    }
    __syncthreads();
    wg_gemm<dd>(ga, M, t1, M, a, M, M, M, M, false, gemm_lds);   // g a
    wg_gemm<dd>(gb, M, t1, M, b, M, M, M, M, false, gemm_lds);   // g b
    wg_gemm<dd>(t1, M, a, M, gb, M, M, M, M, false, gemm_lds);   // a g b
    wg_gemm<dd>(t2, M, b, M, ga, M, M, M, M, false, gemm_lds);   // b g a
    wg_gemm<dd>(a2, M, a, M, ga, M, M, M, M, false, gemm_lds);   // a g a
    wg_gemm<dd>(b2, M, b, M, gb, M, M, M, M, false, gemm_lds);   // b g b
    double amax = 0.0;
    for (int64_t i = tid; i < MM; i += nt) {
      eps_s[i] = c_add(eps_s[i], t1[i]);
      eps[i] = c_add(eps[i], c_add(t1[i], t2[i]));
      a[i] = a2[i];
      b[i] = b2[i];
      amax = fmax(amax, fmax(c_abs1(a2[i]), c_abs1(b2[i])));
    }
    amax = wg_max(amax, sv);
    __syncthreads();
    if (!(amax == amax) || isinf(amax)) {
      flags |= KNIT_P_NONFINITE;
      break;
    }
    if (amax < tol * scale) {
      converged = true;
      break;
    }
  }
  if (!converged) flags |= KNIT_P_NOCONV;

  // g = (z - eps_s)^{-1};  Sigma = Vf g Vb
  for (int64_t i = tid; i < MM; i += nt) {
    const int r = (int)(i / M), c = (int)(i % M);
    C x = c_neg(eps_s[i]);
    if (r == c) x = c_add(x, z);
    X[i] = x;
  }
  __syncthreads();
  flags |= wg_gauss_jordan<dd>(X, M, M, M, q, colj, prow, sv, si);
  wg_invert_perm(q, pinv, M);
  for (int64_t i = tid; i < MM; i += nt) {
    const int r = (int)(i / M), c = (int)(i % M);
    t1[i] = X[(int64_t)r * M + pinv[c]];
  }
  __syncthreads();
  wg_gemm<dd>(t2, M, Vf, M, t1, M, M, M, M, false, gemm_lds);
  wg_gemm<dd>(ga, M, t2, M, Vb, M, M, M, M, false, gemm_lds);
  const double qnan = __builtin_nan("");
  knit_z *out = sigma + (int64_t)e * MM;
  bool bad = (flags & (KNIT_P_SINGULAR | KNIT_P_NONFINITE)) != 0;
  for (int64_t i = tid; i < MM; i += nt) {
    cpx<double> v = {r_to_double(ga[i].re), r_to_double(ga[i].im)};
    if (bad) v = {qnan, qnan};
    st_z(out + i, v);
  }
  if (tid == 0) {
    pstatus[e] = flags;
    if (iters) iters[e] = it > max_iter ? max_iter : it;
  }
}

}  // namespace

size_t decimation_bytes_per_energy(int M) {
  size_t b = (size_t)NBUF * M * M * sizeof(cpx<dd>);
  return (b + 255) & ~size_t(255);
}

static size_t decimation_lds_bytes(int M) {
  size_t b = 2 * (size_t)M * sizeof(int) + 8 + (WG / WAVE) * (sizeof(double) + sizeof(int)) + 32 + 16;
  size_t gj = 2 * (size_t)M * sizeof(cpx<dd>);
  size_t gm = 2 * 32 * 16 * sizeof(cpx<dd>);
  return b + (gj > gm ? gj : gm);
}

hipError_t launch_decimation(const StripDev &s, int side, const double *E, int nE, double eta,
                             double tol, int max_iter, knit_z *sigma, int32_t *iters,
                             int32_t *pstatus, void *ws, size_t per_energy_bytes,
                             hipStream_t stream) {
  size_t lds = decimation_lds_bytes(s.M);
  if (lds > 65536) {
    hipError_t err = hipFuncSetAttribute((const void *)decimation_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
  }
  hipLaunchKernelGGL(decimation_kernel, dim3(nE), dim3(WG), lds, stream, s, side, E, nE, eta, tol,
                     max_iter, sigma, iters, pstatus, reinterpret_cast<char *>(ws), per_energy_bytes);
  return hipGetLastError();
}

}  // namespace knit
