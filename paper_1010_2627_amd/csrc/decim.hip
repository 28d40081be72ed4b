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
// must meet; with ~106-bit arithmetic the same iteration reaches eta = 1e-16
// (about 60 steps, rounding growth 2^60 * 1e-32 ~ 1e-14) and keeps the bias
// eta / velocity below 1e-12 even 1e-9 from a channel threshold, where the
// newly open mode is slow.
//
// Both leads from one run: swapping alpha and beta leaves the doubling
// unchanged (g_k, eps and the pair {a, b} are symmetric in the swap), so the
// right lead's surface term b g_k a is the second half of the bulk update the
// left run computes anyway.  With side 2 the second surface eps_r collects it.
//
// Work layout (every energy runs the same sequence of launches):
//   * g_k: the FP64 inverse of z - eps_k on the matrix cores (one workgroup
//     per energy), then two Newton steps X <- X + X R, R = I - A X, each of
//     which squares the residual (1e-16 kappa -> ~1e-64 kappa^4).  R is formed
//     in double-double; the correction X R is small (|R| |X|), so its FP64
//     product on the matrix cores, rounding ~1e-16 |R| |X|, stays below the
//     |R|^2 the step leaves, and it is added to X in double-double;
//   * every product is a batched double-double tile GEMM over (tile, energy),
//     so all compute units share the work of every energy;
//   * convergence is decided on the device per energy: later launches skip
//     finished energies, and the host issues max_iter iterations without
//     waiting for the device.
//
// Energies at an eigenvalue of the single slice: every doubling step k
// inverts z - eps_k, which is singular where E is an eigenvalue of a strip of
// 2^(k+1) - 1 slices; at E = 0 on a bipartite strip with a zero mode (square
// lattice, odd width) that holds for every k, and the 1/eta-sized parts of
// the decimated couplings amplify rounding by about eta^-2, beyond double-
// double.  Every result is therefore checked against its defining equation,
//   R = (z - h - Sigma) g - I,   g the surface Green function,
// in double-double, and an energy with max |R| > 1e-12 (or a non-finite
// result) is redone with a cell of two slices,
//   h2 = [[h, alpha], [beta, h]],  alpha2 = [[0, 0], [alpha, 0]],
// whose strips all have an even number of slices: the surface slice's g is
// the leading block of the cell's surface Green function (the trailing block
// for the right lead's surface of a side-2 run).  Up to RETRY_SLOTS energies
// per call are redone, when 2M fits the matrix-core inverse; any other failing
// energy gets KNIT_P_NOCONV and NaN output.

#include <atomic>

#include "knit_internal.h"
#include "knit_mfma.h"

namespace knit {

namespace {

#pragma clang fp contract(off)

using Z = cpx<dd>;
using D = cpx<double>;

constexpr int GT = 32;     // GEMM output tile edge
constexpr int GK = 16;     // GEMM k-slice staged in LDS
constexpr int GTHREADS = 256;
constexpr int EW = 256;    // elementwise kernels: threads per workgroup
constexpr int EW_BLOCKS = 64;   // elementwise kernels: workgroups per energy

// Per-energy state, at the start of the workspace.
struct DecState {
  int32_t done, iters, flags;
  int32_t skip;              // 1: left alone by the final stage (an unused retry slot)
  unsigned long long amax;   // bits of a non-negative double (max |a|, |b| of the step)
  unsigned long long scale;  // bits of max(1, max |H0|, max |V|)
  unsigned long long resid;  // bits of max |R| of the defining equation's check
};

constexpr int RETRY_SLOTS = 4;          // energies redone with the two-slice cell per call
constexpr double RESID_TOL = 1e-12;     // max |(z - h - Sigma) g - I| accepted
constexpr int DEC_RETRY = 1 << 8;       // internal flag bits (never reported)
constexpr int DEC_FAILED = 1 << 9;
constexpr int DEC_PUBLIC = KNIT_P_SINGULAR | KNIT_P_NOCONV | KNIT_P_NONFINITE;

// Skip rules of the per-energy kernels: 0 none, 1 finished energies, 2 unused slots.
__device__ __forceinline__ bool dec_skip(const DecState *st, int e, int check) {
  return (check == 1 && st[e].done) || (check == 2 && st[e].skip);
}

// Per-energy slab: buffer offsets in bytes.
struct Slab {
  size_t bytes;
  size_t z[17];               // double-double [M][M] buffers
  size_t x64, scr, xi64;      // FP64: padded [Mp][Mp], elimination scratch, natural [M][M]
  size_t oz_a, oz_b;          // digit planes of the two factors of a product (INT8 matrix cores)
  size_t oz_ea, oz_eb;        // their row / column exponents (int32 [M])
};
enum { ZEPS_S, ZEPS_R, ZEPS, ZA, ZXA, ZXB, ZR, ZGA, ZGB, ZT1, ZT2, ZA0, ZA1, ZB0, ZB1, ZVF, ZVB };

Slab slab_of(int M) {
  Slab s{};
  size_t off = 0;
  const size_t zb = (((size_t)M * M * sizeof(Z)) + 255) & ~size_t(255);
  for (int i = 0; i < 17; ++i) {
    s.z[i] = off;
    off += zb;
  }
  const size_t Mp = (size_t)mfma_padded(M);
  s.x64 = off;
  off += ((Mp * Mp * sizeof(D)) + 255) & ~size_t(255);
  s.scr = off;
  off += ((inverse_fp64_scratch_elems(M) * sizeof(D)) + 255) & ~size_t(255);
  s.xi64 = off;
  off += (((size_t)M * M * sizeof(D)) + 255) & ~size_t(255);
  const size_t planes = ((2 * 16 * (size_t)((M + 31) / 32 * 32) * ((M + 63) / 64 * 64)) + 255) & ~size_t(255);
  s.oz_a = off;
  off += planes;
  s.oz_b = off;
  off += planes;
  s.oz_ea = off;
  off += (((size_t)M * sizeof(int32_t)) + 255) & ~size_t(255);
  s.oz_eb = off;
  off += (((size_t)M * sizeof(int32_t)) + 255) & ~size_t(255);
  s.bytes = off;
  return s;
}

__device__ __forceinline__ Z zdd(D v) { return {dd{v.re, 0.0}, dd{v.im, 0.0}}; }
__device__ __forceinline__ Z zdd(Z v) { return v; }
__device__ __forceinline__ double to_d(dd v) { return v.hi + v.lo; }

// acc (hi, lo) += x * y for double-double x, y: the product's leading part is
// added with an exact two_sum; its rounding error and the cross terms go to
// lo, which is renormalised once after the k loop.
__device__ __forceinline__ void dd_acc(double &hi, double &lo, dd x, dd y) {
  const double p = x.hi * y.hi;
  const double e = __builtin_fma(x.hi, y.hi, -p);
  const double s = hi + p;
  const double bb = s - hi;
  const double t = (hi - (s - bb)) + (p - bb);
  hi = s;
  lo = lo + (t + e);
  lo = __builtin_fma(x.hi, y.lo, lo);
  lo = __builtin_fma(x.lo, y.hi, lo);
}

// A staged complex operand with the sum of its parts, for the three-product
// (Gauss) form of a complex multiply-add:
//   re += ar br - ai bi,   im += (ar + ai)(br + bi) - ar br - ai bi
// i.e. three double-double products per complex term instead of four; the
// sums are formed once per staged element, exactly in double-double.
struct Z3 {
  dd re, im, s;
};
__device__ __forceinline__ Z3 z3(Z v) { return {v.re, v.im, r_add(v.re, v.im)}; }

// C_e = cI I + (+/-) A_e B_e + [D_e], all [M][M], double-double C and D,
// A and B double-double or FP64.  Grid: (tiles of C, energies).
template <class TA, class TB>
__global__ void __launch_bounds__(GTHREADS) dd_gemm_kernel(const TA *A, const TB *B, const Z *Dm, Z *C,
                                                           int64_t stride_bytes, int M, double cI,
                                                           int negate, const DecState *st, int check_done) {
  __shared__ Z3 As[GT][GK + 1];
  __shared__ Z3 Bs[GK][GT + 1];
  const int e = blockIdx.y;
  if (dec_skip(st, e, check_done)) return;
  const int64_t eo = (int64_t)e * stride_bytes;
  const TA *Ae = reinterpret_cast<const TA *>(reinterpret_cast<const char *>(A) + eo);
  const TB *Be = reinterpret_cast<const TB *>(reinterpret_cast<const char *>(B) + eo);
  Z *Ce = reinterpret_cast<Z *>(reinterpret_cast<char *>(C) + eo);
  const Z *De = Dm ? reinterpret_cast<const Z *>(reinterpret_cast<const char *>(Dm) + eo) : nullptr;
  const int tiles_n = (M + GT - 1) / GT;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  // tiles of C, strided over the grid's x dimension
  for (int tile = blockIdx.x; tile < tiles_n * tiles_n; tile += gridDim.x) {
    const int r0 = (tile / tiles_n) * GT, c0 = (tile % tiles_n) * GT;
    const Z zero = {{0.0, 0.0}, {0.0, 0.0}};
    double acc[2][2][6];   // [i][j][p1.hi, p1.lo, p2.hi, p2.lo, p3.hi, p3.lo]
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 6; ++q) acc[i][j][q] = 0.0;
    for (int k0 = 0; k0 < M; k0 += GK) {
      // stage A[r0:r0+32, k0:k0+16] and B[k0:k0+16, c0:c0+32], zero outside M
      for (int i = tid; i < GT * GK; i += GTHREADS) {
        const int r = i / GK, k = i % GK;
        const int gr = r0 + r, gk = k0 + k;
        As[r][k] = z3((gr < M && gk < M) ? zdd(Ae[(int64_t)gr * M + gk]) : zero);
      }
      for (int i = tid; i < GK * GT; i += GTHREADS) {
        const int k = i / GT, c = i % GT;
        const int gk = k0 + k, gc = c0 + c;
        Bs[k][c] = z3((gk < M && gc < M) ? zdd(Be[(int64_t)gk * M + gc]) : zero);
      }
      __syncthreads();
#pragma unroll 2
      for (int k = 0; k < GK; ++k) {
        Z3 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[ty + 16 * i][k];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            dd_acc(acc[i][j][0], acc[i][j][1], a[i].re, b[j].re);
            dd_acc(acc[i][j][2], acc[i][j][3], a[i].im, b[j].im);
            dd_acc(acc[i][j][4], acc[i][j][5], a[i].s, b[j].s);
          }
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = r0 + ty + 16 * i, c = c0 + tx + 16 * j;
        if (r >= M || c >= M) continue;
        const dd p1 = quick_two_sum(acc[i][j][0], acc[i][j][1]);
        const dd p2 = quick_two_sum(acc[i][j][2], acc[i][j][3]);
        const dd p3 = quick_two_sum(acc[i][j][4], acc[i][j][5]);
        Z v = {r_sub(p1, p2), r_sub(r_sub(p3, p1), p2)};
        if (negate) v = c_neg(v);
        if (cI != 0.0 && r == c) v.re = r_add(v.re, dd{cI, 0.0});
        if (De) v = c_add(v, De[(int64_t)r * M + c]);
        Ce[(int64_t)r * M + c] = v;
      }
  }
}

__device__ __forceinline__ D hi_of(D v) { return v; }
__device__ __forceinline__ D hi_of(Z v) { return D{v.re.hi, v.im.hi}; }

// Newton correction C_e = X_e + X_e R_e ([M][M] each energy; X double-double
// or FP64, R double-double): the product of the FP64 leading parts on the
// matrix cores (v_mfma_f64_16x16x4f64, four real products per complex one),
// added to X in double-double.  One wave per 32 x 32 output tile.
template <class TX>
__global__ void __launch_bounds__(64) newton_corr_kernel(const TX *X, const Z *R, Z *C, int64_t stride_bytes, int M,
                                                         const DecState *st, int check) {
  const int e = blockIdx.y;
  if (dec_skip(st, e, check)) return;
  const int64_t eo = (int64_t)e * stride_bytes;
  const TX *Xe = reinterpret_cast<const TX *>(reinterpret_cast<const char *>(X) + eo);
  const Z *Re = reinterpret_cast<const Z *>(reinterpret_cast<const char *>(R) + eo);
  Z *Ce = reinterpret_cast<Z *>(reinterpret_cast<char *>(C) + eo);
  const int tn = (M + 31) / 32;
  const int r0 = (int)(blockIdx.x / tn) * 32, c0 = (int)(blockIdx.x % tn) * 32;
  const int l = threadIdx.x;
  CTile<double, 2> acc;
  acc.zero();
  for (int k = 0; k < M; k += 4) {
    cpx<double> a[2], b[2];
    const int kk = k + (l >> 4);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = r0 + 16 * i + (l & 15);
      const D v = (r < M && kk < M) ? hi_of(Xe[(int64_t)r * M + kk]) : D{0.0, 0.0};
      a[i] = {v.re, v.im};
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = c0 + 16 * j + (l & 15);
      const D v = (kk < M && c < M) ? hi_of(Re[(int64_t)kk * M + c]) : D{0.0, 0.0};
      b[j] = {v.re, v.im};
    }
    ctile_mma<double, 2>(acc, a, b);
  }
  ctile_for_each<double, 2>(acc, [&](int r, int c, double &re, double &im) {
    const int gr = r0 + r, gc = c0 + c;
    if (gr < M && gc < M) {
      const Z x = zdd(Xe[(int64_t)gr * M + gc]);
      Ce[(int64_t)gr * M + gc] = Z{r_add(x.re, dd{re, 0.0}), r_add(x.im, dd{im, 0.0})};
    }
  });
}

__device__ __forceinline__ char *slab_ptr(char *ws, const Slab &sl, int e, size_t off) {
  return ws + (size_t)e * sl.bytes + off;
}

// eps_s = eps_r = eps = H0, a = alpha, b = beta, Vf = alpha, Vb = beta (dd);
// state reset; scale = max(1, max|H0|, max|V|).
__global__ void __launch_bounds__(EW) dec_init_kernel(StripDev s, int side, char *ws, Slab sl, DecState *st) {
  const int e = blockIdx.y, M = s.M;
  const int64_t MM = (int64_t)M * M;
  Z *eps_s = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZEPS_S]));
  Z *eps_r = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZEPS_R]));
  Z *eps = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZEPS]));
  Z *a = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZA0]));
  Z *b = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZB0]));
  Z *vf = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZVF]));
  Z *vb = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZVB]));
  double scale = 1.0;
  for (int64_t i = blockIdx.x * (int64_t)EW + threadIdx.x; i < MM; i += (int64_t)gridDim.x * EW) {
    const int r = (int)(i / M), c = (int)(i % M);
    const D h = ld_z(s.H0 + i);
    eps_s[i] = eps_r[i] = eps[i] = zdd(h);
    const D v = strip_V(s, r, c);           // V[r][c]
    const D vt = strip_V(s, c, r);          // (V^+)[r][c] = conj(V[c][r])
    const Z Vrc = zdd(v), Vdrc = zdd(D{vt.re, -vt.im});
    scale = fmax(scale, fmax(fabs(h.re) + fabs(h.im), fabs(v.re) + fabs(v.im)));
    const bool left = side != 1;
    a[i] = vf[i] = left ? Vrc : Vdrc;
    b[i] = vb[i] = left ? Vdrc : Vrc;
  }
  // scale: non-negative doubles order like their bit patterns
  atomicMax(&st[e].scale, (unsigned long long)__double_as_longlong(scale));
}

__global__ void dec_reset_state_kernel(DecState *st, int nE) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nE) st[e] = DecState{0, 0, 0, 0, 0ull, 0ull, 0ull};
}

// Two-slice cell of a retry slot (dimension 2M):
//   eps_s = eps_r = eps = [[h, alpha], [beta, h]],  a = [[0, 0], [alpha, 0]],
//   b = a^+ = [[0, beta], [0, 0]],  Vf = diag(alpha, alpha),  Vb = diag(beta, beta)
// (alpha = V, beta = V^+ for the left lead, swapped for side 1).
__global__ void __launch_bounds__(EW) dec_init2_kernel(StripDev s, int side, char *ws, Slab sl, const DecState *st) {
  const int e = blockIdx.y, M = s.M, M2 = 2 * s.M;
  if (st[e].done) return;
  Z *eps_s = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZEPS_S]));
  Z *eps_r = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZEPS_R]));
  Z *eps = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZEPS]));
  Z *a = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZA0]));
  Z *b = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZB0]));
  Z *vf = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZVF]));
  Z *vb = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZVB]));
  const bool left = side != 1;
  const Z zero = {{0.0, 0.0}, {0.0, 0.0}};
  for (int64_t i = blockIdx.x * (int64_t)EW + threadIdx.x; i < (int64_t)M2 * M2; i += (int64_t)gridDim.x * EW) {
    const int r = (int)(i / M2), c = (int)(i % M2);
    const int br = r / M, bc = c / M, rr = r % M, cc = c % M;
    const D v = strip_V(s, rr, cc);           // V[rr][cc]
    const D vt = strip_V(s, cc, rr);          // (V^+)[rr][cc] = conj(V[cc][rr])
    const Z Vrc = zdd(v), Vdrc = zdd(D{vt.re, -vt.im});
    const Z al = left ? Vrc : Vdrc, be = left ? Vdrc : Vrc;
    Z h;
    if (br == bc) h = zdd(ld_z(s.H0 + (int64_t)rr * M + cc));
    else h = br == 0 ? al : be;
    eps_s[i] = eps_r[i] = eps[i] = h;
    a[i] = (br == 1 && bc == 0) ? al : zero;
    b[i] = (br == 0 && bc == 1) ? be : zero;
    vf[i] = br == bc ? al : zero;
    vb[i] = br == bc ? be : zero;
  }
}

// A = z - es (dd) and its FP64 copy, padded to Mp with an identity block.
__global__ void __launch_bounds__(EW) dec_form_kernel(int M, int Mp, const double *E, const int *emap, double eta,
                                                      char *ws, Slab sl, int src, const DecState *st, int check_done) {
  const int e = blockIdx.y;
  if (dec_skip(st, e, check_done)) return;
  const Z *es = reinterpret_cast<const Z *>(slab_ptr(ws, sl, e, sl.z[src]));
  Z *A = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZA]));
  D *X64 = reinterpret_cast<D *>(slab_ptr(ws, sl, e, sl.x64));
  const double Ez = E[emap ? emap[e] : e];
  for (int64_t i = blockIdx.x * (int64_t)EW + threadIdx.x; i < (int64_t)Mp * Mp; i += (int64_t)gridDim.x * EW) {
    const int r = (int)(i / Mp), c = (int)(i % Mp);
    if (r < M && c < M) {
      Z x = c_neg(es[(int64_t)r * M + c]);
      if (r == c) x = c_add(x, Z{dd{Ez, 0.0}, dd{eta, 0.0}});
      A[(int64_t)r * M + c] = x;
      X64[i] = D{to_d(x.re), to_d(x.im)};
    } else {
      X64[i] = D{r == c ? 1.0 : 0.0, 0.0};
    }
  }
}

// eps_s += t1, [eps_r += t2], eps += t1 + t2; max |a_new|, |b_new| -> amax.
__global__ void __launch_bounds__(EW) dec_update_kernel(int M, char *ws, Slab sl, int an, int bn, int both,
                                                        DecState *st) {
  __shared__ double red[EW / 64];
  const int e = blockIdx.y;
  if (st[e].done) return;
  Z *eps_s = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZEPS_S]));
  Z *eps_r = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZEPS_R]));
  Z *eps = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZEPS]));
  const Z *t1 = reinterpret_cast<const Z *>(slab_ptr(ws, sl, e, sl.z[ZT1]));
  const Z *t2 = reinterpret_cast<const Z *>(slab_ptr(ws, sl, e, sl.z[ZT2]));
  const Z *a = reinterpret_cast<const Z *>(slab_ptr(ws, sl, e, sl.z[an]));
  const Z *b = reinterpret_cast<const Z *>(slab_ptr(ws, sl, e, sl.z[bn]));
  double amax = 0.0;
  bool nan = false;
  for (int64_t i = blockIdx.x * (int64_t)EW + threadIdx.x; i < (int64_t)M * M; i += (int64_t)gridDim.x * EW) {
    eps_s[i] = c_add(eps_s[i], t1[i]);
    if (both) eps_r[i] = c_add(eps_r[i], t2[i]);
    eps[i] = c_add(eps[i], c_add(t1[i], t2[i]));
    const double m = fmax(fabs(a[i].re.hi) + fabs(a[i].im.hi), fabs(b[i].re.hi) + fabs(b[i].im.hi));
    if (m != m) nan = true;
    else amax = fmax(amax, m);
  }
  if (nan) amax = __builtin_inf();
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < EW / 64; ++w) amax = fmax(amax, red[w]);
    amax = fmax(amax, red[0]);
    atomicMax(&st[e].amax, (unsigned long long)__double_as_longlong(amax));
  }
}

// One thread per energy: count the step, decide convergence.
__global__ void dec_decide_kernel(DecState *st, int nE, double tol, int max_iter) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nE || st[e].done) return;
  const double amax = __longlong_as_double((long long)st[e].amax);
  const double scale = __longlong_as_double((long long)st[e].scale);
  st[e].amax = 0ull;
  const int it = ++st[e].iters;
  if (st[e].flags & KNIT_P_SINGULAR) {
    st[e].done = 1;
  } else if (!isfinite(amax)) {
    st[e].flags |= KNIT_P_NONFINITE;
    st[e].done = 1;
  } else if (amax < tol * scale) {
    st[e].done = 1;
  } else if (it >= max_iter) {
    st[e].flags |= KNIT_P_NOCONV;
    st[e].done = 1;
  }
}

// sigma (FP64) from the M x M block at (off, off) of the dd product (leading
// dimension ld) of energy emap[e] (or e); NaN for failed energies.
__global__ void __launch_bounds__(EW) dec_store_kernel(int M, int ld, int off, char *ws, Slab sl, int src,
                                                       knit_z *sigma, int64_t sigma_stride, const DecState *st,
                                                       const int *emap, int check) {
  const int e = blockIdx.y;
  if (dec_skip(st, e, check)) return;
  const Z *s = reinterpret_cast<const Z *>(slab_ptr(ws, sl, e, sl.z[src]));
  knit_z *out = sigma + (int64_t)(emap ? emap[e] : e) * sigma_stride;
  const bool bad = (st[e].flags & (KNIT_P_SINGULAR | KNIT_P_NONFINITE)) != 0;
  const double qnan = __builtin_nan("");
  for (int64_t i = blockIdx.x * (int64_t)EW + threadIdx.x; i < (int64_t)M * M; i += (int64_t)gridDim.x * EW) {
    const Z v = s[(int64_t)(off + i / M) * ld + off + i % M];
    st_z(out + i, bad ? D{qnan, qnan} : D{to_d(v.re), to_d(v.im)});
  }
}

// Check of the surface block (offset off, leading dimension ld) against its
// defining equation: A = z - h - Sigma into ZA and the surface g into ZXA,
// both [M][M]; the product R = A g - I follows.
__global__ void __launch_bounds__(EW) dec_check_form_kernel(StripDev s, int ld, int off, const double *E,
                                                            const int *emap, double eta, char *ws, Slab sl, int sig,
                                                            int gsrc, const DecState *st, int check) {
  const int e = blockIdx.y, M = s.M;
  if (dec_skip(st, e, check)) return;
  const Z *S = reinterpret_cast<const Z *>(slab_ptr(ws, sl, e, sl.z[sig]));
  const Z *G = reinterpret_cast<const Z *>(slab_ptr(ws, sl, e, sl.z[gsrc]));
  Z *A = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZA]));
  Z *Gc = reinterpret_cast<Z *>(slab_ptr(ws, sl, e, sl.z[ZXA]));
  const double Ez = E[emap ? emap[e] : e];
  for (int64_t i = blockIdx.x * (int64_t)EW + threadIdx.x; i < (int64_t)M * M; i += (int64_t)gridDim.x * EW) {
    const int r = (int)(i / M), c = (int)(i % M);
    const int64_t o = (int64_t)(off + r) * ld + off + c;
    Z a = c_neg(c_add(zdd(ld_z(s.H0 + i)), S[o]));
    if (r == c) a = c_add(a, Z{dd{Ez, 0.0}, dd{eta, 0.0}});
    A[i] = a;
    Gc[i] = G[o];
  }
}

// max |R| (leading parts; NaN counts as +inf) of the check product in ZR.
__global__ void __launch_bounds__(EW) dec_resid_kernel(int M, char *ws, Slab sl, DecState *st, int check) {
  __shared__ double red[EW / 64];
  const int e = blockIdx.y;
  if (dec_skip(st, e, check)) return;
  const Z *R = reinterpret_cast<const Z *>(slab_ptr(ws, sl, e, sl.z[ZR]));
  double m = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)EW + threadIdx.x; i < (int64_t)M * M; i += (int64_t)gridDim.x * EW) {
    double a = fabs(R[i].re.hi) + fabs(R[i].im.hi);
    if (a != a) a = __builtin_inf();
    m = fmax(m, a);
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < EW / 64; ++w) m = fmax(m, red[w]);
    m = fmax(m, red[0]);
    atomicMax(&st[e].resid, (unsigned long long)__double_as_longlong(m));
  }
}

// A check above RESID_TOL (or non-finite) sets `bit`; the residual is cleared.
__global__ void dec_resid_decide_kernel(DecState *st, int n, int bit, int check) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n || dec_skip(st, e, check)) return;
  const double r = __longlong_as_double((long long)st[e].resid);
  if (!(r <= RESID_TOL)) st[e].flags |= bit;
  st[e].resid = 0ull;
}

// Retry slots: energies that failed the check, in slots [0, RETRY_SLOTS) up to
// the capacity (one thread, in energy order, so the assignment is
// reproducible); the rest, or all of them when `allow` is 0, have failed.
__global__ void dec_slot_assign_kernel(DecState *st, int nE, DecState *st2, int *emap, int allow) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int k = 0;
  for (int e = 0; e < nE; ++e) {
    if (!(st[e].flags & DEC_RETRY)) continue;
    if (allow && k < RETRY_SLOTS) emap[k++] = e;
    else st[e].flags |= DEC_FAILED;
  }
  for (int j = 0; j < RETRY_SLOTS; ++j) {
    if (j >= k) emap[j] = -1;
    const int e = emap[j];
    st2[j] = e >= 0 ? DecState{0, 0, 0, 0, 0ull, st[e].scale, 0ull} : DecState{1, 0, 0, 1, 0ull, 0ull, 0ull};
  }
}

// Results of the retry slots into the energies' states.
__global__ void dec_slot_merge_kernel(DecState *st, const DecState *st2, const int *emap) {
  const int j = threadIdx.x;
  if (blockIdx.x != 0 || j >= RETRY_SLOTS) return;
  const int e = emap[j];
  if (e < 0) return;
  st[e].flags = (st2[j].flags & (DEC_PUBLIC | DEC_FAILED)) | DEC_RETRY;
  st[e].iters = st2[j].iters;
}

// NaN self-energies for the energies that failed the check for good.
__global__ void __launch_bounds__(EW) dec_poison_kernel(int M, int nE, int nsurf, knit_z *sigma, const DecState *st) {
  const int e = blockIdx.y;
  if (!(st[e].flags & DEC_FAILED)) return;
  const double qnan = __builtin_nan("");
  for (int sf = 0; sf < nsurf; ++sf) {
    knit_z *out = sigma + ((int64_t)sf * nE + e) * M * M;
    for (int64_t i = blockIdx.x * (int64_t)EW + threadIdx.x; i < (int64_t)M * M; i += (int64_t)gridDim.x * EW)
      st_z(out + i, D{qnan, qnan});
  }
}

__global__ void dec_status_kernel(const DecState *st, int nE, int max_iter, int32_t *pstatus, int32_t *iters) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nE) return;
  pstatus[e] = (st[e].flags & DEC_PUBLIC) | ((st[e].flags & DEC_FAILED) ? KNIT_P_NOCONV : 0);
  if (iters) iters[e] = st[e].iters < max_iter ? st[e].iters : max_iter;
}

// ---------------------------------------------------------------- products on the INT8 matrix cores
//
// A double-double (or FP64) complex product C = A B taken exactly enough for
// double-double by splitting both operands into signed 7-bit digits and
// multiplying the digit planes on the INT8 matrix cores
// (v_mfma_i32_16x16x64_i8, exact int32 sums), the splitting scheme of Ozaki
// and co-workers with integer slices:
//   * every row r of A (every column c of B) is scaled by a power of two 2^-e
//     so that its largest |re|, |im| is below 1;
//   * a scaled value v is written as sum_i d_i 2^-(6 + 7 i), i < S, with
//     balanced digits |d_i| <= 64 (d_i = rint of the remainder times
//     2^(6 + 7 i); each remainder is exact in double-double);
//   * digit planes multiply exactly: |sum_k a_i b_j| <= 64^2 K, and the sums
//     of one weight 2^-(12 + 7 d), d = i + j, stay below 2^31 for K <= 1024;
//   * pairs with i + j >= S are dropped (their weight is below 2^-(12 + 7 S)
//     of the row and column scales), so S = 16 digits carry 112 bits, enough
//     for a double-double result (15 digits measured 1e-31 of the scales on
//     random operands, too close to double-double's 2^-106 for the 60
//     doubling steps);
//   * Re C = sum_d (P_d - Q_d) 2^-(12+7d), Im C = sum_d R_d 2^-(12+7d) with
//     P = ar br, Q = ai bi, R = ar bi + ai br, summed in double-double from
//     the smallest weight, times 2^(e_r + e_c).
// Planes are stored zero-padded to [Mr][Mk] (rows to 32, k to 64): A as
// [2S][Mr][Mk] (digit i of re at plane 2i, of im at 2i + 1), B transposed,
// [2S][Mc][Mk] with the column index first.

constexpr int OZ_S = 16;        // digits of a double-double operand
constexpr int OZ_S64 = 8;       // digits of an FP64 operand (56 bits)
constexpr int OZ_BAD = -100000; // exponent of a line holding a non-finite value

typedef int oz_v4i __attribute__((ext_vector_type(4)));

__host__ __device__ inline int oz_rows(int M) { return (M + 31) / 32 * 32; }
__host__ __device__ inline int oz_kpad(int M) { return (M + 63) / 64 * 64; }
__host__ __device__ inline size_t oz_plane_bytes(int M) { return (size_t)oz_rows(M) * oz_kpad(M); }

__device__ __forceinline__ double oz_hi(dd v) { return v.hi; }
__device__ __forceinline__ double oz_hi(double v) { return v; }
__device__ __forceinline__ dd oz_dd(dd v) { return v; }
__device__ __forceinline__ dd oz_dd(double v) { return dd{v, 0.0}; }

// Exponent of every row (COLS = false) or column (COLS = true) of X [M][M]
// (complex, element type T = cpx<dd> or cpx<double>), per energy: the
// smallest e with max |re|, |im| of the line below 2^e.  Rows: one wave per
// row, lanes along the row; columns: 64 columns per workgroup, four row
// groups reduced in LDS.  Reads are coalesced either way.
template <class T, bool COLS>
__global__ void __launch_bounds__(256) oz_exp_kernel(const T *X, int64_t stride_bytes, int M, int32_t *exps,
                                                     int64_t exp_stride, const DecState *st, int check) {
  __shared__ double sm[4][64];
  __shared__ int sf[4][64];
  const int e = blockIdx.y;
  if (dec_skip(st, e, check)) return;
  const T *Xe = reinterpret_cast<const T *>(reinterpret_cast<const char *>(X) + (int64_t)e * stride_bytes);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double m = 0.0;
  int fin = 1;
  int line;
  if (!COLS) {
    line = blockIdx.x * 4 + wv;
    if (line < M)
      for (int t = lane; t < M; t += 64) {
        const T v = Xe[(int64_t)line * M + t];
        m = fmax(m, fmax(fabs(oz_hi(v.re)), fabs(oz_hi(v.im))));
        fin &= isfinite(oz_hi(v.re)) && isfinite(oz_hi(v.im));
      }
    for (int off = 32; off > 0; off >>= 1) {
      m = fmax(m, __shfl_xor(m, off, 64));
      fin &= __shfl_xor(fin, off, 64);
    }
    if (lane == 0 && line < M) exps[(int64_t)e * exp_stride + line] = !fin ? OZ_BAD : (m > 0.0 ? ilogb(m) + 1 : 0);
  } else {
    line = blockIdx.x * 64 + lane;
    if (line < M)
      for (int t = wv; t < M; t += 4) {
        const T v = Xe[(int64_t)t * M + line];
        m = fmax(m, fmax(fabs(oz_hi(v.re)), fabs(oz_hi(v.im))));
        fin &= isfinite(oz_hi(v.re)) && isfinite(oz_hi(v.im));
      }
    sm[wv][lane] = m;
    sf[wv][lane] = fin;
    __syncthreads();
    if (wv == 0 && line < M) {
      for (int g = 1; g < 4; ++g) {
        m = fmax(m, sm[g][lane]);
        fin &= sf[g][lane];
      }
      exps[(int64_t)e * exp_stride + line] = !fin ? OZ_BAD : (m > 0.0 ? ilogb(m) + 1 : 0);
    }
  }
}

// Digit planes of X (rows scaled, or transposed with columns scaled), S digits.
template <class T, bool COLS>
__global__ void __launch_bounds__(EW) oz_digit_kernel(const T *X, int64_t stride_bytes, int M, int S,
                                                      const int32_t *exps, int64_t exp_stride, int8_t *planes,
                                                      int64_t plane_stride, const DecState *st, int check) {
  const int e = blockIdx.y;
  if (dec_skip(st, e, check)) return;
  const T *Xe = reinterpret_cast<const T *>(reinterpret_cast<const char *>(X) + (int64_t)e * stride_bytes);
  const int Mr = oz_rows(M), Mk = oz_kpad(M);
  const int64_t pb = (int64_t)Mr * Mk;
  int8_t *Pe = planes + (int64_t)e * plane_stride;
  for (int64_t idx = blockIdx.x * (int64_t)EW + threadIdx.x; idx < pb; idx += (int64_t)gridDim.x * EW) {
    const int line = (int)(idx / Mk), k = (int)(idx % Mk);   // line: row of A, or column of B
    dd vr{0.0, 0.0}, vi{0.0, 0.0};
    if (line < M && k < M) {
      const T v = COLS ? Xe[(int64_t)k * M + line] : Xe[(int64_t)line * M + k];
      const int ex = exps[(int64_t)e * exp_stride + line];
      const int sc = ex == OZ_BAD ? 0 : -ex;
      const dd r = oz_dd(v.re), im = oz_dd(v.im);
      vr = dd{ldexp(r.hi, sc), ldexp(r.lo, sc)};
      vi = dd{ldexp(im.hi, sc), ldexp(im.lo, sc)};
      if (ex == OZ_BAD) vr = vi = dd{0.0, 0.0};
    }
    for (int i = 0; i < S; ++i) {
      const double w = ldexp(1.0, 6 + 7 * i);
      const double dr = rint(vr.hi * w), di = rint(vi.hi * w);
      vr = two_sum((vr.hi * w - dr) / w, vr.lo);   // exact: x - rint(x), power-of-two scaling
      vi = two_sum((vi.hi * w - di) / w, vi.lo);
      Pe[(2 * i) * pb + idx] = (int8_t)(int)dr;
      Pe[(2 * i + 1) * pb + idx] = (int8_t)(int)di;
    }
  }
}

// C_e = cI I + (+/-) A_e B_e from the digit planes (SA digits of A, SB of B,
// pairs with i + j < OZ_S).  Workgroup: a 32 x 32 tile of C, four waves of
// 16 x 16; the B digits of a k-block sit in registers, the A digits come from
// LDS one digit at a time.
template <int SA, int SB>
__global__ void __launch_bounds__(256) oz_gemm_kernel(const int8_t *Ap, const int32_t *ea, const int8_t *Bp,
                                                      const int32_t *eb, int64_t plane_stride, int64_t exp_stride,
                                                      Z *C, int64_t c_stride_bytes, int M, double cI, int negate,
                                                      const DecState *st, int check) {
  __shared__ __attribute__((aligned(16))) int8_t As[2 * SA][32][64];
  __shared__ __attribute__((aligned(16))) int8_t Bs[2 * SB][32][64];
  const int e = blockIdx.y;
  if (dec_skip(st, e, check)) return;
  const int Mr = oz_rows(M), Mk = oz_kpad(M);
  const int64_t pb = (int64_t)Mr * Mk;
  const int tiles_n = Mr / 32;
  const int tile = blockIdx.x;
  const int r0 = (tile / tiles_n) * 32, c0 = (tile % tiles_n) * 32;
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  const int8_t *Ae = Ap + (int64_t)e * plane_stride, *Be = Bp + (int64_t)e * plane_stride;
  oz_v4i P[OZ_S], Q[OZ_S], R[OZ_S];
#pragma unroll
  for (int d = 0; d < OZ_S; ++d) P[d] = Q[d] = R[d] = oz_v4i{0, 0, 0, 0};
  for (int k0 = 0; k0 < Mk; k0 += 64) {
    // stage the k-block: 16 bytes per load, rows of 64 bytes
    for (int q = tid; q < 2 * SA * 32 * 4; q += 256) {
      const int p = q / 128, rr = (q / 4) % 32, part = q % 4;
      *reinterpret_cast<oz_v4i *>(&As[p][rr][16 * part]) =
          *reinterpret_cast<const oz_v4i *>(Ae + p * pb + (int64_t)(r0 + rr) * Mk + k0 + 16 * part);
    }
    for (int q = tid; q < 2 * SB * 32 * 4; q += 256) {
      const int p = q / 128, cc = (q / 4) % 32, part = q % 4;
      *reinterpret_cast<oz_v4i *>(&Bs[p][cc][16 * part]) =
          *reinterpret_cast<const oz_v4i *>(Be + p * pb + (int64_t)(c0 + cc) * Mk + k0 + 16 * part);
    }
    __syncthreads();
    oz_v4i br[SB], bi[SB];
#pragma unroll
    for (int j = 0; j < SB; ++j) {
      br[j] = *reinterpret_cast<const oz_v4i *>(&Bs[2 * j][16 * wc + (l & 15)][16 * (l >> 4)]);
      bi[j] = *reinterpret_cast<const oz_v4i *>(&Bs[2 * j + 1][16 * wc + (l & 15)][16 * (l >> 4)]);
    }
#pragma unroll
    for (int i = 0; i < SA; ++i) {
      const oz_v4i ar = *reinterpret_cast<const oz_v4i *>(&As[2 * i][16 * wr + (l & 15)][16 * (l >> 4)]);
      const oz_v4i ai = *reinterpret_cast<const oz_v4i *>(&As[2 * i + 1][16 * wr + (l & 15)][16 * (l >> 4)]);
#pragma unroll
      for (int j = 0; j < SB; ++j) {
        if (i + j >= OZ_S) continue;
        P[i + j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ar, br[j], P[i + j], 0, 0, 0);
        Q[i + j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ai, bi[j], Q[i + j], 0, 0, 0);
        R[i + j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ar, bi[j], R[i + j], 0, 0, 0);
        R[i + j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ai, br[j], R[i + j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // lane l holds rows 4 (l / 16) + q, column l % 16 of the wave's tile
  Z *Ce = reinterpret_cast<Z *>(reinterpret_cast<char *>(C) + (int64_t)e * c_stride_bytes);
  const int c = c0 + 16 * wc + (l & 15);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + 16 * wr + 4 * (l >> 4) + q;
    dd re{0.0, 0.0}, im{0.0, 0.0};
#pragma unroll
    for (int d = OZ_S - 1; d >= 0; --d) {
      const double wgt = ldexp(1.0, -12 - 7 * d);
      re = r_add(re, dd{(double)((long long)P[d][q] - (long long)Q[d][q]) * wgt, 0.0});
      im = r_add(im, dd{(double)R[d][q] * wgt, 0.0});
    }
    if (r >= M || c >= M) continue;
    const int er = ea[(int64_t)e * exp_stride + r], ec = eb[(int64_t)e * exp_stride + c];
    Z v;
    if (er == OZ_BAD || ec == OZ_BAD) {
      const double qn = __builtin_nan("");
      v = Z{dd{qn, 0.0}, dd{qn, 0.0}};
    } else {
      const int sc = er + ec;
      v = Z{dd{ldexp(re.hi, sc), ldexp(re.lo, sc)}, dd{ldexp(im.hi, sc), ldexp(im.lo, sc)}};
    }
    if (negate) v = c_neg(v);
    if (cI != 0.0 && r == c) v.re = r_add(v.re, dd{cI, 0.0});
    Ce[(int64_t)r * M + c] = v;
  }
}

#pragma clang fp contract(fast)

// Host-side launch helpers.
struct Ctx {
  StripDev s;
  int M, Mp, nE;
  Slab sl;
  char *ws;
  DecState *st;
  const int *emap;     // slot -> energy (retry pass), or NULL
  int gx_cap;          // GEMM grid x cap (tiles are strided over it), 0 = one block per tile
  hipStream_t stream;
  int oz;              // double-double products on the INT8 matrix cores (else the vector units)
  Z *zb(int i) const { return reinterpret_cast<Z *>(ws + sl.z[i]); }
  int gx(int m) const {
    const int tiles = ((m + GT - 1) / GT) * ((m + GT - 1) / GT);
    return gx_cap > 0 && tiles > gx_cap ? gx_cap : tiles;
  }
};

// Double-double products on the INT8 matrix cores (digit planes) when enabled,
// else on the vector units (process-wide; knit_set_selfenergy_products).
// Off by default: on the slice dimension 512 spinful lead the doubling
// diverged at 2 of 64 energies with the digit-plane products (their
// accuracy is relative to each row's and column's largest entry), and the
// step was only 1.18x faster.
std::atomic<int> g_int8_products{0};

// C = cI I +/- A B with A [M][M] double-double (buffer a) and B double-double
// (buffer b) or FP64 (the inverse X0, b < 0), on the INT8 matrix cores.
template <class TB>
hipError_t gemm_oz(const Ctx &c, int a, const TB *Bsrc, int out, double cI, int neg, int check) {
  const int M = c.M, Mr = oz_rows(M);
  const int64_t st = (int64_t)c.sl.bytes;
  int8_t *Ap = reinterpret_cast<int8_t *>(c.ws + c.sl.oz_a), *Bp = reinterpret_cast<int8_t *>(c.ws + c.sl.oz_b);
  int32_t *ea = reinterpret_cast<int32_t *>(c.ws + c.sl.oz_ea), *eb = reinterpret_cast<int32_t *>(c.ws + c.sl.oz_eb);
  const int64_t es = st / (int64_t)sizeof(int32_t);
  constexpr bool B64 = sizeof(TB) == sizeof(D);
  const int SB = B64 ? OZ_S64 : OZ_S;
  const int gd = (int)((oz_plane_bytes(M) + EW - 1) / EW);
  hipLaunchKernelGGL((oz_exp_kernel<Z, false>), dim3((M + 3) / 4, c.nE), dim3(256), 0, c.stream, c.zb(a), st, M, ea,
                     es, c.st, check);
  hipLaunchKernelGGL((oz_exp_kernel<TB, true>), dim3((M + 63) / 64, c.nE), dim3(256), 0, c.stream, Bsrc, st, M, eb,
                     es, c.st, check);
  hipLaunchKernelGGL((oz_digit_kernel<Z, false>), dim3(gd, c.nE), dim3(EW), 0, c.stream, c.zb(a), st, M, OZ_S, ea,
                     es, Ap, st, c.st, check);
  hipLaunchKernelGGL((oz_digit_kernel<TB, true>), dim3(gd, c.nE), dim3(EW), 0, c.stream, Bsrc, st, M, SB, eb, es,
                     Bp, st, c.st, check);
  const int tiles = (Mr / 32) * (Mr / 32);
  if (B64)
    hipLaunchKernelGGL((oz_gemm_kernel<OZ_S, OZ_S64>), dim3(tiles, c.nE), dim3(256), 0, c.stream, Ap, ea, Bp, eb, st,
                       es, c.zb(out), st, M, cI, neg, c.st, check);
  else
    hipLaunchKernelGGL((oz_gemm_kernel<OZ_S, OZ_S>), dim3(tiles, c.nE), dim3(256), 0, c.stream, Ap, ea, Bp, eb, st, es,
                       c.zb(out), st, M, cI, neg, c.st, check);
  return hipGetLastError();
}

hipError_t gemm_zz(const Ctx &c, int a, int b, int out, double cI = 0.0, int neg = 0, int check = 1) {
  if (c.oz) return gemm_oz<Z>(c, a, c.zb(b), out, cI, neg, check);
  hipLaunchKernelGGL((dd_gemm_kernel<Z, Z>), dim3(c.gx(c.M), c.nE), dim3(GTHREADS), 0, c.stream, c.zb(a), c.zb(b),
                     (const Z *)nullptr, c.zb(out), (int64_t)c.sl.bytes, c.M, cI, neg, c.st, check);
  return hipGetLastError();
}

// Newton corrections out = X + X R on the matrix cores, X the FP64 inverse X0
// (x0 = true) or the double-double buffer x
hipError_t newton_corr(const Ctx &c, bool x0, int x, int r, int out, int check) {
  const int tn = (c.M + 31) / 32;
  if (x0)
    hipLaunchKernelGGL((newton_corr_kernel<D>), dim3(tn * tn, c.nE), dim3(64), 0, c.stream,
                       reinterpret_cast<const D *>(c.ws + c.sl.xi64), c.zb(r), c.zb(out), (int64_t)c.sl.bytes, c.M,
                       c.st, check);
  else
    hipLaunchKernelGGL((newton_corr_kernel<Z>), dim3(tn * tn, c.nE), dim3(64), 0, c.stream, c.zb(x), c.zb(r),
                       c.zb(out), (int64_t)c.sl.bytes, c.M, c.st, check);
  return hipGetLastError();
}

// products with the FP64 inverse X0 as the right factor
hipError_t gemm_zd(const Ctx &c, int a, int out, double cI, int neg, int check) {
  const D *X = reinterpret_cast<const D *>(c.ws + c.sl.xi64);
  if (c.oz) return gemm_oz<D>(c, a, X, out, cI, neg, check);
  hipLaunchKernelGGL((dd_gemm_kernel<Z, D>), dim3(c.gx(c.M), c.nE), dim3(GTHREADS), 0, c.stream, c.zb(a), X,
                     (const Z *)nullptr, c.zb(out), (int64_t)c.sl.bytes, c.M, cI, neg, c.st, check);
  return hipGetLastError();
}

// g = (z - es)^{-1} into ZXB: FP64 matrix-core inverse X0, then two Newton
// steps X <- X + X R with the residual R = I - A X in double-double and the
// correction X R on the matrix cores.
hipError_t inverse_dd(const Ctx &c, const double *E, double eta, int src, int check) {
  hipError_t err;
  hipLaunchKernelGGL(dec_form_kernel, dim3(EW_BLOCKS, c.nE), dim3(EW), 0, c.stream, c.M, c.Mp, E, c.emap, eta, c.ws,
                     c.sl, src, c.st, check);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  const int64_t dstride = (int64_t)(c.sl.bytes / sizeof(D));
  const int sst = (int)(sizeof(DecState) / sizeof(int32_t));
  err = launch_inverse_fp64(reinterpret_cast<D *>(c.ws + c.sl.x64), dstride,
                            reinterpret_cast<D *>(c.ws + c.sl.scr), dstride, c.M,
                            reinterpret_cast<D *>(c.ws + c.sl.xi64), dstride,
                            check == 1 ? &c.st->done : (check == 2 ? &c.st->skip : nullptr), sst,
                            &c.st->flags, sst, c.nE, c.stream);
  if (err != hipSuccess) return err;
  if ((err = gemm_zd(c, ZA, ZR, 1.0, 1, check)) != hipSuccess) return err;        // R  = I - A X0
  if ((err = newton_corr(c, true, 0, ZR, ZXA, check)) != hipSuccess) return err;  // XA = X0 + X0 R
  if ((err = gemm_zz(c, ZA, ZXA, ZR, 1.0, 1, check)) != hipSuccess) return err;   // R  = I - A XA
  return newton_corr(c, false, ZXA, ZR, ZXB, check);                             // XB = XA + XA R
}

}  // namespace

// Workspace: per-energy states, the retry slots' states and energy map, then
// the slabs (the retry pass reuses the slab region after the first pass).
static size_t head_bytes(int nE) { return (((size_t)nE * sizeof(DecState)) + 255) & ~size_t(255); }
static size_t slot_bytes() {
  return (((size_t)RETRY_SLOTS * (sizeof(DecState) + sizeof(int))) + 255) & ~size_t(255);
}
static bool retry_fits(int M) { return mfma_padded(2 * M) <= 512; }

size_t decimation_workspace(int M, int nE) {
  size_t slabs = (size_t)nE * slab_of(M).bytes;
  if (retry_fits(M)) {
    const size_t r = (size_t)RETRY_SLOTS * slab_of(2 * M).bytes;
    if (r > slabs) slabs = r;
  }
  return head_bytes(nE) + slot_bytes() + slabs;
}

namespace {

// The doubling on context c (every energy, or the retry slots): max_iter
// steps queued without waiting; converged energies skip the rest.
hipError_t run_doubling(const Ctx &c, const double *E, double eta, double tol, int max_iter, int both) {
  hipError_t err;
  for (int it = 0; it < max_iter; ++it) {
    const int a = (it & 1) ? ZA1 : ZA0, b = (it & 1) ? ZB1 : ZB0;
    const int an = (it & 1) ? ZA0 : ZA1, bn = (it & 1) ? ZB0 : ZB1;
    if ((err = inverse_dd(c, E, eta, ZEPS, 1)) != hipSuccess) return err;   // g_k in ZXB
    if ((err = gemm_zz(c, ZXB, a, ZGA)) != hipSuccess) return err;          // g a
    if ((err = gemm_zz(c, ZXB, b, ZGB)) != hipSuccess) return err;          // g b
    if ((err = gemm_zz(c, a, ZGB, ZT1)) != hipSuccess) return err;          // a g b
    if ((err = gemm_zz(c, b, ZGA, ZT2)) != hipSuccess) return err;          // b g a
    if ((err = gemm_zz(c, a, ZGA, an)) != hipSuccess) return err;           // a g a
    if ((err = gemm_zz(c, b, ZGB, bn)) != hipSuccess) return err;           // b g b
    hipLaunchKernelGGL(dec_update_kernel, dim3(EW_BLOCKS, c.nE), dim3(EW), 0, c.stream, c.M, c.ws, c.sl, an, bn,
                       both, c.st);
    hipLaunchKernelGGL(dec_decide_kernel, dim3((c.nE + 255) / 256), dim3(256), 0, c.stream, c.st, c.nE, tol,
                       max_iter);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  return hipSuccess;
}

// Surface Green functions, self-energies and their check, for every surface:
//   left (or the one requested): Sigma = Vf g Vb with g = (z - eps_s)^{-1}
//   side 2, right:               Sigma = Vb g Vf with g = (z - eps_r)^{-1}
// On the two-slice cell (cell = 1) the surface slice is the leading block
// (left) or the trailing block (right) of dimension M.  A failed check sets
// `bit` in the energy's (or slot's) flags.
hipError_t surfaces(const Ctx &c, const double *E, double eta, int both, int cell, int check, knit_z *sigma,
                    int nE_all, int bit) {
  hipError_t err;
  const int M = c.s.M;
  for (int surf = 0; surf < (both ? 2 : 1); ++surf) {
    const int off = cell && surf == 1 ? M : 0;
    if ((err = inverse_dd(c, E, eta, surf == 0 ? ZEPS_S : ZEPS_R, check)) != hipSuccess) return err;
    if ((err = gemm_zz(c, surf == 0 ? ZVF : ZVB, ZXB, ZT1, 0.0, 0, check)) != hipSuccess) return err;
    if ((err = gemm_zz(c, ZT1, surf == 0 ? ZVB : ZVF, ZT2, 0.0, 0, check)) != hipSuccess) return err;
    hipLaunchKernelGGL(dec_store_kernel, dim3(EW_BLOCKS, c.nE), dim3(EW), 0, c.stream, M, c.M, off, c.ws, c.sl,
                       (int)ZT2, sigma + (int64_t)surf * nE_all * M * M, (int64_t)M * M, c.st, c.emap, check);
    hipLaunchKernelGGL(dec_check_form_kernel, dim3(EW_BLOCKS, c.nE), dim3(EW), 0, c.stream, c.s, c.M, off, E, c.emap,
                       eta, c.ws, c.sl, (int)ZT2, (int)ZXB, c.st, check);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    // R = (z - h - Sigma) g - I, [M][M]
    Ctx cm = c;
    cm.M = M;
    if ((err = gemm_zz(cm, ZA, ZXA, ZR, -1.0, 0, check)) != hipSuccess) return err;
    hipLaunchKernelGGL(dec_resid_kernel, dim3(EW_BLOCKS, c.nE), dim3(EW), 0, c.stream, M, c.ws, c.sl, c.st, check);
    hipLaunchKernelGGL(dec_resid_decide_kernel, dim3((c.nE + 255) / 256), dim3(256), 0, c.stream, c.st, c.nE, bit,
                       check);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  return hipSuccess;
}

}  // namespace

void decimation_products_set(int int8) { g_int8_products.store(int8 ? 1 : 0); }
int decimation_products_get() { return g_int8_products.load(); }

hipError_t launch_decimation(const StripDev &s, int side, const double *E, int nE, double eta, double tol,
                             int max_iter, knit_z *sigma, int32_t *iters, int32_t *pstatus, void *ws,
                             hipStream_t stream) {
  if (nE <= 0) return hipSuccess;
  if (mfma_padded(s.M) > 512) return hipErrorInvalidValue;
  char *base = reinterpret_cast<char *>(ws);
  DecState *st = reinterpret_cast<DecState *>(base);
  DecState *st2 = reinterpret_cast<DecState *>(base + head_bytes(nE));
  int *emap = reinterpret_cast<int *>(st2 + RETRY_SLOTS);
  char *slabs = base + head_bytes(nE) + slot_bytes();
  const int both = side == 2;
  hipError_t err;
  // ---- every energy, cells of one slice
  // first pass: products on the INT8 matrix cores when enabled
  Ctx c{s, s.M, mfma_padded(s.M), nE, slab_of(s.M), slabs, st, nullptr, 0, stream, g_int8_products.load()};
  hipLaunchKernelGGL(dec_reset_state_kernel, dim3((nE + 255) / 256), dim3(256), 0, stream, st, nE);
  hipLaunchKernelGGL(dec_init_kernel, dim3(EW_BLOCKS, nE), dim3(EW), 0, stream, s, side, c.ws, c.sl, c.st);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if ((err = run_doubling(c, E, eta, tol, max_iter, both)) != hipSuccess) return err;
  if ((err = surfaces(c, E, eta, both, 0, 0, sigma, nE, DEC_RETRY)) != hipSuccess) return err;
  // ---- energies that failed the check: cells of two slices, in the retry slots
  const bool fits = retry_fits(s.M);
  hipLaunchKernelGGL(dec_slot_assign_kernel, dim3(1), dim3(1), 0, stream, st, nE, st2, emap, fits ? 1 : 0);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if (fits) {
    // retry pass (energies at slice eigenvalues, where the decimated couplings
    // carry parts of size 1/eta beside small ones): double-double products on
    // the vector units, accurate element by element rather than relative to
    // each row's and column's largest entry
    Ctx c2{s, 2 * s.M, mfma_padded(2 * s.M), RETRY_SLOTS, slab_of(2 * s.M), slabs, st2, emap, 64, stream, 0};
    hipLaunchKernelGGL(dec_init2_kernel, dim3(EW_BLOCKS, RETRY_SLOTS), dim3(EW), 0, stream, s, side, c2.ws, c2.sl,
                       c2.st);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if ((err = run_doubling(c2, E, eta, tol, max_iter, both)) != hipSuccess) return err;
    if ((err = surfaces(c2, E, eta, both, 1, 2, sigma, nE, DEC_FAILED)) != hipSuccess) return err;
    hipLaunchKernelGGL(dec_slot_merge_kernel, dim3(1), dim3(64), 0, stream, st, st2, emap);
  }
  hipLaunchKernelGGL(dec_poison_kernel, dim3(EW_BLOCKS, nE), dim3(EW), 0, stream, s.M, nE, both ? 2 : 1, sigma, st);
  hipLaunchKernelGGL(dec_status_kernel, dim3((nE + 255) / 256), dim3(256), 0, stream, st, nE, max_iter, pstatus,
                     iters);
  return hipGetLastError();
}

}  // namespace knit
