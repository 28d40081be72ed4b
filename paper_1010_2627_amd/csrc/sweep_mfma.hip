// Slice recursive Green function sweep on the matrix cores.
//
// Same recursion as the generic sweep (basic recursive Green function
// algorithm, section 1): per slice the stacked matrix X = [A_n; -G_{1,n-1} V^+]
// is reduced by Gauss-Jordan elimination with partial pivoting among the rows
// of A_n, leaving g_n = A_n^{-1} on top and G_1n = G_{1,n-1} V^+ g_n below.
//
// Blocked elimination with panels of NB columns (16 in FP64, 32 in FP32), one workgroup
// (8 waves) per problem, persistent over the problems of the batch:
//   1. panel: the candidate rows [k0, Mp) of the 32 panel columns sit in
//      registers (one row per thread); 32 pivot steps, each a workgroup
//      argmax on |re|+|im| (lowest row on ties), a row swap (registers for
//      the panel, global memory for the other columns) and a rank-1 update
//      of the panel, so the panel ends holding T = (A_PK)^{-1} on its pivot
//      rows and the multipliers -A_rK T on the other candidate rows;
//   2. multipliers of the remaining rows: X[r, K] <- -X[r, K] T   (MFMA)
//   3. update: X[r, c] += X[r, K] X[P, c] for r outside P, c outside K (MFMA)
//   4. pivot rows: X[P, c] <- T X[P, c]                              (MFMA)
// Matrices are padded to Mp = 32 * ceil(M / 32) with an identity block.
//
// Precision modes:
//   FP64         elimination and state in FP64 (v_mfma_f64_16x16x4f64);
//   FP32         elimination and state in FP32 (v_mfma_f32_16x16x4f32);
//   FP32_REFINE  elimination in FP32; g_n and G_1n kept in FP64; per slice one
//                refinement step on the inverse: R = I - A_n X0 with A_n and
//                the product in FP64, then [g_n; G_1n] = [X0; G0] (I + R) with
//                the correction product in FP32.

#include "knit_internal.h"
#include "knit_mfma.h"
#include "knit_slice.h"

namespace knit {

namespace {

constexpr int NT2 = 512;   // threads per workgroup: one panel row per thread
constexpr int MPAD = 32;   // slice dimension padding
// panel width = wave tile edge: 16 for FP64 (a 32-wide FP64 panel row would not
// fit the register file next to the MFMA tiles), 32 for FP32
template <class RG> struct PanelW;
template <> struct PanelW<double> { static constexpr int NB = 16; };
template <> struct PanelW<float> { static constexpr int NB = 16; };

__device__ __forceinline__ void wg_argmax8(double &v, int &i, double *sv, int *si) {
  for (int off = 32; off > 0; off >>= 1) {
    double v2 = __shfl_xor(v, off, 64);
    int i2 = __shfl_xor(i, off, 64);
    argmax_merge(v, i, v2, i2);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sv[w] = v;
    si[w] = i;
  }
  __syncthreads();
  v = sv[0];
  i = si[0];
  const int nw = blockDim.x >> 6;
  for (int k = 1; k < nw; ++k) argmax_merge(v, i, sv[k], si[k]);
  __syncthreads();
}

// Phase 1.  Requires Mp <= blockDim.x.  Returns status bits.  The pivot loop
// is not unrolled: register column j is picked with selects, which keeps the
// panel row (NB complex values) in registers without spilling.
template <class RG, int NB = PanelW<RG>::NB>
__device__ int gj_panel(cpx<RG> *X, int Mp, int k0, int *q, cpx<RG> *xchg, cpx<RG> *prow, double *sv,
                        int *si) {
  const int t = threadIdx.x, nt = blockDim.x;
  const bool cand = t >= k0 && t < Mp;
  cpx<RG> x[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) x[c] = cand ? X[(int64_t)t * Mp + k0 + c] : c_zero<RG>();
  int flags = 0;
#pragma unroll 1
  for (int j = 0; j < NB; ++j) {
    const int pj = k0 + j;
    cpx<RG> xj = x[0];
#pragma unroll
    for (int c = 1; c < NB; ++c)
      if (c == j) xj = x[c];
    double v = -1.0;
    int idx = 0x7fffffff;
    if (t >= pj && t < Mp) {
      v = c_abs1(xj);
      idx = t;
    }
    wg_argmax8(v, idx, sv, si);
    const int p = (idx >= pj && idx < Mp) ? idx : pj;
    if (!(v > 0.0)) flags |= (v == 0.0) ? KNIT_P_SINGULAR : KNIT_P_NONFINITE;
    if (!isfinite(v)) flags |= KNIT_P_NONFINITE;
    if (p != pj) {
      if (t == p)
#pragma unroll
        for (int c = 0; c < NB; ++c) xchg[c] = x[c];
      if (t == pj)
#pragma unroll
        for (int c = 0; c < NB; ++c) xchg[NB + c] = x[c];
      for (int c = t; c < Mp; c += nt) {
        if (c >= k0 && c < k0 + NB) continue;
        cpx<RG> a = X[(int64_t)pj * Mp + c], b = X[(int64_t)p * Mp + c];
        X[(int64_t)pj * Mp + c] = b;
        X[(int64_t)p * Mp + c] = a;
      }
      if (t == 0) {
        int s2 = q[pj];
        q[pj] = q[p];
        q[p] = s2;
      }
      __syncthreads();
      if (t == pj)
#pragma unroll
        for (int c = 0; c < NB; ++c) x[c] = xchg[c];
      if (t == p)
#pragma unroll
        for (int c = 0; c < NB; ++c) x[c] = xchg[NB + c];
      xj = x[0];
#pragma unroll
      for (int c = 1; c < NB; ++c)
        if (c == j) xj = x[c];
    }
    if (t == pj) {
      const cpx<RG> d = c_inv(xj);
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        x[c] = (c == j) ? d : c_mul(x[c], d);
        prow[c] = x[c];
      }
    }
    __syncthreads();
    if (cand && t != pj) {
      const cpx<RG> mdf = c_neg(xj);
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const cpx<RG> base = (c == j) ? c_zero<RG>() : x[c];
        x[c] = c_fma(mdf, prow[c], base);
      }
    }
  }
  if (cand)
#pragma unroll
    for (int c = 0; c < NB; ++c) X[(int64_t)t * Mp + k0 + c] = x[c];
  return flags;
}

// Phases 2-4 of one block step; R rows in X (Mp or 2 Mp).
template <class RG, int NB = PanelW<RG>::NB>
__device__ void gj_block_update(cpx<RG> *X, int Mp, int R, int k0) {
  constexpr int NBLK = NB / 16;
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int pt = k0 / NB, ntr = R / NB, ntc = Mp / NB;
  const cpx<RG> *T = X + (int64_t)k0 * Mp + k0;         // pivot block, ld Mp
  // 2. multipliers of the rows that were not candidates: [0, k0) and [Mp, R)
  {
    const int n_above = pt, n_below = (R - Mp) / NB;
    for (int i = wave; i < n_above + n_below; i += nwaves) {
      const int rt = i < n_above ? i : (Mp / NB) + (i - n_above);
      CTile<RG, NBLK> acc;
      acc.zero();
      ctile_gemm<RG, NBLK>(acc, X + k0, Mp, rt * NB, T, Mp, 0, NB);
      ctile_for_each<RG, NBLK>(acc, [&](int r, int c, RG &re, RG &im) {
        X[(int64_t)(rt * NB + r) * Mp + k0 + c] = cpx<RG>{-re, -im};
      });
    }
  }
  __syncthreads();
  // 3. rank-NB update of everything outside pivot rows / panel columns
  {
    const int ntiles = (ntr - 1) * (ntc - 1);
    for (int i = wave; i < ntiles; i += nwaves) {
      int rt = i / (ntc - 1), ct = i % (ntc - 1);
      rt += (rt >= pt);
      ct += (ct >= pt);
      CTile<RG, NBLK> acc;
      cpx<RG> *C = X + (int64_t)rt * NB * Mp + ct * NB;
      ctile_for_each<RG, NBLK>(acc, [&](int r, int c, RG &re, RG &im) {
        cpx<RG> v = C[(int64_t)r * Mp + c];
        re = v.re;
        im = v.im;
      });
      ctile_gemm<RG, NBLK>(acc, X + k0, Mp, rt * NB, X + (int64_t)k0 * Mp, Mp, ct * NB, NB);
      ctile_for_each<RG, NBLK>(acc, [&](int r, int c, RG &re, RG &im) { C[(int64_t)r * Mp + c] = cpx<RG>{re, im}; });
    }
  }
  __syncthreads();
  // 4. pivot rows: X[P, c] <- T X[P, c]
  {
    for (int i = wave; i < ntc - 1; i += nwaves) {
      const int ct = i + (i >= pt);
      CTile<RG, NBLK> acc;
      acc.zero();
      ctile_gemm<RG, NBLK>(acc, T, Mp, 0, X + (int64_t)k0 * Mp, Mp, ct * NB, NB);
      ctile_for_each<RG, NBLK>(acc, [&](int r, int c, RG &re, RG &im) {
        X[(int64_t)(k0 + r) * Mp + ct * NB + c] = cpx<RG>{re, im};
      });
    }
  }
  __syncthreads();
}

template <class RG, int NB = PanelW<RG>::NB>
__device__ int gj_blocked(cpx<RG> *X, int Mp, int R, int *q, cpx<RG> *xchg, cpx<RG> *prow, double *sv,
                          int *si) {
  for (int i = threadIdx.x; i < Mp; i += blockDim.x) q[i] = i;
  __syncthreads();
  int flags = 0;
  for (int k0 = 0; k0 < Mp; k0 += NB) {
    flags |= gj_panel<RG>(X, Mp, k0, q, xchg, prow, sv, si);
    __syncthreads();
    gj_block_update<RG>(X, Mp, R, k0);
  }
  return flags;
}

// A_n (and B_n) into X (type RG, padded), from g_{n-1}, G_{1,n-1} (type RS, natural order).
// With REFINE also writes A_n in FP64 to A64.
template <class RG, class RS, bool REFINE>
__device__ void form_padded(cpx<RG> *X, cpx<double> *A64, const StripDev &s, int Mp, double E,
                            const knit_z *D, const knit_z *sL, const knit_z *sR, bool first, bool last,
                            const cpx<RS> *g, const cpx<RS> *G1) {
  const int M = s.M, no = s.norb;
  const int64_t E2 = (int64_t)Mp * Mp;
  for (int64_t i = threadIdx.x; i < E2; i += blockDim.x) {
    const int a = (int)(i / Mp), b = (int)(i % Mp);
    cpx<double> v;
    if (a < M && b < M) {
      const int sa = a / no, oa = a % no, sb = b / no, ob = b % no;
      cpx<double> h = ld_z(s.H0 + (int64_t)a * M + b);
      if (sa == sb) {
        cpx<double> d = ld_z(D + ((int64_t)sa * no + oa) * no + ob);
        h.re += d.re;
        h.im += d.im;
      }
      if (first) {
        cpx<double> x = ld_z(sL + (int64_t)a * M + b);
        h.re += x.re;
        h.im += x.im;
      }
      if (last) {
        cpx<double> x = ld_z(sR + (int64_t)a * M + b);
        h.re += x.re;
        h.im += x.im;
      }
      v = {(a == b ? E : 0.0) - h.re, -h.im};
      if (!first) {
        const int ca = s.vcol[sa], cb = s.vcol[sb];
        if (ca >= 0 && cb >= 0) {
          cpx<double> acc = {0.0, 0.0};
          for (int ii = 0; ii < no; ++ii) {
            cpx<double> va = vblk_at(s, sa, oa, ii);
            cpx<double> inner = {0.0, 0.0};
            for (int jj = 0; jj < no; ++jj)
              inner = c_fma(cvt<double>(g[(int64_t)(ca * no + ii) * Mp + cb * no + jj]),
                            c_conj(vblk_at(s, sb, ob, jj)), inner);
            acc = c_fma(va, inner, acc);
          }
          v = c_sub(v, acc);
        }
      }
    } else {
      v = {a == b ? 1.0 : 0.0, 0.0};
    }
    X[i] = cvt<RG>(v);
    if (REFINE) A64[i] = v;
    if (!first) {
      cpx<double> w = {0.0, 0.0};
      if (a < M && b < M) {
        const int sb = b / no, ob = b % no, cb = s.vcol[sb];
        if (cb >= 0)
          for (int jj = 0; jj < no; ++jj)
            w = c_fma(cvt<double>(G1[(int64_t)a * Mp + cb * no + jj]), c_conj(vblk_at(s, sb, ob, jj)), w);
      }
      X[E2 + i] = cvt<RG>(cpx<double>{-w.re, -w.im});
    }
  }
}

template <class RS>
__device__ void gather_vg(cpx<RS> *Y, const cpx<RS> *Gm, const StripDev &s, int Mp) {
  // Y = V Gm (rows of Gm gathered through vcol), padded rows zero
  const int M = s.M, no = s.norb;
  const int64_t E2 = (int64_t)Mp * Mp;
  for (int64_t i = threadIdx.x; i < E2; i += blockDim.x) {
    const int a = (int)(i / Mp), b = (int)(i % Mp);
    cpx<double> acc = {0.0, 0.0};
    if (a < M && b < M) {
      const int sa = a / no, oa = a % no, ca = s.vcol[sa];
      if (ca >= 0)
        for (int ii = 0; ii < no; ++ii)
          acc = c_fma(vblk_at(s, sa, oa, ii), cvt<double>(Gm[(int64_t)(ca * no + ii) * Mp + b]), acc);
    }
    Y[i] = cvt<RS>(acc);
  }
}

__global__ void reset_queue_kernel(unsigned int *counter) { *counter = 0u; }

template <class RG, class RS, bool REFINE>
__global__ void __launch_bounds__(NT2) sweep_mfma_kernel(StripTable tab, const knit_problem *probs, int P,
                                                         const knit_z *onsite, const knit_z *sigmaL,
                                                         const knit_z *sigmaR, knit_z *G1N, knit_z *GN1,
                                                         knit_z *GNN, int32_t *pstatus, char *ws,
                                                         size_t slab_bytes, int Mpmax,
                                                         unsigned int *queue) {
  __shared__ int next_p;
  __shared__ int q[NT2];
  __shared__ int pinv[NT2];
  __shared__ double sv[16];
  __shared__ int si[16];
  __shared__ cpx<RG> xchg[2 * 32];
  __shared__ cpx<RG> prow[32];

  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t EE = (int64_t)Mpmax * Mpmax;
  char *slab = ws + (size_t)blockIdx.x * slab_bytes;
  cpx<RG> *X = reinterpret_cast<cpx<RG> *>(slab);                 // [2 Mp][Mp]
  cpx<RS> *g = reinterpret_cast<cpx<RS> *>(X + 2 * EE);           // [Mp][Mp]
  cpx<RS> *G1 = g + EE;                                           // [Mp][Mp]
  cpx<RS> *N1a = G1 + EE;                                         // [Mp][Mp]
  cpx<RS> *N1b = N1a + EE;                                        // [Mp][Mp]
  cpx<double> *A64 = reinterpret_cast<cpx<double> *>(N1b + EE);   // [Mp][Mp]   (REFINE)
  cpx<float> *Xn = reinterpret_cast<cpx<float> *>(A64 + (REFINE ? EE : 0));   // [2 Mp][Mp] (REFINE)
  cpx<float> *Rr = Xn + (REFINE ? 2 * EE : 0);                    // [Mp][Mp]   (REFINE)
  const bool want_n1 = GN1 != nullptr;
  const double qnan = __builtin_nan("");

  // problems are handed out by an atomic counter; every workgroup leaves the
  // loop once the counter has passed P
  for (;;) {
    if (tid == 0) next_p = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int p = next_p;
    __syncthreads();
    if (p >= P) break;
    const knit_problem pr = probs[p];
    const StripDev s = tab.s[pr.strip];
    const int M = s.M, no = s.norb, L = pr.L;
    const int Mp = (M + MPAD - 1) / MPAD * MPAD;
    const int64_t E2 = (int64_t)Mp * Mp;
    const knit_z *sL = sigmaL + pr.sigma_off, *sR = sigmaR + pr.sigma_off;
    int flags = 0;
    for (int n = 0; n < L; ++n) {
      const knit_z *D = onsite + pr.onsite_off + (int64_t)n * M * no;
      form_padded<RG, RS, REFINE>(X, A64, s, Mp, pr.E, D, sL, sR, n == 0, n == L - 1, g, G1);
      __syncthreads();
      const int R = n > 0 ? 2 * Mp : Mp;
      flags |= gj_blocked<RG>(X, Mp, R, q, xchg, prow, sv, si);
      for (int i = tid; i < Mp; i += nt) pinv[q[i]] = i;
      __syncthreads();
      if (!REFINE) {
        for (int64_t i = tid; i < (int64_t)R * Mp; i += nt) {
          const int a = (int)(i / Mp), b = (int)(i % Mp);
          cpx<RG> v = X[(int64_t)a * Mp + pinv[b]];
          if (a < Mp) g[i] = cvt<RS>(v);
          else G1[i - E2] = cvt<RS>(v);
        }
        __syncthreads();
      } else {
        // X0 (and G0) in natural column order
        for (int64_t i = tid; i < (int64_t)R * Mp; i += nt) {
          const int a = (int)(i / Mp), b = (int)(i % Mp);
          Xn[i] = cvt<float>(X[(int64_t)a * Mp + pinv[b]]);
        }
        __syncthreads();
        // residual R = I - A_n X0, FP64 product
        wg_gemm_mfma<double>(Mp, Mp, Mp, A64, Mp, Xn, Mp, [&](int r, int c, double &re, double &im) {
          Rr[(int64_t)r * Mp + c] = cpx<float>{(float)((r == c ? 1.0 : 0.0) - re), (float)(-im)};
        });
        __syncthreads();
        // [g; G1] = [X0; G0] + [X0; G0] R, correction in FP32
        wg_gemm_mfma<float>(R, Mp, Mp, Xn, Mp, Rr, Mp, [&](int r, int c, float &re, float &im) {
          const int64_t o = (int64_t)r * Mp + c;
          cpx<double> v = {(double)Xn[o].re + (double)re, (double)Xn[o].im + (double)im};
          if (r < Mp) g[o] = cvt<RS>(v);
          else G1[o - E2] = cvt<RS>(v);
        });
        __syncthreads();
      }
      if (n == 0) {
        for (int64_t i = tid; i < E2; i += nt) G1[i] = g[i];
        __syncthreads();
      }
      if (want_n1) {
        if (n == 0) {
          for (int64_t i = tid; i < E2; i += nt) N1a[i] = g[i];
        } else {
          gather_vg<RS>(N1b, N1a, s, Mp);
          __syncthreads();
          wg_gemm_mfma<RS>(Mp, Mp, Mp, g, Mp, N1b, Mp, [&](int r, int c, RS &re, RS &im) {
            N1a[(int64_t)r * Mp + c] = cpx<RS>{re, im};
          });
        }
        __syncthreads();
      }
    }
    // outputs (the leading M x M blocks)
    double bad = 0.0;
    const int64_t mm = (int64_t)M * M;
    for (int64_t i = tid; i < mm; i += nt) {
      const int a = (int)(i / M), b = (int)(i % M);
      const int64_t o = (int64_t)a * Mp + b;
      bad = fmax(bad, c_abs1(G1[o]));
      if (GNN) bad = fmax(bad, c_abs1(g[o]));
      if (want_n1) bad = fmax(bad, c_abs1(N1a[o]));
    }
    // workgroup max over 8 waves
    if (bad != bad) bad = INFINITY;
    for (int off = 32; off > 0; off >>= 1) bad = fmax(bad, __shfl_xor(bad, off, 64));
    if ((tid & 63) == 0) sv[tid >> 6] = bad;
    __syncthreads();
    bad = sv[0];
    for (int w = 1; w < (nt >> 6); ++w) bad = fmax(bad, sv[w]);
    __syncthreads();
    if (!isfinite(bad)) flags |= KNIT_P_NONFINITE;
    const bool kill = (flags & (KNIT_P_SINGULAR | KNIT_P_NONFINITE)) != 0;
    const cpx<double> nanz = {qnan, qnan};
    for (int64_t i = tid; i < mm; i += nt) {
      const int a = (int)(i / M), b = (int)(i % M);
      const int64_t o = (int64_t)a * Mp + b;
      st_z(G1N + pr.out_off + i, kill ? nanz : cvt<double>(G1[o]));
      if (GNN) st_z(GNN + pr.out_off + i, kill ? nanz : cvt<double>(g[o]));
      if (want_n1) st_z(GN1 + pr.out_off + i, kill ? nanz : cvt<double>(N1a[o]));
    }
    if (tid == 0) pstatus[p] = flags;
    __syncthreads();
  }
}

}  // namespace

int mfma_padded(int M) { return (M + MPAD - 1) / MPAD * MPAD; }

size_t sweep_mfma_slab_bytes(int Mmax, int precision) {
  const size_t Mp = (size_t)mfma_padded(Mmax);
  const size_t EE = Mp * Mp;
  size_t b;
  if (precision == KNIT_FP64) b = EE * (2 * 16 + 4 * 16);
  else if (precision == KNIT_FP32) b = EE * (2 * 8 + 4 * 8);
  else b = EE * (2 * 8 + 4 * 16 + 16 + 2 * 8 + 8);
  return (b + 255) & ~size_t(255);
}

bool sweep_mfma_supports(int Mmax) { return mfma_padded(Mmax) <= NT2; }

// Workspace: a 256-byte header (queue counter) then one slab per workgroup.
size_t sweep_mfma_workspace(int Mmax, int precision, int P) {
  const int grid = P < SWEEP_MAX_GRID ? P : SWEEP_MAX_GRID;
  return 256 + sweep_mfma_slab_bytes(Mmax, precision) * (size_t)grid;
}

hipError_t launch_sweep_mfma(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                             const knit_z *sigmaL, const knit_z *sigmaR, int precision, knit_z *G1N,
                             knit_z *GN1, knit_z *GNN, int32_t *pstatus, void *ws, int Mmax,
                             hipStream_t stream) {
  unsigned int *queue = reinterpret_cast<unsigned int *>(ws);
  char *w = reinterpret_cast<char *>(ws) + 256;
  const size_t slab = sweep_mfma_slab_bytes(Mmax, precision);
  const int Mpmax = mfma_padded(Mmax);
  // one resident workgroup per compute unit (8 waves of up to 256 VGPRs)
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  int grid = ncu < SWEEP_MAX_GRID ? ncu : SWEEP_MAX_GRID;
  if (grid > P) grid = P;
  hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(1), 0, stream, queue);
  if (precision == KNIT_FP64)
    hipLaunchKernelGGL((sweep_mfma_kernel<double, double, false>), dim3(grid), dim3(NT2), 0, stream, tab,
                       probs, P, onsite, sigmaL, sigmaR, G1N, GN1, GNN, pstatus, w, slab, Mpmax, queue);
  else if (precision == KNIT_FP32)
    hipLaunchKernelGGL((sweep_mfma_kernel<float, float, false>), dim3(grid), dim3(NT2), 0, stream, tab,
                       probs, P, onsite, sigmaL, sigmaR, G1N, GN1, GNN, pstatus, w, slab, Mpmax, queue);
  else
    hipLaunchKernelGGL((sweep_mfma_kernel<float, double, true>), dim3(grid), dim3(NT2), 0, stream, tab,
                       probs, P, onsite, sigmaL, sigmaR, G1N, GN1, GNN, pstatus, w, slab, Mpmax, queue);
  return hipGetLastError();
}

}  // namespace knit
