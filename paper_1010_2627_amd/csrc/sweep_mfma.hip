// Slice recursive Green function sweep on the matrix cores.
//
// Same recursion as the generic sweep (basic recursive Green function
// algorithm, section 1): per slice the stacked matrix X = [A_n; -G_{1,n-1} V^+]
// (2 Mp x Mp, Mp = M rounded up to 32, padded with an identity block) is
// reduced by Gauss-Jordan elimination with partial pivoting among the rows of
// A_n, leaving g_n = A_n^{-1} on top and G_1n = G_{1,n-1} V^+ g_n below.
//
// One workgroup per problem, persistent over a queue of problems (atomic
// counter over an order written by order_kernel, longest first by default).
// The elimination is blocked in two levels (gj_two_level):
//   * inner panels of 16 columns, factorised in registers (gj_panel): one
//     logical row per thread, pivot = largest |re|+|im| found by wavefront
//     reductions of a 32-bit key, rows never move in memory (a logical ->
//     physical row map in LDS is permuted instead);
//   * outer panels of 64 or 128 columns: the inner panels are applied to the
//     outer panel's columns only, then one rank-NO update (multipliers, new
//     pivot rows, and the update of everything else) touches the rest of the
//     matrix once per outer panel;
//   * every block product is a 32 x 32 (or 16 x 16) complex tile on MFMA
//     (tile_gemm_window_flat: 4 real products per complex product, operands
//     double-buffered in registers).
// Two elimination buffers alternate between slices: slice n+1 assembles
// A_{n+1} (form_blocks, one norb x norb site block per thread) directly from
// slice n's result through its row and column permutations.
//
// Precision modes:
//   FP64         elimination and state in FP64 (v_mfma_f64_16x16x4f64);
//   FP32         elimination and state in FP32 (v_mfma_f32_16x16x4f32);
//   FP32_REFINE  elimination of A_n alone in FP32 (X0 ~ A_n^{-1}); one
//                refinement step on the inverse: R = I - A_n X0 with A_n and
//                the product in FP64, g_n = X0 + X0 R (correction product in
//                FP32, sum in FP64); the propagator is then an FP64 product
//                of the refined inverse, G_1n = (G_{1,n-1} V^+) g_n (or
//                P_n = (P_{n-1} V^+) g_n), so nothing the recursion carries
//                from slice to slice is ever rounded to FP32.  A slice whose
//                largest |R| exceeds the refine threshold hands its problem
//                to a second, FP64 pass of the same call (KNIT_P_FALLBACK).
//
// The same machinery serves the batched FP64 inverse of the lead decimation
// (inverse_fp64_kernel) and the LDOS backward sweep (ldos_mfma_kernel).

#include <atomic>
#include <mutex>
#include <type_traits>

#include "knit_internal.h"
#include "knit_mfma.h"
#include "knit_slice.h"

namespace knit {

namespace {

constexpr int MPAD = 32;   // slice dimension padding
constexpr int NO_MAX = 128;  // widest outer panel (scratch is sized for it)
// inner panel width = wave tile edge of the inner phases
template <class RG> struct PanelW;
template <> struct PanelW<double> { static constexpr int NB = 16; };
template <> struct PanelW<float> { static constexpr int NB = 16; };

extern "C" __device__ unsigned int __ockl_wfred_max_u32(unsigned int);

// Workgroup argmax of a non-negative magnitude, lowest index on ties.  Each
// thread offers (v, idx) or v < 0 for "no candidate".  The key is the float
// bit pattern of v (monotonic for v >= 0) and the complement of idx, reduced
// by two 32-bit wavefront max-reductions and one LDS exchange across waves.
// key (double buffered by the caller: one barrier suffices) holds 2 words per wave.
__device__ __forceinline__ void wg_argmax_key(double v, int idx, unsigned int *key, float &vbest,
                                              int &ibest) {
  const bool valid = v >= 0.0 || v != v;
  const unsigned int hi = valid ? __float_as_uint((float)v) : 0u;
  const unsigned int whi = __ockl_wfred_max_u32(hi);
  const unsigned int lo = (valid && hi == whi) ? 0xffffffffu - (unsigned int)idx : 0u;
  const unsigned int wlo = __ockl_wfred_max_u32(lo);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    key[2 * w] = whi;
    key[2 * w + 1] = wlo;
  }
  __syncthreads();
  unsigned int bh = key[0], bl = key[1];
  const int nw = blockDim.x >> 6;
  for (int k = 1; k < nw; ++k) {
    const unsigned int h = key[2 * k], l2 = key[2 * k + 1];
    if (h > bh || (h == bh && l2 > bl)) {
      bh = h;
      bl = l2;
    }
  }
  vbest = bl ? __uint_as_float(bh) : -1.0f;
  ibest = bl ? (int)(0xffffffffu - bl) : 0x7fffffff;
}

// Workgroup maximum of a double, NaN if any thread holds NaN.  sv: one slot per
// wave; ends with a barrier, so sv is free again on return.
__device__ __forceinline__ double wg_max_nan(double v, double *sv) {
  double nanflag = (v != v) ? 1.0 : 0.0;
  double m = (v != v) ? 0.0 : v;
  for (int off = 32; off > 0; off >>= 1) {
    m = fmax(m, __shfl_xor(m, off, 64));
    nanflag = fmax(nanflag, __shfl_xor(nanflag, off, 64));
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sv[threadIdx.x >> 6] = nanflag > 0.0 ? -1.0 : m;
  __syncthreads();
  double r = 0.0;
  bool nan = false;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    const double x = sv[w];
    if (x < 0.0) nan = true;
    else r = fmax(r, x);
  }
  __syncthreads();
  return nan ? __builtin_nan("") : r;
}

// Columns of a factor C ([M][M] row-major, row stride M) up to its last
// column with a nonzero (or NaN) entry: the number of columns that take part
// in C C^+.  Called by the whole workgroup.
__device__ int factor_columns(const knit_z *C, int M, double *sv) {
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < (int64_t)M * M; i += blockDim.x) {
    const cpx<double> c = ld_z(C + i);
    if (c.re != 0.0 || c.im != 0.0) m = fmax(m, (double)(i % M + 1));
  }
  return (int)wg_max_nan(m, sv);
}

// Rows of X are addressed through a logical -> physical map: pivoting permutes
// the map (kept in LDS), never the rows in memory.  Rows >= Mp (the stacked
// propagator rows) are never permuted.
struct RowMap {
  const int *phys;
  int Mp;
  __device__ __forceinline__ int operator()(int r) const { return r < Mp ? phys[r] : r; }
};

// Phase 1: elimination restricted to the NB panel columns [k0, k0+NB) and the
// candidate rows [k0, Mp), one logical row per thread (requires Mp <=
// blockDim.x).  Pivot: largest |re|+|im| in the column among rows not yet
// used, lowest row on ties.  The pivot loop is not unrolled: register column
// j is picked with selects.  Returns status bits.
template <class RG, int NB = PanelW<RG>::NB>
__device__ int gj_panel(cpx<RG> *X, int Mp, int k0, int *phys, cpx<RG> *xchg, cpx<RG> *prow, double *sv,
                        int *si) {
  const int t = threadIdx.x;
  const bool cand = t >= k0 && t < Mp;
  const int64_t myrow = cand ? (int64_t)phys[t] * Mp : 0;
  cpx<RG> x[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) x[c] = cand ? X[myrow + k0 + c] : c_zero<RG>();
  int flags = 0;
#pragma unroll 1
  for (int j = 0; j < NB; ++j) {
    const int pj = k0 + j;
    cpx<RG> xj = x[0];
#pragma unroll
    for (int c = 1; c < NB; ++c)
      if (c == j) xj = x[c];
    float vb;
    int idx;
    wg_argmax_key((t >= pj && t < Mp) ? c_abs1(xj) : -1.0, t, reinterpret_cast<unsigned int *>(si) + (j & 1) * 32,
                  vb, idx);
    const int p = (idx >= pj && idx < Mp) ? idx : pj;
    if (!(vb > 0.0f)) flags |= (vb == 0.0f) ? KNIT_P_SINGULAR : KNIT_P_NONFINITE;
    if (!isfinite(vb)) flags |= KNIT_P_NONFINITE;
    // the pivot row (at position p) moves to position pj, scaled; the row at pj moves to p
    if (t == p) {
      const cpx<RG> d = c_inv(xj);
#pragma unroll
      for (int c = 0; c < NB; ++c) prow[c] = (c == j) ? d : c_mul(x[c], d);
    }
    if (t == pj && p != pj)
#pragma unroll
      for (int c = 0; c < NB; ++c) xchg[c] = x[c];
    if (t == 0 && p != pj) {
      const int s2 = phys[pj];
      phys[pj] = phys[p];
      phys[p] = s2;
    }
    __syncthreads();
    if (t == pj) {
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = prow[c];
    } else if (cand) {
      if (t == p)
#pragma unroll
        for (int c = 0; c < NB; ++c) x[c] = xchg[c];
      cpx<RG> f = x[0];
#pragma unroll
      for (int c = 1; c < NB; ++c)
        if (c == j) f = x[c];
      const cpx<RG> mf = c_neg(f);
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const cpx<RG> base = (c == j) ? c_zero<RG>() : x[c];
        x[c] = c_fma(mf, prow[c], base);
      }
    }
  }
  __syncthreads();   // phys is final for this panel
  if (cand) {
    const int64_t row = (int64_t)phys[t] * Mp;
#pragma unroll
    for (int c = 0; c < NB; ++c) X[row + k0 + c] = x[c];
  }
  return flags;
}

// Index map of a window of tiles: tile i starts at
//   base1 + step * i            for i < n1
//   base2 + step * (i - n1)     otherwise,
// shifted past [hole, hole + hole_len) when it would start inside or after it.
struct IdxMap {
  int base1, n1, base2, n, hole, hole_len;
  __device__ __forceinline__ int at(int i, int step) const {
    int r = i < n1 ? base1 + step * i : base2 + step * (i - n1);
    if (hole_len && r >= hole) r += hole_len;
    return r;
  }
};
__device__ __forceinline__ IdxMap imap(int base1, int n, int hole = 0, int hole_len = 0) {
  return IdxMap{base1, n, 0, n, hole, hole_len};
}
__device__ __forceinline__ IdxMap imap2(int base1, int n1, int base2, int n) {
  return IdxMap{base1, n1, base2, n, 0, 0};
}

// For every tile (r0 = rows.at(i), c0 = cols.at(j)) of the window:
//   out[r, c] = (negate ? -1 : 1) * sum_k X[arow + r, acol + k] X[krow0 + k, c + bshift]  (+ out if accumulate)
// with logical rows of X mapped through rm; out is X (rows mapped) or a plain
// scratch matrix S with leading dimension lds.  Out of line: one body serves
// every phase.
template <class RG, int NBLK, int KT, int NT>
__device__ __attribute__((noinline)) void tile_gemm_window_flat(
    const cpx<RG> *X, cpx<RG> *S, int lds, const int *phys, int Mp, int rb1, int rn1, int rb2, int rn, int rh,
    int rhl, int cb1, int cn1, int cb2, int cn, int ch, int chl, int K, int arow, int acol, int krow0,
    int bshift, int flags) {
  const RowMap rm{phys, Mp};
  const IdxMap rows{rb1, rn1, rb2, rn, rh, rhl}, cols{cb1, cn1, cb2, cn, ch, chl};
  const bool accumulate = flags & 1, negate = flags & 2;
  const int l = lane_id();
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int ntot = rows.n * cols.n;
  for (int it = wave; it < ntot; it += nwaves) {
    const int r0 = rows.at(it / cols.n, 16 * NBLK), c0 = cols.at(it % cols.n, 16 * NBLK);
    int64_t aoff[NBLK];
#pragma unroll
    for (int i = 0; i < NBLK; ++i) aoff[i] = (int64_t)rm(arow + r0 + 16 * i + (l & 15)) * Mp + acol + (l >> 4);
    cpx<RG> *Xw = const_cast<cpx<RG> *>(X);
    auto dst_of = [=](int r, int c) -> cpx<RG> * {
      return S ? S + (int64_t)(r0 + r) * lds + c0 + c : Xw + (int64_t)rm(r0 + r) * Mp + c0 + c;
    };
    CTile<RG, NBLK> acc;
    if (accumulate)
      ctile_for_each<RG, NBLK>(acc, [=](int r, int c, RG &re, RG &im) {
        const cpx<RG> v = *dst_of(r, c);
        re = v.re;
        im = v.im;
      });
    else
      acc.zero();
    // operands in double-buffered chunks of CH k-slices: the loads of chunk
    // c + 1 are in flight while the MFMAs of chunk c run.  KT > 0: K = KT,
    // fully unrolled; KT == 0: K is a runtime multiple of 8 CH, walked in
    // pairs of chunks so that both buffers keep static indices
    constexpr int CH = NBLK == 1 ? 4 : 2, NCH = KT / 4 / CH;
    cpx<RG> a[2][CH][NBLK], b[2][CH][NBLK];
    auto load = [&](int ch, int buf) {
#pragma unroll
      for (int q2 = 0; q2 < CH; ++q2) {
        const int ks = ch * CH + q2;
#pragma unroll
        for (int i = 0; i < NBLK; ++i) a[buf][q2][i] = X[aoff[i] + 4 * ks];
        const int64_t brow = (int64_t)rm(krow0 + 4 * ks + (l >> 4)) * Mp + c0 + bshift + (l & 15);
#pragma unroll
        for (int jb = 0; jb < NBLK; ++jb) b[buf][q2][jb] = X[brow + 16 * jb];
      }
    };
    load(0, 0);
    if constexpr (KT > 0) {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        if (ch + 1 < NCH) load(ch + 1, (ch + 1) & 1);
#pragma unroll
        for (int q2 = 0; q2 < CH; ++q2) ctile_mma<RG, NBLK>(acc, a[ch & 1][q2], b[ch & 1][q2]);
      }
    } else {
      const int nch = K / (4 * CH);   // even
#pragma unroll 1
      for (int ch = 0; ch < nch; ch += 2) {
        load(ch + 1, 1);
#pragma unroll
        for (int q2 = 0; q2 < CH; ++q2) ctile_mma<RG, NBLK>(acc, a[0][q2], b[0][q2]);
        if (ch + 2 < nch) load(ch + 2, 0);
#pragma unroll
        for (int q2 = 0; q2 < CH; ++q2) ctile_mma<RG, NBLK>(acc, a[1][q2], b[1][q2]);
      }
    }
    ctile_for_each<RG, NBLK>(acc, [=](int r, int c, RG &re, RG &im) {
      *dst_of(r, c) = negate ? cpx<RG>{-re, -im} : cpx<RG>{re, im};
    });
  }
}

// Block products of the outer update with 64 x 32 wave tiles, for the 64-row
// tiles rows.at(i, 64) and 32-column tiles cols.at(j, 32):
//   out[r, c] = (negate ? -1 : 1) * sum_k X[arow + r, acol + k] X[krow0 + k, c + bshift]  (+ out if accumulate)
// with out X (rows mapped) or the scratch S (leading dimension lds).  Twice the
// rows of tile_gemm_window's tiles: the operand every row tile re-reads (pivot
// rows, or the panel's own block) is read half as often.  K is a multiple of 32.
// The output target and sign are template parameters: each instance keeps
// its k-loop within the register budget.
template <class RG, int NT, bool TO_S, bool ACC, bool NEG>
__device__ __attribute__((noinline)) void tile_gemm_64x32(cpx<RG> *X, cpx<RG> *S, int lds, const int *phys, int Mp,
                                                          int rb1, int rn1, int rb2, int rn, int rh, int rhl, int cb1,
                                                          int cn, int ch, int chl, int K, int arow, int acol,
                                                          int krow0, int bshift) {
  constexpr int NBR = 4, NBC = 2;
  const RowMap rm{phys, Mp};
  const IdxMap rows{rb1, rn1, rb2, rn, rh, rhl}, cols{cb1, cn, 0, cn, ch, chl};
  const int l = lane_id();
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int ntot = rows.n * cols.n;
  for (int it = wave; it < ntot; it += nwaves) {
    const int r0 = rows.at(it / cols.n, 64), c0 = cols.at(it % cols.n, 32);
    int64_t aoff[NBR];
#pragma unroll
    for (int i = 0; i < NBR; ++i) aoff[i] = (int64_t)rm(arow + r0 + 16 * i + (l & 15)) * Mp + acol + (l >> 4);
    auto dst_of = [=](int r, int c) -> cpx<RG> * {
      if constexpr (TO_S) return S + (int64_t)(r0 + r) * lds + c0 + c;
      else return X + (int64_t)rm(r0 + r) * Mp + c0 + c;
    };
    CTileRC<RG, NBR, NBC> acc;
    ctile_for_each_rc<RG, NBR, NBC>(acc, [=](int r, int c, RG &re, RG &im) {
      if constexpr (ACC) {
        const cpx<RG> v = *dst_of(r, c);
        re = v.re;
        im = v.im;
      } else {
        re = RG(0);
        im = RG(0);
      }
    });
    // operands in chunks of two k-slices, double-buffered: the loads of chunk
    // c + 1 are in flight while the 64 products of chunk c run
    cpx<RG> a[2][2][NBR], b[2][2][NBC];
    auto load = [&](int ch, int buf) {
#pragma unroll
      for (int q2 = 0; q2 < 2; ++q2) {
        const int ks = 2 * ch + q2;
#pragma unroll
        for (int i = 0; i < NBR; ++i) a[buf][q2][i] = X[aoff[i] + 4 * ks];
        const int64_t brow = (int64_t)rm(krow0 + 4 * ks + (l >> 4)) * Mp + c0 + bshift + (l & 15);
#pragma unroll
        for (int j = 0; j < NBC; ++j) b[buf][q2][j] = X[brow + 16 * j];
      }
    };
    const int nch = K / 8;   // even
    load(0, 0);
#pragma unroll 1
    for (int ch = 0; ch < nch; ch += 2) {
      load(ch + 1, 1);
#pragma unroll
      for (int q2 = 0; q2 < 2; ++q2) ctile_mma_rc<RG, NBR, NBC>(acc, a[0][q2], b[0][q2]);
      if (ch + 2 < nch) load(ch + 2, 0);
#pragma unroll
      for (int q2 = 0; q2 < 2; ++q2) ctile_mma_rc<RG, NBR, NBC>(acc, a[1][q2], b[1][q2]);
    }
    ctile_for_each_rc<RG, NBR, NBC>(acc, [=](int r, int c, RG &re, RG &im) {
      *dst_of(r, c) = NEG ? cpx<RG>{-re, -im} : cpx<RG>{re, im};
    });
  }
}

// LDS staging of the FP64 block products below.  The workgroup's waves form
// WR x WC wave tiles of 64 x 32 (2 x 4 at 512 threads, 2 x 2 at 256), so one
// group of tiles covers AR = 128 rows and BC = 32 WC columns; a k-chunk holds
// KC slices of the group's A rows (AR x KC) and B columns (KC x BC).  Two
// buffers, each its own LDS object, so that the compiler can tell a read of
// one from a pending direct load into the other.
template <int NT, int WR_ = 2> struct UpdStage {
  static constexpr int NW = NT / 64, WR = WR_, WC = NW / WR;
  static constexpr int KC = NT == 512 ? 16 : 8;
  static constexpr int AR = 64 * WR, BC = 32 * WC;
  static constexpr int A_EL = AR * KC, B_EL = KC * BC;
};
// (at 256 threads the 1 x 4 shape, 64 rows by 128 columns, needs the same
// stage size as the 2 x 2 one: 64 x 8 + 8 x 128 = 128 x 8 + 8 x 64 elements)
static_assert(UpdStage<256, 1>::A_EL + UpdStage<256, 1>::B_EL == UpdStage<256>::A_EL + UpdStage<256>::B_EL, "");
template <int NT> __device__ __forceinline__ cpx<double> *upd_stage0() {
  __shared__ cpx<double> buf[UpdStage<NT>::A_EL + UpdStage<NT>::B_EL];
  return buf;
}
template <int NT> __device__ __forceinline__ cpx<double> *upd_stage1() {
  __shared__ cpx<double> buf[UpdStage<NT>::A_EL + UpdStage<NT>::B_EL];
  return buf;
}

// Position of A element (row, k) of a chunk in its stage buffer: rows of KC
// slots, the slot XOR-swizzled by the row so that the 16 rows one operand
// read touches fall on 16 different 16-byte bank groups.
template <int KC>
__device__ __forceinline__ int upd_a_slot(int row, int k) {
  return row * KC + (k ^ (KC == 16 ? (row & 15) : ((row >> 1) & 7)));
}

// Direct global -> LDS copy of 16 bytes per lane: lane i of the wave writes
// dst + 16 i (dst wave-uniform).
__device__ __forceinline__ void lds_copy16(const cpx<double> *src, cpx<double> *dst) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                   (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
}

// tile_gemm_64x32 in FP64 with the operands staged through LDS: the
// workgroup walks groups of WR x WC wave tiles; for each group the k-chunks
// of its A rows and B columns are copied by direct global -> LDS loads into
// one buffer while the waves multiply the chunk in the other.  Each wave
// reads its operands from LDS and takes every output element's k-terms in
// the same order as tile_gemm_64x32, so the results are bitwise the same.
// The A rows of a group are read once per group instead of once per wave
// tile, the B columns once per group instead of once per row tile.  Called
// by the whole workgroup; K a multiple of 32.  tail = 1: the last row tile
// has only its first 32 rows (the others are neither read nor written).
// A group reads all of its A rows and B columns before it writes any output,
// and no other group writes them: the output may overwrite the group's own
// A rows when the group spans every output column (WC tiles of 32 >= the
// columns), or its B columns when it spans every output row.
template <int NT, bool TO_S, bool ACC, bool NEG, int WR_ = 2>
__device__ __attribute__((noinline)) void tile_gemm_64x32_lds(cpx<double> *X, cpx<double> *S, int lds,
                                                              const int *phys, int Mp, int rb1, int rn1, int rb2,
                                                              int rn, int rh, int rhl, int cb1, int cn, int ch,
                                                              int chl, int K, int arow, int acol, int krow0,
                                                              int bshift, int tail) {
  using U = UpdStage<NT, WR_>;
  constexpr int KC = U::KC, AR = U::AR, BC = U::BC, WC = U::WC, NW = U::NW, WR = U::WR;
  constexpr int A_INS = U::A_EL / 64 / NW, B_INS = U::B_EL / 64 / NW;   // copies per wave per chunk
  constexpr int A_ROWS = 64 / KC;                                       // rows per A copy
  // the row map lives in LDS: read it as LDS (a generic load would also wait
  // for the direct loads in flight)
  const __attribute__((address_space(3))) int *pl = (const __attribute__((address_space(3))) int *)phys;
  auto rm = [=](int r) { return r < Mp ? pl[r] : r; };
  const IdxMap rows{rb1, rn1, rb2, rn, rh, rhl}, cols{cb1, cn, 0, cn, ch, chl};
  const int l = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wave / WC, wc = wave % WC;
  const int ngr = (rows.n + WR - 1) / WR, ngc = (cols.n + WC - 1) / WC;
  const int nch = K / KC;   // even
  cpx<double> *st0 = upd_stage0<NT>(), *st1 = upd_stage1<NT>();
  for (int g = 0; g < ngr * ngc; ++g) {
    const int gr = g / ngc, gc = g % ngc;
    const int ti = WR * gr + wr, tj = WC * gc + wc;
    const bool mine = ti < rows.n && tj < cols.n;
    const int vrows = (tail && ti == rows.n - 1) ? 32 : 64;   // valid rows of this wave's tile
    const int r0 = rows.at(ti < rows.n ? ti : WR * gr, 64), c0 = cols.at(tj < cols.n ? tj : WC * gc, 32);
    // this lane's source rows and columns of the group's copies (a tile
    // outside the window takes the group's first tile: in bounds, unused)
    int64_t asrc[A_INS];
    bool aok[A_INS];
#pragma unroll
    for (int q = 0; q < A_INS; ++q) {
      const int j = wave * A_INS + q, row = j * A_ROWS + l / KC, u = row / 64;
      aok[q] = WR * gr + u < rows.n && !(tail && WR * gr + u == rows.n - 1 && row % 64 >= 32);
      const int p = l % KC, k = p ^ (KC == 16 ? (row & 15) : ((row >> 1) & 7));
      asrc[q] = (int64_t)rm(arow + rows.at(aok[q] ? WR * gr + u : WR * gr, 64) + row % 64) * Mp + acol + k;
    }
    int bkrow[B_INS];
    int64_t bcol[B_INS];
#pragma unroll
    for (int q = 0; q < B_INS; ++q) {
      const int s = (wave * B_INS + q) * 64 + l, k = s / BC, col = s % BC, u = col / 32;
      bkrow[q] = krow0 + k;
      bcol[q] = cols.at(WC * gc + u < cols.n ? WC * gc + u : WC * gc, 32) + bshift + col % 32;
    }
    auto stage = [&](int chunk, cpx<double> *buf) {
      const int kb = chunk * KC;
#pragma unroll
      for (int q = 0; q < A_INS; ++q)
        if (aok[q]) lds_copy16(X + asrc[q] + kb, buf + (wave * A_INS + q) * 64);
#pragma unroll
      for (int q = 0; q < B_INS; ++q)
        // B rows krow0 + k (k < K) are pivot rows, below Mp: always mapped
        lds_copy16(X + (int64_t)pl[bkrow[q] + kb] * Mp + bcol[q], buf + U::A_EL + (wave * B_INS + q) * 64);
    };
    auto dst_of = [=](int r, int c) -> cpx<double> * {
      if constexpr (TO_S) return S + (int64_t)(r0 + r) * lds + c0 + c;
      else return X + (int64_t)rm(r0 + r) * Mp + c0 + c;
    };
    CTileRC<double, 4, 2> acc;
    if (ACC && mine)
      ctile_for_each_rc<double, 4, 2>(acc, [=](int r, int c, double &re, double &im) {
        if (r < vrows) {
          const cpx<double> v = *dst_of(r, c);
          re = v.re;
          im = v.im;
        } else {
          re = 0.0;
          im = 0.0;
        }
      });
    else
      ctile_for_each_rc<double, 4, 2>(acc, [=](int, int, double &re, double &im) {
        re = 0.0;
        im = 0.0;
      });
    auto multiply = [&](const cpx<double> *buf) {
      const cpx<double> *sa = buf, *sb = buf + U::A_EL;
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        cpx<double> a[4], b[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = sa[upd_a_slot<KC>(wr * 64 + 16 * i + (l & 15), 4 * ks + (l >> 4))];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = sb[(4 * ks + (l >> 4)) * BC + wc * 32 + 16 * j + (l & 15)];
        ctile_mma_rc<double, 4, 2>(acc, a, b);
      }
    };
    stage(0, st0);
    __syncthreads();
#pragma unroll 1
    for (int c = 0; c < nch; c += 2) {
      stage(c + 1, st1);
      if (mine) multiply(st0);
      __syncthreads();
      if (c + 2 < nch) stage(c + 2, st0);
      if (mine) multiply(st1);
      __syncthreads();
    }
    if (mine)
      ctile_for_each_rc<double, 4, 2>(acc, [=](int r, int c, double &re, double &im) {
        if (r < vrows) *dst_of(r, c) = NEG ? cpx<double>{-re, -im} : cpx<double>{re, im};
      });
  }
}

// FP64 products go through the LDS-staged routine, FP32 ones through the
// per-wave one.
template <class RG, int NT, bool TO_S, bool ACC, bool NEG>
__device__ __forceinline__ void tile_gemm_64x32_any(cpx<RG> *X, cpx<RG> *S, int lds, const int *phys, int Mp,
                                                    int rb1, int rn1, int rb2, int rn, int rh, int rhl, int cb1,
                                                    int cn, int ch, int chl, int K, int arow, int acol, int krow0,
                                                    int bshift) {
  if constexpr (std::is_same<RG, double>::value)
    tile_gemm_64x32_lds<NT, TO_S, ACC, NEG>(X, S, lds, phys, Mp, rb1, rn1, rb2, rn, rh, rhl, cb1, cn, ch, chl, K,
                                            arow, acol, krow0, bshift, 0);
  else
    tile_gemm_64x32<RG, NT, TO_S, ACC, NEG>(X, S, lds, phys, Mp, rb1, rn1, rb2, rn, rh, rhl, cb1, cn, ch, chl, K,
                                            arow, acol, krow0, bshift);
}

// D = A B (+ Add) in FP64 for plain row-major operands: rows r < Mr and
// columns c < Nc (multiples of 32), K a multiple of 32.  The staging of
// tile_gemm_64x32_lds (groups of 64 x 32 wave tiles, k-chunks copied by
// direct global -> LDS loads into two buffers while the other is multiplied;
// the last row tile may hold 32 rows), with every output element's k-terms
// in ascending order from zero, as wg_gemm_mfma takes them: the results are
// bitwise those of wg_gemm_mfma with a storing (or adding) epilogue.  D may
// not overlap A or B.  Called by the whole workgroup.
template <int NT>
__device__ __attribute__((noinline)) void gemm_lds(int Mr, int Nc, int K, const cpx<double> *A, int64_t lda,
                                                   const cpx<double> *B, int64_t ldb, cpx<double> *D, int64_t ldd,
                                                   const cpx<double> *Add, int64_t ldadd) {
  using U = UpdStage<NT>;
  constexpr int KC = U::KC, BC = U::BC, WC = U::WC, WR = U::WR, NW = U::NW;
  constexpr int A_INS = U::A_EL / 64 / NW, B_INS = U::B_EL / 64 / NW;
  constexpr int A_ROWS = 64 / KC;
  const int l = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wave / WC, wc = wave % WC;
  const int nrt = (Mr + 63) / 64, nct = Nc / 32;
  const int ngr = (nrt + WR - 1) / WR, ngc = (nct + WC - 1) / WC;
  const int nch = K / KC;   // even
  cpx<double> *st0 = upd_stage0<NT>(), *st1 = upd_stage1<NT>();
  for (int g = 0; g < ngr * ngc; ++g) {
    const int gr = g / ngc, gc = g % ngc;
    const int ti = WR * gr + wr, tj = WC * gc + wc;
    const bool mine = ti < nrt && tj < nct;
    const int r0 = 64 * ti, c0 = 32 * tj;
    const int vrows = Mr - r0 < 64 ? Mr - r0 : 64;   // valid rows of this wave's tile
    int64_t asrc[A_INS];
    bool aok[A_INS];
#pragma unroll
    for (int q = 0; q < A_INS; ++q) {
      const int j = wave * A_INS + q, row = j * A_ROWS + l / KC;
      const int grow = 64 * WR * gr + row;   // A row of this copy
      aok[q] = grow < Mr;                    // uniform over the copy (A_ROWS divides 32)
      const int p = l % KC, k = p ^ (KC == 16 ? (row & 15) : ((row >> 1) & 7));
      asrc[q] = (int64_t)(aok[q] ? grow : 0) * lda + k;
    }
    int bk[B_INS];
    int64_t bcol[B_INS];
#pragma unroll
    for (int q = 0; q < B_INS; ++q) {
      const int s = (wave * B_INS + q) * 64 + l, k = s / BC, col = s % BC;
      const int gcol = 32 * WC * gc + col;
      bk[q] = k;
      bcol[q] = gcol < Nc ? gcol : col % 32;   // a column outside the window reads column tile 0
    }
    auto stage = [&](int chunk, cpx<double> *buf) {
      const int kb = chunk * KC;
#pragma unroll
      for (int q = 0; q < A_INS; ++q)
        if (aok[q]) lds_copy16(A + asrc[q] + kb, buf + (wave * A_INS + q) * 64);
#pragma unroll
      for (int q = 0; q < B_INS; ++q)
        lds_copy16(B + (int64_t)(kb + bk[q]) * ldb + bcol[q], buf + U::A_EL + (wave * B_INS + q) * 64);
    };
    CTileRC<double, 4, 2> acc;
    ctile_for_each_rc<double, 4, 2>(acc, [=](int, int, double &re, double &im) {
      re = 0.0;
      im = 0.0;
    });
    auto multiply = [&](const cpx<double> *buf) {
      const cpx<double> *sa = buf, *sb = buf + U::A_EL;
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        cpx<double> a[4], b[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = sa[upd_a_slot<KC>(wr * 64 + 16 * i + (l & 15), 4 * ks + (l >> 4))];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = sb[(4 * ks + (l >> 4)) * BC + wc * 32 + 16 * j + (l & 15)];
        ctile_mma_rc<double, 4, 2>(acc, a, b);
      }
    };
    stage(0, st0);
    __syncthreads();
#pragma unroll 1
    for (int c = 0; c < nch; c += 2) {
      stage(c + 1, st1);
      if (mine) multiply(st0);
      __syncthreads();
      if (c + 2 < nch) stage(c + 2, st0);
      if (mine) multiply(st1);
      __syncthreads();
    }
    if (mine)
      ctile_for_each_rc<double, 4, 2>(acc, [=](int r, int c, double &re, double &im) {
        if (r < vrows) {
          const int64_t o = (int64_t)(r0 + r) * ldd + c0 + c;
          if (Add) {
            const cpx<double> x = Add[(int64_t)(r0 + r) * ldadd + c0 + c];
            D[o] = cpx<double>{x.re + re, x.im + im};
          } else {
            D[o] = cpx<double>{re, im};
          }
        }
      });
  }
}

// The update inside an outer panel after its inner panel at k0:
//   X[r, c] += sum_{k < 16} X[r, k0 + k] X[k0 + k, c]
// for the 16-row tiles rows.at(i, 16) and 16-column tiles cols.at(j, 16).  A
// wave takes a row strip, keeps its 16 x 16 multipliers in registers and walks
// the column tiles, loading the next tile's accumulator and pivot-row block
// while the current tile's products run (same products, in the same order, as
// tile_gemm_window with one 16 x 16 block).
template <class RG, int NT>
__device__ __attribute__((noinline)) void inner_update_strips(cpx<RG> *X, const int *phys, int Mp, int rb1, int rn,
                                                              int rh, int rhl, int cb1, int cn, int ch, int chl,
                                                              int k0) {
  using M = Mfma<RG>;
  const RowMap rm{phys, Mp};
  const IdxMap rows{rb1, rn, 0, rn, rh, rhl}, cols{cb1, cn, 0, cn, ch, chl};
  const int l = lane_id();
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  int64_t brow[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) brow[ks] = (int64_t)rm(k0 + 4 * ks + (l >> 4)) * Mp + (l & 15);
  for (int it = wave; it < rows.n; it += nwaves) {
    const int r0 = rows.at(it, 16);
    cpx<RG> a[4][1];
    const int64_t arow = (int64_t)rm(r0 + (l & 15)) * Mp + k0 + (l >> 4);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) a[ks][0] = X[arow + 4 * ks];
    int64_t crow[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) crow[e] = (int64_t)rm(r0 + M::row(l, e)) * Mp + (l & 15);
    cpx<RG> cb[2][4], bb[2][4][1];
    auto load = [&](int j, int buf) {
      const int c0 = cols.at(j, 16);
#pragma unroll
      for (int e = 0; e < 4; ++e) cb[buf][e] = X[crow[e] + c0];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) bb[buf][ks][0] = X[brow[ks] + c0];
    };
    auto step = [&](int j, int buf) {
      CTile<RG, 1> acc;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc.re[0][0][e] = cb[buf][e].re;
        acc.im[0][0][e] = cb[buf][e].im;
      }
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) ctile_mma<RG, 1>(acc, a[ks], bb[buf][ks]);
      const int c0 = cols.at(j, 16);
#pragma unroll
      for (int e = 0; e < 4; ++e) X[crow[e] + c0] = cpx<RG>{acc.re[0][0][e], acc.im[0][0][e]};
    };
    load(0, 0);
#pragma unroll 1
    for (int j = 0; j < cols.n; j += 2) {
      if (j + 1 < cols.n) load(j + 1, 1);
      step(j, 0);
      if (j + 1 < cols.n) {
        if (j + 2 < cols.n) load(j + 2, 0);
        step(j + 1, 1);
      }
    }
  }
}

template <class RG, int NBLK, int NT>
__device__ __forceinline__ void tile_gemm_window(const cpx<RG> *X, cpx<RG> *S, int lds, RowMap rm, IdxMap rows,
                                                 IdxMap cols, int K, int arow, int acol, int krow0, int bshift,
                                                 bool accumulate, bool negate) {
  const int fl = (accumulate ? 1 : 0) | (negate ? 2 : 0);
#define KNIT_TGW(KT)                                                                                              \
  tile_gemm_window_flat<RG, NBLK, KT, NT>(X, S, lds, rm.phys, rm.Mp, rows.base1, rows.n1, rows.base2, rows.n,        \
                                      rows.hole, rows.hole_len, cols.base1, cols.n1, cols.base2, cols.n,         \
                                      cols.hole, cols.hole_len, K, arow, acol, krow0, bshift, fl)
  if (NBLK == 1) KNIT_TGW(16);            // inner panels: K = 16
  else if (K == 64) KNIT_TGW(64);         // outer panels of 64
  else KNIT_TGW(0);                       // any other multiple of 32 (runtime K)
#undef KNIT_TGW
}

// Gauss-Jordan with partial pivoting in two levels: outer panels of NO columns
// (NO = 64 or 128, the last one may be narrower by multiples of 32) whose
// restricted elimination runs as
// NI = PanelW steps confined to the outer panel's columns and to the logical
// rows [K0, Mp); then one rank-NO update of the rest of the matrix.  The whole
// matrix is touched once per outer panel instead of once per inner panel.
// Sb ([R][NO]) and Sd ([NO][Mp]) hold the two products that cannot be formed
// in place.  phys (LDS, Mp entries) receives the final row order.
template <class RG, int NT, int NO, int NI = PanelW<RG>::NB>
__device__ int gj_two_level(cpx<RG> *X, int Mp, int R, int *phys, cpx<RG> *xchg, cpx<RG> *prow, double *sv,
                            int *si, cpx<RG> *Sb, cpx<RG> *Sd) {
  constexpr int BI = NI / 16;      // inner tile blocks
  for (int i = threadIdx.x; i < Mp; i += blockDim.x) phys[i] = i;
  __syncthreads();
  const RowMap rm{phys, Mp};
  int flags = 0;
  for (int K0 = 0; K0 < Mp; K0 += NO) {
    const int NOe = Mp - K0 < NO ? Mp - K0 : NO;
    // ---- restricted elimination of the outer panel
    for (int k0 = K0; k0 < K0 + NOe; k0 += NI) {
      flags |= gj_panel<RG, NI>(X, Mp, k0, phys, xchg, prow, sv, si);
      __syncthreads();
      const int npan = NOe / NI, pi = (k0 - K0) / NI;
      const IdxMap pcols = imap(K0, npan - 1, k0, NI);   // outer-panel columns minus the inner panel
      // multipliers of the earlier pivot rows of this outer panel: rows [K0, k0)
      if (pi > 0)
        tile_gemm_window<RG, BI, NT>(X, nullptr, 0, rm, imap(K0, pi), imap(k0, 1), NI, 0, k0, k0, 0, false, true);
      __syncthreads();
      // update inside the outer panel: rows [K0, Mp) minus the pivot rows
      if (npan > 1) {
        if constexpr (NI == 16)
          inner_update_strips<RG, NT>(X, phys, Mp, K0, (Mp - K0) / NI - 1, k0, NI, pcols.base1, pcols.n, pcols.hole,
                                      pcols.hole_len, k0);
        else
          tile_gemm_window<RG, BI, NT>(X, nullptr, 0, rm, imap(K0, (Mp - K0) / NI - 1, k0, NI), pcols, NI, 0, k0, k0,
                                   0, true, false);
      }
      // pivot rows across the outer panel (into Sd: in place would race)
      if (npan > 1)
        tile_gemm_window<RG, BI, NT>(X, Sd, Mp, rm, imap(0, 1), pcols, NI, k0, k0, k0, 0, false, false);
      __syncthreads();
      for (int e = threadIdx.x; e < NI * NOe; e += blockDim.x) {
        const int r = e / NOe, c = K0 + e % NOe;
        if (c >= k0 && c < k0 + NI) continue;
        X[(int64_t)phys[k0 + r] * Mp + c] = Sd[(int64_t)r * Mp + c];
      }
      __syncthreads();
    }
    if (NOe == Mp && R == Mp) continue;
    // ---- rank-NO update of the rest
    const int n_above = K0 / 32, n_below = (R - Mp) / 32;
    const IdxMap ocols = imap(0, (Mp - NOe) / 32, K0, NOe);
    // (b) multipliers of the rows outside [K0, Mp): -X[r, K] T; (c) the
    // update X[r, c] += X[r, K] X[P, c] of those rows and of the rows below P
    // (with the old pivot rows X[P, c]); (d) the new pivot rows T X[P, c], for
    // c outside the panel.
    constexpr int NW = NT / 64;
    constexpr bool LDSP = std::is_same<RG, double>::value;
    // FP64: the LDS-staged products.  (b) writes X[r, K] in place when one
    // group spans the panel's columns; (d) writes X[P, c] in place after (c)
    // has used the old rows (a group spans all of P).  No copies.
    // (at 256 threads with 128-wide panels the groups take the 1 x 4 shape)
    constexpr int BWR = UpdStage<NT>::BC >= NO ? 2 : 1;
    constexpr bool B_INPLACE = LDSP && UpdStage<NT, BWR>::BC >= NO;
    if (n_above + n_below > 0) {
      const int a64 = n_above / 2, b64 = n_below / 2;
      if constexpr (B_INPLACE) {
        tile_gemm_64x32_lds<NT, false, false, true, BWR>(X, nullptr, 0, rm.phys, Mp, 0, a64, Mp,
                                                    a64 + b64 + (n_below & 1), 0, 0, K0, NOe / 32, 0, 0, NOe, 0, K0,
                                                    K0, 0, n_below & 1);
      } else if ((a64 + b64) * (NOe / 32) < 2 * NW) {
        // (64-row tiles where there are at least two per wave: the rows above
        // P come in pairs of 32, the rows below Mp too except an odd last 32,
        // which the 32 x 32 routine takes; otherwise 32 x 32 tiles throughout)
        tile_gemm_window<RG, 2, NT>(X, Sb, NO, rm, imap2(0, n_above, Mp, n_above + n_below), imap(0, NOe / 32), NOe,
                                0, K0, K0, K0, false, true);
      } else {
        if (a64 + b64 > 0)
          tile_gemm_64x32_any<RG, NT, true, false, true>(X, Sb, NO, rm.phys, Mp, 0, a64, Mp, a64 + b64, 0, 0, 0,
                                                     NOe / 32, 0, 0, NOe, 0, K0, K0, K0);
        if (n_below & 1)
          tile_gemm_window<RG, 2, NT>(X, Sb, NO, rm, imap(R - 32, 1), imap(0, NOe / 32), NOe, 0, K0, K0, K0, false,
                                  true);
      }
    }
    if constexpr (!LDSP) {
      // (d) into Sd (64-row tiles when the panel width allows and there are at
      // least two per wave)
      if (Mp > NOe) {
        if (NOe % 64 == 0 && (NOe / 64) * ocols.n >= 2 * NW)
          tile_gemm_64x32_any<RG, NT, true, false, false>(X, Sd, Mp, rm.phys, Mp, 0, NOe / 64, 0, NOe / 64, 0, 0,
                                                      ocols.base1, ocols.n, ocols.hole, ocols.hole_len, NOe, K0, K0,
                                                      K0, 0);
        else
          tile_gemm_window<RG, 2, NT>(X, Sd, Mp, rm, imap(0, NOe / 32), ocols, NOe, K0, K0, K0, 0, false, false);
      }
    }
    __syncthreads();
    if constexpr (!B_INPLACE) {
      for (int e = threadIdx.x; e < (n_above + n_below) * 32 * NOe; e += blockDim.x) {
        const int rr = e / NOe, c = e % NOe;
        const int r = rr < n_above * 32 ? rr : Mp + (rr - n_above * 32);
        X[(int64_t)rm(r) * Mp + K0 + c] = Sb[(int64_t)r * NO + c];
      }
      __syncthreads();
    }
    // (c): 64-row tiles where there are at least two per wave (K0 is a
    // multiple of 64, so none straddles P), and the last 32 rows on their own
    // when the count of 32-row tiles is odd (they follow P); otherwise 32 x 32
    // tiles throughout
    if (Mp > NOe) {
      const int n32 = R / 32 - NOe / 32;
      const bool tall = (n32 / 2) * ocols.n >= 2 * NW;
      const int n64 = tall ? n32 / 2 : 0;
      const IdxMap rest = tall ? imap(R - 32, n32 & 1) : imap(0, n32, K0, NOe);
      if (n64 > 0)
        tile_gemm_64x32_any<RG, NT, false, true, false>(X, nullptr, 0, rm.phys, Mp, 0, n64, 0, n64, K0, NOe, ocols.base1,
                                                    ocols.n, ocols.hole, ocols.hole_len, NOe, 0, K0, K0, 0);
      if (rest.n > 0)
        tile_gemm_window<RG, 2, NT>(X, nullptr, 0, rm, rest, ocols, NOe, 0, K0, K0, 0, true, false);
    }
    __syncthreads();
    if constexpr (LDSP) {
      // (d) in place: rows P = [K0, K0 + NOe) in 64-row tiles (the last one 32
      // rows when NOe is an odd multiple of 32)
      if (Mp > NOe) {
        const int np = (NOe + 63) / 64;
        tile_gemm_64x32_lds<NT, false, false, false>(X, nullptr, 0, rm.phys, Mp, K0, np, 0, np, 0, 0, ocols.base1,
                                                     ocols.n, ocols.hole, ocols.hole_len, NOe, 0, K0, K0, 0,
                                                     (NOe % 64) != 0);
      }
    } else {
      for (int e = threadIdx.x; e < NOe * Mp; e += blockDim.x) {
        const int r = e / Mp, c = e % Mp;
        if (c >= K0 && c < K0 + NOe) continue;
        X[(int64_t)phys[K0 + r] * Mp + c] = Sd[(int64_t)r * Mp + c];
      }
    }
    __syncthreads();
  }
  return flags;
}

// A_n (and B_n = -G_{1,n-1} V^+) into X (type RG, padded to Mp with an
// identity block), one norb x norb site block per thread.  gprev(r, c) and
// G1prev(r, c) return g_{n-1} and G_{1,n-1} in natural order; with REFINE
// A_n is also written in FP64 to A64.
template <int no, class RG, bool REFINE, bool BOTTOM, class GAcc, class G1Acc>
__device__ __forceinline__ void form_blocks_n(cpx<RG> *X, cpx<double> *A64, StripDev s, int Mp,
                                                        double E, const knit_z *D, const knit_z *sL,
                                                        const knit_z *sR, bool first, bool last, GAcc gprev,
                                                        G1Acc G1prev, int nbot, bool couple) {
  const int M = s.M, W = M / no, Wp = Mp / no;
  const int64_t E2 = (int64_t)Mp * Mp;
  // top: site blocks (sa, sb), one output row oa at a time
  for (int blk = threadIdx.x; blk < Wp * Wp; blk += blockDim.x) {
    const int sa = blk / Wp, sb = blk % Wp;
    const bool real = sa < W && sb < W;
    const bool cpl = couple && real;
    const int ca = cpl ? s.vcol[sa] : -1, cb = cpl ? s.vcol[sb] : -1;
    const bool vgv = !first && ca >= 0 && cb >= 0;
    const bool inband = s.h0_band == 0 || (sa > sb ? sa - sb : sb - sa) <= s.h0_band;
    cpx<double> gb[no][no];
    if (vgv)
#pragma unroll
      for (int i = 0; i < no; ++i)
#pragma unroll
        for (int j = 0; j < no; ++j) gb[i][j] = gprev(ca * no + i, cb * no + j);
#pragma unroll
    for (int oa = 0; oa < no; ++oa) {
      cpx<double> u[no];          // row oa of v_a g
      if (vgv)
#pragma unroll
        for (int j = 0; j < no; ++j) {
          cpx<double> acc = {0.0, 0.0};
#pragma unroll
          for (int i = 0; i < no; ++i) acc = c_fma(vblk_at(s, sa, oa, i), gb[i][j], acc);
          u[j] = acc;
        }
#pragma unroll
      for (int ob = 0; ob < no; ++ob) {
        cpx<double> out;
        if (real) {
          const int64_t e = (int64_t)(sa * no + oa) * M + sb * no + ob;
          // H0 outside its stated band is zero: not read
          cpx<double> h = inband ? ld_z(s.H0 + e) : cpx<double>{0.0, 0.0};
          if (s.onsite_dense || sa == sb) {
            const cpx<double> d = ld_z(D + (s.onsite_dense ? e : ((int64_t)sa * no + oa) * no + ob));
            h.re += d.re;
            h.im += d.im;
          }
          if (first) {
            const cpx<double> x = ld_z(sL + e);
            h.re += x.re;
            h.im += x.im;
          }
          if (last) {
            const cpx<double> x = ld_z(sR + e);
            h.re += x.re;
            h.im += x.im;
          }
          if (vgv) {
            cpx<double> acc = {0.0, 0.0};
#pragma unroll
            for (int j = 0; j < no; ++j) acc = c_fma(u[j], c_conj(vblk_at(s, sb, ob, j)), acc);
            h.re += acc.re;
            h.im += acc.im;
          }
          out = {(sa == sb && oa == ob ? E : 0.0) - h.re, -h.im};
        } else {
          out = {(sa == sb && oa == ob) ? 1.0 : 0.0, 0.0};
        }
        const int64_t o = (int64_t)(sa * no + oa) * Mp + sb * no + ob;
        X[o] = cvt<RG>(out);
        if (REFINE) A64[o] = out;
      }
    }
  }
  if (first || !BOTTOM || !couple) return;
  // bottom: row a, site block sb: -(G_{1,n-1} V^+)[a, sb]; rows a >= nbot (up to
  // the next multiple of MPAD) are zero
  const int Mb = (nbot + MPAD - 1) / MPAD * MPAD;
  for (int blk = threadIdx.x; blk < Mb * Wp; blk += blockDim.x) {
    const int a = blk / Wp, sb = blk % Wp;
    const int cb = (sb < W && a < nbot) ? s.vcol[sb] : -1;
    cpx<double> gr[no];
    if (cb >= 0)
#pragma unroll
      for (int j = 0; j < no; ++j) gr[j] = G1prev(a, cb * no + j);
#pragma unroll
    for (int ob = 0; ob < no; ++ob) {
      cpx<double> w = {0.0, 0.0};
      if (cb >= 0)
#pragma unroll
        for (int j = 0; j < no; ++j) w = c_fma(gr[j], c_conj(vblk_at(s, sb, ob, j)), w);
      X[E2 + (int64_t)a * Mp + sb * no + ob] = cvt<RG>(cpx<double>{-w.re, -w.im});
    }
  }
}

// couple = false leaves out the coupling terms (V g V^+ and the stacked rows):
// with a dense V they are formed by dense_coupling afterwards.
template <class RG, bool REFINE, bool BOTTOM = true, class GAcc, class G1Acc>
__device__ void form_blocks(cpx<RG> *X, cpx<double> *A64, const StripDev &s, int Mp, double E,
                            const knit_z *D, const knit_z *sL, const knit_z *sR, bool first, bool last,
                            GAcc gprev, G1Acc G1prev, int nbot = -1, bool couple = true) {
  if (nbot < 0) nbot = s.M;
  switch (s.norb) {
    case 1: form_blocks_n<1, RG, REFINE, BOTTOM>(X, A64, s, Mp, E, D, sL, sR, first, last, gprev, G1prev, nbot, couple); break;
    case 2: form_blocks_n<2, RG, REFINE, BOTTOM>(X, A64, s, Mp, E, D, sL, sR, first, last, gprev, G1prev, nbot, couple); break;
    default: form_blocks_n<4, RG, REFINE, BOTTOM>(X, A64, s, Mp, E, D, sL, sR, first, last, gprev, G1prev, nbot, couple); break;
  }
}

// Dense inter-slice hopping V (general hopping matrices of Eq. (1)): the
// coupling terms of the slice matrix as complex products on the matrix cores,
// after form_blocks(couple = false) has written the rest:
//   top:     A_n -= (V g_{n-1}) V^+              (two Mp^3 products, Tv scratch)
//   stacked: X[Mp + r] = -(G_{1,n-1} V^+)[r]     for the first nbp rows
// Vd = V and Vh = V^+ ([Mp][Mp], zero padded), g and G1 in natural order.
// With REFINE the top is accumulated in FP64 in A64 and rounded into X.
// Called by the whole workgroup; ends with a barrier.
template <class RG, class RS, bool REFINE>
__device__ __attribute__((noinline)) void dense_coupling(cpx<RG> *X, cpx<double> *A64, const cpx<RS> *Vd,
                                                         const cpx<RS> *Vh, const cpx<RS> *g, const cpx<RS> *G1,
                                                         cpx<RS> *Tv, int Mp, int nbp) {
  const int64_t E2 = (int64_t)Mp * Mp;
  wg_gemm_mfma<RS>(Mp, Mp, Mp, Vd, Mp, g, Mp, [&](int r, int c, RS &re, RS &im) {
    Tv[(int64_t)r * Mp + c] = cpx<RS>{re, im};
  });
  __syncthreads();
  wg_gemm_mfma<RS>(Mp, Mp, Mp, Tv, Mp, Vh, Mp, [&](int r, int c, RS &re, RS &im) {
    const int64_t o = (int64_t)r * Mp + c;
    if constexpr (REFINE) {
      const cpx<double> a = {A64[o].re - (double)re, A64[o].im - (double)im};
      A64[o] = a;
      X[o] = cvt<RG>(a);
    } else {
      const cpx<RG> x = X[o];
      X[o] = cpx<RG>{x.re - (RG)re, x.im - (RG)im};
    }
  });
  if (nbp > 0)
    wg_gemm_mfma<RS>(nbp, Mp, Mp, G1, Mp, Vh, Mp, [&](int r, int c, RS &re, RS &im) {
      X[E2 + (int64_t)r * Mp + c] = cpx<RG>{(RG)-re, (RG)-im};
    });
  __syncthreads();
}

// Vd = V and Vh = V^+ of a dense-coupling strip, zero padded to [Mp][Mp].
template <class RS>
__device__ void load_dense_v(cpx<RS> *Vd, cpx<RS> *Vh, const StripDev &s, int Mp) {
  const int M = s.M;
  for (int64_t i = threadIdx.x; i < (int64_t)Mp * Mp; i += blockDim.x) {
    const int a = (int)(i / Mp), b = (int)(i % Mp);
    cpx<double> v = {0.0, 0.0}, vt = {0.0, 0.0};
    if (a < M && b < M) {
      v = ld_z(s.V + (int64_t)a * M + b);
      const cpx<double> w = ld_z(s.V + (int64_t)b * M + a);
      vt = {w.re, -w.im};
    }
    Vd[i] = cvt<RS>(v);
    Vh[i] = cvt<RS>(vt);
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

// Y = Gm V^+ (columns of Gm gathered through vcol) on the first `nrows` rows
// (default all Mp), padded rows and columns zero
template <class RS>
__device__ void gather_gvdag(cpx<RS> *Y, const cpx<RS> *Gm, const StripDev &s, int Mp, int nrows = -1) {
  const int M = s.M, no = s.norb;
  const int64_t E2 = (int64_t)(nrows < 0 ? Mp : nrows) * Mp;
  for (int64_t i = threadIdx.x; i < E2; i += blockDim.x) {
    const int a = (int)(i / Mp), b = (int)(i % Mp);
    cpx<double> acc = {0.0, 0.0};
    if (a < M && b < M) {
      const int sb = b / no, ob = b % no, cb = s.vcol[sb];
      if (cb >= 0)
        for (int j = 0; j < no; ++j)
          acc = c_fma(cvt<double>(Gm[(int64_t)a * Mp + cb * no + j]), c_conj(vblk_at(s, sb, ob, j)), acc);
    }
    Y[i] = cvt<RS>(acc);
  }
}

// Workgroup sum of a non-negative double, NaN if any thread holds NaN.  sv: one
// slot per wave; ends with a barrier, so sv is free again on return.
__device__ __forceinline__ double wg_sum_nan(double v, double *sv) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sv[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sv[w];
  __syncthreads();
  return r;
}

// Refined inverse of a slice (precision extension), called by the whole
// workgroup after the FP32 elimination of A_n.  X0 (the elimination result X
// through the row map q and column map pinv) goes to Xn in natural order;
// then Newton steps on the inverse,
//   R_k = I - A_n X_k  (FP64 product, A_n and X_k exact in FP64),
//   X_{k+1} = X_k + X_k R_k  (correction product in FP32, sum in FP64),
// each of which squares the residual: ||I - A_n X_{k+1}|| <= ||R_k||^2 plus
// the FP32 rounding of the correction (about 6e-8 ||R_k|| relative).  Steps
// continue while ||R_k||_F > REFINE_TARGET (at most REFINE_MAX_STEPS), so a
// refined inverse carries a relative error below about REFINE_TARGET^2.  g
// receives X_final in FP64.  Returns the number of steps, or 0 (g undefined)
// when ||R_0||_F exceeds tol or is NaN, or when the steps stop shrinking the
// residual above the target: the problem then goes to the FP64 pass.  Rr holds
// R_k in FP32 (only its leading digits enter the correction).  Out of line:
// shared by the sweep and the LDOS kernels.
constexpr double REFINE_TARGET = 1e-5;
constexpr int REFINE_MAX_STEPS = 4;
template <class RS>
__device__ __attribute__((noinline)) int refine_inverse(const cpx<float> *X, const int *q, const int *pinv, int Mp,
                                                        const cpx<double> *A64, cpx<float> *Xn, cpx<float> *Rr,
                                                        cpx<RS> *g, double tol, double *sv) {
  const int64_t E2 = (int64_t)Mp * Mp;
  for (int64_t i = threadIdx.x; i < E2; i += blockDim.x) {
    const int a = (int)(i / Mp), b = (int)(i % Mp);
    Xn[i] = X[(int64_t)q[a] * Mp + pinv[b]];
  }
  __syncthreads();
  double fprev = 0.0;
  for (int k = 0; k < REFINE_MAX_STEPS; ++k) {
    // residual of the current inverse (X0 in FP32 at k = 0, g in FP64 after)
    double ss = 0.0;
    auto resid = [&](int r, int c, double &re, double &im) {
      const double rr = (r == c ? 1.0 : 0.0) - re, ri = -im;
      ss += rr * rr + ri * ri;
      Rr[(int64_t)r * Mp + c] = cpx<float>{(float)rr, (float)ri};
    };
    if (k == 0) wg_gemm_mfma<double>(Mp, Mp, Mp, A64, Mp, Xn, Mp, resid);
    else wg_gemm_mfma<double>(Mp, Mp, Mp, A64, Mp, g, Mp, resid);
    const double f = sqrt(wg_sum_nan(ss, sv));
    if (k == 0 ? !(f <= tol) : !(f < fprev)) return 0;
    if (k > 0) {
      // the FP32 operand of the correction
      for (int64_t i = threadIdx.x; i < E2; i += blockDim.x) Xn[i] = cvt<float>(g[i]);
      __syncthreads();
    }
    // X_{k+1} = X_k + X_k R_k; every element of g is read and written by the
    // lane that owns it in the epilogue only
    wg_gemm_mfma<float>(Mp, Mp, Mp, Xn, Mp, Rr, Mp, [&](int r, int c, float &re, float &im) {
      const int64_t o = (int64_t)r * Mp + c;
      const cpx<double> x = k == 0 ? cvt<double>(Xn[o]) : cvt<double>(g[o]);
      g[o] = cvt<RS>(cpx<double>{x.re + (double)re, x.im + (double)im});
    });
    __syncthreads();
    if (f <= REFINE_TARGET) return k + 1;
    fprev = f;
  }
  return 0;
}

// Propagator of the refined sweep as an FP64 product of the refined inverse g
// (natural order), in place in G1:
//   slice 1 (n == 0): G_11 = g_1, or P_1 = C_L^+ g_1 with CLp = C_L (rows >= rl zero)
//   later:            G_1n = (G_{1,n-1} V^+) g_n, or P_n = (P_{n-1} V^+) g_n
// on the first nb rows (Mp, or the projected rows rounded up to 32).  Tb is
// [nb][Mp] scratch; Vh = V^+ for a dense V (else V is gathered through vcol).
template <class RS>
__device__ __attribute__((noinline)) void refined_propagator(cpx<RS> *G1, cpx<RS> *Tb, const cpx<RS> *g,
                                                             StripDev s, int Mp, int n, const knit_z *CLp, int rl,
                                                             int nb, const cpx<RS> *Vh) {
  const int64_t E2 = (int64_t)Mp * Mp;
  const int M = s.M;
  if (n == 0 && !CLp) {
    for (int64_t i = threadIdx.x; i < E2; i += blockDim.x) G1[i] = g[i];
    __syncthreads();
    return;
  }
  if (n == 0) {
    for (int64_t i = threadIdx.x; i < (int64_t)nb * Mp; i += blockDim.x) {
      const int a = (int)(i / Mp), b = (int)(i % Mp);
      cpx<double> v = {0.0, 0.0};
      if (a < rl && b < M) {
        const cpx<double> c = ld_z(CLp + (int64_t)b * M + a);
        v = {c.re, -c.im};
      }
      Tb[i] = cvt<RS>(v);
    }
  } else if (Vh) {
    // dense V: G_{1,n-1} V^+ as a product
    wg_gemm_mfma<double>(nb, Mp, Mp, G1, Mp, Vh, Mp, [&](int r, int c, double &re, double &im) {
      Tb[(int64_t)r * Mp + c] = cvt<RS>(cpx<double>{re, im});
    });
  } else {
    gather_gvdag<RS>(Tb, G1, s, Mp, nb);
  }
  __syncthreads();
  wg_gemm_mfma<double>(nb, Mp, Mp, Tb, Mp, g, Mp, [&](int r, int c, double &re, double &im) {
    G1[(int64_t)r * Mp + c] = cvt<RS>(cpx<double>{re, im});
  });
  __syncthreads();
}

// Queue order for the persistent sweep.  policy 0: problem order.  policy 1:
// longest processing time first, on the cost Mp^2 R L (R = rows of the stacked
// elimination: 2 Mp, or Mp plus the projected rows when `rows` is given),
// binned at 16 bins per doubling (a counting sort, one workgroup; order within
// a bin is whatever the atomics give, which does not change any result).  Also
// clears the queue.
constexpr int LPT_BINS = 1024;   // 16 bins per doubling of the cost (4.4 % wide)
__global__ void __launch_bounds__(1024) order_kernel(StripTable tab, const knit_problem *probs, int P, int policy,
                                                     const int *rows, int *order, unsigned int *queue) {
  __shared__ unsigned int cnt[LPT_BINS];
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) *queue = 0u;
  if (policy == 0) {
    for (int p = tid; p < P; p += nt) order[p] = p;
    return;
  }
  auto bin_of = [&](int p) {
    const knit_problem pr = probs[p];
    const int mp = (tab.s[pr.strip].M + MPAD - 1) / MPAD * MPAD;
    const double Mp = (double)mp;
    // rows of the stacked elimination: Mp + Mp, or Mp + the projected rows
    const double R = Mp + (rows ? (double)((rows[p] + MPAD - 1) / MPAD * MPAD) : Mp);
    const double cost = Mp * Mp * R * (double)(pr.L > 0 ? pr.L : 1);
    int b = (int)(16.0 * log2(cost));
    return b < 0 ? 0 : (b >= LPT_BINS ? LPT_BINS - 1 : b);
  };
  for (int b = tid; b < LPT_BINS; b += nt) cnt[b] = 0u;
  __syncthreads();
  for (int p = tid; p < P; p += nt) atomicAdd(&cnt[bin_of(p)], 1u);
  __syncthreads();
  if (tid == 0) {   // start of each bin, costliest bin first
    unsigned int run = 0;
    for (int b = LPT_BINS - 1; b >= 0; --b) {
      const unsigned int c = cnt[b];
      cnt[b] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int p = tid; p < P; p += nt) order[atomicAdd(&cnt[bin_of(p)], 1u)] = p;
}

// Rows of the projected propagator, per problem: the columns of its C_L up to
// the last nonzero one.  One workgroup per problem.
__global__ void __launch_bounds__(256) proj_rows_kernel(StripTable tab, const knit_problem *probs, int P,
                                                        const knit_z *CL, int *rows) {
  __shared__ double sv[4];
  const int p = blockIdx.x;
  if (p >= P) return;
  const knit_problem pr = probs[p];
  const int M = tab.s[pr.strip].M;
  const int r = factor_columns(CL + pr.sigma_off, M, sv);
  if (threadIdx.x == 0) rows[p] = r < M ? r : M;
}

template <class RG, class RS, bool REFINE, int NT, bool PROJ = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) sweep_mfma_kernel(StripTable tab, const knit_problem *probs, int P,
                                                        const knit_z *onsite, const knit_z *sigmaL,
                                                        const knit_z *sigmaR, knit_z *G1N, knit_z *GN1,
                                                        knit_z *GNN, int32_t *pstatus, char *ws,
                                                        size_t slab_bytes, int Mpmax, unsigned int *queue,
                                                        const int *order, double refine_tol, const int32_t *redo,
                                                        int outer, const knit_z *CL, const int *rows) {
  __shared__ int next_p;
  __shared__ int qa[NT], qb[NT];        // row order of the current / previous elimination
  __shared__ int pa[NT], pb[NT];        // and its inverse (column order of the inverse)
  __shared__ double sv[32];
  __shared__ int si[64];
  __shared__ cpx<RG> xchg[2 * 32];
  __shared__ cpx<RG> prow[32];

  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t EE = (int64_t)Mpmax * Mpmax;
  char *slab = ws + (size_t)blockIdx.x * slab_bytes;
  // the refined sweep eliminates A_n alone: its elimination buffers hold Mp rows
  constexpr int XROWS = REFINE ? 1 : 2;
  cpx<RG> *Xa = reinterpret_cast<cpx<RG> *>(slab);                // [2 Mp][Mp]  ([Mp][Mp] refined)
  cpx<RG> *Xb = Xa + XROWS * EE;                                   // [2 Mp][Mp]  ([Mp][Mp] refined)
  cpx<RS> *g = reinterpret_cast<cpx<RS> *>(Xb + XROWS * EE);      // [Mp][Mp]  natural order (refine / G_n1)
  cpx<RS> *G1 = g + EE;                                           // [Mp][Mp]
  cpx<RS> *N1a = G1 + EE;                                         // [Mp][Mp]
  cpx<RS> *N1b = N1a + EE;                                        // [Mp][Mp]
  cpx<double> *A64 = reinterpret_cast<cpx<double> *>(N1b + EE);   // [Mp][Mp]   (REFINE)
  cpx<RS> *Tb = reinterpret_cast<cpx<RS> *>(A64 + (REFINE ? EE : 0));   // [Mp][Mp] (REFINE) G_{1,n-1} V^+
  cpx<float> *Xn = reinterpret_cast<cpx<float> *>(Tb + (REFINE ? EE : 0));    // [Mp][Mp] (REFINE)
  cpx<float> *Rr = Xn + (REFINE ? EE : 0);                        // [Mp][Mp]   (REFINE)
  cpx<RG> *Sb = reinterpret_cast<cpx<RG> *>(Rr + (REFINE ? EE : 0));   // [2 Mp][NO] scratch
  cpx<RG> *Sd = Sb + (int64_t)2 * Mpmax * NO_MAX;                       // [NO][Mp]   scratch
  // dense V (present in the slab only when the batch has a dense-coupling strip)
  cpx<RS> *Vd = reinterpret_cast<cpx<RS> *>(Sd + (int64_t)NO_MAX * Mpmax);   // [Mp][Mp] V
  cpx<RS> *Vh = Vd + EE;                                                      // [Mp][Mp] V^+
  cpx<RS> *Tv = Vh + EE;                                                      // [Mp][Mp] V g
  const bool want_n1 = GN1 != nullptr;
  const double qnan = __builtin_nan("");

  // problems are handed out by an atomic counter; every workgroup leaves the
  // loop once the counter has passed P
  for (;;) {
    if (tid == 0) next_p = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int pi = next_p;
    __syncthreads();
    if (pi >= P) break;
    const int p = order[pi];
    // second pass of a refined sweep: only the problems the first pass gave up on
    if (redo && !(redo[p] & KNIT_P_FALLBACK)) continue;
    const knit_problem pr = probs[p];
    const StripDev s = tab.s[pr.strip];
    const int M = s.M, no = s.norb, L = pr.L;
    const int Mp = (M + MPAD - 1) / MPAD * MPAD;
    const int64_t E2 = (int64_t)Mp * Mp;
    const knit_z *sL = sigmaL + pr.sigma_off, *sR = sigmaR + pr.sigma_off;
    // projected propagator: C_L^+ G_1n, rl rows (Gamma_L = C_L C_L^+, C_L with rl
    // columns up to its last nonzero one)
    const int rl = PROJ ? rows[p] : 0;
    const int rlp = (rl + MPAD - 1) / MPAD * MPAD;
    const int nbot = PROJ ? rl : M;
    // dense V: coupling terms as matrix-core products of natural-order g and G_1n
    const bool dense = s.V != nullptr;
    if (dense) {
      load_dense_v<RS>(Vd, Vh, s, Mp);
      __syncthreads();
    }
    int flags = 0;
    int *q = qa, *pinv = pa, *qp = qb, *pinvp = pb;
    cpx<RG> *X = Xa, *Xp = Xb;
    for (int n = 0; n < L; ++n) {
      const knit_z *D = onsite + pr.onsite_off + (int64_t)n * s.onsite_stride();
      if (REFINE || n == 0 || dense) {
        form_blocks<RG, REFINE, !REFINE>(X, A64, s, Mp, pr.E, D, sL, sR, n == 0, n == L - 1,
                                [=](int r, int c) { return cvt<double>(g[(int64_t)r * Mp + c]); },
                                [=](int r, int c) { return cvt<double>(G1[(int64_t)r * Mp + c]); }, -1, !dense);
        if (dense && n > 0) {
          __syncthreads();
          dense_coupling<RG, RS, REFINE>(X, A64, Vd, Vh, g, G1, Tv, Mp, REFINE ? 0 : (PROJ ? rlp : Mp));
        }
      } else {
        // previous result in Xp: logical row r at physical row qp[r], column c of the
        // inverse at column pinvp[c]; G_11 = g_1 is the top of slice 1's result
        // (projected: C_L^+ G_11 is already the bottom of slice 1's result)
        const bool top = n == 1 && !PROJ;
        form_blocks<RG, false>(X, A64, s, Mp, pr.E, D, sL, sR, false, n == L - 1,
                               [=](int r, int c) { return cvt<double>(Xp[(int64_t)qp[r] * Mp + pinvp[c]]); },
                               [=](int r, int c) {
                                 return cvt<double>(top ? Xp[(int64_t)qp[r] * Mp + pinvp[c]]
                                                        : Xp[(int64_t)(Mp + r) * Mp + pinvp[c]]);
                               },
                               nbot);
      }
      if (PROJ && !REFINE && n == 0) {
        // bottom block of slice 1: -C_L^+ (rows >= rl zero)
        for (int64_t i = tid; i < (int64_t)rlp * Mp; i += nt) {
          const int a = (int)(i / Mp), b = (int)(i % Mp);
          cpx<double> v = {0.0, 0.0};
          if (a < rl && b < M) {
            const cpx<double> c = ld_z(CL + pr.sigma_off + (int64_t)b * M + a);
            v = {-c.re, c.im};
          }
          X[E2 + i] = cvt<RG>(v);
        }
      }
      __syncthreads();
      const int R = REFINE ? Mp : (PROJ ? Mp + rlp : (n > 0 ? 2 * Mp : Mp));
      flags |= outer == 128 ? gj_two_level<RG, NT, 128>(X, Mp, R, q, xchg, prow, sv, si, Sb, Sd)
                            : gj_two_level<RG, NT, 64>(X, Mp, R, q, xchg, prow, sv, si, Sb, Sd);
      for (int i = tid; i < Mp; i += nt) pinv[q[i]] = i;
      __syncthreads();
      // logical row a of the result sits in physical row q[a] (a < Mp)
      if constexpr (REFINE) {
        // one FP64-residual step on the FP32 inverse, then the propagator as an
        // FP64 product of the refined inverse; a slice too poor for one step
        // hands the problem to the FP64 pass
        if (refine_inverse<RS>(X, q, pinv, Mp, A64, Xn, Rr, g, refine_tol, sv) == 0) {
          flags |= KNIT_P_FALLBACK;
          break;
        }
        refined_propagator<RS>(G1, Tb, g, s, Mp, n, PROJ ? CL + pr.sigma_off : nullptr, rl, PROJ ? rlp : Mp,
                               dense ? Vh : nullptr);
      } else if (want_n1 || n == L - 1 || dense) {
        // natural-order g_n (and G_1n) when G_n1 is carried, and for the outputs
        for (int64_t i = tid; i < (int64_t)R * Mp; i += nt) {
          const int a = (int)(i / Mp), b = (int)(i % Mp);
          cpx<RG> v = X[(int64_t)(a < Mp ? q[a] : a) * Mp + pinv[b]];
          if (a < Mp) g[i] = cvt<RS>(v);
          else G1[i - E2] = cvt<RS>(v);
        }
        __syncthreads();
        if (n == 0 && !PROJ) {
          for (int64_t i = tid; i < E2; i += nt) G1[i] = g[i];
          __syncthreads();
        }
      }
      if (want_n1) {
        if (n == 0) {
          for (int64_t i = tid; i < E2; i += nt) N1a[i] = g[i];
        } else {
          if (dense)
            wg_gemm_mfma<RS>(Mp, Mp, Mp, Vd, Mp, N1a, Mp, [&](int r, int c, RS &re, RS &im) {
              N1b[(int64_t)r * Mp + c] = cpx<RS>{re, im};
            });
          else
            gather_vg<RS>(N1b, N1a, s, Mp);
          __syncthreads();
          wg_gemm_mfma<RS>(Mp, Mp, Mp, g, Mp, N1b, Mp, [&](int r, int c, RS &re, RS &im) {
            N1a[(int64_t)r * Mp + c] = cpx<RS>{re, im};
          });
        }
        __syncthreads();
      }
      // the result of this slice becomes the previous one
      int *t1 = q; q = qp; qp = t1;
      int *t2 = pinv; pinv = pinvp; pinvp = t2;
      cpx<RG> *t3 = X; X = Xp; Xp = t3;
    }
    // outputs (the leading M x M blocks); a problem the refined pass gave up on
    // only records that, the FP64 pass writes its outputs
    if (redo) flags |= KNIT_P_FALLBACK;
    if (redo || !(flags & KNIT_P_FALLBACK)) {
      double bad = 0.0;
      const int64_t mm = (int64_t)M * M;
      for (int64_t i = tid; i < mm; i += nt) {
        const int a = (int)(i / M), b = (int)(i % M);
        const int64_t o = (int64_t)a * Mp + b;
        if (a < nbot) bad = fmax(bad, c_abs1(G1[o]));
        if (GNN) bad = fmax(bad, c_abs1(g[o]));
        if (want_n1) bad = fmax(bad, c_abs1(N1a[o]));
      }
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
        st_z(G1N + pr.out_off + i, kill ? nanz : (a < nbot ? cvt<double>(G1[o]) : cpx<double>{0.0, 0.0}));
        if (GNN) st_z(GNN + pr.out_off + i, kill ? nanz : cvt<double>(g[o]));
        if (want_n1) st_z(GN1 + pr.out_off + i, kill ? nanz : cvt<double>(N1a[o]));
      }
    }
    if (tid == 0) pstatus[p] = flags;
    __syncthreads();
  }
}

// Batched FP64 inverse on the matrix cores, one workgroup per matrix: X_e
// ([Mp][Mp], padded with an identity block) is reduced in place by the
// two-level elimination and its inverse, in natural order, goes to out_e
// ([M][M]).  Matrices whose skip flag is set are left alone; a singular pivot
// sets KNIT_P_SINGULAR in flags[e].
template <int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
inverse_fp64_kernel(cpx<double> *X, int64_t xstride, cpx<double> *scratch, int64_t sstride, int M, int Mp,
                    cpx<double> *out, int64_t ostride, const int32_t *skip, int skip_stride, int32_t *flags,
                    int flags_stride) {
  __shared__ int q[NT];
  __shared__ int pinv[NT];
  __shared__ double sv[32];
  __shared__ int si[64];
  __shared__ cpx<double> xchg[2 * 32];
  __shared__ cpx<double> prow[32];
  const int e = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  if (skip && skip[(int64_t)e * skip_stride]) return;
  cpx<double> *Xe = X + (int64_t)e * xstride;
  cpx<double> *Sb = scratch + (int64_t)e * sstride;
  cpx<double> *Sd = Sb + (int64_t)2 * Mp * NO_MAX;
  const int fl = Mp >= 128 ? gj_two_level<double, NT, 128>(Xe, Mp, Mp, q, xchg, prow, sv, si, Sb, Sd)
                           : gj_two_level<double, NT, 64>(Xe, Mp, Mp, q, xchg, prow, sv, si, Sb, Sd);
  for (int i = tid; i < Mp; i += nt) pinv[q[i]] = i;
  __syncthreads();
  cpx<double> *o = out + (int64_t)e * ostride;
  for (int64_t i = tid; i < (int64_t)M * M; i += nt) {
    const int a = (int)(i / M), b = (int)(i % M);
    o[i] = Xe[(int64_t)q[a] * Mp + pinv[b]];
  }
  if (fl && tid == 0) atomicOr(flags + (int64_t)e * flags_stride, fl);
}

// Local density of states on every slice (section 5.3-C sewing, the on-site
// Green function of section 7.1-D) on the matrix cores, one workgroup per
// problem from the same queue as the sweep:
//   forward:  g_n = A_n^{-1} (elimination of A_n alone, unpermuted to natural
//             order), g_{k st - 1} kept as checkpoint k;
//   reverse:  per segment, g_n recomputed from its checkpoint, then
//             G_LL = g_L,  G_nn = g_n + (g_n V^+) G_{n+1,n+1} (V g_n)
//             with the two products on MFMA;  LDOS_n[i] = -Im (G_nn)_ii / pi.
// RG is the elimination type, RS the type of everything kept (g_n, the
// checkpoints, G_nn and the products).  REFINE (RG float, RS double): each
// g_n is the FP32 inverse X0 plus one FP64-residual step, X0 + X0 (I - A_n X0),
// as in the refined sweep, and a slice whose residual exceeds the refine
// threshold hands the problem to a second, FP64 pass (KNIT_P_FALLBACK).
// Slab (Mp^2 elements each): X (RG), Gnn, U, W, T (RS), the segment's g
// [max(st, 2)], checkpoints [ceil(Lmax / st)] (RS), with REFINE A_n (FP64),
// X0 and R (FP32), then the elimination scratch (RG).
template <class RG, class RS, bool REFINE, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
ldos_mfma_kernel(StripTable tab, const knit_problem *probs, int P, const knit_z *onsite, const knit_z *sigmaL,
                 const knit_z *sigmaR, int stride, double *ldos, int32_t *pstatus, char *ws, size_t slab_bytes,
                 int Mpmax, int Lmax, unsigned int *queue, const int *order, int outer, double refine_tol,
                 const int32_t *redo) {
  using C = cpx<RG>;
  using S = cpx<RS>;
  __shared__ int next_p;
  __shared__ int q[NT], pinv[NT];
  __shared__ double sv[32];
  __shared__ int si[64];
  __shared__ C xchg[2 * 32];
  __shared__ C prow[32];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t EE = (int64_t)Mpmax * Mpmax;
  const int segbuf = stride < 2 ? 2 : stride;
  const int nsegmax = (Lmax + stride - 1) / stride;
  char *slab = ws + (size_t)blockIdx.x * slab_bytes;
  C *X = reinterpret_cast<C *>(slab);
  S *Gnn = reinterpret_cast<S *>(X + EE), *U = Gnn + EE, *W = U + EE, *T1 = W + EE;
  S *seg = T1 + EE;                              // [segbuf][Mp][Mp]
  S *cps = seg + (int64_t)segbuf * EE;           // [nsegmax][Mp][Mp]
  cpx<double> *A64 = reinterpret_cast<cpx<double> *>(cps + (int64_t)nsegmax * EE);   // (REFINE)
  cpx<float> *Xn = reinterpret_cast<cpx<float> *>(A64 + (REFINE ? EE : 0));           // (REFINE)
  cpx<float> *Rr = Xn + (REFINE ? EE : 0);                                             // (REFINE)
  C *Sb = reinterpret_cast<C *>(Rr + (REFINE ? EE : 0));   // [2 Mp][NO] scratch
  C *Sd = Sb + (int64_t)2 * Mpmax * NO_MAX;                // [NO][Mp]   scratch
  // dense V (present in the slab only when the batch has a dense-coupling strip)
  S *Vd = reinterpret_cast<S *>(Sd + (int64_t)NO_MAX * Mpmax);   // [Mp][Mp] V
  S *Vh = Vd + EE;                                               // [Mp][Mp] V^+
  const double qnan = __builtin_nan("");
  const double inv_pi = 0.318309886183790671537767526745;
  for (;;) {
    if (tid == 0) next_p = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int pi = next_p;
    __syncthreads();
    if (pi >= P) break;
    const int p = order[pi];
    // second pass of a refined call: only the problems the first pass gave up on
    if (redo && !(redo[p] & KNIT_P_FALLBACK)) continue;
    const knit_problem pr = probs[p];
    const StripDev s = tab.s[pr.strip];
    const int M = s.M, no = s.norb, L = pr.L;
    const int Mp = (M + MPAD - 1) / MPAD * MPAD;
    const int64_t E2 = (int64_t)Mp * Mp;
    const knit_z *sL = sigmaL + pr.sigma_off, *sR = sigmaR + pr.sigma_off;
    const int nseg = (L + stride - 1) / stride;
    const bool dense = s.V != nullptr;
    if (dense) {
      load_dense_v<RS>(Vd, Vh, s, Mp);
      __syncthreads();
    }
    int flags = 0;
    // g_n (natural order, into dst) from g_{n-1} (natural order, or none for n = 0);
    // false when a refined slice is too poor for one step (uniform over the workgroup)
    auto step = [&](int n, const S *gprev, S *dst) -> bool {
      const knit_z *D = onsite + pr.onsite_off + (int64_t)n * s.onsite_stride();
      form_blocks<RG, REFINE, false>(X, A64, s, Mp, pr.E, D, sL, sR, n == 0, n == L - 1,
                                     [=](int r, int c) { return cvt<double>(gprev[(int64_t)r * Mp + c]); },
                                     [=](int r, int c) { return cpx<double>{0.0, 0.0}; }, -1, !dense);
      __syncthreads();
      // dense V: A_n -= (V g_{n-1}) V^+ on the matrix cores (T1 is free here)
      if (dense && n > 0) dense_coupling<RG, RS, REFINE>(X, A64, Vd, Vh, gprev, nullptr, T1, Mp, 0);
      flags |= outer == 128 ? gj_two_level<RG, NT, 128>(X, Mp, Mp, q, xchg, prow, sv, si, Sb, Sd)
                            : gj_two_level<RG, NT, 64>(X, Mp, Mp, q, xchg, prow, sv, si, Sb, Sd);
      for (int i = tid; i < Mp; i += nt) pinv[q[i]] = i;
      __syncthreads();
      if constexpr (REFINE) {
        if (refine_inverse<RS>(X, q, pinv, Mp, A64, Xn, Rr, dst, refine_tol, sv) == 0) return false;
      } else {
        for (int64_t i = tid; i < E2; i += nt) {
          const int a = (int)(i / Mp), b = (int)(i % Mp);
          dst[i] = cvt<RS>(X[(int64_t)q[a] * Mp + pinv[b]]);
        }
      }
      __syncthreads();
      return true;
    };
    bool ok = true;
    // forward pass: checkpoint k holds g_{k st - 1} (k >= 1)
    {
      S *cur = seg, *prev = seg + E2;
      for (int n = 0; n < L && ok; ++n) {
        ok = step(n, prev, cur);
        if (ok && (n + 1) % stride == 0 && n + 1 < L) {
          S *cp = cps + (int64_t)((n + 1) / stride) * E2;
          for (int64_t i = tid; i < E2; i += nt) cp[i] = cur[i];
          __syncthreads();
        }
        S *t = cur;
        cur = prev;
        prev = t;
      }
    }
    // reverse pass, one segment at a time
    double *out = ldos + pr.ldos_off;
    for (int k = nseg - 1; k >= 0 && ok; --k) {
      const int n0 = k * stride, n1 = min(L, n0 + stride);
      for (int n = n0; n < n1 && ok; ++n) {
        const S *gprev = n == n0 ? (k > 0 ? cps + (int64_t)k * E2 : seg) : seg + (int64_t)(n - n0 - 1) * E2;
        ok = step(n, gprev, seg + (int64_t)(n - n0) * E2);
      }
      for (int n = n1 - 1; n >= n0 && ok; --n) {
        const S *g = seg + (int64_t)(n - n0) * E2;
        if (n == L - 1) {
          for (int64_t i = tid; i < E2; i += nt) Gnn[i] = g[i];
        } else {
          if (dense) {
            wg_gemm_mfma<RS>(Mp, Mp, Mp, g, Mp, Vh, Mp, [&](int r, int c, RS &re, RS &im) {
              U[(int64_t)r * Mp + c] = S{re, im};      // g V^+
            });
            wg_gemm_mfma<RS>(Mp, Mp, Mp, Vd, Mp, g, Mp, [&](int r, int c, RS &re, RS &im) {
              W[(int64_t)r * Mp + c] = S{re, im};      // V g
            });
          } else {
            gather_gvdag<RS>(U, g, s, Mp);     // g V^+
            gather_vg<RS>(W, g, s, Mp);        // V g
          }
          __syncthreads();
          wg_gemm_mfma<RS>(Mp, Mp, Mp, U, Mp, Gnn, Mp, [&](int r, int c, RS &re, RS &im) {
            T1[(int64_t)r * Mp + c] = S{re, im};
          });
          __syncthreads();
          wg_gemm_mfma<RS>(Mp, Mp, Mp, T1, Mp, W, Mp, [&](int r, int c, RS &re, RS &im) {
            const int64_t o = (int64_t)r * Mp + c;
            Gnn[o] = S{g[o].re + re, g[o].im + im};
          });
        }
        __syncthreads();
        for (int i = tid; i < M; i += nt) out[(int64_t)n * M + i] = -(double)Gnn[(int64_t)i * Mp + i].im * inv_pi;
        __syncthreads();
      }
    }
    if (!ok) flags |= KNIT_P_FALLBACK;
    // a problem the refined pass gave up on only records that; the FP64 pass
    // writes its outputs
    if (redo) flags |= KNIT_P_FALLBACK;
    if (redo || ok) {
      // non-finite check over the outputs
      double bad = 0.0;
      for (int64_t i = tid; i < (int64_t)L * M; i += nt) bad = fmax(bad, fabs(out[i]));
      if (bad != bad) bad = INFINITY;
      bad = wg_max_nan(bad, sv);
      if (!(bad <= 1.79e308)) flags |= KNIT_P_NONFINITE;
      if (flags & (KNIT_P_SINGULAR | KNIT_P_NONFINITE))
        for (int64_t i = tid; i < (int64_t)L * M; i += nt) out[i] = qnan;
    }
    if (tid == 0) pstatus[p] = flags;
    __syncthreads();
  }
}

// Y = V^+ Gm on the first `ncols` columns for a block-monomial V: row block
// vcol[a] of Y is vblk[a]^+ times row block a of Gm (each site of slice n-1
// receives from at most one site of slice n); other rows are zero.
template <class RS>
__device__ void scatter_vdag(cpx<RS> *Y, const cpx<RS> *Gm, const StripDev &s, int Mp, int ncols) {
  const int M = s.M, no = s.norb, W = M / no;
  for (int64_t i = threadIdx.x; i < (int64_t)Mp * Mp; i += blockDim.x) Y[i] = cpx<RS>{0, 0};
  __syncthreads();
  for (int64_t i = threadIdx.x; i < (int64_t)W * ncols; i += blockDim.x) {
    const int a = (int)(i / ncols), c = (int)(i % ncols), cb = s.vcol[a];
    if (cb < 0) continue;
    for (int ob = 0; ob < no; ++ob) {
      cpx<double> acc = {0.0, 0.0};
      for (int oa = 0; oa < no; ++oa)
        acc = c_fma(c_conj(vblk_at(s, a, oa, ob)), cvt<double>(Gm[(int64_t)(a * no + oa) * Mp + c]), acc);
      Y[(int64_t)(cb * no + ob) * Mp + c] = cvt<RS>(acc);
    }
  }
}

// Lesser Green function of injection from the left lead and its local
// observables (section 2.3: G_L^< = i G Gamma_L G^+; sections 5.3-D and 6:
// local densities, currents and spin accumulation), FP64, on the matrix
// cores, one workgroup per problem from the same queue as the sweep.  With
// Gamma_L = C_L C_L^+ (r columns), A_L = -i G_L^< = Q Q^+ where the slice
// blocks Q_n = G_{n1} C_L of the full Green function follow from
//   forward:  g_n = A_n^{-1},  N_1 = g_1 C_L,  N_n = g_n (V N_{n-1})
//             (N_n = g^L_{n1} C_L, left-connected; g_n and N_n kept every
//             `stride` slices as checkpoints),
//   reverse:  Q_L = N_L,  Q_n = N_n + g_n (V^+ Q_{n+1})   (Dyson's equation
//             across the cut between slices n and n+1), segment by segment
//             from the checkpoints.
// Per slice n and site s (orbitals o of s, k < r):
//   blk[n][s][o][o']  = sum_k Q_n[o,k] conj(Q_n[o',k])          (on-site block of A_L)
//   jtran[n][s]       = 2 Im sum_o sum_k (H0 Q_n)[o,k] conj(Q_n[o,k])  (inflow from slice n's other sites)
//   jlong[n+1][s]     = 2 Im sum_o sum_k (V Q_n)[o,k] conj(Q_{n+1}[o,k]) (inflow from slice n)
// (the on-site terms D_n and the diagonal blocks of H0 drop out of the
// imaginary parts: Tr of a product of two Hermitian matrices is real);
// jlong[0] = 0.  With full on-site matrices (onsite_dense) their inter-site
// terms join H0 in the transverse currents.  Slab (Mp^2 elements each): X,
// the slice Hamiltonian H_n padded, U, Qa, Qb, the segment's g and N
// [max(st, 2)] each, their checkpoints [ceil(Lmax / st)] each, V and V^+
// (used with a dense V, reserved in every slab), then the elimination scratch.
template <int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
lesser_mfma_kernel(StripTable tab, const knit_problem *probs, int P, const knit_z *onsite, const knit_z *sigmaL,
                   const knit_z *sigmaR, const knit_z *CL, const int *rows, int stride, knit_z *blk,
                   const int64_t *blk_off, double *jlong, double *jtran, int32_t *pstatus, char *ws,
                   size_t slab_bytes, int Mpmax, int Lmax, unsigned int *queue, const int *order, int outer) {
  using C = cpx<double>;
  __shared__ int next_p;
  __shared__ int q[NT], pinv[NT];
  __shared__ double sv[32];
  __shared__ int si[64];
  __shared__ C xchg[2 * 32];
  __shared__ C prow[32];
  __shared__ double rowv[512];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nw = nt >> 6, wave = tid >> 6, lane = tid & 63;
  const int64_t EE = (int64_t)Mpmax * Mpmax;
  const int segbuf = stride < 2 ? 2 : stride;
  const int nsegmax = (Lmax + stride - 1) / stride;
  char *slab = ws + (size_t)blockIdx.x * slab_bytes;
  C *X = reinterpret_cast<C *>(slab);
  C *H0p = X + EE, *U = H0p + EE, *Qa = U + EE, *Qb = Qa + EE;
  C *segg = Qb + EE;                               // [segbuf][Mp][Mp]
  C *segN = segg + (int64_t)segbuf * EE;           // [segbuf][Mp][Mp]
  C *cpg = segN + (int64_t)segbuf * EE;            // [nsegmax][Mp][Mp]
  C *cpN = cpg + (int64_t)nsegmax * EE;            // [nsegmax][Mp][Mp]
  C *Vd = cpN + (int64_t)nsegmax * EE, *Vh = Vd + EE;   // dense V only
  C *Sb = Vh + EE;                                 // [2 Mp][NO] scratch
  C *Sd = Sb + (int64_t)2 * Mpmax * NO_MAX;        // [NO][Mp]   scratch
  const double qnan = __builtin_nan("");
  for (;;) {
    if (tid == 0) next_p = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int pi = next_p;
    __syncthreads();
    if (pi >= P) break;
    const int p = order[pi];
    const knit_problem pr = probs[p];
    const StripDev s = tab.s[pr.strip];
    const int M = s.M, no = s.norb, W = M / no, L = pr.L;
    const int Mp = (M + MPAD - 1) / MPAD * MPAD;
    const int64_t E2 = (int64_t)Mp * Mp;
    const knit_z *sL = sigmaL + pr.sigma_off, *sR = sigmaR + pr.sigma_off;
    const int r = rows[p], rp = (r + MPAD - 1) / MPAD * MPAD;
    const int nseg = (L + stride - 1) / stride;
    const bool dense = s.V != nullptr;
    int flags = 0;
    for (int64_t i = tid; i < E2; i += nt) {
      const int a = (int)(i / Mp), b = (int)(i % Mp);
      H0p[i] = (a < M && b < M) ? ld_z(s.H0 + (int64_t)a * M + b) : C{0.0, 0.0};
    }
    if (dense) load_dense_v<double>(Vd, Vh, s, Mp);
    __syncthreads();
    // g_n and N_n (natural order) from g_{n-1} and N_{n-1}
    auto step = [&](int n, const C *gprev, const C *Nprev, C *gdst, C *Ndst) {
      const knit_z *D = onsite + pr.onsite_off + (int64_t)n * s.onsite_stride();
      form_blocks<double, false, false>(X, nullptr, s, Mp, pr.E, D, sL, sR, n == 0, n == L - 1,
                                        [=](int rr, int c) { return gprev[(int64_t)rr * Mp + c]; },
                                        [=](int rr, int c) { return C{0.0, 0.0}; }, -1, !dense);
      __syncthreads();
      if (dense && n > 0) dense_coupling<double, double, false>(X, nullptr, Vd, Vh, gprev, nullptr, U, Mp, 0);
      flags |= outer == 128 ? gj_two_level<double, NT, 128>(X, Mp, Mp, q, xchg, prow, sv, si, Sb, Sd)
                            : gj_two_level<double, NT, 64>(X, Mp, Mp, q, xchg, prow, sv, si, Sb, Sd);
      for (int i = tid; i < Mp; i += nt) pinv[q[i]] = i;
      __syncthreads();
      for (int64_t i = tid; i < E2; i += nt) {
        const int a = (int)(i / Mp), b = (int)(i % Mp);
        gdst[i] = X[(int64_t)q[a] * Mp + pinv[b]];
      }
      // U = C_L (slice 1) or V N_{n-1}, on rp columns
      if (n == 0) {
        for (int64_t i = tid; i < E2; i += nt) {
          const int a = (int)(i / Mp), c = (int)(i % Mp);
          U[i] = (a < M && c < r) ? ld_z(CL + pr.sigma_off + (int64_t)a * M + c) : C{0.0, 0.0};
        }
      } else if (dense) {
        gemm_lds<NT>(Mp, rp, Mp, Vd, Mp, Nprev, Mp, U, Mp, nullptr, 0);
      } else {
        gather_vg<double>(U, Nprev, s, Mp);
      }
      __syncthreads();
      gemm_lds<NT>(Mp, rp, Mp, gdst, Mp, U, Mp, Ndst, Mp, nullptr, 0);
      __syncthreads();
    };
    // per-row 2 Im sum_k Y[o,k] conj(Z[o,k]) summed over each site's orbitals into out[W]
    auto site_current = [&](const C *Y, const C *Z, double *out) {
      for (int o = wave; o < M; o += nw) {
        double acc = 0.0;
        for (int k = lane; k < r; k += 64) {
          const C y = Y[(int64_t)o * Mp + k], z = Z[(int64_t)o * Mp + k];
          acc += y.im * z.re - y.re * z.im;          // Im(y conj(z))
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) rowv[o] = 2.0 * acc;
      }
      __syncthreads();
      for (int a = tid; a < W; a += nt) {
        double v = 0.0;
        for (int o = 0; o < no; ++o) v += rowv[a * no + o];
        out[a] = v;
      }
      __syncthreads();
    };
    // forward pass: checkpoint k holds g and N of slice k st - 1 (k >= 1)
    {
      C *cg = segg, *pg = segg + E2, *cN = segN, *pN = segN + E2;
      for (int n = 0; n < L; ++n) {
        step(n, pg, pN, cg, cN);
        if ((n + 1) % stride == 0 && n + 1 < L) {
          const int64_t k = (n + 1) / stride;
          for (int64_t i = tid; i < E2; i += nt) {
            cpg[k * E2 + i] = cg[i];
            cpN[k * E2 + i] = cN[i];
          }
          __syncthreads();
        }
        C *t = cg; cg = pg; pg = t;
        t = cN; cN = pN; pN = t;
      }
    }
    // reverse pass, one segment at a time; Qn is Q_n, Qnext Q_{n+1}
    C *Qn = Qa, *Qnext = Qb;
    double *jl = jlong + pr.ldos_off, *jt = jtran + pr.ldos_off;
    knit_z *bo = blk + blk_off[p];
    for (int k = nseg - 1; k >= 0; --k) {
      const int n0 = k * stride, n1 = min(L, n0 + stride);
      for (int n = n0; n < n1; ++n) {
        const int64_t prevoff = (int64_t)(n - n0 - 1) * E2;
        const C *gprev = n == n0 ? (k > 0 ? cpg + (int64_t)k * E2 : segg) : segg + prevoff;
        const C *Nprev = n == n0 ? (k > 0 ? cpN + (int64_t)k * E2 : segN) : segN + prevoff;
        step(n, gprev, Nprev, segg + (int64_t)(n - n0) * E2, segN + (int64_t)(n - n0) * E2);
      }
      for (int n = n1 - 1; n >= n0; --n) {
        const C *g = segg + (int64_t)(n - n0) * E2, *N = segN + (int64_t)(n - n0) * E2;
        if (n == L - 1) {
          for (int64_t i = tid; i < E2; i += nt) Qn[i] = N[i];
        } else {
          // Q_n = N_n + g_n (V^+ Q_{n+1})
          if (dense)
            gemm_lds<NT>(Mp, rp, Mp, Vh, Mp, Qnext, Mp, U, Mp, nullptr, 0);
          else
            scatter_vdag<double>(U, Qnext, s, Mp, rp);
          __syncthreads();
          gemm_lds<NT>(Mp, rp, Mp, g, Mp, U, Mp, Qn, Mp, N, Mp);
        }
        __syncthreads();
        // on-site blocks of A_L = Q Q^+
        for (int e = wave; e < M * no; e += nw) {
          const int o = e / no, o2 = (o / no) * no + e % no;    // orbital o, partner o2 of the same site
          C acc = {0.0, 0.0};
          for (int kk = lane; kk < r; kk += 64)
            acc = c_fma(Qn[(int64_t)o * Mp + kk], c_conj(Qn[(int64_t)o2 * Mp + kk]), acc);
          for (int off = 32; off > 0; off >>= 1) {
            acc.re += __shfl_xor(acc.re, off, 64);
            acc.im += __shfl_xor(acc.im, off, 64);
          }
          if (lane == 0) st_z(bo + (int64_t)n * M * no + e, acc);
        }
        // inflow into slice n+1 from slice n: 2 Im (V Q_n) . conj(Q_{n+1})
        if (n < L - 1) {
          if (dense)
            gemm_lds<NT>(Mp, rp, Mp, Vd, Mp, Qn, Mp, U, Mp, nullptr, 0);
          else
            gather_vg<double>(U, Qn, s, Mp);
          __syncthreads();
          site_current(U, Qnext, jl + (int64_t)(n + 1) * W);
        } else {
          __syncthreads();
        }
        // inflow from the other sites of slice n: 2 Im (H_n Q_n) . conj(Q_n); the site
        // blocks of H_n drop out, so H0 serves unless the on-site terms are full matrices
        if (s.onsite_dense) {
          const knit_z *D = onsite + pr.onsite_off + (int64_t)n * s.onsite_stride();
          for (int64_t i = tid; i < E2; i += nt) {
            const int a = (int)(i / Mp), b = (int)(i % Mp);
            C h = {0.0, 0.0};
            if (a < M && b < M) {
              const C h0 = ld_z(s.H0 + (int64_t)a * M + b), d = ld_z(D + (int64_t)a * M + b);
              h = C{h0.re + d.re, h0.im + d.im};
            }
            H0p[i] = h;
          }
          __syncthreads();
        }
        gemm_lds<NT>(Mp, rp, Mp, H0p, Mp, Qn, Mp, U, Mp, nullptr, 0);
        __syncthreads();
        site_current(U, Qn, jt + (int64_t)n * W);
        C *t = Qn; Qn = Qnext; Qnext = t;
      }
    }
    for (int a = tid; a < W; a += nt) jl[a] = 0.0;
    // non-finite check over the outputs
    double bad = 0.0;
    for (int64_t i = tid; i < (int64_t)L * W; i += nt) bad = fmax(bad, fabs(jl[i]) + fabs(jt[i]));
    for (int64_t i = tid; i < (int64_t)L * M * no; i += nt) bad = fmax(bad, fabs(bo[i].re) + fabs(bo[i].im));
    if (bad != bad) bad = INFINITY;
    bad = wg_max_nan(bad, sv);
    if (!(bad <= 1.79e308)) flags |= KNIT_P_NONFINITE;
    if (flags & (KNIT_P_SINGULAR | KNIT_P_NONFINITE)) {
      for (int64_t i = tid; i < (int64_t)L * W; i += nt) jl[i] = jt[i] = qnan;
      for (int64_t i = tid; i < (int64_t)L * M * no; i += nt) st_z(bo + i, C{qnan, qnan});
    }
    if (tid == 0) pstatus[p] = flags;
    __syncthreads();
  }
}

// The reverse coupling of the right-connected recursion, X -= V^+ gR V, for a
// block-monomial V: site block (b, b') receives vblk[a]^+ gR[a, a'] vblk[a']
// with a, a' the sites bonded to b, b' (inv = the inverse of vcol, -1 where
// none).  gR natural order, [Mp][Mp].  One site block per thread.
template <class RS>
__device__ void reverse_coupling_blocks(cpx<double> *X, const StripDev &s, const int *inv, const cpx<RS> *gR,
                                        int Mp) {
  const int no = s.norb, W = s.M / no;
  for (int blk = threadIdx.x; blk < W * W; blk += blockDim.x) {
    const int b = blk / W, b2 = blk % W;
    const int a = inv[b], a2 = inv[b2];
    if (a < 0 || a2 < 0) continue;
    for (int ob = 0; ob < no; ++ob)
      for (int ob2 = 0; ob2 < no; ++ob2) {
        cpx<double> acc = {0.0, 0.0};
        for (int i = 0; i < no; ++i) {
          cpx<double> inner = {0.0, 0.0};
          for (int j = 0; j < no; ++j)
            inner = c_fma(cvt<double>(gR[(int64_t)(a * no + i) * Mp + a2 * no + j]), vblk_at(s, a2, j, ob2), inner);
          acc = c_fma(c_conj(vblk_at(s, a, i, ob)), inner, acc);
        }
        cpx<double> &x = X[(int64_t)(b * no + ob) * Mp + b2 * no + ob2];
        x = cpx<double>{x.re - acc.re, x.im - acc.im};
      }
  }
}

// Y = Gm V on the first `nrows` rows for a block-monomial V: column block b of Y
// is column block inv[b] of Gm times vblk[inv[b]] (zero where inv[b] < 0).
template <class RS>
__device__ void right_mul_v_blocks(cpx<RS> *Y, const cpx<RS> *Gm, const StripDev &s, const int *inv, int Mp,
                                   int nrows) {
  const int M = s.M, no = s.norb;
  for (int64_t i = threadIdx.x; i < (int64_t)nrows * Mp; i += blockDim.x) {
    const int r = (int)(i / Mp), c = (int)(i % Mp);
    cpx<double> acc = {0.0, 0.0};
    if (c < M) {
      const int b = c / no, ob = c % no, a = inv[b];
      if (a >= 0)
        for (int oa = 0; oa < no; ++oa)
          acc = c_fma(cvt<double>(Gm[(int64_t)r * Mp + a * no + oa]), vblk_at(s, a, oa, ob), acc);
    }
    Y[i] = cvt<RS>(acc);
  }
}

constexpr int MT_MAX_LEADS = 8;   // left, right and up to six side leads

// Conductance matrix of a strip with leads on several slices (section 2.3,
// T_kl = Tr[Gamma_k G_kl Gamma_l G_kl^+]; section 6.1, the conductance matrix),
// FP64, one workgroup per problem.  Lead 0 is the left lead (slice 0, Sigma_L,
// C_L), lead 1 the right lead (slice L-1, Sigma_R, C_R), leads 2.. are the side
// leads of the call (slice, Sigma_k = sigmaX + off, C_k = CX + off), every
// Gamma_k = C_k C_k^+.  With A_n the local slice matrix (E - H_n minus every
// self-energy attached to slice n):
//   forward:  left-connected g^L_n = (A_n - V g^L_{n-1} V^+)^{-1}, checkpoints;
//   reverse:  right-connected g^R_n = (A_n - V^+ g^R_{n+1} V)^{-1}; at a slice
//             hosting leads the full block
//             G_nn = (A_n - V g^L_{n-1} V^+ - V^+ g^R_{n+1} V)^{-1};
//             each lead l at slice n starts its column Y_l = G_nn C_l and row
//             R_l = C_l^+ G_nn, which move one slice down per step by Dyson's
//             equation across the cut (n-1 | n):
//               Y_l <- g^L_{n-1} V^+ Y_l     (= G_{n-1, s_l} C_l)
//               R_k <- R_k V g^L_{n-1}       (= C_k^+ G_{s_k, n-1});
//   T_kl      = || C_k^+ Y_l ||_F^2 when the sweep reaches s_k <= s_l,
//             = || R_k C_l ||_F^2   when it reaches s_l <  s_k.
// Slab (Mp^2 elements each): X, U, U2, gRa, gRb, Gnn, C (one lead's factor,
// padded), Y[K], R[K], the segment's g^L [max(st, 2)], checkpoints
// [ceil(Lmax / st)], V, V^+, then the elimination scratch.
template <int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
multiterminal_mfma_kernel(StripTable tab, const knit_problem *probs, int P, const knit_z *onsite,
                          const knit_z *sigmaL, const knit_z *sigmaR, const knit_z *CL, const knit_z *CR,
                          int n_side, const knit_lead *side, const knit_z *sigmaX, const knit_z *CX, int stride,
                          double *Tout, int32_t *pstatus, char *ws, size_t slab_bytes, int Mpmax, int Lmax,
                          unsigned int *queue, const int *order, int outer) {
  using C = cpx<double>;
  __shared__ int next_p;
  __shared__ int q[NT], pinv[NT];
  __shared__ int vinv[NT];
  __shared__ double sv[32];
  __shared__ int si[64];
  __shared__ C xchg[2 * 32];
  __shared__ C prow[32];
  __shared__ int lslice[MT_MAX_LEADS], lrank[MT_MAX_LEADS];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int K = n_side + 2;
  const int64_t EE = (int64_t)Mpmax * Mpmax;
  const int segbuf = stride < 2 ? 2 : stride;
  const int nsegmax = (Lmax + stride - 1) / stride;
  char *slab = ws + (size_t)blockIdx.x * slab_bytes;
  C *X = reinterpret_cast<C *>(slab);
  C *U = X + EE, *U2 = U + EE, *gRa = U2 + EE, *gRb = gRa + EE, *Gnn = gRb + EE, *Cb = Gnn + EE;
  C *Yb = Cb + EE;                                  // [K][Mp][Mp]
  C *Rb = Yb + (int64_t)K * EE;                     // [K][Mp][Mp]
  C *segg = Rb + (int64_t)K * EE;                   // [segbuf][Mp][Mp]
  C *cpg = segg + (int64_t)segbuf * EE;             // [nsegmax][Mp][Mp]
  C *Vd = cpg + (int64_t)nsegmax * EE, *Vh = Vd + EE;
  C *Sb = Vh + EE;                                  // [2 Mp][NO] scratch
  C *Sd = Sb + (int64_t)2 * Mpmax * NO_MAX;         // [NO][Mp]   scratch
  const double qnan = __builtin_nan("");
  for (;;) {
    if (tid == 0) next_p = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int pi = next_p;
    __syncthreads();
    if (pi >= P) break;
    const int p = order[pi];
    const knit_problem pr = probs[p];
    const StripDev s = tab.s[pr.strip];
    const int M = s.M, no = s.norb, W = M / no, L = pr.L;
    const int Mp = (M + MPAD - 1) / MPAD * MPAD;
    const int64_t E2 = (int64_t)Mp * Mp;
    const knit_z *sL = sigmaL + pr.sigma_off, *sR = sigmaR + pr.sigma_off;
    const knit_lead *sd = side + (int64_t)p * n_side;
    const bool dense = s.V != nullptr;
    const int nseg = (L + stride - 1) / stride;
    int flags = 0;
    // factor of lead k (device, [M][M], row stride M)
    auto factor = [&](int k) -> const knit_z * {
      return k == 0 ? CL + pr.sigma_off : (k == 1 ? CR + pr.sigma_off : CX + sd[k - 2].sigma_off);
    };
    // lead slices, ranks (columns of C up to the last nonzero one), vcol inverse, V
    if (tid < K) lslice[tid] = tid == 0 ? 0 : (tid == 1 ? L - 1 : min(max(sd[tid - 2].slice, 0), L - 1));
    for (int k = 0; k < K; ++k) {
      const int r = factor_columns(factor(k), M, sv);
      if (tid == 0) lrank[k] = r < M ? r : M;
    }
    if (!dense) {
      for (int b = tid; b < W; b += nt) vinv[b] = -1;
      __syncthreads();
      for (int a = tid; a < W; a += nt)
        if (s.vcol[a] >= 0) vinv[s.vcol[a]] = a;
    } else {
      load_dense_v<double>(Vd, Vh, s, Mp);
    }
    __syncthreads();
    // local slice matrix of slice n into X (natural order): E - H_n - the self-energies
    // attached to it, plus the forward coupling with gl (g^L_{n-1}, or null) and the
    // reverse coupling with gr (g^R_{n+1}, or null)
    auto assemble = [&](int n, const C *gl, const C *gr) {
      const knit_z *D = onsite + pr.onsite_off + (int64_t)n * s.onsite_stride();
      form_blocks<double, false, false>(X, nullptr, s, Mp, pr.E, D, sL, sR, n == 0, n == L - 1,
                                        [=](int rr, int c) { return gl[(int64_t)rr * Mp + c]; },
                                        [=](int rr, int c) { return C{0.0, 0.0}; }, -1, gl != nullptr && !dense);
      __syncthreads();
      for (int k = 2; k < K; ++k) {
        if (lslice[k] != n) continue;
        const knit_z *sg = sigmaX + sd[k - 2].sigma_off;
        for (int64_t i = tid; i < (int64_t)M * M; i += nt) {
          const int a = (int)(i / M), b = (int)(i % M);
          const C v = ld_z(sg + i);
          C &x = X[(int64_t)a * Mp + b];
          x = C{x.re - v.re, x.im - v.im};
        }
        __syncthreads();
      }
      if (dense && gl) dense_coupling<double, double, false>(X, nullptr, Vd, Vh, gl, nullptr, U, Mp, 0);
      if (gr) {
        if (dense) {
          // X -= V^+ (gR V)
          gemm_lds<NT>(Mp, Mp, Mp, gr, Mp, Vd, Mp, U, Mp, nullptr, 0);
          __syncthreads();
          wg_gemm_mfma<double>(Mp, Mp, Mp, Vh, Mp, U, Mp, [&](int rr, int c, double &re, double &im) {
            C &x = X[(int64_t)rr * Mp + c];
            x = C{x.re - re, x.im - im};
          });
        } else {
          reverse_coupling_blocks<double>(X, s, vinv, gr, Mp);
        }
        __syncthreads();
      }
    };
    // inverse of the assembled X into dst (natural order)
    auto invert = [&](C *dst) {
      flags |= outer == 128 ? gj_two_level<double, NT, 128>(X, Mp, Mp, q, xchg, prow, sv, si, Sb, Sd)
                            : gj_two_level<double, NT, 64>(X, Mp, Mp, q, xchg, prow, sv, si, Sb, Sd);
      for (int i = tid; i < Mp; i += nt) pinv[q[i]] = i;
      __syncthreads();
      for (int64_t i = tid; i < E2; i += nt) {
        const int a = (int)(i / Mp), b = (int)(i % Mp);
        dst[i] = X[(int64_t)q[a] * Mp + pinv[b]];
      }
      __syncthreads();
    };
    // lead k's factor, padded: Cb[a][c] = C_k[a][c] (cols < rank), or its adjoint
    auto load_factor = [&](int k, bool adjoint) {
      const knit_z *Ck = factor(k);
      const int r = lrank[k];
      for (int64_t i = tid; i < E2; i += nt) {
        const int a = (int)(i / Mp), c = (int)(i % Mp);
        C v = {0.0, 0.0};
        if (!adjoint && a < M && c < r) v = ld_z(Ck + (int64_t)a * M + c);
        if (adjoint && c < M && a < r) {
          const C w = ld_z(Ck + (int64_t)c * M + a);
          v = C{w.re, -w.im};
        }
        Cb[i] = v;
      }
      __syncthreads();
    };
    auto rp_of = [&](int k) { return (lrank[k] + MPAD - 1) / MPAD * MPAD; };
    // || A B ||_F^2 with A [ra][Mp] and B [Mp][rb] (both padded)
    auto frob_product = [&](const C *A, int ra, const C *B, int rb) -> double {
      double ss = 0.0;
      wg_gemm_mfma<double>(ra, rb, Mp, A, Mp, B, Mp, [&](int rr, int c, double &re, double &im) {
        ss += re * re + im * im;
      });
      __syncthreads();
      double t = ss;
      for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
      if ((tid & 63) == 0) sv[tid >> 6] = t;
      __syncthreads();
      double tot = 0.0;
      for (int w = 0; w < (nt >> 6); ++w) tot += sv[w];
      __syncthreads();
      return tot;
    };
    double *Tp = Tout + (int64_t)p * K * K;
    // ---- forward: left-connected g^L_n, checkpoint k holds g^L of slice k st - 1
    {
      C *cur = segg, *prev = segg + E2;
      for (int n = 0; n < L; ++n) {
        assemble(n, n > 0 ? prev : nullptr, nullptr);
        invert(cur);
        if ((n + 1) % stride == 0 && n + 1 < L) {
          C *cp = cpg + (int64_t)((n + 1) / stride) * E2;
          for (int64_t i = tid; i < E2; i += nt) cp[i] = cur[i];
          __syncthreads();
        }
        C *t = cur; cur = prev; prev = t;
      }
    }
    // ---- reverse
    C *gR = gRa, *gRn = gRb;     // g^R_{n+1} and the one being formed
    bool have_gR = false;
    for (int kseg = nseg - 1; kseg >= 0; --kseg) {
      const int n0 = kseg * stride, n1 = min(L, n0 + stride);
      // g^L of the segment (slot j holds slice n0 + j)
      for (int n = n0; n < n1; ++n) {
        const C *gprev = n == n0 ? (kseg > 0 ? cpg + (int64_t)kseg * E2 : nullptr) : segg + (int64_t)(n - n0 - 1) * E2;
        assemble(n, n > 0 ? gprev : nullptr, nullptr);
        invert(segg + (int64_t)(n - n0) * E2);
      }
      for (int n = n1 - 1; n >= n0; --n) {
        const C *gl_prev = n > n0 ? segg + (int64_t)(n - n0 - 1) * E2 : (kseg > 0 ? cpg + (int64_t)kseg * E2 : nullptr);
        bool here = false;
        for (int k = 0; k < K; ++k) here = here || lslice[k] == n;
        if (here) {
          // full diagonal block and the leads attached here
          assemble(n, n > 0 ? gl_prev : nullptr, have_gR ? gR : nullptr);
          invert(Gnn);
          for (int k = 0; k < K; ++k) {
            if (lslice[k] != n) continue;
            const int rp = rp_of(k);
            load_factor(k, false);
            gemm_lds<NT>(Mp, rp, Mp, Gnn, Mp, Cb, Mp, Yb + (int64_t)k * EE, Mp, nullptr, 0);
            __syncthreads();
            load_factor(k, true);
            gemm_lds<NT>(rp, Mp, Mp, Cb, Mp, Gnn, Mp, Rb + (int64_t)k * EE, Mp, nullptr, 0);
            __syncthreads();
          }
          // transmissions whose lower slice is n
          for (int k = 0; k < K; ++k)
            for (int l = 0; l < K; ++l) {
              const int sk = lslice[k], sl = lslice[l];
              if (min(sk, sl) != n) continue;
              double t;
              if (sk == n) {                                   // sink here: || C_k^+ Y_l ||^2
                load_factor(k, true);
                t = frob_product(Cb, rp_of(k), Yb + (int64_t)l * EE, rp_of(l));
              } else {                                         // source here, sink above: || R_k C_l ||^2
                load_factor(l, false);
                t = frob_product(Rb + (int64_t)k * EE, rp_of(k), Cb, rp_of(l));
              }
              if (tid == 0) Tp[k * K + l] = t;
            }
        }
        // right-connected g^R_n for the next slice down (not needed below slice 0)
        if (n > 0) {
          assemble(n, nullptr, have_gR ? gR : nullptr);
          invert(gRn);
          C *t = gR; gR = gRn; gRn = t;
          have_gR = true;
          // move the active columns and rows down to slice n-1 with g^L_{n-1}
          const C *gl = gl_prev;
          for (int k = 0; k < K; ++k) {
            if (lslice[k] < n) continue;
            const int rp = rp_of(k);
            C *Y = Yb + (int64_t)k * EE, *R = Rb + (int64_t)k * EE;
            // Y <- g^L_{n-1} (V^+ Y)
            if (dense)
              gemm_lds<NT>(Mp, rp, Mp, Vh, Mp, Y, Mp, U, Mp, nullptr, 0);
            else
              scatter_vdag<double>(U, Y, s, Mp, rp);
            __syncthreads();
            gemm_lds<NT>(Mp, rp, Mp, gl, Mp, U, Mp, Y, Mp, nullptr, 0);
            __syncthreads();
            // R <- (R V) g^L_{n-1}
            if (dense)
              gemm_lds<NT>(rp, Mp, Mp, R, Mp, Vd, Mp, U2, Mp, nullptr, 0);
            else
              right_mul_v_blocks<double>(U2, R, s, vinv, Mp, rp);
            __syncthreads();
            gemm_lds<NT>(rp, Mp, Mp, U2, Mp, gl, Mp, R, Mp, nullptr, 0);
            __syncthreads();
          }
        }
      }
    }
    // non-finite check
    double bad = 0.0;
    for (int i = tid; i < K * K; i += nt) bad = fmax(bad, fabs(Tp[i]));
    if (bad != bad) bad = INFINITY;
    bad = wg_max_nan(bad, sv);
    if (!(bad <= 1.79e308)) flags |= KNIT_P_NONFINITE;
    if (flags & (KNIT_P_SINGULAR | KNIT_P_NONFINITE))
      for (int i = tid; i < K * K; i += nt) Tp[i] = qnan;
    if (tid == 0) pstatus[p] = flags;
    __syncthreads();
  }
}

}  // namespace

int mfma_padded(int M) { return (M + MPAD - 1) / MPAD * MPAD; }

static size_t order_bytes(int P) { return (((size_t)P * sizeof(int)) + 255) & ~size_t(255); }

size_t sweep_mfma_slab_bytes(int Mmax, int precision, bool dense) {
  const size_t Mp = (size_t)mfma_padded(Mmax);
  const size_t EE = Mp * Mp;
  const size_t gs = precision == KNIT_FP64 ? 16 : 8;     // elimination element size
  const size_t ss = precision == KNIT_FP32 ? 8 : 16;     // kept state element size
  size_t b = dense ? 3 * EE * ss : 0;                    // V, V^+, V g

  if (precision == KNIT_FP64) b += EE * (4 * 16 + 4 * 16);
  else if (precision == KNIT_FP32) b += EE * (4 * 8 + 4 * 8);
  else b += EE * (2 * 8 + 4 * 16 + 16 + 16 + 8 + 8);   // Xa, Xb (Mp rows); g, G1, N1a, N1b; A64; Tb; Xn; Rr
  b += (2 * Mp * NO_MAX + NO_MAX * Mp) * gs;              // Sb, Sd scratch
  return (b + 255) & ~size_t(255);
}

bool sweep_mfma_supports(int Mmax) { return mfma_padded(Mmax) <= 512; }

size_t ldos_mfma_slab_bytes(int Mmax, int Lmax, int stride, int precision, bool dense) {
  const size_t Mp = (size_t)mfma_padded(Mmax);
  const size_t EE = Mp * Mp;
  const size_t gs = precision == KNIT_FP64 ? 16 : 8;                   // elimination element
  const size_t ss = precision == KNIT_FP32 ? 8 : 16;                   // kept state element
  const size_t segbuf = stride < 2 ? 2 : stride;
  const size_t nseg = (Lmax + stride - 1) / stride;
  size_t b = EE * gs + (4 + segbuf + nseg) * EE * ss + (2 * Mp * NO_MAX + NO_MAX * Mp) * gs;
  if (precision == KNIT_FP32_REFINE) b += EE * (16 + 8 + 8);            // A_n, X0, R
  if (dense) b += 2 * EE * ss;                                          // V, V^+
  return (b + 255) & ~size_t(255);
}

// The refined call's second (FP64) pass shares the workspace.
static size_t ldos_slab_for(int Mmax, int Lmax, int stride, int precision, bool dense) {
  size_t s = ldos_mfma_slab_bytes(Mmax, Lmax, stride, precision, dense);
  if (precision == KNIT_FP32_REFINE) {
    const size_t s64 = ldos_mfma_slab_bytes(Mmax, Lmax, stride, KNIT_FP64, dense);
    if (s64 > s) s = s64;
  }
  return s;
}

size_t ldos_mfma_workspace(int Mmax, int Lmax, int stride, int precision, int P, bool dense) {
  const int grid = P < SWEEP_MAX_GRID ? P : SWEEP_MAX_GRID;
  return 256 + order_bytes(P) + ldos_slab_for(Mmax, Lmax, stride, precision, dense) * (size_t)grid;
}

bool table_has_dense(const StripTable &tab) {
  for (int i = 0; i < tab.n; ++i)
    if (tab.s[i].V) return true;
  return false;
}

hipError_t launch_ldos_mfma(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                            const knit_z *sigmaL, const knit_z *sigmaR, int precision, int stride, double *ldos,
                            int32_t *pstatus, void *ws, int Mmax, int Lmax, hipStream_t stream) {
  unsigned int *queue = reinterpret_cast<unsigned int *>(ws);
  int *order = reinterpret_cast<int *>(reinterpret_cast<char *>(ws) + 256);
  char *w = reinterpret_cast<char *>(ws) + 256 + order_bytes(P);
  const int Mpmax = mfma_padded(Mmax);
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  const double rtol = sweep_get_refine_threshold();
  auto pass = [&](int prec, const int32_t *redo) -> hipError_t {
    const knit_sweep_tuning tune = sweep_tuning_get(prec, Mpmax);
    const size_t slab = ldos_mfma_slab_bytes(Mmax, Lmax, stride, prec, table_has_dense(tab));
    int grid = tune.wg_per_cu * ncu;
    if (grid > SWEEP_MAX_GRID) grid = SWEEP_MAX_GRID;
    if (grid > P) grid = P;
    hipLaunchKernelGGL(order_kernel, dim3(1), dim3(1024), 0, stream, tab, probs, P, tune.order, (const int *)nullptr,
                       order, queue);
#define KNIT_LAUNCH(RG, RS, RF, NT)                                                                            \
  hipLaunchKernelGGL((ldos_mfma_kernel<RG, RS, RF, NT>), dim3(grid), dim3(NT), 0, stream, tab, probs, P, onsite,   \
                     sigmaL, sigmaR, stride, ldos, pstatus, w, slab, Mpmax, Lmax, queue, order, tune.outer, rtol,  \
                     redo)
    const bool small = tune.threads == 256;
    if (prec == KNIT_FP64) {
      if (small) KNIT_LAUNCH(double, double, false, 256); else KNIT_LAUNCH(double, double, false, 512);
    } else if (prec == KNIT_FP32) {
      if (small) KNIT_LAUNCH(float, float, false, 256); else KNIT_LAUNCH(float, float, false, 512);
    } else {
      if (small) KNIT_LAUNCH(float, double, true, 256); else KNIT_LAUNCH(float, double, true, 512);
    }
#undef KNIT_LAUNCH
    return hipGetLastError();
  };
  hipError_t err = pass(precision, nullptr);
  if (err != hipSuccess || precision != KNIT_FP32_REFINE) return err;
  return pass(KNIT_FP64, pstatus);
}

size_t lesser_mfma_slab_bytes(int Mmax, int Lmax, int stride, bool dense) {
  const size_t Mp = (size_t)mfma_padded(Mmax);
  const size_t EE = Mp * Mp;
  const size_t segbuf = stride < 2 ? 2 : stride;
  const size_t nseg = (Lmax + stride - 1) / stride;
  (void)dense;   // V and V^+ sit before the elimination scratch in every slab
  size_t b = (7 + 2 * segbuf + 2 * nseg) * EE * 16 + (2 * Mp * NO_MAX + NO_MAX * Mp) * 16;
  return (b + 255) & ~size_t(255);
}

size_t lesser_mfma_workspace(int Mmax, int Lmax, int stride, int P, bool dense) {
  const int grid = P < SWEEP_MAX_GRID ? P : SWEEP_MAX_GRID;
  return 256 + 2 * order_bytes(P) + lesser_mfma_slab_bytes(Mmax, Lmax, stride, dense) * (size_t)grid;
}

hipError_t launch_lesser_mfma(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                              const knit_z *sigmaL, const knit_z *sigmaR, const knit_z *CL, int stride,
                              knit_z *blk, const int64_t *blk_off, double *jlong, double *jtran, int32_t *pstatus,
                              void *ws, int Mmax, int Lmax, hipStream_t stream) {
  unsigned int *queue = reinterpret_cast<unsigned int *>(ws);
  int *order = reinterpret_cast<int *>(reinterpret_cast<char *>(ws) + 256);
  int *rows = reinterpret_cast<int *>(reinterpret_cast<char *>(ws) + 256 + order_bytes(P));
  char *w = reinterpret_cast<char *>(ws) + 256 + 2 * order_bytes(P);
  const int Mpmax = mfma_padded(Mmax);
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  const knit_sweep_tuning tune = sweep_tuning_get(KNIT_FP64, Mpmax);
  const size_t slab = lesser_mfma_slab_bytes(Mmax, Lmax, stride, table_has_dense(tab));
  int grid = tune.wg_per_cu * ncu;
  if (grid > SWEEP_MAX_GRID) grid = SWEEP_MAX_GRID;
  if (grid > P) grid = P;
  hipLaunchKernelGGL(proj_rows_kernel, dim3(P), dim3(256), 0, stream, tab, probs, P, CL, rows);
  hipLaunchKernelGGL(order_kernel, dim3(1), dim3(1024), 0, stream, tab, probs, P, tune.order, (const int *)rows,
                     order, queue);
  if (tune.threads == 256)
    hipLaunchKernelGGL(lesser_mfma_kernel<256>, dim3(grid), dim3(256), 0, stream, tab, probs, P, onsite, sigmaL,
                       sigmaR, CL, (const int *)rows, stride, blk, blk_off, jlong, jtran, pstatus, w, slab, Mpmax,
                       Lmax, queue, order, tune.outer);
  else
    hipLaunchKernelGGL(lesser_mfma_kernel<512>, dim3(grid), dim3(512), 0, stream, tab, probs, P, onsite, sigmaL,
                       sigmaR, CL, (const int *)rows, stride, blk, blk_off, jlong, jtran, pstatus, w, slab, Mpmax,
                       Lmax, queue, order, tune.outer);
  return hipGetLastError();
}

size_t multiterminal_mfma_slab_bytes(int Mmax, int Lmax, int stride, int n_side) {
  const size_t Mp = (size_t)mfma_padded(Mmax);
  const size_t EE = Mp * Mp;
  const size_t segbuf = stride < 2 ? 2 : stride;
  const size_t nseg = (Lmax + stride - 1) / stride;
  const size_t K = (size_t)n_side + 2;
  size_t b = (7 + 2 * K + segbuf + nseg + 2) * EE * 16 + (2 * Mp * NO_MAX + NO_MAX * Mp) * 16;
  return (b + 255) & ~size_t(255);
}

size_t multiterminal_mfma_workspace(int Mmax, int Lmax, int stride, int n_side, int P) {
  const int grid = P < SWEEP_MAX_GRID ? P : SWEEP_MAX_GRID;
  return 256 + order_bytes(P) + multiterminal_mfma_slab_bytes(Mmax, Lmax, stride, n_side) * (size_t)grid;
}

hipError_t launch_multiterminal_mfma(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                                     const knit_z *sigmaL, const knit_z *sigmaR, const knit_z *CL, const knit_z *CR,
                                     int n_side, const knit_lead *side, const knit_z *sigmaX, const knit_z *CX,
                                     int stride, double *T, int32_t *pstatus, void *ws, int Mmax, int Lmax,
                                     hipStream_t stream) {
  unsigned int *queue = reinterpret_cast<unsigned int *>(ws);
  int *order = reinterpret_cast<int *>(reinterpret_cast<char *>(ws) + 256);
  char *w = reinterpret_cast<char *>(ws) + 256 + order_bytes(P);
  const int Mpmax = mfma_padded(Mmax);
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  const knit_sweep_tuning tune = sweep_tuning_get(KNIT_FP64, Mpmax);
  const size_t slab = multiterminal_mfma_slab_bytes(Mmax, Lmax, stride, n_side);
  int grid = tune.wg_per_cu * ncu;
  if (grid > SWEEP_MAX_GRID) grid = SWEEP_MAX_GRID;
  if (grid > P) grid = P;
  hipLaunchKernelGGL(order_kernel, dim3(1), dim3(1024), 0, stream, tab, probs, P, tune.order, (const int *)nullptr,
                     order, queue);
  if (tune.threads == 256)
    hipLaunchKernelGGL(multiterminal_mfma_kernel<256>, dim3(grid), dim3(256), 0, stream, tab, probs, P, onsite,
                       sigmaL, sigmaR, CL, CR, n_side, side, sigmaX, CX, stride, T, pstatus, w, slab, Mpmax, Lmax,
                       queue, order, tune.outer);
  else
    hipLaunchKernelGGL(multiterminal_mfma_kernel<512>, dim3(grid), dim3(512), 0, stream, tab, probs, P, onsite,
                       sigmaL, sigmaR, CL, CR, n_side, side, sigmaX, CX, stride, T, pstatus, w, slab, Mpmax, Lmax,
                       queue, order, tune.outer);
  return hipGetLastError();
}

hipError_t launch_sweep_projected(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                                  const knit_z *sigmaL, const knit_z *sigmaR, const knit_z *CL, int precision,
                                  knit_z *G1Np, knit_z *GNN, int32_t *pstatus, void *ws, int Mmax, int max_grid,
                                  hipStream_t stream) {
  unsigned int *queue = reinterpret_cast<unsigned int *>(ws);
  int *order = reinterpret_cast<int *>(reinterpret_cast<char *>(ws) + 256);
  int *rows = reinterpret_cast<int *>(reinterpret_cast<char *>(ws) + 256 + order_bytes(P));
  char *w = reinterpret_cast<char *>(ws) + 256 + 2 * order_bytes(P);
  const int Mpmax = mfma_padded(Mmax);
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  const double rtol = sweep_get_refine_threshold();
  hipLaunchKernelGGL(proj_rows_kernel, dim3(P), dim3(256), 0, stream, tab, probs, P, CL, rows);
  // one pass at `prec`; redo != NULL restricts it to the problems flagged KNIT_P_FALLBACK
  auto pass = [&](int prec, const int32_t *redo) -> hipError_t {
    const knit_sweep_tuning tune = sweep_tuning_get(prec, Mpmax);
    const size_t slab = sweep_mfma_slab_bytes(Mmax, prec, table_has_dense(tab));
    int grid = tune.wg_per_cu * ncu;
    if (grid > SWEEP_MAX_GRID) grid = SWEEP_MAX_GRID;
    if (max_grid > 0 && grid > max_grid) grid = max_grid;
    if (grid > P) grid = P;
    hipLaunchKernelGGL(order_kernel, dim3(1), dim3(1024), 0, stream, tab, probs, P, tune.order, (const int *)rows,
                       order, queue);
#define KNIT_LAUNCH(RG, RS, RF, NT)                                                                            \
  hipLaunchKernelGGL((sweep_mfma_kernel<RG, RS, RF, NT, true>), dim3(grid), dim3(NT), 0, stream, tab, probs, P,     \
                     onsite, sigmaL, sigmaR, G1Np, (knit_z *)nullptr, GNN, pstatus, w, slab, Mpmax, queue, order,  \
                     rtol, redo, tune.outer, CL, rows)
    const bool small = tune.threads == 256;
    if (prec == KNIT_FP64) {
      if (small) KNIT_LAUNCH(double, double, false, 256); else KNIT_LAUNCH(double, double, false, 512);
    } else if (prec == KNIT_FP32) {
      if (small) KNIT_LAUNCH(float, float, false, 256); else KNIT_LAUNCH(float, float, false, 512);
    } else {
      if (small) KNIT_LAUNCH(float, double, true, 256); else KNIT_LAUNCH(float, double, true, 512);
    }
#undef KNIT_LAUNCH
    return hipGetLastError();
  };
  hipError_t err = pass(precision, nullptr);
  if (err != hipSuccess || precision != KNIT_FP32_REFINE) return err;
  return pass(KNIT_FP64, pstatus);
}

size_t inverse_fp64_scratch_elems(int M) {
  const size_t Mp = (size_t)mfma_padded(M);
  return 2 * Mp * NO_MAX + NO_MAX * Mp;
}

hipError_t launch_inverse_fp64(cpx<double> *X, int64_t xstride, cpx<double> *scratch, int64_t sstride, int M,
                               cpx<double> *out, int64_t ostride, const int32_t *skip, int skip_stride,
                               int32_t *flags, int flags_stride, int n, hipStream_t stream) {
  const int Mp = mfma_padded(M);
  if (Mp > 512) return hipErrorInvalidValue;
  if (n <= 0) return hipSuccess;
  if (Mp <= 256)
    hipLaunchKernelGGL(inverse_fp64_kernel<256>, dim3(n), dim3(256), 0, stream, X, xstride, scratch, sstride, M,
                       Mp, out, ostride, skip, skip_stride, flags, flags_stride);
  else
    hipLaunchKernelGGL(inverse_fp64_kernel<512>, dim3(n), dim3(512), 0, stream, X, xstride, scratch, sstride, M,
                       Mp, out, ostride, skip, skip_stride, flags, flags_stride);
  return hipGetLastError();
}

// Workspace: a 256-byte header (queue counter), the queue order [P] and the
// projected rows [P] (each padded to 256 bytes), then one slab per workgroup.

// The refined sweep's second (FP64) pass shares the workspace.
static size_t slab_for(int Mmax, int precision, bool dense) {
  size_t s = sweep_mfma_slab_bytes(Mmax, precision, dense);
  if (precision == KNIT_FP32_REFINE) {
    const size_t s64 = sweep_mfma_slab_bytes(Mmax, KNIT_FP64, dense);
    if (s64 > s) s = s64;
  }
  return s;
}

size_t sweep_mfma_workspace(int Mmax, int precision, int P, bool dense) {
  const int grid = P < SWEEP_MAX_GRID ? P : SWEEP_MAX_GRID;
  return 256 + 2 * order_bytes(P) + slab_for(Mmax, precision, dense) * (size_t)grid;
}

int sweep_mfma_grid_within(size_t bytes, int Mmax, int precision, int P, bool dense) {
  const size_t head = 256 + 2 * order_bytes(P);
  if (bytes <= head) return 0;
  const size_t n = (bytes - head) / slab_for(Mmax, precision, dense);
  return n > (size_t)SWEEP_MAX_GRID ? SWEEP_MAX_GRID : (int)n;
}

namespace {
std::atomic<double> refine_threshold{0.25};
}

int sweep_set_refine_threshold(double t) {
  refine_threshold.store(t);
  return 0;
}
double sweep_get_refine_threshold() { return refine_threshold.load(); }

// Launch tuning per (precision, padded-slice class), set by the autotuner.
namespace {
std::mutex tuning_mu;
knit_sweep_tuning tuning_table[3][KNIT_TUNING_CLASSES];
bool tuning_set_flag[3][KNIT_TUNING_CLASSES];
}  // namespace

knit_sweep_tuning sweep_default_tuning(int Mpmax) {
  knit_sweep_tuning t;
  t.threads = Mpmax <= 256 ? 256 : 512;
  t.wg_per_cu = Mpmax <= 256 ? 2 : 1;
  t.order = 1;
  t.outer = Mpmax >= 128 ? 128 : 64;
  return t;
}

bool sweep_tuning_valid(int Mpmax, const knit_sweep_tuning &t) {
  if (t.threads != 256 && t.threads != 512) return false;
  if (t.threads < Mpmax) return false;                 // one panel row per thread
  if (t.wg_per_cu < 1 || t.wg_per_cu > 2) return false;
  if (t.order != 0 && t.order != 1) return false;
  if (t.outer != 64 && t.outer != 128) return false;
  return true;
}

int sweep_tuning_set(int precision, int cls, const knit_sweep_tuning *t) {
  std::lock_guard<std::mutex> lk(tuning_mu);
  if (t) {
    tuning_table[precision][cls] = *t;
    tuning_set_flag[precision][cls] = true;
  } else {
    tuning_set_flag[precision][cls] = false;
  }
  return 0;
}

knit_sweep_tuning sweep_tuning_get(int precision, int Mpmax) {
  const int cls = Mpmax / 32 - 1;
  std::lock_guard<std::mutex> lk(tuning_mu);
  if (cls >= 0 && cls < KNIT_TUNING_CLASSES && tuning_set_flag[precision][cls] &&
      sweep_tuning_valid(Mpmax, tuning_table[precision][cls]))
    return tuning_table[precision][cls];
  return sweep_default_tuning(Mpmax);
}

hipError_t launch_sweep_mfma(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                             const knit_z *sigmaL, const knit_z *sigmaR, int precision, knit_z *G1N,
                             knit_z *GN1, knit_z *GNN, int32_t *pstatus, void *ws, int Mmax, int max_grid,
                             hipStream_t stream) {
  unsigned int *queue = reinterpret_cast<unsigned int *>(ws);
  int *order = reinterpret_cast<int *>(reinterpret_cast<char *>(ws) + 256);
  char *w = reinterpret_cast<char *>(ws) + 256 + 2 * order_bytes(P);
  const int Mpmax = mfma_padded(Mmax);
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  const double rtol = sweep_get_refine_threshold();
  // one pass at `prec`; redo != NULL restricts it to the problems flagged KNIT_P_FALLBACK
  auto pass = [&](int prec, const int32_t *redo) -> hipError_t {
    // workgroup size, workgroups per compute unit and queue order from the
    // tuning table (default: 256 threads, two per compute unit, when the padded
    // slice fits one panel row per thread, else 512 threads, one per unit; LPT)
    const knit_sweep_tuning tune = sweep_tuning_get(prec, Mpmax);
    const bool small = tune.threads == 256;
    const size_t slab = sweep_mfma_slab_bytes(Mmax, prec, table_has_dense(tab));
    int grid = tune.wg_per_cu * ncu;
    if (grid > SWEEP_MAX_GRID) grid = SWEEP_MAX_GRID;
    if (max_grid > 0 && grid > max_grid) grid = max_grid;
    if (grid > P) grid = P;
    hipLaunchKernelGGL(order_kernel, dim3(1), dim3(1024), 0, stream, tab, probs, P, tune.order, (const int *)nullptr, order,
                     queue);
#define KNIT_LAUNCH(RG, RS, RF, NT)                                                                          \
  hipLaunchKernelGGL((sweep_mfma_kernel<RG, RS, RF, NT>), dim3(grid), dim3(NT), 0, stream, tab, probs, P, onsite, \
                     sigmaL, sigmaR, G1N, GN1, GNN, pstatus, w, slab, Mpmax, queue, order, rtol, redo, tune.outer,  \
                     (const knit_z *)nullptr, (const int *)nullptr)
    if (prec == KNIT_FP64) {
      if (small) KNIT_LAUNCH(double, double, false, 256); else KNIT_LAUNCH(double, double, false, 512);
    } else if (prec == KNIT_FP32) {
      if (small) KNIT_LAUNCH(float, float, false, 256); else KNIT_LAUNCH(float, float, false, 512);
    } else {
      if (small) KNIT_LAUNCH(float, double, true, 256); else KNIT_LAUNCH(float, double, true, 512);
    }
#undef KNIT_LAUNCH
    return hipGetLastError();
  };
  hipError_t err = pass(precision, nullptr);
  if (err != hipSuccess || precision != KNIT_FP32_REFINE) return err;
  return pass(KNIT_FP64, pstatus);
}

}  // namespace knit
