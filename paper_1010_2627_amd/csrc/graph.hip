// Knitting of a system of any geometry (section 1; section 5.3-D, FIG. 9), FP64.
//
// The host plan (knit_graph_plan_create) fixes the order of the sites and,
// for every step, which earlier sites the new one couples to and where each
// kept site lives: every site held at a step owns a "slot", a block of norb
// rows and columns of the matrix the knitting updates, and a slot is handed
// to a later site once its site has no neighbour left to add (lead sites are
// kept to the end).  The plan is the same for every problem of a call, so
// the device only replays it.
//
// One workgroup per problem (a grid stride over the problems):
//   1. lead 0's sites as one block: G = (E - H_00 - Sigma_0)^{-1} by
//      Gauss-Jordan with partial pivoting in the workgroup's slab;
//   2. every further site i by Dyson's equation with the sites it couples to
//      (their slots s_j, hopping blocks H_{i,s_j} and H_{s_j,i}):
//        u = G[:, nb] H_{nb,i},  v = H_{i,nb} G[nb, :]          (D x m, m x D)
//        g = (E - H_ii - H_{i,nb} u[nb])^{-1}                   (m x m)
//        G += u (g v),   G[:, s_i] = u g,  G[s_i, :] = g v,  G[s_i, s_i] = g
//      over the D = (highest slot in use + 1) * m leading rows and columns;
//   3. the other leads' self-energies on the lead block:
//        G_LL <- (I - G_LL Sigma')^{-1} G_LL,  Sigma' = diag(0, Sigma_1, ..);
//   4. T_kl = Re sum_{a in k, d in l} conj(G_ad) (Gamma G Gamma)_ad with
//      Gamma block-diagonal over the leads.
//
// The matrix of step 2 lives in registers when D <= 128: each thread owns an
// RPT x CPT set of entries (rows tr + 16 a, columns tc + TC b), the columns
// and rows of the coupled slots are staged through LDS by their owners, and
// the rank-m update touches no memory.  Larger interfaces keep it in the
// workgroup's slab (L2-resident for moderate D).

#include <algorithm>
#include <cstdlib>
#include <functional>
#include <new>
#include <queue>
#include <vector>

#include "knit_internal.h"
#include "knit_wg.h"
#include "../../include/knit_graph.h"

// ---------------------------------------------------------------- host plan

struct knit_graph_plan {
  int N = 0, m = 0, K = 0;      // sites, orbitals per site (per group in a blocked plan), leads
  std::vector<int32_t> order;   // full knitting order (lead 0's sites first)
  std::vector<int32_t> image;   // device image of the plan (int32 words)
  knit_graph_info info{};
  // blocked plans: groups of `block` sites knitted as one site of block * norb
  // orbitals; `gmap` (device words) says how the groups' blocks are gathered
  int block = 1;
  std::vector<int32_t> gmap;
};

namespace knit {
namespace {

using Z = cpx<double>;

// word offsets in the plan image header
enum {
  H_N, H_M, H_K, H_N0, H_NSTEPS, H_DIM, H_LDIM, H_LEADOFF, H_LSLOT, H_LSITE, H_INIT, H_REC, H_STEPS,
  H_NLS, H_WORDS = 16
};

constexpr int NPAIR = KNIT_GRAPH_MAX_PAIRS;
constexpr int MMAX = KNIT_MAX_NORB;

// ---------------------------------------------------------------- device helpers

// B <- A^{-1} B by Gauss-Jordan with partial pivoting (largest |re|+|im|,
// lowest row on ties); A [n][n] (leading dimension lda) is destroyed, rows are
// swapped physically.  fcol: n scratch elements.  Returns nonzero on a zero
// pivot (then B is garbage).
__device__ int wg_gj_solve(Z *A, int lda, Z *B, int ldb, int n, int nrhs, Z *fcol, double *sv, int *si) {
  const int tid = threadIdx.x, nt = blockDim.x;
  int bad = 0;
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int bi = n;
    for (int r = k + tid; r < n; r += nt) argmax_merge(best, bi, c_abs1(A[(int64_t)r * lda + k]), r);
    wg_argmax(best, bi, sv, si);
    if (!(best > 0.0)) bad = 1;   // a zero (or NaN) pivot: keep going, the caller discards the result
    if (bi != k && bi < n) {
      for (int c = k + tid; c < n; c += nt) {
        const Z t = A[(int64_t)k * lda + c];
        A[(int64_t)k * lda + c] = A[(int64_t)bi * lda + c];
        A[(int64_t)bi * lda + c] = t;
      }
      for (int c = tid; c < nrhs; c += nt) {
        const Z t = B[(int64_t)k * ldb + c];
        B[(int64_t)k * ldb + c] = B[(int64_t)bi * ldb + c];
        B[(int64_t)bi * ldb + c] = t;
      }
    }
    __syncthreads();
    const Z piv = c_inv(A[(int64_t)k * lda + k]);
    // multipliers of the other rows, taken before the pivot row is scaled
    for (int r = tid; r < n; r += nt) fcol[r] = r == k ? Z{0.0, 0.0} : A[(int64_t)r * lda + k];
    __syncthreads();
    for (int c = k + 1 + tid; c < n; c += nt) A[(int64_t)k * lda + c] = c_mul(A[(int64_t)k * lda + c], piv);
    for (int c = tid; c < nrhs; c += nt) B[(int64_t)k * ldb + c] = c_mul(B[(int64_t)k * ldb + c], piv);
    __syncthreads();
    const int wa = n - k - 1, wt = wa + nrhs;
    for (int64_t e = tid; e < (int64_t)n * wt; e += nt) {
      const int r = (int)(e / wt), c = (int)(e % wt);
      if (r == k) continue;
      const Z f = fcol[r];
      if (c < wa) {
        Z &x = A[(int64_t)r * lda + k + 1 + c];
        x = c_fms(f, A[(int64_t)k * lda + k + 1 + c], x);
      } else {
        Z &x = B[(int64_t)r * ldb + c - wa];
        x = c_fms(f, B[(int64_t)k * ldb + c - wa], x);
      }
    }
    __syncthreads();
  }
  return bad;
}

// M x M inverse by Gauss-Jordan with partial pivoting, one thread; every
// index is static (row exchanges by selection), so nothing leaves registers.
template <int M>
__device__ __forceinline__ int small_inverse(Z (&a)[M][M], Z (&g)[M][M]) {
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) g[i][j] = i == j ? Z{1.0, 0.0} : Z{0.0, 0.0};
  int bad = 0;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    int p = k;
    double best = c_abs1(a[k][k]);
#pragma unroll
    for (int r = k + 1; r < M; ++r) {
      const double v = c_abs1(a[r][k]);
      if (v > best) {
        best = v;
        p = r;
      }
    }
    if (!(best > 0.0)) bad = 1;
#pragma unroll
    for (int r = k + 1; r < M; ++r)
      if (r == p)
#pragma unroll
        for (int c = 0; c < M; ++c) {
          Z t = a[k][c];
          a[k][c] = a[r][c];
          a[r][c] = t;
          t = g[k][c];
          g[k][c] = g[r][c];
          g[r][c] = t;
        }
    const Z piv = c_inv(a[k][k]);
#pragma unroll
    for (int c = 0; c < M; ++c) {
      a[k][c] = c_mul(a[k][c], piv);
      g[k][c] = c_mul(g[k][c], piv);
    }
#pragma unroll
    for (int r = 0; r < M; ++r) {
      if (r == k) continue;
      const Z f = a[r][k];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        a[r][c] = c_fms(f, a[k][c], a[r][c]);
        g[r][c] = c_fms(f, g[k][c], g[r][c]);
      }
    }
  }
  return bad;
}

// g = (E - H_ii - sum_j hr[j][:] u[pcol_j][:])^{-1} for one m x m block
template <int M>
__device__ __forceinline__ int step_block_inverse(int npairs, const int *pcol, const Z (*hr)[KNIT_MAX_NORB],
                                                  const Z *u, const knit_z *Hii, double E,
                                                  Z (*gsh)[KNIT_MAX_NORB]) {
  Z a[M][M], g[M][M];
#pragma unroll
  for (int k = 0; k < M; ++k)
#pragma unroll
    for (int l = 0; l < M; ++l) {
      const knit_z h = Hii[k * M + l];
      a[k][l] = Z{(k == l ? E : 0.0) - h.re, -h.im};
    }
  for (int j = 0; j < npairs; ++j) {
    const int r = pcol[j];
#pragma unroll
    for (int k = 0; k < M; ++k)
#pragma unroll
      for (int l = 0; l < M; ++l) a[k][l] = c_fms(hr[j][k], u[r * KNIT_MAX_NORB + l], a[k][l]);
  }
  const int bad = small_inverse<M>(a, g);
#pragma unroll
  for (int k = 0; k < M; ++k)
#pragma unroll
    for (int l = 0; l < M; ++l) gsh[k][l] = g[k][l];
  return bad;
}

__device__ __forceinline__ Z ldz(const knit_z *p) { return Z{p->re, p->im}; }
__device__ __forceinline__ void stz(knit_z *p, Z v) {
  p->re = v.re;
  p->im = v.im;
}

__device__ __forceinline__ double wg_sum_d(double v, double *sv) {
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

// Gamma_k[a][b] = i (Sigma_k[a][b] - conj(Sigma_k[b][a])) of the lead block that
// holds lead indices a, b (both in lead k, block offset o, dimension nk).
__device__ __forceinline__ Z gamma_ab(const knit_z *S, int nk, int a, int b) {
  const Z s1 = ldz(S + (int64_t)a * nk + b), s2 = ldz(S + (int64_t)b * nk + a);
  // i (s1 - conj(s2)) = i ((s1.re - s2.re) + i (s1.im + s2.im))
  return Z{-(s1.im + s2.im), s1.re - s2.re};
}

// the register-resident matrix of the knitting steps: entry (tr + 16 a, tc + TC b)
template <int RPT, int CPT>
struct RegG {
  Z x[RPT][CPT];
};

struct Buffers {   // per-workgroup working arrays of the knitting steps
  Z *u, *ug, *w;   // [D][MMAX], [D][MMAX], [MMAX][ldw]
  int ldw;
};

// Phases 2-4 of one knitting step (shared by both storage modes).  On entry
// pcol/hr/hc hold the coupled orbitals and blocks, and u (D x m) / w (v, m x D)
// have been formed by the caller's phase 2; this forms g and turns v into
// w = g v and u into ug = u g.
template <int M>
__device__ __forceinline__ void step_inverse(int npairs, const int *pcol, const Z (*hr)[MMAX], const Z *u,
                                             const knit_z *Hii, double E, Z (*gsh)[MMAX], int *flag) {
  if (threadIdx.x == 0) {
    if (step_block_inverse<M>(npairs, pcol, hr, u, Hii, E, gsh)) *flag |= KNIT_P_SINGULAR;
  }
}

template <int NT, int RPT, int CPT, bool REG, int M>
__global__ __launch_bounds__(NT) void graph_knit_kernel(const int32_t *img, const knit_graph_problem *probs, int P,
                                                        const knit_z *hop, const knit_z *onsite,
                                                        const knit_z *sigma, double *Tout, knit_z *GLL,
                                                        int32_t *pstatus, char *ws, int64_t slab_elems) {
  constexpr int TC = NT / 16;            // threads along a row of the register tile
  constexpr int DM = REG ? 16 * RPT : 1; // register-tile dimension
  static_assert(!REG || 16 * RPT == TC * CPT, "square register tile");
  __shared__ Z Gc[REG ? NPAIR : 1][DM], Gr[REG ? NPAIR : 1][DM];
  __shared__ Z su[REG ? DM * MMAX : 1], sug[REG ? DM * MMAX : 1], sw[REG ? MMAX * DM : 1];
  __shared__ Z sf[REG ? DM : 1];
  __shared__ Z hr[NPAIR][MMAX], hc[NPAIR][MMAX], gsh[MMAX][MMAX];
  __shared__ int pcol[NPAIR];
  // register mode: step records and coupling blocks, double-buffered
  __shared__ int srec[4][REG ? 4 + 3 * NPAIR : 1], spcol[2][REG ? NPAIR : 1];
  // register mode: own[t & 1][c] = (t << 5) | j when column (and row) c of the
  // matrix is coupled orbital j of step t, written two steps ahead
  __shared__ int own[2][REG ? DM : 1];
  __shared__ Z shr[2][REG ? NPAIR : 1][M], shc[2][REG ? NPAIR : 1][M], shii[2][M * M];
  __shared__ double sv[NT / WAVE];
  __shared__ int si[NT / WAVE];
  __shared__ int sflag;

  const int tid = threadIdx.x;
  constexpr int m = M;   // orbitals per site
  const int N = img[H_N], K = img[H_K], n0 = img[H_N0], nsteps = img[H_NSTEPS];
  const int D = img[H_DIM], LD = img[H_LDIM];
  const int32_t *leadoff = img + img[H_LEADOFF];   // [K + 1], in lead orbitals
  const int32_t *lslot = img + img[H_LSLOT];       // slot of every lead site, lead order
  const int32_t *lsite = img + img[H_LSITE];       // site of every lead site
  const int32_t *init = img + img[H_INIT];         // count, then (a, b, e) per hop inside lead 0
  const int R = img[H_REC];                         // words per step record
  const int32_t *steps = img + img[H_STEPS];
  const int mm = m * m;
  (void)N;

  Z *slab = reinterpret_cast<Z *>(ws) + (int64_t)blockIdx.x * slab_elems;
  const int64_t DD = (int64_t)D * D, LL = (int64_t)LD * LD;
  // S0, S1: [LD][LD] (lead 0's block, d0 <= LD, and the lead block); S2: the
  // register dump [D][D] (register mode) or [LD][LD]; SG: the matrix of the
  // steps (slab mode)
  Z *S0 = slab, *S1 = slab + LL, *S2 = slab + 2 * LL;
  Z *SG = S2 + (REG ? DD : LL);
  Z *gu = SG + (REG ? 0 : DD), *gug = gu + (int64_t)D * MMAX, *gw = gug + (int64_t)D * MMAX;
  Z *gf = gw + (int64_t)MMAX * D;
  Buffers bf = REG ? Buffers{su, sug, sw, DM} : Buffers{gu, gug, gw, D};
  Z *fcol = REG ? sf : gf;

  const int tc = tid % TC, tr = tid / TC;

  for (int p = blockIdx.x; p < P; p += gridDim.x) {
    const knit_graph_problem pr = probs[p];
    const knit_z *ons = onsite + pr.onsite_off;
    const knit_z *sig = sigma + pr.sigma_off;
    if (tid == 0) sflag = 0;
    __syncthreads();

    // ---- 1. lead 0's block: S0 = E - H_00 - Sigma_0, S1 = I, S1 <- S0^{-1} S1
    const int d0 = n0 * m;
    for (int e = tid; e < d0 * d0; e += NT) {
      const int a = e / d0, b = e % d0;
      const int sa = a / m, oa = a % m, sb = b / m, ob = b % m;
      Z v = ldz(sig + (int64_t)a * d0 + b);
      v = Z{-v.re, -v.im};
      if (sa == sb) {
        const Z h = ldz(ons + (int64_t)lsite[sa] * mm + oa * m + ob);
        v = Z{v.re - h.re + (oa == ob ? pr.E : 0.0), v.im - h.im};
      }
      S0[(int64_t)a * d0 + b] = v;
      S1[(int64_t)a * d0 + b] = a == b ? Z{1.0, 0.0} : Z{0.0, 0.0};
    }
    __syncthreads();
    for (int q = tid; q < init[0]; q += NT) {   // hops between lead-0 sites: distinct blocks, no races
      const int a = init[1 + 3 * q], b = init[2 + 3 * q], e = init[3 + 3 * q];
      for (int k = 0; k < m; ++k)
        for (int l = 0; l < m; ++l) {
          Z &x = S0[(int64_t)(a * m + k) * d0 + b * m + l];
          const Z h = ldz(hop + (int64_t)e * mm + k * m + l);
          x = Z{x.re - h.re, x.im - h.im};
        }
    }
    __syncthreads();
    int bad = wg_gj_solve(S0, d0, S1, d0, d0, d0, fcol, sv, si);

    // the initial matrix: slots 0 .. n0-1 are lead 0's sites in lead order
    RegG<RPT, CPT> G;
    if constexpr (REG) {
#pragma unroll
      for (int a = 0; a < RPT; ++a)
#pragma unroll
        for (int b = 0; b < CPT; ++b) {
          const int r = tr + 16 * a, c = tc + TC * b;
          G.x[a][b] = (r < d0 && c < d0) ? S1[(int64_t)r * d0 + c] : Z{0.0, 0.0};
        }
    } else {
      for (int e = tid; e < d0 * d0; e += NT) SG[(int64_t)(e / d0) * D + e % d0] = S1[e];
    }
    __syncthreads();

    // ---- 2. the sites one at a time
    if constexpr (REG) {
      // Two barriers per step.  Step t's record sits in LDS slot t & 3 and its
      // coupling blocks in buffer t & 1; the record of step t+3 and the blocks
      // of step t+1 are loaded into registers at the top of step t and stored
      // at its end, so their latency hides behind the step.
      for (int e = tid; e < 3 * R; e += NT) {
        const int tt = e / R;
        srec[tt][e % R] = tt < nsteps ? steps[(int64_t)tt * R + e % R] : 0;
      }
      for (int e = tid; e < 2 * DM; e += NT) own[e / DM][e % DM] = -1;
      __syncthreads();
      for (int tt = 0; tt < 2 && tt < nsteps; ++tt)
        if (tid < srec[tt][3] * M) own[tt][srec[tt][4 + 3 * (tid / M)] * M + tid % M] = (tt << 5) | tid;
      if (nsteps > 0) {
        const int nent0 = srec[0][3];
        for (int e = tid; e < nent0 * mm; e += NT) {
          const int j = e / M, k = e % M, en = j / M, q = j % M;
          shr[0][j][k] = ldz(hop + (int64_t)srec[0][5 + 3 * en] * mm + k * M + q);
          shc[0][j][k] = ldz(hop + (int64_t)srec[0][6 + 3 * en] * mm + q * M + k);
        }
        if (tid < mm) shii[0][tid] = ldz(ons + (int64_t)srec[0][0] * mm + tid);
      }
      __syncthreads();
      // Every load issued so far (the register matrix above all) completes
      // here.  Otherwise the compiler, meeting those loads still in flight at
      // the loop's entry, waits for all vector memory at the first staging
      // store of every step, the three-steps-ahead prefetch included.
      __builtin_amdgcn_s_waitcnt(0);
      for (int t = 0; t < nsteps; ++t) {
        const int cur = t & 1, nxt = cur ^ 1, rc = t & 3, rn = (t + 1) & 3;
        const int sl = srec[rc][1], Da = srec[rc][2], nent = srec[rc][3];
        const int np = nent * M;
        // prefetch: record t+3, blocks of step t+1
        const bool has1 = t + 1 < nsteps, has3 = t + 3 < nsteps;
        int recv = 0;
        if (has3 && tid < R) recv = steps[(int64_t)(t + 3) * R + tid];
        const int nent1 = has1 ? srec[rn][3] : 0;
        Z phr = {0.0, 0.0}, phc = {0.0, 0.0}, phii = {0.0, 0.0};
        if (tid < nent1 * mm) {
          const int j = tid / M, k = tid % M, en = j / M, q = j % M;
          phr = ldz(hop + (int64_t)srec[rn][5 + 3 * en] * mm + k * M + q);
          phc = ldz(hop + (int64_t)srec[rn][6 + 3 * en] * mm + q * M + k);
        }
        if (has1 && tid < mm) phii = ldz(ons + (int64_t)srec[rn][0] * mm + tid);
        // phase 1: the owners stage the coupled columns and rows, looked up in
        // the ownership table (a fixed count of tests per thread, whatever the
        // step couples); every register is addressed statically
        if (tid < np) spcol[cur][tid] = srec[rc][4 + 3 * (tid / M)] * M + tid % M;
#pragma unroll
        for (int b = 0; b < CPT; ++b) {
          const int v = own[cur][tc + TC * b];
          if ((v >> 5) == t) {
            const int j = v & 31;
#pragma unroll
            for (int a = 0; a < RPT; ++a) Gc[j][tr + 16 * a] = G.x[a][b];
          }
        }
#pragma unroll
        for (int a = 0; a < RPT; ++a) {
          const int v = own[cur][tr + 16 * a];
          if ((v >> 5) == t) {
            const int j = v & 31;
#pragma unroll
            for (int b = 0; b < CPT; ++b) Gr[j][tc + TC * b] = G.x[a][b];
          }
        }
        __syncthreads();
        // every thread: g = (E - H_ii - H_{i,nb} G[nb, nb] H_{nb,i})^{-1} from the
        // staged columns (G[nb, nb] are their rows pcol)
        Z g[M][M];
        {
          Z a[M][M];
#pragma unroll
          for (int k = 0; k < M; ++k)
#pragma unroll
            for (int l = 0; l < M; ++l) {
              const Z h = shii[cur][k * M + l];
              a[k][l] = Z{(k == l ? pr.E : 0.0) - h.re, -h.im};
            }
          for (int j = 0; j < np; ++j) {
            const int r = spcol[cur][j];
            Z ul[M];
#pragma unroll
            for (int l = 0; l < M; ++l) ul[l] = Z{0.0, 0.0};
            for (int i = 0; i < np; ++i) {
              const Z gv = Gc[i][r];
#pragma unroll
              for (int l = 0; l < M; ++l) ul[l] = c_fma(gv, shc[cur][i][l], ul[l]);
            }
#pragma unroll
            for (int k = 0; k < M; ++k)
#pragma unroll
              for (int l = 0; l < M; ++l) a[k][l] = c_fms(shr[cur][j][k], ul[l], a[k][l]);
          }
          if (small_inverse<M>(a, g) && tid == 0) sflag |= KNIT_P_SINGULAR;
        }
        // phase 2: u = G[:, nb] H_{nb,i} (D x m), w = g H_{i,nb} G[nb, :] (m x D),
        // with the new slot s folded in so that phase 3 is one uniform update:
        // u's rows of s are the identity and w's columns of s are g, so that
        // 0 + u w gives G[s, s] = g, G[s, :] = w, G[:, s] = u g
        const int s0 = sl * M;
        for (int e = tid; e < Da * M; e += NT) {
          const int r = e / M, k = e % M;
          Z sum = {0.0, 0.0};
          for (int j = 0; j < np; ++j) sum = c_fma(Gc[j][r], shc[cur][j][k], sum);
          if (r >= s0 && r < s0 + M) sum = Z{r - s0 == k ? 1.0 : 0.0, 0.0};
          su[r * MMAX + k] = sum;
        }
        for (int c = tid; c < Da; c += NT) {
          Z v[M];
#pragma unroll
          for (int l = 0; l < M; ++l) v[l] = Z{0.0, 0.0};
          for (int j = 0; j < np; ++j) {
            const Z gv = Gr[j][c];
#pragma unroll
            for (int l = 0; l < M; ++l) v[l] = c_fma(shr[cur][j][l], gv, v[l]);
          }
          const bool cs = c >= s0 && c < s0 + M;
#pragma unroll
          for (int k = 0; k < M; ++k) {
            Z sum = {0.0, 0.0};
#pragma unroll
            for (int l = 0; l < M; ++l) sum = c_fma(g[k][l], v[l], sum);
            if (cs) {
#pragma unroll
              for (int l = 0; l < M; ++l)
                if (c - s0 == l) sum = g[k][l];
            }
            sw[k * DM + c] = sum;
          }
        }
        __syncthreads();
        // phase 3: G <- (0 on the rows and columns of s, else G) + u w
        Z wc[CPT][M];   // w on the thread's columns
#pragma unroll
        for (int b = 0; b < CPT; ++b)
#pragma unroll
          for (int k = 0; k < M; ++k) wc[b][k] = sw[k * DM + tc + TC * b];   // inside the LDS array
#pragma unroll
        for (int a = 0; a < RPT; ++a) {
          const int r = tr + 16 * a;
          const bool rin = r < Da, rs = r >= s0 && r < s0 + M;
          Z ur[M];
#pragma unroll
          for (int k = 0; k < M; ++k) ur[k] = su[r * MMAX + k];
#pragma unroll
          for (int b = 0; b < CPT; ++b) {
            const int c = tc + TC * b;
            if (rin && c < Da) {
              const bool cs = c >= s0 && c < s0 + M;
              Z x = (rs || cs) ? Z{0.0, 0.0} : G.x[a][b];
#pragma unroll
              for (int k = 0; k < M; ++k) x = c_fma(ur[k], wc[b][k], x);
              G.x[a][b] = x;
            }
          }
        }
        // the prefetched record and blocks (their slots are no longer read by any
        // thread: record t-1's slot, step t-1's blocks)
        if (has3 && tid < R) srec[(t + 3) & 3][tid] = recv;
        if (t + 2 < nsteps) {   // ownership of step t+2 (its record arrived a step ago)
          const int r2 = (t + 2) & 3;
          if (tid < srec[r2][3] * M) own[cur][srec[r2][4 + 3 * (tid / M)] * M + tid % M] = ((t + 2) << 5) | tid;
        }
        if (tid < nent1 * mm) {
          shr[nxt][tid / M][tid % M] = phr;
          shc[nxt][tid / M][tid % M] = phc;
        }
        if (has1 && tid < mm) shii[nxt][tid] = phii;
      }
    } else {
      for (int t = 0; t < nsteps; ++t) {
        const int32_t *st = steps + (int64_t)t * R;
        const int site = st[0], sl = st[1], Da = st[2], nent = st[3];
        const int np = nent * m;
        if (tid < np) {
          const int j = tid, en = j / m, q = j % m;
          const int slot = st[4 + 3 * en], erow = st[5 + 3 * en], ecol = st[6 + 3 * en];
          pcol[j] = slot * m + q;
          for (int k = 0; k < m; ++k) {
            hr[j][k] = ldz(hop + (int64_t)erow * mm + k * m + q);   // H_{i,nb}[k][q]
            hc[j][k] = ldz(hop + (int64_t)ecol * mm + q * m + k);   // H_{nb,i}[q][k]
          }
        }
        __syncthreads();
        // u = G[:, nb] H_{nb,i} (D x m), v = H_{i,nb} G[nb, :] (m x D, into w)
        for (int e = tid; e < Da * m; e += NT) {
          const int r = e / m, k = e % m;
          Z sum = {0.0, 0.0};
          for (int j = 0; j < np; ++j) sum = c_fma(SG[(int64_t)r * D + pcol[j]], hc[j][k], sum);
          bf.u[r * MMAX + k] = sum;
        }
        for (int e = tid; e < Da * m; e += NT) {
          const int k = e / Da, c = e % Da;
          Z sum = {0.0, 0.0};
          for (int j = 0; j < np; ++j) sum = c_fma(hr[j][k], SG[(int64_t)pcol[j] * D + c], sum);
          bf.w[k * bf.ldw + c] = sum;
        }
        __syncthreads();
        step_inverse<M>(np, pcol, hr, bf.u, ons + (int64_t)site * mm, pr.E, gsh, &sflag);
        __syncthreads();
        // w = g v (per column), ug = u g (per row)
        for (int c = tid; c < Da; c += NT) {
          Z v[M];
#pragma unroll
          for (int k = 0; k < M; ++k) v[k] = bf.w[k * bf.ldw + c];
#pragma unroll
          for (int k = 0; k < M; ++k) {
            Z sum = {0.0, 0.0};
#pragma unroll
            for (int l = 0; l < M; ++l) sum = c_fma(gsh[k][l], v[l], sum);
            bf.w[k * bf.ldw + c] = sum;
          }
        }
        for (int r = tid; r < Da; r += NT)
#pragma unroll
          for (int k = 0; k < M; ++k) {
            Z sum = {0.0, 0.0};
#pragma unroll
            for (int l = 0; l < M; ++l) sum = c_fma(bf.u[r * MMAX + l], gsh[l][k], sum);
            bf.ug[r * MMAX + k] = sum;
          }
        __syncthreads();
        const int s0 = sl * m;
        for (int64_t e = tid; e < (int64_t)Da * Da; e += NT) {
          const int r = (int)(e / Da), c = (int)(e % Da);
          const bool rs = r >= s0 && r < s0 + m, cs = c >= s0 && c < s0 + m;
          Z &x = SG[(int64_t)r * D + c];
          if (rs && cs) x = gsh[r - s0][c - s0];
          else if (rs) x = bf.w[(r - s0) * bf.ldw + c];
          else if (cs) x = bf.ug[r * MMAX + c - s0];
          else {
            Z sum = x;
#pragma unroll
            for (int k = 0; k < M; ++k) sum = c_fma(bf.u[r * MMAX + k], bf.w[k * bf.ldw + c], sum);
            x = sum;
          }
        }
        __syncthreads();
      }
    }

    // ---- 3. the lead block, then the other leads' self-energies
    __syncthreads();
    const Z *Gsrc = SG;
    if constexpr (REG) {
#pragma unroll
      for (int a = 0; a < RPT; ++a)
#pragma unroll
        for (int b = 0; b < CPT; ++b) {
          const int r = tr + 16 * a, c = tc + TC * b;
          if (r < D && c < D) S2[(int64_t)r * D + c] = G.x[a][b];
        }
      Gsrc = S2;
    }
    __syncthreads();
    // S1 = G_LL (lead orbitals a, b -> rows lslot*m + o)
    for (int e = tid; e < LD * LD; e += NT) {
      const int a = e / LD, b = e % LD;
      const int ra = lslot[a / m] * m + a % m, rb = lslot[b / m] * m + b % m;
      S1[e] = Gsrc[(int64_t)ra * D + rb];
    }
    __syncthreads();
    // S0 = I - G_LL Sigma' (Sigma' = 0 on lead 0's block)
    if (K > 1) {
      for (int e = tid; e < LD * LD; e += NT) {
        const int a = e / LD, b = e % LD;
        int k = 0;
        while (b >= leadoff[k + 1]) ++k;
        Z s = a == b ? Z{1.0, 0.0} : Z{0.0, 0.0};
        if (k > 0) {
          const int o = leadoff[k], nk = leadoff[k + 1] - o;
          int64_t so = 0;
          for (int j = 0; j < k; ++j) so += (int64_t)(leadoff[j + 1] - leadoff[j]) * (leadoff[j + 1] - leadoff[j]);
          const knit_z *Sk = sig + so;
          for (int c = 0; c < nk; ++c) s = c_fms(S1[(int64_t)a * LD + o + c], ldz(Sk + (int64_t)c * nk + b - o), s);
        }
        S0[e] = s;
      }
      __syncthreads();
      bad |= wg_gj_solve(S0, LD, S1, LD, LD, LD, fcol, sv, si);
    }
    // ---- 4. Q = Gamma G_LL Gamma (block-diagonal Gamma), then T_kl
    for (int e = tid; e < LD * LD; e += NT) {   // S0 = G_LL Gamma
      const int a = e / LD, b = e % LD;
      int k = 0;
      while (b >= leadoff[k + 1]) ++k;
      const int o = leadoff[k], nk = leadoff[k + 1] - o;
      int64_t so = 0;
      for (int j = 0; j < k; ++j) so += (int64_t)(leadoff[j + 1] - leadoff[j]) * (leadoff[j + 1] - leadoff[j]);
      Z s = {0.0, 0.0};
      for (int c = 0; c < nk; ++c) s = c_fma(S1[(int64_t)a * LD + o + c], gamma_ab(sig + so, nk, c, b - o), s);
      S0[e] = s;
    }
    __syncthreads();
    for (int e = tid; e < LD * LD; e += NT) {   // S2 = Gamma S0
      const int a = e / LD, b = e % LD;
      int k = 0;
      while (a >= leadoff[k + 1]) ++k;
      const int o = leadoff[k], nk = leadoff[k + 1] - o;
      int64_t so = 0;
      for (int j = 0; j < k; ++j) so += (int64_t)(leadoff[j + 1] - leadoff[j]) * (leadoff[j + 1] - leadoff[j]);
      Z s = {0.0, 0.0};
      for (int c = 0; c < nk; ++c) s = c_fma(gamma_ab(sig + so, nk, a - o, c), S0[(int64_t)(o + c) * LD + b], s);
      S2[e] = s;
    }
    __syncthreads();
    const bool fail = bad || sflag;
    for (int k = 0; k < K; ++k)
      for (int l = 0; l < K; ++l) {
        const int ok = leadoff[k], nk = leadoff[k + 1] - ok, ol = leadoff[l], nl = leadoff[l + 1] - ol;
        double s = 0.0;
        for (int e = tid; e < nk * nl; e += NT) {
          const int a = ok + e / nl, d = ol + e % nl;
          const Z g = S1[(int64_t)a * LD + d], q = S2[(int64_t)a * LD + d];
          s += g.re * q.re + g.im * q.im;   // Re(conj(g) q)
        }
        s = wg_sum_d(s, sv);
        if (tid == 0) Tout[(int64_t)p * K * K + k * K + l] = fail ? NAN : s;
      }
    if (GLL)
      for (int e = tid; e < LD * LD; e += NT) stz(GLL + pr.gll_off + e, fail ? Z{NAN, NAN} : S1[e]);
    if (tid == 0) {
      int f = sflag | (bad ? KNIT_P_SINGULAR : 0);
      bool fin = true;
      for (int q = 0; q < K * K; ++q) fin = fin && isfinite(Tout[(int64_t)p * K * K + q]);
      if (!fail && !fin) f |= KNIT_P_NONFINITE;
      pstatus[p] = f;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- blocked plans

// words of a blocked plan's group map (header, then the arrays it points at)
enum { GM_NC, GM_MB, GM_B, GM_M, GM_NNZ, GM_MEM, GM_INPTR, GM_IN, GM_EPTR, GM_E, GM_WORDS = 16 };

// Hopping blocks of the group graph: block (a, b) of group edge (g, h) is the
// hopping block from member a of g to member b of h, zero where they are not
// coupled.  One element per thread, grid-strided.
__global__ void __launch_bounds__(256) group_hop_kernel(const int32_t *gm, const knit_z *hop, knit_z *ghop) {
  const int nnzc = gm[GM_NNZ], MB = gm[GM_MB], m = gm[GM_M];
  const int32_t *eptr = gm + gm[GM_EPTR], *et = gm + gm[GM_E];
  const int64_t n = (int64_t)nnzc * MB * MB;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int ec = (int)(i / (MB * MB)), r = (int)(i / MB % MB), c = (int)(i % MB);
    const int a = r / m, bq = c / m;
    knit_z v{0.0, 0.0};
    for (int q = eptr[ec]; q < eptr[ec + 1]; ++q)
      if (et[3 * q] == a && et[3 * q + 1] == bq) v = hop[(int64_t)et[3 * q + 2] * m * m + (r % m) * m + c % m];
    ghop[i] = v;
  }
}

// On-site blocks of the groups for every problem: the members' on-site blocks
// on the diagonal, the hoppings between members off it, E - H = 1 (and no
// coupling) on padding orbitals; and the problem table that points at them.
__global__ void __launch_bounds__(256) group_onsite_kernel(const int32_t *gm, const knit_graph_problem *probs, int P,
                                                           const knit_z *hop, const knit_z *onsite, knit_z *gons,
                                                           knit_graph_problem *gprobs) {
  const int Nc = gm[GM_NC], MB = gm[GM_MB], b = gm[GM_B], m = gm[GM_M];
  const int32_t *mem = gm + gm[GM_MEM], *inptr = gm + gm[GM_INPTR], *it = gm + gm[GM_IN];
  const int64_t per = (int64_t)Nc * MB * MB, n = per * P;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(i / per);
    const int64_t j = i % per;
    const int g = (int)(j / (MB * MB)), r = (int)(j / MB % MB), c = (int)(j % MB);
    const int a = r / m, bq = c / m;
    const knit_graph_problem pr = probs[p];
    knit_z v{0.0, 0.0};
    if (a == bq) {
      const int s = mem[(int64_t)g * b + a];
      if (s >= 0) v = onsite[pr.onsite_off + (int64_t)s * m * m + (r % m) * m + c % m];
      else if (r == c) v = knit_z{pr.E - 1.0, 0.0};
    } else {
      for (int q = inptr[g]; q < inptr[g + 1]; ++q)
        if (it[3 * q] == a && it[3 * q + 1] == bq) v = hop[(int64_t)it[3 * q + 2] * m * m + (r % m) * m + c % m];
    }
    gons[i] = v;
    if (j == 0) {
      knit_graph_problem q = pr;
      q.onsite_off = (int64_t)p * per;
      gprobs[p] = q;
    }
  }
}

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

// workspace bytes of a blocked plan's gathered blocks (group map, hopping
// blocks, per-problem on-site blocks, problem table)
size_t group_bytes(const knit_graph_plan *p, int P) {
  if (p->block <= 1) return 0;
  const int32_t *gm = p->gmap.data();
  const size_t bb = (size_t)gm[GM_MB] * gm[GM_MB] * sizeof(knit_z);
  return round256(p->gmap.size() * 4) + round256((size_t)gm[GM_NNZ] * bb) + round256((size_t)P * gm[GM_NC] * bb) +
         round256((size_t)P * sizeof(knit_graph_problem));
}

constexpr int GRAPH_MAX_GRID = 1024;

int64_t slab_elems_of(int D, int LD, bool reg) {
  const int64_t DD = (int64_t)D * D, LL = (int64_t)LD * LD;
  return 2 * LL + (reg ? DD : LL) + (reg ? 0 : DD + 3 * (int64_t)D * MMAX + D) + 64;
}

bool reg_mode(int D) { return D <= 128; }

size_t image_bytes(const knit_graph_plan *p) { return (p->image.size() * 4 + 255) / 256 * 256; }

}  // namespace
}  // namespace knit

// ---------------------------------------------------------------- C ABI

using namespace knit;

namespace knit {
namespace {

// Validates the graph and the leads, fixes the order and replays it (slots,
// interface, step records) into *pl.  Nothing is kept on failure.
int build_plan(int32_t nsite, int32_t norb, const int32_t *row_ptr, const int32_t *col, int32_t n_leads,
               const knit_graph_lead *leads, const int32_t *order, knit_graph_plan *pl) {
  if (nsite < 1 || norb < 1 || norb > KNIT_MAX_NORB || !row_ptr || !leads || n_leads < 1 ||
      n_leads > KNIT_GRAPH_MAX_LEADS)
    return KNIT_E_ARG;
  const int N = nsite, m = norb, K = n_leads;
  if (row_ptr[0] != 0) return KNIT_E_ARG;
  for (int i = 0; i < N; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return KNIT_E_ARG;
  const int64_t nnz = row_ptr[N];
  if (nnz > 0 && !col) return KNIT_E_ARG;
  if (nnz > INT32_MAX / 4) return KNIT_E_UNSUPPORTED;
  // edges: in range, no self loop, no repeat, structurally symmetric
  std::vector<std::vector<int32_t>> nbr(N);
  for (int i = 0; i < N; ++i)
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int j = col[e];
      if (j < 0 || j >= N || j == i) return KNIT_E_ARG;
      nbr[i].push_back(j);
    }
  auto edge_of = [&](int i, int j) -> int {   // CSR index of (i, j) or -1
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
      if (col[e] == j) return e;
    return -1;
  };
  for (int i = 0; i < N; ++i) {
    std::vector<int32_t> s = nbr[i];
    std::sort(s.begin(), s.end());
    if (std::adjacent_find(s.begin(), s.end()) != s.end()) return KNIT_E_ARG;
    for (int j : s)
      if (edge_of(j, i) < 0) return KNIT_E_ARG;
  }
  // leads: sites in range, distinct, in at most one lead
  std::vector<int> lead_of(N, -1), pos_in(N, -1);
  int nls = 0;
  for (int k = 0; k < K; ++k) {
    if (leads[k].nsite < 1 || !leads[k].sites) return KNIT_E_ARG;
    for (int q = 0; q < leads[k].nsite; ++q) {
      const int s = leads[k].sites[q];
      if (s < 0 || s >= N || lead_of[s] >= 0) return KNIT_E_ARG;
      lead_of[s] = k;
      pos_in[s] = q;
    }
    nls += leads[k].nsite;
  }
  // the order: lead 0's sites, then the rest
  std::vector<int32_t> ord;
  ord.reserve(N);
  std::vector<char> taken(N, 0);
  for (int q = 0; q < leads[0].nsite; ++q) {
    ord.push_back(leads[0].sites[q]);
    taken[leads[0].sites[q]] = 1;
  }
  if (order) {
    std::vector<char> seen(N, 0);
    for (int t = 0; t < N; ++t) {
      const int s = order[t];
      if (s < 0 || s >= N || seen[s]) return KNIT_E_ARG;
      seen[s] = 1;
      if (!taken[s]) {
        ord.push_back(s);
        taken[s] = 1;
      }
    }
  } else {
    size_t head = 0;
    int next_root = 0;
    while ((int)ord.size() < N) {
      if (head == ord.size()) {   // start a new component
        while (taken[next_root]) ++next_root;
        ord.push_back(next_root);
        taken[next_root] = 1;
      }
      const int s = ord[head++];
      for (int j : nbr[s])
        if (!taken[j]) {
          ord.push_back(j);
          taken[j] = 1;
        }
    }
  }
  // replay: slots, interface, steps
  const int n0 = leads[0].nsite;
  std::vector<int> remaining(N), slot(N, -1);
  for (int i = 0; i < N; ++i) remaining[i] = (int)nbr[i].size();
  std::vector<char> added(N, 0);
  std::priority_queue<int, std::vector<int>, std::greater<int>> free_slots;   // lowest free slot on top
  int hw = 0, max_slots = 0, max_pairs = 0;
  std::vector<int32_t> steps, stepoff;
  std::vector<int> used_count;   // slots in use (for the high-water mark)
  std::vector<char> in_use;
  auto take_slot = [&]() -> int {
    int s;
    if (!free_slots.empty()) {
      s = free_slots.top();
      free_slots.pop();
    } else {
      s = hw++;
      in_use.push_back(0);
    }
    in_use[s] = 1;
    return s;
  };
  auto release = [&](int s) {
    in_use[s] = 0;
    free_slots.push(s);
  };
  auto top_in_use = [&]() -> int {
    int t = (int)in_use.size() - 1;
    while (t >= 0 && !in_use[t]) --t;
    return t + 1;
  };
  auto after_add = [&](int i) {
    added[i] = 1;
    for (int j : nbr[i]) --remaining[j];
  };
  auto maybe_release = [&](int i) {
    if (added[i] && slot[i] >= 0 && remaining[i] == 0 && lead_of[i] < 0) {
      release(slot[i]);
      slot[i] = -1;
    }
  };
  for (int q = 0; q < n0; ++q) slot[ord[q]] = take_slot();
  for (int q = 0; q < n0; ++q) after_add(ord[q]);
  max_slots = top_in_use();
  double flops = 0.0, bytes = 0.0;
  for (int t = n0; t < N; ++t) {
    const int i = ord[t];
    std::vector<int32_t> ent;
    for (int j : nbr[i])
      if (added[j]) {
        if (slot[j] < 0) return KNIT_E_ARG;   // cannot happen: j still has i to add
        ent.push_back(slot[j]);
        ent.push_back(edge_of(i, j));
        ent.push_back(edge_of(j, i));
      }
    const int nent = (int)ent.size() / 3;
    if (nent * m > KNIT_GRAPH_MAX_PAIRS) return KNIT_E_UNSUPPORTED;
    max_pairs = std::max(max_pairs, nent * m);
    slot[i] = take_slot();
    const int Da = top_in_use() * m;
    max_slots = std::max(max_slots, Da / m);
    stepoff.push_back((int32_t)steps.size());
    steps.push_back(i);
    steps.push_back(slot[i]);
    steps.push_back(Da);
    steps.push_back(nent);
    steps.insert(steps.end(), ent.begin(), ent.end());
    flops += 8.0 * m * (double)Da * Da;
    bytes += 32.0 * (double)Da * Da;
    after_add(i);
    maybe_release(i);
    for (int j : nbr[i]) maybe_release(j);
  }
  stepoff.push_back((int32_t)steps.size());
  const int D = max_slots * m, LD = nls * m;
  if (D > KNIT_GRAPH_MAX_DIM) return KNIT_E_UNSUPPORTED;

  pl->N = N;
  pl->m = m;
  pl->K = K;
  pl->order = ord;
  std::vector<int32_t> &img = pl->image;
  img.assign(H_WORDS, 0);
  img[H_N] = N;
  img[H_M] = m;
  img[H_K] = K;
  img[H_N0] = n0;
  img[H_NSTEPS] = N - n0;
  img[H_DIM] = D;
  img[H_LDIM] = LD;
  img[H_NLS] = nls;
  img[H_LEADOFF] = (int32_t)img.size();
  {
    int o = 0;
    for (int k = 0; k < K; ++k) {
      img.push_back(o);
      o += leads[k].nsite * m;
    }
    img.push_back(o);
  }
  img[H_LSLOT] = (int32_t)img.size();
  for (int k = 0; k < K; ++k)
    for (int q = 0; q < leads[k].nsite; ++q) img.push_back(slot[leads[k].sites[q]]);
  img[H_LSITE] = (int32_t)img.size();
  for (int k = 0; k < K; ++k)
    for (int q = 0; q < leads[k].nsite; ++q) img.push_back(leads[k].sites[q]);
  img[H_INIT] = (int32_t)img.size();
  {
    std::vector<int32_t> tri;
    for (int a = 0; a < n0; ++a) {
      const int i = leads[0].sites[a];
      for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
        if (lead_of[col[e]] == 0) {
          tri.push_back(a);
          tri.push_back(pos_in[col[e]]);
          tri.push_back(e);
        }
    }
    img.push_back((int32_t)(tri.size() / 3));
    img.insert(img.end(), tri.begin(), tri.end());
  }
  // fixed-size step records (site, slot, D_t, n, then n x (slot, edge i->j, edge j->i)),
  // so that a workgroup can fetch any step's record without an index
  const int R = 4 + 3 * std::max(1, max_pairs / m);
  img[H_REC] = R;
  img[H_STEPS] = (int32_t)img.size();
  for (size_t t = 0; t + 1 < stepoff.size(); ++t) {
    const size_t n = stepoff[t + 1] - stepoff[t];
    img.insert(img.end(), steps.begin() + stepoff[t], steps.begin() + stepoff[t + 1]);
    img.insert(img.end(), R - n, 0);
  }

  knit_graph_info &in = pl->info;
  in.nsite = N;
  in.norb = m;
  in.n_leads = K;
  in.max_slots = max_slots;
  in.dim = D;
  in.lead_dim = LD;
  in.max_pairs = max_pairs;
  in.n_steps = N - n0;
  int64_t ss = 0;
  for (int k = 0; k < K; ++k) ss += (int64_t)leads[k].nsite * m * leads[k].nsite * m;
  in.sigma_size = ss;
  in.nnz = nnz;
  in.update_flops = flops;
  in.update_bytes = bytes;
  in.block = 1;
  return KNIT_OK;
}

}  // namespace
}  // namespace knit

extern "C" int knit_graph_plan_create(int32_t nsite, int32_t norb, const int32_t *row_ptr, const int32_t *col,
                                      int32_t n_leads, const knit_graph_lead *leads, const int32_t *order,
                                      knit_graph_plan **plan) {
  return knit_graph_plan_create_blocked(nsite, norb, row_ptr, col, n_leads, leads, order, 1, plan);
}

namespace knit {
namespace {

// The group plan of a validated site plan: groups of b sites (each lead's
// sites b at a time in lead order, the others b at a time in the site order),
// the graph of the groups with their member-to-member hops, and the plan of
// that graph with b * norb orbitals per group, knitted in the order in which
// the groups' first members come in the site order.
int build_blocked(const knit_graph_plan &fine, const int32_t *row_ptr, const int32_t *col, int K,
                  const knit_graph_lead *leads, int b, knit_graph_plan *out) {
  const int N = fine.N, m = fine.m, MB = b * m;
  std::vector<int> grp(N, -1), gpos(N, -1);
  std::vector<int32_t> members;   // [groups][b]: member sites, -1 for padding
  auto new_group = [&]() {
    members.insert(members.end(), b, -1);
    return (int)(members.size() / b) - 1;
  };
  auto put = [&](int g, int a, int s) {
    grp[s] = g;
    gpos[s] = a;
    members[(size_t)g * b + a] = s;
  };
  std::vector<std::vector<int32_t>> lgroups(K);
  for (int k = 0; k < K; ++k)
    for (int q = 0; q < leads[k].nsite; ++q) {
      if (q % b == 0) lgroups[k].push_back(new_group());
      put(lgroups[k].back(), q % b, leads[k].sites[q]);
    }
  int cur = -1, fill = b;
  for (int s : fine.order) {
    if (grp[s] >= 0) continue;
    if (fill == b) {
      cur = new_group();
      fill = 0;
    }
    put(cur, fill++, s);
  }
  const int Nc = (int)(members.size() / b);
  std::vector<int32_t> gorder;
  std::vector<char> seen(Nc, 0);
  for (int s : fine.order)
    if (!seen[grp[s]]) {
      seen[grp[s]] = 1;
      gorder.push_back(grp[s]);
    }
  std::vector<int32_t> grow(Nc + 1, 0), gcol, eptr{0}, etri, inptr{0}, intri;
  for (int g = 0; g < Nc; ++g) {
    std::vector<int32_t> nb;
    for (int a = 0; a < b; ++a) {
      const int s = members[(size_t)g * b + a];
      if (s < 0) continue;
      for (int e = row_ptr[s]; e < row_ptr[s + 1]; ++e) {
        const int h = grp[col[e]];
        if (h == g) {
          intri.push_back(a);
          intri.push_back(gpos[col[e]]);
          intri.push_back(e);
        } else {
          nb.push_back(h);
        }
      }
    }
    inptr.push_back((int32_t)(intri.size() / 3));
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    for (int h : nb) {
      gcol.push_back(h);
      for (int a = 0; a < b; ++a) {
        const int s = members[(size_t)g * b + a];
        if (s < 0) continue;
        for (int e = row_ptr[s]; e < row_ptr[s + 1]; ++e)
          if (grp[col[e]] == h) {
            etri.push_back(a);
            etri.push_back(gpos[col[e]]);
            etri.push_back(e);
          }
      }
      eptr.push_back((int32_t)(etri.size() / 3));
    }
    grow[g + 1] = (int32_t)gcol.size();
  }
  std::vector<knit_graph_lead> gl(K);
  for (int k = 0; k < K; ++k) gl[k] = knit_graph_lead{(int32_t)lgroups[k].size(), 0, lgroups[k].data()};
  const int rc = build_plan(Nc, MB, grow.data(), gcol.empty() ? nullptr : gcol.data(), K, gl.data(), gorder.data(),
                            out);
  if (rc != KNIT_OK) return rc;
  out->order = fine.order;
  out->block = b;
  out->info.nsite = N;
  out->info.norb = m;
  out->info.nnz = fine.info.nnz;
  out->info.block = b;
  std::vector<int32_t> &gm = out->gmap;
  gm.assign(GM_WORDS, 0);
  gm[GM_NC] = Nc;
  gm[GM_MB] = MB;
  gm[GM_B] = b;
  gm[GM_M] = m;
  gm[GM_NNZ] = (int32_t)gcol.size();
  gm[GM_MEM] = (int32_t)gm.size();
  gm.insert(gm.end(), members.begin(), members.end());
  gm[GM_INPTR] = (int32_t)gm.size();
  gm.insert(gm.end(), inptr.begin(), inptr.end());
  gm[GM_IN] = (int32_t)gm.size();
  gm.insert(gm.end(), intri.begin(), intri.end());
  gm[GM_EPTR] = (int32_t)gm.size();
  gm.insert(gm.end(), eptr.begin(), eptr.end());
  gm[GM_E] = (int32_t)gm.size();
  gm.insert(gm.end(), etri.begin(), etri.end());
  return KNIT_OK;
}

}  // namespace
}  // namespace knit

extern "C" int knit_graph_plan_create_blocked(int32_t nsite, int32_t norb, const int32_t *row_ptr, const int32_t *col,
                                              int32_t n_leads, const knit_graph_lead *leads, const int32_t *order,
                                              int32_t block, knit_graph_plan **plan) {
  if (!plan) return KNIT_E_ARG;
  *plan = nullptr;
  if (block < 0) return KNIT_E_ARG;
  knit_graph_plan *fine = new (std::nothrow) knit_graph_plan();
  if (!fine) return KNIT_E_ARG;
  const int rc = build_plan(nsite, norb, row_ptr, col, n_leads, leads, order, fine);
  if (rc != KNIT_OK || block == 1) {
    if (rc == KNIT_OK) *plan = fine;
    else delete fine;
    return rc;
  }
  auto fits = [&](int b) {
    if (b * norb > KNIT_MAX_NORB) return false;
    for (int k = 0; k < n_leads; ++k)
      if (leads[k].nsite % b) return false;
    return true;
  };
  if (block > 1) {
    if (!fits(block)) {
      delete fine;
      return KNIT_E_ARG;
    }
    knit_graph_plan *bp = new (std::nothrow) knit_graph_plan();
    const int rb = bp ? build_blocked(*fine, row_ptr, col, n_leads, leads, block, bp) : KNIT_E_ARG;
    delete fine;
    if (rb != KNIT_OK) {
      delete bp;
      return rb;
    }
    *plan = bp;
    return KNIT_OK;
  }
  // Automatic.  With the interface in registers a step has a fixed part that
  // groups share and a part that grows with the square of the orbitals it
  // couples (every thread forms the group's block): groups of two one-orbital
  // sites, kept in the same register kernel (dimension up to 64, or up to
  // 128), else site by site.  With the interface in the slab every step is a
  // pass over it in memory, which groups share; the serial group inverse
  // grows with the group, so groups of about three orbitals come first, then
  // the larger of two equally close sizes.
  if (reg_mode(fine->info.dim)) {
    if (norb == 1 && fits(2)) {
      knit_graph_plan *bp = new (std::nothrow) knit_graph_plan();
      const int lim = fine->info.dim <= 64 ? 64 : 128;
      if (bp && build_blocked(*fine, row_ptr, col, n_leads, leads, 2, bp) == KNIT_OK && bp->info.dim <= lim) {
        delete fine;
        *plan = bp;
        return KNIT_OK;
      }
      delete bp;
    }
    *plan = fine;
    return KNIT_OK;
  }
  std::vector<int> cand;
  for (int b = 2; b * norb <= KNIT_MAX_NORB; ++b)
    if (fits(b)) cand.push_back(b);
  std::sort(cand.begin(), cand.end(), [&](int x, int y) {
    const int dx = std::abs(x * norb - 3), dy = std::abs(y * norb - 3);
    return dx != dy ? dx < dy : x > y;
  });
  for (int b : cand) {
    knit_graph_plan *bp = new (std::nothrow) knit_graph_plan();
    if (!bp) break;
    if (build_blocked(*fine, row_ptr, col, n_leads, leads, b, bp) == KNIT_OK) {
      delete fine;
      *plan = bp;
      return KNIT_OK;
    }
    delete bp;
  }
  *plan = fine;
  return KNIT_OK;
}

extern "C" int knit_graph_plan_info(const knit_graph_plan *plan, knit_graph_info *info) {
  if (!plan || !info) return KNIT_E_ARG;
  *info = plan->info;
  return KNIT_OK;
}

extern "C" int knit_graph_plan_order(const knit_graph_plan *plan, int32_t *order) {
  if (!plan || !order) return KNIT_E_ARG;
  std::copy(plan->order.begin(), plan->order.end(), order);
  return KNIT_OK;
}

extern "C" void knit_graph_plan_destroy(knit_graph_plan *plan) { delete plan; }

namespace knit {
namespace {
template <int M>
void launch_graph(int D, int LD, int grid, hipStream_t s, const int32_t *img, const knit_graph_problem *probs, int P,
                  const knit_z *hop, const knit_z *onsite, const knit_z *sigma, double *T, knit_z *GLL,
                  int32_t *pstatus, char *slabs) {
  if (D <= 64)
    hipLaunchKernelGGL((graph_knit_kernel<256, 4, 4, true, M>), dim3(grid), dim3(256), 0, s, img, probs, P, hop,
                       onsite, sigma, T, GLL, pstatus, slabs, slab_elems_of(D, LD, true));
  else if (D <= 128)
    hipLaunchKernelGGL((graph_knit_kernel<512, 8, 4, true, M>), dim3(grid), dim3(512), 0, s, img, probs, P, hop,
                       onsite, sigma, T, GLL, pstatus, slabs, slab_elems_of(D, LD, true));
  else
    hipLaunchKernelGGL((graph_knit_kernel<512, 1, 1, false, M>), dim3(grid), dim3(512), 0, s, img, probs, P, hop,
                       onsite, sigma, T, GLL, pstatus, slabs, slab_elems_of(D, LD, false));
}

// resident workgroups: up to 1024 in register mode, one per CU in slab mode
int graph_grid(int P, int D) {
  const int cap = reg_mode(D) ? GRAPH_MAX_GRID : 256;
  return P < cap ? P : cap;
}
}  // namespace
}  // namespace knit

extern "C" size_t knit_graph_workspace(const knit_graph_plan *plan, int32_t P) {
  if (!plan || P < 1) return 0;
  const int D = plan->info.dim, LD = plan->info.lead_dim;
  return image_bytes(plan) + group_bytes(plan, P) +
         (size_t)graph_grid(P, D) * (size_t)slab_elems_of(D, LD, reg_mode(D)) * sizeof(Z);
}

extern "C" int knit_graph_transmission(const knit_graph_plan *plan, const knit_graph_problem *probs, int32_t P,
                                       const knit_z *hop, const knit_z *onsite, const knit_z *sigma, double *T,
                                       knit_z *GLL, int32_t *pstatus, void *ws, size_t ws_bytes, void *stream) {
  if (!plan || P < 0) return KNIT_E_ARG;
  if (P == 0) return KNIT_OK;
  if (!probs || !onsite || !sigma || !T || !pstatus) return KNIT_E_ARG;
  if (plan->info.nnz > 0 && !hop) return KNIT_E_ARG;
  const size_t need = knit_graph_workspace(plan, P);
  if (!ws || ws_bytes < need) return KNIT_E_WORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int32_t *img = reinterpret_cast<int32_t *>(ws);
  if (hipMemcpyAsync(img, plan->image.data(), plan->image.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess)
    return KNIT_E_DEVICE;
  char *next = reinterpret_cast<char *>(ws) + image_bytes(plan);
  if (plan->block > 1) {   // gather the groups' blocks, then knit the groups
    const int32_t *gmh = plan->gmap.data();
    const size_t bb = (size_t)gmh[GM_MB] * gmh[GM_MB] * sizeof(knit_z);
    int32_t *gm = reinterpret_cast<int32_t *>(next);
    next += round256(plan->gmap.size() * 4);
    knit_z *ghop = reinterpret_cast<knit_z *>(next);
    next += round256((size_t)gmh[GM_NNZ] * bb);
    knit_z *gons = reinterpret_cast<knit_z *>(next);
    next += round256((size_t)P * gmh[GM_NC] * bb);
    knit_graph_problem *gprobs = reinterpret_cast<knit_graph_problem *>(next);
    next += round256((size_t)P * sizeof(knit_graph_problem));
    if (hipMemcpyAsync(gm, gmh, plan->gmap.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess) return KNIT_E_DEVICE;
    const int64_t nh = (int64_t)gmh[GM_NNZ] * gmh[GM_MB] * gmh[GM_MB];
    const int64_t no = (int64_t)P * gmh[GM_NC] * gmh[GM_MB] * gmh[GM_MB];
    if (nh > 0)
      hipLaunchKernelGGL(group_hop_kernel, dim3((unsigned)std::min<int64_t>((nh + 255) / 256, 4096)), dim3(256), 0,
                         s, gm, hop, ghop);
    hipLaunchKernelGGL(group_onsite_kernel, dim3((unsigned)std::min<int64_t>((no + 255) / 256, 16384)), dim3(256),
                       0, s, gm, probs, P, hop, onsite, gons, gprobs);
    hop = ghop;
    onsite = gons;
    probs = gprobs;
  }
  char *slabs = next;
  const int D = plan->info.dim, LD = plan->info.lead_dim, grid = graph_grid(P, D);
  switch (plan->m) {
    case 1: launch_graph<1>(D, LD, grid, s, img, probs, P, hop, onsite, sigma, T, GLL, pstatus, slabs); break;
    case 2: launch_graph<2>(D, LD, grid, s, img, probs, P, hop, onsite, sigma, T, GLL, pstatus, slabs); break;
    case 3: launch_graph<3>(D, LD, grid, s, img, probs, P, hop, onsite, sigma, T, GLL, pstatus, slabs); break;
    default: launch_graph<4>(D, LD, grid, s, img, probs, P, hop, onsite, sigma, T, GLL, pstatus, slabs); break;
  }
  return hipGetLastError() == hipSuccess ? KNIT_OK : KNIT_E_DEVICE;
}
