// Fisher-Lee transmission (section 2.3, T_kl = G_kl Gamma_l G_lk^+ Gamma_k),
// FP64, one workgroup per problem.
//
// With Gamma = i (Sigma - Sigma^+) Hermitian,
//   Re Tr[Ga G Gb G^+] = Re sum_{a,c} (Ga G)[a,c] * conj((G Gb)[a,c]),
// so one pass over 32 x 32 output tiles forms both products (Gamma built on
// the fly from Sigma) and reduces their elementwise product.

#include "knit_internal.h"
#include "knit_wg.h"

namespace knit {

namespace {

using Z = cpx<double>;

__device__ __forceinline__ Z gamma_at(const knit_z *sig, int M, int a, int b) {
  // i (S[a][b] - conj(S[b][a]))
  Z x = ld_z(sig + (int64_t)a * M + b), y = ld_z(sig + (int64_t)b * M + a);
  Z d = {x.re - y.re, x.im + y.im};
  return {-d.im, d.re};
}

// Re Tr[Gamma_A G Gamma_B G^+] for one problem; every thread gets the result.
__device__ double fl_trace(const knit_z *sA, const knit_z *G, const knit_z *sB, int M, Z *lds,
                           double *sv) {
  constexpr int T = 32, TK = 16;
  Z *GA = lds;                 // [T][TK]  Gamma_A[a0+r][b0+k]
  Z *Gk = GA + T * TK;         // [TK][T]  G[b0+k][c0+c]
  Z *Ga = Gk + TK * T;         // [T][TK]  G[a0+r][b0+k]
  Z *GB = Ga + T * TK;         // [TK][T]  Gamma_B[b0+k][c0+c]
  const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
  double part = 0.0;
  for (int a0 = 0; a0 < M; a0 += T)
    for (int c0 = 0; c0 < M; c0 += T) {
      Z x[2][2], y[2][2];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) x[i][j] = y[i][j] = Z{0.0, 0.0};
      for (int b0 = 0; b0 < M; b0 += TK) {
        for (int e = tid; e < T * TK; e += blockDim.x) {
          int r = e / TK, k = e % TK;
          bool ok = a0 + r < M && b0 + k < M;
          GA[e] = ok ? gamma_at(sA, M, a0 + r, b0 + k) : Z{0.0, 0.0};
          Ga[e] = ok ? ld_z(G + (int64_t)(a0 + r) * M + b0 + k) : Z{0.0, 0.0};
          int k2 = e / T, c = e % T;
          bool ok2 = b0 + k2 < M && c0 + c < M;
          Gk[e] = ok2 ? ld_z(G + (int64_t)(b0 + k2) * M + c0 + c) : Z{0.0, 0.0};
          GB[e] = ok2 ? gamma_at(sB, M, b0 + k2, c0 + c) : Z{0.0, 0.0};
        }
        __syncthreads();
        for (int k = 0; k < TK; ++k) {
          Z a0v = GA[(tr * 2) * TK + k], a1v = GA[(tr * 2 + 1) * TK + k];
          Z g0 = Gk[k * T + tc * 2], g1 = Gk[k * T + tc * 2 + 1];
          x[0][0] = c_fma(a0v, g0, x[0][0]);
          x[0][1] = c_fma(a0v, g1, x[0][1]);
          x[1][0] = c_fma(a1v, g0, x[1][0]);
          x[1][1] = c_fma(a1v, g1, x[1][1]);
          Z h0 = Ga[(tr * 2) * TK + k], h1 = Ga[(tr * 2 + 1) * TK + k];
          Z b0v = GB[k * T + tc * 2], b1v = GB[k * T + tc * 2 + 1];
          y[0][0] = c_fma(h0, b0v, y[0][0]);
          y[0][1] = c_fma(h0, b1v, y[0][1]);
          y[1][0] = c_fma(h1, b0v, y[1][0]);
          y[1][1] = c_fma(h1, b1v, y[1][1]);
        }
        __syncthreads();
      }
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          if (a0 + tr * 2 + i < M && c0 + tc * 2 + j < M)
            part += x[i][j].re * y[i][j].re + x[i][j].im * y[i][j].im;   // Re(x conj(y))
    }
  // workgroup sum
  for (int off = WAVE / 2; off > 0; off >>= 1) part += __shfl_xor(part, off, WAVE);
  if (tid % WAVE == 0) sv[tid / WAVE] = part;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) s += sv[w];
  __syncthreads();
  return s;
}

__global__ void __launch_bounds__(WG) transmission_kernel(StripTable tab, const knit_problem *probs,
                                                          int P, const knit_z *sigmaL,
                                                          const knit_z *sigmaR, const knit_z *G1N,
                                                          const knit_z *GN1, const knit_z *GNN,
                                                          double *T, double *T_RL, double *T_ward) {
  __shared__ Z lds[4 * 32 * 16];
  __shared__ double sv[WG / WAVE];
  const int p = blockIdx.x;
  if (p >= P) return;
  const knit_problem pr = probs[p];
  const int M = tab.s[pr.strip].M;
  const knit_z *sL = sigmaL + pr.sigma_off, *sR = sigmaR + pr.sigma_off;
  double t = fl_trace(sL, G1N + pr.out_off, sR, M, lds, sv);
  if (threadIdx.x == 0) T[p] = t;
  if (T_RL && GN1) {
    double t2 = fl_trace(sR, GN1 + pr.out_off, sL, M, lds, sv);
    if (threadIdx.x == 0) T_RL[p] = t2;
  }
  if (T_ward && GNN) {
    const knit_z *G = GNN + pr.out_off;
    // Re Tr[Gamma_R i (G - G^+)] = Re sum_{a,b} GR[a][b] * i (G[b][a] - conj(G[a][b]))
    double part = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)M * M; e += blockDim.x) {
      const int a = (int)(e / M), b = (int)(e % M);
      Z gr = gamma_at(sR, M, a, b);
      Z x = ld_z(G + (int64_t)b * M + a), y = ld_z(G + (int64_t)a * M + b);
      Z d = {x.re - y.re, x.im + y.im};   // G[b][a] - conj(G[a][b])
      Z id = {-d.im, d.re};
      part += gr.re * id.re - gr.im * id.im;
    }
    for (int off = WAVE / 2; off > 0; off >>= 1) part += __shfl_xor(part, off, WAVE);
    __syncthreads();
    if (threadIdx.x % WAVE == 0) sv[threadIdx.x / WAVE] = part;
    __syncthreads();
    double s1 = 0.0;
    for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) s1 += sv[w];
    __syncthreads();
    double s2 = fl_trace(sR, G, sR, M, lds, sv);
    if (threadIdx.x == 0) T_ward[p] = s1 - s2;
  }
}

// Gamma = C C^+ by Cholesky with diagonal pivoting (left-looking), one
// workgroup per matrix: at step k the largest remaining diagonal entry d_p is
// the pivot, column k of C is (Gamma[:, p] - sum_{j<k} C[:, j] conj(C[p, j])) / sqrt(d_p),
// and every remaining diagonal entry loses |C[i, k]|^2.  Stops when the
// largest remaining entry is <= tol * max_i |Sigma_ii| (the scale of the
// rounding noise in Gamma, so that a Gamma of pure noise, outside the band,
// gets rank 0); the step count is the numerical rank (for a lead: its open
// channels).  C is [M][M] row-major,
// columns >= rank zero.  d and the chosen flags live in LDS.
__global__ void __launch_bounds__(WG) gamma_factor_kernel(int M, const knit_z *sigma, double tol, knit_z *Cout,
                                                          int32_t *rank) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double *d = reinterpret_cast<double *>(lds_raw);          // [M] remaining diagonal
  int *chosen = reinterpret_cast<int *>(d + M);             // [M]
  __shared__ double sv[WG / WAVE];
  __shared__ int si[WG / WAVE];
  const int e = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const knit_z *sig = sigma + (int64_t)e * M * M;
  knit_z *C = Cout + (int64_t)e * M * M;
  for (int64_t i = tid; i < (int64_t)M * M; i += nt) st_z(C + i, Z{0.0, 0.0});
  double smax = 0.0;
  for (int i = tid; i < M; i += nt) {
    d[i] = gamma_at(sig, M, i, i).re;
    chosen[i] = 0;
    const Z sd = ld_z(sig + (int64_t)i * M + i);
    double a = sqrt(sd.re * sd.re + sd.im * sd.im);
    if (a != a) a = INFINITY;
    smax = fmax(smax, a);
  }
  smax = wg_max(smax, sv);   // NaN or Inf anywhere on the diagonal gives +inf
  if (!(smax < INFINITY)) {
    // a non-finite Sigma: C of NaN so that every later step reports it
    const double qn = __builtin_nan("");
    for (int64_t i = tid; i < (int64_t)M * M; i += nt) st_z(C + i, Z{qn, qn});
    if (tid == 0) rank[e] = -1;
    return;
  }
  __syncthreads();
  int k = 0;
  for (; k < M; ++k) {
    // pivot: largest remaining diagonal entry (lowest index on ties)
    double best = -1.0;
    int bi = M;
    for (int i = tid; i < M; i += nt)
      if (!chosen[i] && (d[i] > best)) {
        best = d[i];
        bi = i;
      }
    wg_argmax(best, bi, sv, si);
    const int p = bi;
    const double dp = best;
    if (!(dp > tol * smax) || p >= M) break;
    const double inv = 1.0 / sqrt(dp);
    // column k: (Gamma[:, p] - sum_{j<k} C[:, j] conj(C[p, j])) / sqrt(d_p)
    for (int i = tid; i < M; i += nt) {
      Z acc = gamma_at(sig, M, i, p);
      const knit_z *ci = C + (int64_t)i * M, *cp = C + (int64_t)p * M;
      for (int j = 0; j < k; ++j) acc = c_sub(acc, c_mul(ld_z(ci + j), c_conj(ld_z(cp + j))));
      // the pivot entry is (d_p) / sqrt(d_p): written as sqrt(d_p), exactly real
      acc = i == p ? Z{dp * inv, 0.0} : Z{acc.re * inv, acc.im * inv};
      st_z(C + (int64_t)i * M + k, acc);
      d[i] = i == p ? 0.0 : d[i] - (acc.re * acc.re + acc.im * acc.im);
    }
    __syncthreads();
    if (tid == 0) chosen[p] = 1;
    __syncthreads();
  }
  if (tid == 0) rank[e] = k;
}

// T = || P C_R ||_F^2 with P = C_L^+ G_1N (the projected propagator, [M][M]
// with rows beyond C_L's columns zero) and Gamma_R = C_R C_R^+: equal to
// Re Tr[Gamma_L G_1N Gamma_R G_1N^+].  Rows of P after its last nonzero row and
// columns of C_R after its last nonzero column add nothing and are skipped.
// One workgroup per problem (WG = 256: a 16 x 16 thread grid over 32 x 32 tiles).
__global__ void __launch_bounds__(WG) transmission_proj_kernel(StripTable tab, const knit_problem *probs, int P,
                                                               const knit_z *CR, const knit_z *G1Np, double *T) {
  constexpr int TT = 32, TK = 16;
  __shared__ Z As[TT * TK];
  __shared__ Z Bs[TK * TT];
  __shared__ double sv[WG / WAVE];
  const int p = blockIdx.x;
  if (p >= P) return;
  const knit_problem pr = probs[p];
  const int M = tab.s[pr.strip].M;
  const knit_z *Pm = G1Np + pr.out_off, *Cm = CR + pr.sigma_off;
  const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
  double lr = 0.0, lc = 0.0;
  for (int64_t i = tid; i < (int64_t)M * M; i += blockDim.x) {
    const Z a = ld_z(Pm + i), c = ld_z(Cm + i);
    if (a.re != 0.0 || a.im != 0.0) lr = fmax(lr, (double)(i / M + 1));
    if (c.re != 0.0 || c.im != 0.0) lc = fmax(lc, (double)(i % M + 1));
  }
  const int rl = (int)wg_max(lr, sv);
  const int rr = (int)wg_max(lc, sv);
  double part = 0.0;
  for (int a0 = 0; a0 < rl; a0 += TT)
    for (int c0 = 0; c0 < rr; c0 += TT) {
      Z x[2][2];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) x[i][j] = Z{0.0, 0.0};
      for (int b0 = 0; b0 < M; b0 += TK) {
        for (int e = tid; e < TT * TK; e += blockDim.x) {
          const int r = e / TK, k = e % TK;
          As[e] = (a0 + r < rl && b0 + k < M) ? ld_z(Pm + (int64_t)(a0 + r) * M + b0 + k) : Z{0.0, 0.0};
          const int k2 = e / TT, c = e % TT;
          Bs[e] = (b0 + k2 < M && c0 + c < rr) ? ld_z(Cm + (int64_t)(b0 + k2) * M + c0 + c) : Z{0.0, 0.0};
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
        for (int j = 0; j < 2; ++j) part += x[i][j].re * x[i][j].re + x[i][j].im * x[i][j].im;
    }
  for (int off = WAVE / 2; off > 0; off >>= 1) part += __shfl_xor(part, off, WAVE);
  if (tid % WAVE == 0) sv[tid / WAVE] = part;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) s += sv[w];
    T[p] = s;
  }
}

}  // namespace

hipError_t launch_gamma_factor(int M, const knit_z *sigma, int n, double tol, knit_z *C, int32_t *rank,
                               hipStream_t stream) {
  const size_t lds = (size_t)M * (sizeof(double) + sizeof(int));
  hipLaunchKernelGGL(gamma_factor_kernel, dim3(n), dim3(WG), lds, stream, M, sigma, tol, C, rank);
  return hipGetLastError();
}

hipError_t launch_transmission_proj(const StripTable &tab, const knit_problem *probs, int P, const knit_z *CR,
                                    const knit_z *G1Np, double *T, hipStream_t stream) {
  hipLaunchKernelGGL(transmission_proj_kernel, dim3(P), dim3(WG), 0, stream, tab, probs, P, CR, G1Np, T);
  return hipGetLastError();
}

hipError_t launch_transmission(const StripTable &tab, const knit_problem *probs, int P,
                               const knit_z *sigmaL, const knit_z *sigmaR, const knit_z *G1N,
                               const knit_z *GN1, const knit_z *GNN, double *T, double *T_RL,
                               double *T_ward, hipStream_t stream) {
  hipLaunchKernelGGL(transmission_kernel, dim3(P), dim3(WG), 0, stream, tab, probs, P, sigmaL, sigmaR,
                     G1N, GN1, GNN, T, T_RL, T_ward);
  return hipGetLastError();
}

}  // namespace knit
