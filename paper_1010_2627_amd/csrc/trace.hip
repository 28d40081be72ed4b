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

}  // namespace

hipError_t launch_transmission(const StripTable &tab, const knit_problem *probs, int P,
                               const knit_z *sigmaL, const knit_z *sigmaR, const knit_z *G1N,
                               const knit_z *GN1, const knit_z *GNN, double *T, double *T_RL,
                               double *T_ward, hipStream_t stream) {
  hipLaunchKernelGGL(transmission_kernel, dim3(P), dim3(WG), 0, stream, tab, probs, P, sigmaL, sigmaR,
                     G1N, GN1, GNN, T, T_RL, T_ward);
  return hipGetLastError();
}

}  // namespace knit
