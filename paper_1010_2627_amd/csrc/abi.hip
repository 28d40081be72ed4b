// Host side of the C ABI declared in include/knit.h: argument validation
// (before any HIP call), workspace sizing and kernel launches.

#include <math.h>
#include <string.h>

#include "knit_internal.h"

using namespace knit;

namespace {

bool strip_ok(const knit_strip *s) {
  if (!s) return false;
  if (s->M < 1 || s->M > KNIT_MAX_M) return false;
  if (s->norb < 1 || s->norb > KNIT_MAX_NORB) return false;
  if (s->M % s->norb != 0) return false;
  if (!s->H0) return false;
  if (!s->V && (!s->vcol || !s->vblk)) return false;
  if (s->onsite_dense != 0 && s->onsite_dense != 1) return false;
  if (s->h0_band < 0) return false;
  return true;
}

StripDev strip_dev(const knit_strip &s) {
  return StripDev{s.M, s.norb, s.H0, s.vcol, s.vblk, s.V, s.onsite_dense, s.h0_band};
}

// Dense couplings and dense on-site terms run on the matrix-core kernels only.
bool generic_ok(const knit_strip *strips, int32_t n_strips) {
  for (int i = 0; i < n_strips; ++i)
    if (strips[i].V || strips[i].onsite_dense) return false;
  return true;
}

bool any_dense_v(const knit_strip *strips, int32_t n_strips) {
  for (int i = 0; i < n_strips; ++i)
    if (strips[i].V) return true;
  return false;
}

bool table_ok(const knit_strip *strips, int32_t n_strips) {
  if (!strips || n_strips < 1 || n_strips > KNIT_MAX_STRIPS) return false;
  for (int i = 0; i < n_strips; ++i)
    if (!strip_ok(strips + i)) return false;
  return true;
}

// Validates the problem table; returns largest M and L through the pointers.
bool problems_ok(const knit_strip *strips, int32_t n_strips, const knit_problem *ph, int32_t P,
                 int *Mmax, int *Lmax) {
  if (P < 0) return false;
  if (P > 0 && !ph) return false;
  int mm = 0, lm = 0;
  for (int i = 0; i < P; ++i) {
    const knit_problem &p = ph[i];
    if (p.strip < 0 || p.strip >= n_strips) return false;
    if (p.L < 1) return false;
    if (!isfinite(p.E)) return false;
    if (p.onsite_off < 0 || p.sigma_off < 0 || p.out_off < 0 || p.ldos_off < 0) return false;
    mm = strips[p.strip].M > mm ? strips[p.strip].M : mm;
    lm = p.L > lm ? p.L : lm;
  }
  if (Mmax) *Mmax = mm;
  if (Lmax) *Lmax = lm;
  return true;
}

StripTable make_table(const knit_strip *strips, int32_t n) {
  StripTable t;
  memset(&t, 0, sizeof(t));
  t.n = n;
  for (int i = 0; i < n; ++i) t.s[i] = strip_dev(strips[i]);
  return t;
}

bool precision_ok(int32_t p) { return p == KNIT_FP64 || p == KNIT_FP32_REFINE || p == KNIT_FP32; }

}  // namespace

namespace knit {

bool batch_ok(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host, int32_t P,
              int32_t precision, int *Mmax) {
  int Lmax = 0;
  return table_ok(strips, n_strips) && precision_ok(precision) &&
         problems_ok(strips, n_strips, probs_host, P, Mmax, &Lmax);
}

StripTable strip_table_of(const knit_strip *strips, int32_t n) { return make_table(strips, n); }

}  // namespace knit

namespace {

int resolve_stride(int stride, int Lmax) {
  if (stride > 0) return stride;
  int s = (int)ceil(sqrt((double)Lmax));
  return s < 1 ? 1 : s;
}

}  // namespace

extern "C" {

int knit_abi_version(void) { return KNIT_ABI_VERSION; }

const char *knit_status_string(int code) {
  switch (code) {
    case KNIT_OK: return "ok";
    case KNIT_E_ARG: return "invalid argument";
    case KNIT_E_DEVICE: return "HIP device error";
    case KNIT_E_WORKSPACE: return "workspace missing or too small";
    case KNIT_E_UNSUPPORTED: return "not supported by this library";
    case KNIT_E_SCRATCH: return "request does not fit the library's static scratch";
    case KNIT_P_SINGULAR: return "singular slice";
    case KNIT_P_NOCONV: return "decimation not converged";
    case KNIT_P_NONFINITE: return "non-finite value";
    case KNIT_P_FALLBACK: return "refinement gave up; recomputed in FP64";
    default: return "combination of problem status bits or unknown code";
  }
}

size_t knit_lead_selfenergy_workspace(const knit_strip *strip, int32_t nE) {
  if (!strip_ok(strip) || nE < 0) return 0;
  return decimation_workspace(strip->M, nE);
}

int knit_lead_selfenergy(const knit_strip *strip, int32_t side, const double *E, int32_t nE,
                         double eta, double tol, int32_t max_iter, knit_z *sigma, int32_t *iters,
                         int32_t *pstatus, void *ws, size_t ws_bytes, void *stream) {
  if (!strip_ok(strip)) return KNIT_E_ARG;
  if (side < 0 || side > 2) return KNIT_E_ARG;
  if (nE < 0) return KNIT_E_ARG;
  if (!(eta > 0.0) || !isfinite(eta)) return KNIT_E_ARG;
  if (!(tol > 0.0) || !isfinite(tol)) return KNIT_E_ARG;
  if (max_iter < 1) return KNIT_E_ARG;
  if (strip->M > KNIT_MAX_SELFENERGY_M) return KNIT_E_UNSUPPORTED;
  if (nE == 0) return KNIT_OK;
  if (!E || !sigma || !pstatus) return KNIT_E_ARG;
  const size_t need = knit_lead_selfenergy_workspace(strip, nE);
  if (!ws || ws_bytes < need) return KNIT_E_WORKSPACE;
  const StripDev s = strip_dev(*strip);
  hipError_t err = launch_decimation(s, side, E, nE, eta, tol, max_iter, sigma, iters, pstatus, ws,
                                     (hipStream_t)stream);
  return err == hipSuccess ? KNIT_OK : KNIT_E_DEVICE;
}

size_t knit_rgf_sweep_workspace(const knit_strip *strips, int32_t n_strips,
                                const knit_problem *probs_host, int32_t P, int32_t precision,
                                int32_t want_gn1) {
  (void)want_gn1;
  int Mmax = 0, Lmax = 0;
  if (!table_ok(strips, n_strips) || !precision_ok(precision)) return 0;
  if (!problems_ok(strips, n_strips, probs_host, P, &Mmax, &Lmax)) return 0;
  if (P == 0) return 0;
  if (sweep_mfma_supports(Mmax)) return sweep_mfma_workspace(Mmax, precision, P, any_dense_v(strips, n_strips));
  if (precision == KNIT_FP32_REFINE || !generic_ok(strips, n_strips)) return 0;
  return sweep_slab_bytes(Mmax, precision) * (size_t)sweep_grid(P);
}

int knit_rgf_sweep(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                   const knit_problem *probs_dev, int32_t P, const knit_z *onsite,
                   const knit_z *sigmaL, const knit_z *sigmaR, int32_t precision, knit_z *G1N,
                   knit_z *GN1, knit_z *GNN, int32_t *pstatus, void *ws, size_t ws_bytes,
                   void *stream) {
  int Mmax = 0, Lmax = 0;
  if (!table_ok(strips, n_strips) || !precision_ok(precision)) return KNIT_E_ARG;
  if (!problems_ok(strips, n_strips, probs_host, P, &Mmax, &Lmax)) return KNIT_E_ARG;
  if (P == 0) return KNIT_OK;
  if (!probs_dev || !onsite || !sigmaL || !sigmaR || !G1N || !pstatus) return KNIT_E_ARG;
  const bool fast = sweep_mfma_supports(Mmax);
  if (!fast && (precision == KNIT_FP32_REFINE || !generic_ok(strips, n_strips))) return KNIT_E_UNSUPPORTED;
  const size_t need = knit_rgf_sweep_workspace(strips, n_strips, probs_host, P, precision, GN1 != nullptr);
  if (!ws || ws_bytes < need) return KNIT_E_WORKSPACE;
  StripTable tab = make_table(strips, n_strips);
  hipError_t err;
  if (fast)
    err = launch_sweep_mfma(tab, probs_dev, P, onsite, sigmaL, sigmaR, precision, G1N, GN1, GNN, pstatus, ws,
                            Mmax, 0, (hipStream_t)stream);
  else
    err = launch_sweep(tab, probs_dev, P, onsite, sigmaL, sigmaR, precision, G1N, GN1, GNN, pstatus, ws,
                       sweep_slab_bytes(Mmax, precision), Mmax, (hipStream_t)stream);
  return err == hipSuccess ? KNIT_OK : KNIT_E_DEVICE;
}

int knit_set_refine_threshold(double threshold) {
  if (!(threshold >= 0.0)) return KNIT_E_ARG;   // also rejects NaN
  sweep_set_refine_threshold(threshold);
  return KNIT_OK;
}

double knit_get_refine_threshold(void) { return sweep_get_refine_threshold(); }

int knit_set_selfenergy_products(int32_t mode) {
  if (mode != KNIT_PRODUCTS_VECTOR && mode != KNIT_PRODUCTS_INT8) return KNIT_E_ARG;
  decimation_products_set(mode == KNIT_PRODUCTS_INT8);
  return KNIT_OK;
}

int32_t knit_get_selfenergy_products(void) {
  return decimation_products_get() ? KNIT_PRODUCTS_INT8 : KNIT_PRODUCTS_VECTOR;
}

int knit_sweep_tuning_set(int32_t precision, int32_t cls, const knit_sweep_tuning *t) {
  if (!precision_ok(precision) || cls < 0 || cls >= KNIT_TUNING_CLASSES) return KNIT_E_ARG;
  if (t && !sweep_tuning_valid(32 * (cls + 1), *t)) return KNIT_E_ARG;
  sweep_tuning_set(precision, cls, t);
  return KNIT_OK;
}

int knit_sweep_tuning_get(int32_t precision, int32_t cls, knit_sweep_tuning *t) {
  if (!precision_ok(precision) || cls < 0 || cls >= KNIT_TUNING_CLASSES || !t) return KNIT_E_ARG;
  *t = sweep_tuning_get(precision, 32 * (cls + 1));
  return KNIT_OK;
}

int knit_transmission(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                      const knit_problem *probs_dev, int32_t P, const knit_z *sigmaL,
                      const knit_z *sigmaR, const knit_z *G1N, const knit_z *GN1,
                      const knit_z *GNN, double *T, double *T_RL, double *T_ward, void *stream) {
  if (!table_ok(strips, n_strips)) return KNIT_E_ARG;
  if (!problems_ok(strips, n_strips, probs_host, P, nullptr, nullptr)) return KNIT_E_ARG;
  if (P == 0) return KNIT_OK;
  if (!probs_dev || !sigmaL || !sigmaR || !G1N || !T) return KNIT_E_ARG;
  if (T_RL && !GN1) return KNIT_E_ARG;
  if (T_ward && !GNN) return KNIT_E_ARG;
  StripTable tab = make_table(strips, n_strips);
  hipError_t err = launch_transmission(tab, probs_dev, P, sigmaL, sigmaR, G1N, GN1, GNN, T, T_RL,
                                       T_ward, (hipStream_t)stream);
  return err == hipSuccess ? KNIT_OK : KNIT_E_DEVICE;
}

size_t knit_ldos_workspace(const knit_strip *strips, int32_t n_strips,
                           const knit_problem *probs_host, int32_t P, int32_t precision,
                           int32_t checkpoint_stride) {
  int Mmax = 0, Lmax = 0;
  if (!table_ok(strips, n_strips) || !precision_ok(precision)) return 0;
  if (!problems_ok(strips, n_strips, probs_host, P, &Mmax, &Lmax)) return 0;
  if (P == 0) return 0;
  const int st = resolve_stride(checkpoint_stride, Lmax);
  if (sweep_mfma_supports(Mmax)) return ldos_mfma_workspace(Mmax, Lmax, st, precision, P, any_dense_v(strips, n_strips));
  if (precision == KNIT_FP32_REFINE || !generic_ok(strips, n_strips)) return 0;
  const int grid = P < 1024 ? P : 1024;
  return ldos_slab_bytes(Mmax, Lmax, st, precision) * (size_t)grid;
}

int knit_ldos(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
              const knit_problem *probs_dev, int32_t P, const knit_z *onsite,
              const knit_z *sigmaL, const knit_z *sigmaR, int32_t precision,
              int32_t checkpoint_stride, double *ldos, int32_t *pstatus, void *ws,
              size_t ws_bytes, void *stream) {
  int Mmax = 0, Lmax = 0;
  if (!table_ok(strips, n_strips) || !precision_ok(precision)) return KNIT_E_ARG;
  if (!problems_ok(strips, n_strips, probs_host, P, &Mmax, &Lmax)) return KNIT_E_ARG;
  if (P == 0) return KNIT_OK;
  if (!probs_dev || !onsite || !sigmaL || !sigmaR || !ldos || !pstatus) return KNIT_E_ARG;
  if (!sweep_mfma_supports(Mmax) && (precision == KNIT_FP32_REFINE || !generic_ok(strips, n_strips)))
    return KNIT_E_UNSUPPORTED;
  const int st = resolve_stride(checkpoint_stride, Lmax);
  const size_t need = knit_ldos_workspace(strips, n_strips, probs_host, P, precision, checkpoint_stride);
  if (!ws || ws_bytes < need) return KNIT_E_WORKSPACE;
  StripTable tab = make_table(strips, n_strips);
  hipError_t err;
  if (sweep_mfma_supports(Mmax))
    err = launch_ldos_mfma(tab, probs_dev, P, onsite, sigmaL, sigmaR, precision, st, ldos, pstatus, ws, Mmax, Lmax,
                           (hipStream_t)stream);
  else
    err = launch_ldos(tab, probs_dev, P, onsite, sigmaL, sigmaR, precision, st, ldos, pstatus, ws,
                      ldos_slab_bytes(Mmax, Lmax, st, precision), Mmax, (hipStream_t)stream);
  return err == hipSuccess ? KNIT_OK : KNIT_E_DEVICE;
}

int knit_gamma_factor(int32_t M, const knit_z *sigma, int32_t n, double tol, knit_z *C, int32_t *rank,
                      void *stream) {
  if (M < 1 || M > KNIT_MAX_M || n < 0 || isnan(tol)) return KNIT_E_ARG;
  if (n == 0) return KNIT_OK;
  if (!sigma || !C || !rank) return KNIT_E_ARG;
  if (!(tol > 0.0)) tol = 1e-10;
  hipError_t err = launch_gamma_factor(M, sigma, n, tol, C, rank, (hipStream_t)stream);
  return err == hipSuccess ? KNIT_OK : KNIT_E_DEVICE;
}

int knit_rgf_sweep_projected(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                             const knit_problem *probs_dev, int32_t P, const knit_z *onsite,
                             const knit_z *sigmaL, const knit_z *sigmaR, const knit_z *CL, int32_t precision,
                             knit_z *G1Np, knit_z *GNN, int32_t *pstatus, void *ws, size_t ws_bytes, void *stream) {
  int Mmax = 0, Lmax = 0;
  if (!table_ok(strips, n_strips) || !precision_ok(precision)) return KNIT_E_ARG;
  if (!problems_ok(strips, n_strips, probs_host, P, &Mmax, &Lmax)) return KNIT_E_ARG;
  if (P == 0) return KNIT_OK;
  if (!probs_dev || !onsite || !sigmaL || !sigmaR || !CL || !G1Np || !pstatus) return KNIT_E_ARG;
  if (!sweep_mfma_supports(Mmax)) return KNIT_E_UNSUPPORTED;
  const size_t need = knit_rgf_sweep_workspace(strips, n_strips, probs_host, P, precision, 0);
  if (!ws || ws_bytes < need) return KNIT_E_WORKSPACE;
  StripTable tab = make_table(strips, n_strips);
  hipError_t err = launch_sweep_projected(tab, probs_dev, P, onsite, sigmaL, sigmaR, CL, precision, G1Np, GNN,
                                          pstatus, ws, Mmax, 0, (hipStream_t)stream);
  return err == hipSuccess ? KNIT_OK : KNIT_E_DEVICE;
}

int knit_transmission_projected(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                                const knit_problem *probs_dev, int32_t P, const knit_z *CR,
                                const knit_z *G1Np, double *T, void *stream) {
  if (!table_ok(strips, n_strips)) return KNIT_E_ARG;
  if (!problems_ok(strips, n_strips, probs_host, P, nullptr, nullptr)) return KNIT_E_ARG;
  if (P == 0) return KNIT_OK;
  if (!probs_dev || !CR || !G1Np || !T) return KNIT_E_ARG;
  StripTable tab = make_table(strips, n_strips);
  hipError_t err = launch_transmission_proj(tab, probs_dev, P, CR, G1Np, T, (hipStream_t)stream);
  return err == hipSuccess ? KNIT_OK : KNIT_E_DEVICE;
}

size_t knit_transmission_eigenvalues_workspace(const knit_strip *strips, int32_t n_strips,
                                               const knit_problem *probs_host, int32_t P) {
  int Mmax = 0, Lmax = 0;
  if (!table_ok(strips, n_strips)) return 0;
  if (!problems_ok(strips, n_strips, probs_host, P, &Mmax, &Lmax)) return 0;
  if (P == 0) return 0;
  return transmission_eigs_workspace(Mmax, P);
}

int knit_transmission_eigenvalues(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                                  const knit_problem *probs_dev, int32_t P, const knit_z *CR, const knit_z *G1Np,
                                  int32_t ld, double *tn, int32_t *nch, double *T, double *fano, void *ws,
                                  size_t ws_bytes, void *stream) {
  int Mmax = 0, Lmax = 0;
  if (!table_ok(strips, n_strips)) return KNIT_E_ARG;
  if (!problems_ok(strips, n_strips, probs_host, P, &Mmax, &Lmax)) return KNIT_E_ARG;
  if (P == 0) return KNIT_OK;
  if (!probs_dev || !CR || !G1Np || !tn || ld < Mmax) return KNIT_E_ARG;
  const size_t need = knit_transmission_eigenvalues_workspace(strips, n_strips, probs_host, P);
  if (!ws || ws_bytes < need) return KNIT_E_WORKSPACE;
  StripTable tab = make_table(strips, n_strips);
  hipError_t err = launch_transmission_eigs(tab, probs_dev, P, Mmax, CR, G1Np, ld, tn, nch, T, fano, ws,
                                            (hipStream_t)stream);
  return err == hipSuccess ? KNIT_OK : KNIT_E_DEVICE;
}

size_t knit_local_observables_workspace(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                                        int32_t P, int32_t checkpoint_stride) {
  int Mmax = 0, Lmax = 0;
  if (!table_ok(strips, n_strips)) return 0;
  if (!problems_ok(strips, n_strips, probs_host, P, &Mmax, &Lmax)) return 0;
  if (P == 0 || !sweep_mfma_supports(Mmax)) return 0;
  return lesser_mfma_workspace(Mmax, Lmax, resolve_stride(checkpoint_stride, Lmax), P, any_dense_v(strips, n_strips));
}

int knit_local_observables(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                           const knit_problem *probs_dev, int32_t P, const knit_z *onsite, const knit_z *sigmaL,
                           const knit_z *sigmaR, const knit_z *CL, int32_t checkpoint_stride, knit_z *blk,
                           const int64_t *blk_off, double *jlong, double *jtran, int32_t *pstatus, void *ws,
                           size_t ws_bytes, void *stream) {
  int Mmax = 0, Lmax = 0;
  if (!table_ok(strips, n_strips)) return KNIT_E_ARG;
  if (!problems_ok(strips, n_strips, probs_host, P, &Mmax, &Lmax)) return KNIT_E_ARG;
  if (P == 0) return KNIT_OK;
  if (!probs_dev || !onsite || !sigmaL || !sigmaR || !CL || !blk || !blk_off || !jlong || !jtran || !pstatus)
    return KNIT_E_ARG;
  if (!sweep_mfma_supports(Mmax)) return KNIT_E_UNSUPPORTED;
  const int st = resolve_stride(checkpoint_stride, Lmax);
  const size_t need = knit_local_observables_workspace(strips, n_strips, probs_host, P, checkpoint_stride);
  if (!ws || ws_bytes < need) return KNIT_E_WORKSPACE;
  StripTable tab = make_table(strips, n_strips);
  hipError_t err = launch_lesser_mfma(tab, probs_dev, P, onsite, sigmaL, sigmaR, CL, st, blk, blk_off, jlong, jtran,
                                      pstatus, ws, Mmax, Lmax, (hipStream_t)stream);
  return err == hipSuccess ? KNIT_OK : KNIT_E_DEVICE;
}

size_t knit_conductance_matrix_workspace(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                                         int32_t P, int32_t n_side, int32_t checkpoint_stride) {
  int Mmax = 0, Lmax = 0;
  if (!table_ok(strips, n_strips)) return 0;
  if (!problems_ok(strips, n_strips, probs_host, P, &Mmax, &Lmax)) return 0;
  if (P == 0 || n_side < 0 || n_side > KNIT_MAX_SIDE_LEADS || !sweep_mfma_supports(Mmax)) return 0;
  return multiterminal_mfma_workspace(Mmax, Lmax, resolve_stride(checkpoint_stride, Lmax), n_side, P);
}

int knit_conductance_matrix(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                            const knit_problem *probs_dev, int32_t P, const knit_z *onsite, const knit_z *sigmaL,
                            const knit_z *sigmaR, const knit_z *CL, const knit_z *CR, int32_t n_side,
                            const knit_lead *side_host, const knit_lead *side_dev, const knit_z *sigmaX,
                            const knit_z *CX, int32_t checkpoint_stride, double *T, int32_t *pstatus, void *ws,
                            size_t ws_bytes, void *stream) {
  int Mmax = 0, Lmax = 0;
  if (!table_ok(strips, n_strips)) return KNIT_E_ARG;
  if (!problems_ok(strips, n_strips, probs_host, P, &Mmax, &Lmax)) return KNIT_E_ARG;
  if (n_side < 0 || n_side > KNIT_MAX_SIDE_LEADS) return KNIT_E_ARG;
  if (P == 0) return KNIT_OK;
  if (!probs_dev || !onsite || !sigmaL || !sigmaR || !CL || !CR || !T || !pstatus) return KNIT_E_ARG;
  if (n_side > 0) {
    if (!side_host || !side_dev || !sigmaX || !CX) return KNIT_E_ARG;
    for (int p = 0; p < P; ++p)
      for (int j = 0; j < n_side; ++j) {
        const knit_lead &l = side_host[(int64_t)p * n_side + j];
        if (l.slice < 0 || l.slice >= probs_host[p].L || l.sigma_off < 0) return KNIT_E_ARG;
      }
  }
  if (!sweep_mfma_supports(Mmax)) return KNIT_E_UNSUPPORTED;
  const int st = resolve_stride(checkpoint_stride, Lmax);
  const size_t need = knit_conductance_matrix_workspace(strips, n_strips, probs_host, P, n_side, checkpoint_stride);
  if (!ws || ws_bytes < need) return KNIT_E_WORKSPACE;
  StripTable tab = make_table(strips, n_strips);
  hipError_t err = launch_multiterminal_mfma(tab, probs_dev, P, onsite, sigmaL, sigmaR, CL, CR, n_side, side_dev,
                                             sigmaX, CX, st, T, pstatus, ws, Mmax, Lmax, (hipStream_t)stream);
  return err == hipSuccess ? KNIT_OK : KNIT_E_DEVICE;
}

}  // extern "C"
