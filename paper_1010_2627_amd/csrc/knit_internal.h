// Internal declarations shared by the libknit host layer and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/knit.h"
#include "knit_num.h"

namespace knit {

// Strip class as the kernels see it (device pointers, by value in kernel args).
struct StripDev {
  int M, norb;
  const knit_z *H0;
  const int32_t *vcol;
  const knit_z *vblk;
  const knit_z *V;        // dense [M][M] inter-slice hopping, or null (block-monomial vcol / vblk)
  int onsite_dense;       // on-site terms as [M][M] per slice instead of site blocks
  int h0_band;            // 0, or the site-block half-bandwidth of H0 (blocks outside it are zero)
  // elements of one slice's on-site term in the on-site buffer
  __host__ __device__ int64_t onsite_stride() const {
    return onsite_dense ? (int64_t)M * M : (int64_t)M * norb;
  }
};

struct StripTable {
  int n;
  StripDev s[KNIT_MAX_STRIPS];
};

// H0[a][b] and the dense inter-slice hopping V[a][b] = H_{n,n-1}(a, b) of a strip.
__device__ __forceinline__ cpx<double> ld_z(const knit_z *p) { return {p->re, p->im}; }
__device__ __forceinline__ void st_z(knit_z *p, cpx<double> v) {
  p->re = v.re;
  p->im = v.im;
}
__device__ __forceinline__ cpx<double> strip_V(const StripDev &s, int a, int b) {
  if (s.V) return ld_z(s.V + (int64_t)a * s.M + b);
  const int no = s.norb;
  const int sa = a / no, oa = a % no, sb = b / no, ob = b % no;
  if (s.vcol[sa] != sb) return {0.0, 0.0};
  return ld_z(s.vblk + ((int64_t)sa * no + oa) * no + ob);
}

// Host-side validation shared by the entry points (abi.hip): the strip table,
// the precision and the problem table (largest slice dimension to *Mmax).
bool batch_ok(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host, int32_t P,
              int32_t precision, int *Mmax);
StripTable strip_table_of(const knit_strip *strips, int32_t n);

// Launch wrappers (defined in the .hip files).
hipError_t launch_decimation(const StripDev &s, int side, const double *E, int nE, double eta,
                             double tol, int max_iter, knit_z *sigma, int32_t *iters,
                             int32_t *pstatus, void *ws, hipStream_t stream);
size_t decimation_workspace(int M, int nE);
// Double-double products of the decimation: 1 on the INT8 matrix cores, 0 on the vector units.
void decimation_products_set(int int8);
int decimation_products_get();

// Matrix-core FP64 inverses of n identity-padded [Mp][Mp] matrices (Mp = the
// slice padding of M, at most 512), in place; natural-order inverses to out.
int mfma_padded(int M);
size_t inverse_fp64_scratch_elems(int M);
hipError_t launch_inverse_fp64(cpx<double> *X, int64_t xstride, cpx<double> *scratch, int64_t sstride, int M,
                               cpx<double> *out, int64_t ostride, const int32_t *skip, int skip_stride,
                               int32_t *flags, int flags_stride, int n, hipStream_t stream);

constexpr int SWEEP_MAX_GRID = 512;   // upper bound of resident sweep workgroups

bool sweep_mfma_supports(int Mmax);
int sweep_tuning_set(int precision, int cls, const knit_sweep_tuning *t);
int sweep_set_refine_threshold(double t);
double sweep_get_refine_threshold();
knit_sweep_tuning sweep_tuning_get(int precision, int Mpmax);
knit_sweep_tuning sweep_default_tuning(int Mpmax);
bool sweep_tuning_valid(int Mpmax, const knit_sweep_tuning &t);
// dense: the batch has a strip with a dense inter-slice hopping (extra slab buffers)
size_t sweep_mfma_workspace(int Mmax, int precision, int P, bool dense);
// Resident workgroups of a matrix-core sweep whose workspace fits in `bytes`
// (0 if not even one does).
int sweep_mfma_grid_within(size_t bytes, int Mmax, int precision, int P, bool dense);
// max_grid > 0 caps the number of resident workgroups (the workspace then
// needs room for that many slabs only).
hipError_t launch_sweep_mfma(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                             const knit_z *sigmaL, const knit_z *sigmaR, int precision, knit_z *G1N,
                             knit_z *GN1, knit_z *GNN, int32_t *pstatus, void *ws, int Mmax, int max_grid,
                             hipStream_t stream);

size_t sweep_slab_bytes(int Mmax, int precision);
int sweep_grid(int P);
hipError_t launch_sweep(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                        const knit_z *sigmaL, const knit_z *sigmaR, int precision, knit_z *G1N,
                        knit_z *GN1, knit_z *GNN, int32_t *pstatus, void *ws, size_t slab_bytes,
                        int Mmax, hipStream_t stream);

hipError_t launch_sweep_projected(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                                  const knit_z *sigmaL, const knit_z *sigmaR, const knit_z *CL, int precision,
                                  knit_z *G1Np, knit_z *GNN, int32_t *pstatus, void *ws, int Mmax, int max_grid,
                                  hipStream_t stream);
hipError_t launch_gamma_factor(int M, const knit_z *sigma, int n, double tol, knit_z *C, int32_t *rank,
                               hipStream_t stream);
hipError_t launch_transmission_proj(const StripTable &tab, const knit_problem *probs, int P, const knit_z *CR,
                                    const knit_z *G1Np, double *T, hipStream_t stream);

size_t lesser_mfma_workspace(int Mmax, int Lmax, int stride, int P, bool dense);
hipError_t launch_lesser_mfma(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                              const knit_z *sigmaL, const knit_z *sigmaR, const knit_z *CL, int stride,
                              knit_z *blk, const int64_t *blk_off, double *jlong, double *jtran, int32_t *pstatus,
                              void *ws, int Mmax, int Lmax, hipStream_t stream);

size_t multiterminal_mfma_workspace(int Mmax, int Lmax, int stride, int n_side, int P);
hipError_t launch_multiterminal_mfma(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                                     const knit_z *sigmaL, const knit_z *sigmaR, const knit_z *CL, const knit_z *CR,
                                     int n_side, const knit_lead *side, const knit_z *sigmaX, const knit_z *CX,
                                     int stride, double *T, int32_t *pstatus, void *ws, int Mmax, int Lmax,
                                     hipStream_t stream);

size_t transmission_eigs_workspace(int Mmax, int P);
hipError_t launch_transmission_eigs(const StripTable &tab, const knit_problem *probs, int P, int Mmax,
                                    const knit_z *CR, const knit_z *G1Np, int ld, double *tn, int32_t *nch,
                                    double *T, double *fano, void *ws, hipStream_t stream);

hipError_t launch_transmission(const StripTable &tab, const knit_problem *probs, int P,
                               const knit_z *sigmaL, const knit_z *sigmaR, const knit_z *G1N,
                               const knit_z *GN1, const knit_z *GNN, double *T, double *T_RL,
                               double *T_ward, hipStream_t stream);

size_t ldos_slab_bytes(int Mmax, int Lmax, int stride, int precision);
size_t ldos_mfma_workspace(int Mmax, int Lmax, int stride, int precision, int P, bool dense);
hipError_t launch_ldos_mfma(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                            const knit_z *sigmaL, const knit_z *sigmaR, int precision, int stride, double *ldos,
                            int32_t *pstatus, void *ws, int Mmax, int Lmax, hipStream_t stream);
hipError_t launch_ldos(const StripTable &tab, const knit_problem *probs, int P, const knit_z *onsite,
                       const knit_z *sigmaL, const knit_z *sigmaR, int precision, int stride,
                       double *ldos, int32_t *pstatus, void *ws, size_t slab_bytes, int Mmax,
                       hipStream_t stream);

}  // namespace knit
