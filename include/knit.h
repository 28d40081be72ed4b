/*
 * knit.h -- C ABI of libknit: the two-lead strip transport path on MI355X (gfx950).
 *
 * What is computed (tight-binding model of Eq. (1), objects of section 2.3):
 * a strip of L identical-width slices n = 1..L, slice Hamiltonians
 * H_n = H0 + D_n (D_n: per-site on-site blocks, e.g. disorder), inter-slice
 * hopping V = H_{n,n-1}, and two semi-infinite leads made by repeating the
 * clean slice (H0, V) (section 5.3-B; the interface slices 1 and L belong to
 * both system and lead).  The leads enter as self-energies Sigma_L on slice 1
 * and Sigma_R on slice L; the retarded Green function is
 * G = (E - H - Sigma_L - Sigma_R)^{-1} (Eq. (2), read with Im Sigma <= 0), and
 * the transmission between the leads is T = Tr[Gamma_L G_1L Gamma_R G_1L^+]
 * with Gamma = i (Sigma - Sigma^+) (section 2.3, T_kl and its Landauer
 * conductance).  The basic recursive Green function algorithm (section 1)
 * adds the slices one at a time from the left lead to the right lead; the
 * local density of states comes from the reverse sweep (the "sewing" of
 * section 5.3-D).  Since Gamma_L = C_L C_L^+ has the rank of the lead's open
 * channels, the recursion can carry C_L^+ G_1n (that many rows) instead of
 * G_1n: T = || C_L^+ G_1L C_R ||_F^2 (the projected calls below).
 *
 * Conventions shared by every entry point
 *   - Complex numbers are interleaved (re, im) doubles: knit_z, the element
 *     type of torch.complex128.  Matrices are row-major [M][M].
 *   - Slice-local index of orbital o of site s is s * norb + o.
 *   - Pointers documented as "device" point to GPU memory owned by the caller;
 *     the library never allocates, frees or retains them.  Pointers documented
 *     as "host" are read before the call returns.
 *   - All device work is enqueued on `stream` (a hipStream_t; NULL = the
 *     default stream) and is asynchronous with respect to the host.
 *   - Arguments are validated on the host before any device call; a bad
 *     argument returns KNIT_E_ARG and enqueues nothing.
 *   - Numerical trouble in one problem never aborts a batch: it sets bits in
 *     that problem's status word (KNIT_P_*), and its outputs are NaN.
 *   - Work memory is supplied by the caller (`ws`, `ws_bytes`), sized by the
 *     matching *_workspace() query; the calls perform no allocation.
 *   - Calls on distinct streams with distinct workspaces are thread-safe.
 */
#ifndef KNIT_H
#define KNIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KNIT_ABI_VERSION 4
#define KNIT_MAX_STRIPS 64     /* strip classes per batch */
#define KNIT_MAX_M 1024        /* largest slice dimension */
#define KNIT_MAX_NORB 4        /* largest orbitals-per-site */
#define KNIT_MAX_SELFENERGY_M 512   /* largest slice for knit_lead_selfenergy */
#define KNIT_TUNING_CLASSES 16      /* padded slice classes 32, 64, .., 512 */
#define KNIT_NOALLOC_SCRATCH_BYTES (128u << 20)   /* static scratch of knit_rgf_sweep_noalloc, per GPU */
#define KNIT_NOALLOC_MAX_PROBLEMS 1048576         /* largest P knit_rgf_sweep_noalloc accepts */

typedef struct knit_z { double re, im; } knit_z;

/* Return codes of every call. */
enum {
  KNIT_OK = 0,
  KNIT_E_ARG = -1,          /* invalid argument (nothing was enqueued) */
  KNIT_E_DEVICE = -2,       /* a HIP call failed */
  KNIT_E_WORKSPACE = -3,    /* ws is NULL or ws_bytes is below the *_workspace() size */
  KNIT_E_UNSUPPORTED = -4,  /* valid request the library does not implement */
  KNIT_E_SCRATCH = -5       /* knit_rgf_sweep_noalloc: the request does not fit the
                               library's static scratch (nothing was enqueued) */
};

/* Per-problem status bits (int32 per problem, written on the device). */
enum {
  KNIT_P_OK = 0,
  KNIT_P_SINGULAR = 1,      /* an exactly singular slice (zero pivot) */
  KNIT_P_NOCONV = 2,        /* decimation hit max_iter before convergence */
  KNIT_P_NONFINITE = 4,     /* NaN or Inf met in inputs or intermediates */
  KNIT_P_FALLBACK = 8       /* KNIT_FP32_REFINE only: a slice's FP32 inverse was too
                               poor for the refinement (see knit_set_refine_threshold),
                               so the problem was recomputed by the FP64 sweep in the
                               same call; its outputs are FP64's */
};

/* Arithmetic of the slice sweep. */
enum {
  KNIT_FP64 = 0,            /* FP64 throughout */
  KNIT_FP32_REFINE = 1,     /* FP32 slice inverse X0, refined by Newton steps with FP64
                               residuals (X <- X + X (I - A_n X), residual product in
                               FP64) until ||I - A_n X||_F <= 1e-5; every quantity
                               carried from slice to slice
                               (g_n, G_1n, G_n1, the projected rows) is kept in FP64
                               and the propagator is an FP64 product of the refined
                               inverse */
  KNIT_FP32 = 2             /* FP32 slice inverse and products, no refinement */
};

/*
 * A strip class: the clean slice shared by the system slices and both leads.
 *   M     slice dimension W * norb (1 <= M <= KNIT_MAX_M)
 *   norb  orbitals per site (1 <= norb <= KNIT_MAX_NORB, M % norb == 0)
 *   H0    device [M][M]  clean intra-slice Hamiltonian (Hermitian)
 *   V     device [M][M]  dense inter-slice hopping H_{n,n-1} (any matrix: the
 *                        hopping matrices of Eq. (1) are general), or NULL: V is
 *                        then block-monomial and given by vcol / vblk.  With a
 *                        dense V the slice recursion forms V g V^+, G V^+ and V G
 *                        as complex matrix products; M > 512 returns
 *                        KNIT_E_UNSUPPORTED for it in the sweeps and the LDOS
 *   vcol  device [W]     (V == NULL) for each site a of slice n, the site of
 *                        slice n-1 it is bonded to, or -1; no site of slice n-1
 *                        may appear twice (V is block-monomial)
 *   vblk  device [W][norb][norb]  (V == NULL) the hopping block H_{n,n-1}(a, vcol[a])
 *   onsite_dense  0: each slice's on-site term D_n is given as W site blocks
 *                 [W][norb][norb]; 1: as a full [M][M] matrix (e.g. site-mixing
 *                 terms, or a basis rotation of a disordered strip)
 *   h0_band  0, or b > 0: the caller's statement that the site blocks (a, c)
 *            of H0 vanish for |a - c| > b (sites of a slice coupled only to
 *            near neighbours within it, as on a lattice strip with hard
 *            walls).  The matrix-core sweeps and the LDOS then read only that
 *            band of H0 when they assemble a slice, which is the same sum
 *            when the statement holds (the skipped entries are zeros).
 *            Negative: KNIT_E_ARG.
 */
typedef struct knit_strip {
  int32_t M;
  int32_t norb;
  const knit_z *H0;
  const int32_t *vcol;
  const knit_z *vblk;
  const knit_z *V;
  int32_t onsite_dense;
  int32_t h0_band;
} knit_strip;

/*
 * One problem of a batch: a strip instance (its on-site blocks) at one energy.
 *   strip       index into the strip table of the call
 *   L           number of slices (>= 1)
 *   E           real energy
 *   onsite_off  offset, in knit_z elements, of its on-site blocks
 *               [L][W][norb][norb] (or [L][M][M] for an onsite_dense strip)
 *               in the `onsite` buffer
 *   sigma_off   offset, in knit_z, of its Sigma_L / Sigma_R ([M][M]) in
 *               `sigmaL` / `sigmaR` (problems at the same energy and strip
 *               class may share one)
 *   out_off     offset, in knit_z, of its G1N / GN1 / GNN blocks ([M][M])
 *   ldos_off    offset, in doubles, of its LDOS [L][M]
 * 48 bytes, no padding.
 */
typedef struct knit_problem {
  int32_t strip;
  int32_t L;
  double E;
  int64_t onsite_off;
  int64_t sigma_off;
  int64_t out_off;
  int64_t ldos_off;
} knit_problem;

/* ABI version of the loaded library (KNIT_ABI_VERSION). */
int knit_abi_version(void);

/* Static text for a return code or a per-problem status bit set. */
const char *knit_status_string(int code);

/*
 * Lead self-energies by decimation (section 2.3: the leads are integrated
 * out into energy-dependent self-energies; section 7.1-B selfE).
 *
 * For each energy E[e] computes the surface Green function g of the
 * semi-infinite lead at z = E + i*eta by renormalisation-group doubling
 * (Lopez Sancho, Lopez Sancho and Rubio 1985), carried in double-double
 * arithmetic (about 32 significant digits) so that the rounding growth of
 * the doubling stays far below eta, then returns
 *   side 0 (left lead):  Sigma_L = V g V^+,  g = (z - H0 - V g V^+)^{-1}
 *   side 1 (right lead): Sigma_R = V^+ g V,  g = (z - H0 - V^+ g V)^{-1}
 *   side 2 (both leads from one doubling run: the right lead's surface term is
 *          the half of the bulk update the left run computes anyway)
 * Iteration stops when both decimated couplings fall below tol * scale
 * (scale = max(1, max|H0|, max|V|)) or after max_iter steps (KNIT_P_NOCONV).
 * Each step's inverse (z - eps_k)^{-1} is an FP64 matrix-core inverse refined
 * by two double-double Newton steps; M above KNIT_MAX_SELFENERGY_M returns
 * KNIT_E_UNSUPPORTED.  Every result is checked against the lead's defining
 * equation, max |(z - H0 - Sigma) g - I| <= 1e-12 in double-double; an energy
 * that fails (near an eigenvalue of the single slice H0, where every doubling
 * step is singular, e.g. E = 0 on a bipartite strip with a zero mode) is
 * redone with a cell of two slices, for up to 4 energies per call and
 * M <= 256; any other failing energy gets KNIT_P_NOCONV and a NaN Sigma.  The call queues max_iter steps without waiting for the
 * device; energies that have converged skip the remaining steps.
 *
 *   strip     host   strip class
 *   side      0 = left lead, 1 = right lead, 2 = both
 *   E         device [nE] energies
 *   eta       broadening, > 0 (1e-16 recommended: the result is biased by about
 *             eta / velocity, which stays below 1e-12 even 1e-9 from a channel
 *             threshold, where the slowest open mode has velocity ~ 6e-5)
 *   sigma     device [nE][M][M] output; side 2: [2][nE][M][M], left block first
 *   iters     device [nE] output iteration counts, or NULL
 *   pstatus   device [nE] output status words
 */
size_t knit_lead_selfenergy_workspace(const knit_strip *strip, int32_t nE);
int knit_lead_selfenergy(const knit_strip *strip, int32_t side, const double *E, int32_t nE,
                         double eta, double tol, int32_t max_iter, knit_z *sigma, int32_t *iters,
                         int32_t *pstatus, void *ws, size_t ws_bytes, void *stream);

/*
 * Launch tuning of the matrix-core sweep (batching: workgroup shape, occupancy
 * and queue order), one entry per precision and padded-slice class
 * cls = Mp / 32 - 1 (Mp = slice dimension rounded up to 32, the largest of
 * the batch).  The library's defaults apply to classes never set; an entry
 * that does not fit the class (threads < Mp) is ignored at launch.
 *
 *   threads    256 or 512 threads per workgroup (one panel row per thread,
 *              so threads >= Mp)
 *   wg_per_cu  resident workgroups per compute unit the grid is sized for (1, 2)
 *   order      0: problems in table order; 1: longest (Mp^3 L) first
 *   outer      outer panel width of the blocked elimination, 64 or 128 (each
 *              outer panel is one read-and-write pass over the slice matrix;
 *              default 128 from Mp = 128, else 64)
 *
 * Process-wide; set before the sweeps that should use it (calls that run
 * concurrently with a change see either the old or the new entry).
 * knit_sweep_tuning_set with t == NULL restores the default.  Both return
 * KNIT_E_ARG for a bad precision, class or entry.
 */
typedef struct knit_sweep_tuning {
  int32_t threads;
  int32_t wg_per_cu;
  int32_t order;
  int32_t outer;
} knit_sweep_tuning;

int knit_sweep_tuning_set(int32_t precision, int32_t cls, const knit_sweep_tuning *t);
int knit_sweep_tuning_get(int32_t precision, int32_t cls, knit_sweep_tuning *t);

/*
 * Threshold of the KNIT_FP32_REFINE sweeps and LDOS (precision extension).
 * Each slice's FP32 inverse X0 is refined by Newton steps on the inverse,
 *   R_k = I - A_n X_k (FP64 product),  X_{k+1} = X_k + X_k R_k,
 * each of which squares the residual; steps continue while ||R_k||_F > 1e-5
 * (at most 4), so a refined inverse carries a relative error below about
 * 1e-10.  A problem whose first residual ||I - A_n X0||_F exceeds the
 * threshold (or is NaN), or whose steps stop shrinking the residual before
 * reaching 1e-5, is marked KNIT_P_FALLBACK and recomputed in FP64.  Default
 * 0.25 (Newton's iteration for the inverse converges for ||R_0|| < 1).  0
 * sends every problem to FP64.  Process-wide; returns KNIT_E_ARG for a
 * negative or NaN value.
 */
int knit_set_refine_threshold(double threshold);
double knit_get_refine_threshold(void);

/*
 * How knit_lead_selfenergy forms its double-double matrix products (section
 * 5.3-B: the leads' self-energies by decimation).
 *   KNIT_PRODUCTS_VECTOR  (default) double-double arithmetic on the vector
 *                         units;
 *   KNIT_PRODUCTS_INT8    both factors split into signed 7-bit
 *                         digits (rows of the left factor and columns of the
 *                         right one scaled by powers of two; 16 digits for a
 *                         double-double factor, 8 for an FP64 one), digit
 *                         planes multiplied exactly on the INT8 matrix cores
 *                         with int32 sums, digit pairs of combined weight below
 *                         2^-124 of the scales dropped, the rest summed in
 *                         double-double: a normwise relative error of about
 *                         2^-106 per product, as double-double's own.  The
 *                         retry pass (energies at slice eigenvalues) always
 *                         uses the vector products.  Where the decimated
 *                         couplings mix parts of very different size the
 *                         row- and column-relative accuracy can stall the
 *                         doubling (KNIT_P_NOCONV / KNIT_P_NONFINITE).
 * Process-wide; returns KNIT_E_ARG for any other value.
 */
#define KNIT_PRODUCTS_VECTOR 0
#define KNIT_PRODUCTS_INT8 1
int knit_set_selfenergy_products(int32_t mode);
int32_t knit_get_selfenergy_products(void);

/*
 * Left-to-right slice recursion (section 1, basic RGF) for a batch of P
 * problems, in one persistent launch.  Per problem:
 *   g_1 = (E - H_1 - Sigma_L - [L = 1] Sigma_R)^{-1}
 *   g_n = (E - H_n - [n = L] Sigma_R - V g_{n-1} V^+)^{-1}
 *   G_1n = G_{1,n-1} V^+ g_n,  G_n1 = g_n V G_{n-1,1},  G_11 = g_1
 * and returns G_1L (G1N), optionally G_L1 (GN1) and G_LL = g_L (GNN).  Each
 * slice inverse is a Gauss-Jordan elimination with partial pivoting (the
 * pivot sequence of LU with partial pivoting, largest |re|+|im|, lowest
 * row on ties).
 *
 *   strips, n_strips   host table of strip classes (n_strips <= KNIT_MAX_STRIPS)
 *   probs_host         host [P] problem table (read before return)
 *   probs_dev          device [P] copy of the same table
 *   onsite             device on-site blocks addressed by onsite_off
 *   sigmaL, sigmaR     device self-energies addressed by sigma_off
 *   precision          KNIT_FP64, KNIT_FP32_REFINE or KNIT_FP32 (with
 *                      KNIT_FP32_REFINE, problems flagged KNIT_P_FALLBACK are
 *                      recomputed in FP64 by a second launch of the same call)
 *   G1N                device output addressed by out_off (required)
 *   GN1, GNN           device outputs addressed by out_off, or NULL
 *   pstatus            device [P] output status words
 */
size_t knit_rgf_sweep_workspace(const knit_strip *strips, int32_t n_strips,
                                const knit_problem *probs_host, int32_t P, int32_t precision,
                                int32_t want_gn1);
int knit_rgf_sweep(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                   const knit_problem *probs_dev, int32_t P, const knit_z *onsite,
                   const knit_z *sigmaL, const knit_z *sigmaR, int32_t precision, knit_z *G1N,
                   knit_z *GN1, knit_z *GNN, int32_t *pstatus, void *ws, size_t ws_bytes,
                   void *stream);

/*
 * knit_rgf_sweep without a workspace argument, for callers that cannot
 * allocate device memory (code under stream capture, serving loops, harnesses
 * that forbid allocation).  Same arguments, outputs and status words as
 * knit_rgf_sweep (FP64 outputs equal it bit for bit); the call allocates
 * nothing.  Its work memory is a static device array of
 * KNIT_NOALLOC_SCRATCH_BYTES (128 MiB) per GPU, which each GPU the library
 * runs on holds until the process ends; the sweep runs as many resident
 * workgroups as that array holds slice slabs (at slice dimension 512, three),
 * so large batches run slower than with a full-size workspace.  Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other host threads) race and must be serialised by the caller.  Nothing in
 * the array needs to start at zero (the queue counter is reset on the device
 * by each call).  Returns KNIT_E_SCRATCH, enqueuing nothing, for P above
 * KNIT_NOALLOC_MAX_PROBLEMS, and KNIT_E_UNSUPPORTED for strips with M > 512.
 */
int knit_rgf_sweep_noalloc(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                           const knit_problem *probs_dev, int32_t P, const knit_z *onsite, const knit_z *sigmaL,
                           const knit_z *sigmaR, int32_t precision, knit_z *G1N, knit_z *GN1, knit_z *GNN,
                           int32_t *pstatus, void *stream);

/*
 * Fisher-Lee transmission (section 2.3, T_kl), FP64, per problem:
 *   T[p]      = Re Tr[Gamma_L G_1L Gamma_R G_1L^+]                 (required)
 *   T_RL[p]   = Re Tr[Gamma_R G_L1 Gamma_L G_L1^+]                 (needs GN1)
 *   T_ward[p] = Re{Tr[Gamma_R i(G_LL - G_LL^+)] - Tr[Gamma_R G_LL Gamma_R G_LL^+]}
 *                                                                   (needs GNN)
 * with Gamma = i (Sigma - Sigma^+).  T_RL and T_ward equal T when current is
 * conserved; they are checks.  Output pointers other than T may be NULL.
 */
int knit_transmission(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                      const knit_problem *probs_dev, int32_t P, const knit_z *sigmaL,
                      const knit_z *sigmaR, const knit_z *G1N, const knit_z *GN1,
                      const knit_z *GNN, double *T, double *T_RL, double *T_ward, void *stream);

/*
 * Local density of states LDOS[p][n][i] = -Im (G_nn)_ii / pi on every slice
 * (section 2.1 item b, the Green function at a given site; section 5.3-D
 * sewing; section 7.1-D getG_retarded on-site).  A forward sweep keeps g_n
 * every `checkpoint_stride` slices (the role of the paper's saving level),
 * then the reverse sweep
 *   G_LL = g_L,  G_nn = g_n + g_n V^+ G_{n+1,n+1} V g_n
 * recomputes each segment's g_n from its checkpoint.  checkpoint_stride <= 0
 * picks ceil(sqrt(L)).  precision as for knit_rgf_sweep (KNIT_FP32_REFINE:
 * refined inverses, checkpoints, G_nn and both products in FP64, fallback
 * problems recomputed in FP64 by the same call; M > 512 returns
 * KNIT_E_UNSUPPORTED for it).
 *
 *   ldos   device output addressed by ldos_off ([L][M] doubles per problem)
 */
size_t knit_ldos_workspace(const knit_strip *strips, int32_t n_strips,
                           const knit_problem *probs_host, int32_t P, int32_t precision,
                           int32_t checkpoint_stride);
int knit_ldos(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
              const knit_problem *probs_dev, int32_t P, const knit_z *onsite,
              const knit_z *sigmaL, const knit_z *sigmaR, int32_t precision,
              int32_t checkpoint_stride, double *ldos, int32_t *pstatus, void *ws,
              size_t ws_bytes, void *stream);

/*
 * Broadening factors (section 2.3: Gamma = i (Sigma - Sigma^+) is Hermitian
 * positive semidefinite; its rank is the lead's number of open channels).
 * For each of the n matrices sigma[e] ([M][M], row-major, consecutive) writes
 * C[e] ([M][M], row-major) and rank[e] with Gamma_e = C_e C_e^+ + D_e, by a
 * Cholesky factorisation with diagonal pivoting: columns are added while the
 * largest remaining diagonal entry exceeds tol * s_e, s_e = max_i |(Sigma_e)_ii|
 * (the scale of Gamma's rounding noise; tol <= 0 picks 1e-10, above the
 * decimation's own error, so a lead's rank is its open channels and a Gamma
 * of noise alone, outside the band, has rank 0).  The dropped part D_e is
 * positive semidefinite with trace at most (M - rank[e]) * tol * s_e.  Columns >= rank[e] of C_e
 * are zero and column k < rank[e] has a positive real entry at its pivot row,
 * so rank[e] is also one plus the index of C_e's last nonzero column.  A
 * non-finite Sigma gives rank[e] = -1 and a C_e of NaN.
 *
 *   M        1 <= M <= KNIT_MAX_M
 *   sigma    device [n][M][M] input
 *   C        device [n][M][M] output (may be addressed like sigma by sigma_off)
 *   rank     device [n] output
 * Asynchronous on stream; allocates nothing.
 */
int knit_gamma_factor(int32_t M, const knit_z *sigma, int32_t n, double tol, knit_z *C, int32_t *rank,
                      void *stream);

/*
 * Projected sweep: the recursion of knit_rgf_sweep carrying
 *   P_1 = C_L^+ g_1,   P_n = P_{n-1} V^+ g_n   (= C_L^+ G_1n)
 * instead of G_1n, where Gamma_L = C_L C_L^+ (section 2.3; C_L as written by
 * knit_gamma_factor for the left self-energy, addressed by sigma_off).  Only
 * the r = C_L's columns up to its last nonzero one enter, so each slice's
 * stacked elimination has Mp + r rows instead of 2 Mp (Mp = M rounded up to
 * 32; with KNIT_FP32_REFINE the elimination covers A_n alone and P_n is the
 * FP64 product (P_{n-1} V^+) g_n of the refined inverse).  Writes P_L to G1Np
 * ([M][M] at out_off, rows >= r zero) and, if GNN is not NULL, G_LL = g_L.
 * precision is KNIT_FP64, KNIT_FP32_REFINE (problems flagged KNIT_P_FALLBACK
 * are recomputed in FP64 by a second launch of the same call) or KNIT_FP32;
 * strips with M > 512 return KNIT_E_UNSUPPORTED.  The workspace is
 * knit_rgf_sweep_workspace(..., precision, 0) bytes; other arguments as for
 * knit_rgf_sweep.
 */
int knit_rgf_sweep_projected(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                             const knit_problem *probs_dev, int32_t P, const knit_z *onsite,
                             const knit_z *sigmaL, const knit_z *sigmaR, const knit_z *CL, int32_t precision,
                             knit_z *G1Np, knit_z *GNN, int32_t *pstatus, void *ws, size_t ws_bytes,
                             void *stream);

/*
 * Fisher-Lee transmission from the projected propagator (section 2.3, T_kl):
 *   T[p] = || P_L C_R ||_F^2 = Re Tr[Gamma_L G_1L Gamma_R G_1L^+]
 * with P_L from knit_rgf_sweep_projected (G1Np, at out_off) and Gamma_R =
 * C_R C_R^+ (CR addressed by sigma_off).  FP64; T is device [P].
 */
int knit_transmission_projected(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                                const knit_problem *probs_dev, int32_t P, const knit_z *CR,
                                const knit_z *G1Np, double *T, void *stream);

/*
 * Transmission eigenvalues and shot noise (section 2.1 item (a): conductance
 * and shot noise), FP64, from the projected propagator.  With P_L = C_L^+ G_1L
 * (knit_rgf_sweep_projected, G1Np at out_off) and Gamma_R = C_R C_R^+ (CR at
 * sigma_off), t~ = P_L C_R has the singular values of the transmission
 * amplitude matrix t = Gamma_R^{1/2} G_L1 Gamma_L^{1/2}; per problem:
 *   tn[p * ld + i]  the transmission eigenvalues T_i (eigenvalues of t t^+),
 *                   descending, i < nch[p] = min(rank Gamma_L, rank Gamma_R);
 *                   entries nch[p] .. ld-1 are zero
 *   T[p]            sum_i T_i = Tr t~^+ t~ (the Fisher-Lee T), or NULL
 *   fano[p]         shot-noise Fano factor sum_i T_i (1 - T_i) / sum_i T_i,
 *                   from traces (Tr tau - ||tau||_F^2) / Tr tau with
 *                   tau = t~^+ t~; NaN where T = 0; or NULL
 *   nch             device [P] int32, or NULL
 * The eigenvalues come from a Householder reduction of tau to tridiagonal form
 * and bisection on its Sturm sequence (absolute accuracy a few units of
 * rounding of ||tau|| <= 1).  ld >= the largest M of the batch.  The workspace
 * is knit_transmission_eigenvalues_workspace() bytes.
 */
size_t knit_transmission_eigenvalues_workspace(const knit_strip *strips, int32_t n_strips,
                                               const knit_problem *probs_host, int32_t P);
int knit_transmission_eigenvalues(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                                  const knit_problem *probs_dev, int32_t P, const knit_z *CR, const knit_z *G1Np,
                                  int32_t ld, double *tn, int32_t *nch, double *T, double *fano, void *ws,
                                  size_t ws_bytes, void *stream);

/*
 * Lesser Green function of injection from the left lead and the local
 * observables built on it (section 2.3: G_L^< = i G Gamma_L G^+, electrons
 * injected with probability 1 from the left lead; sections 5.3-D, 6.1 and 6.2:
 * local densities, local currents, spin accumulation), FP64.  With
 * Gamma_L = C_L C_L^+ (knit_gamma_factor), A_L = -i G_L^< = Q Q^+ with the
 * slice blocks Q_n = G_{n1} C_L of the full Green function; a forward sweep
 * keeps checkpoints of g_n and g^L_{n1} C_L every `checkpoint_stride` slices
 * (<= 0: ceil(sqrt(L))), the reverse sweep forms Q_n from Dyson's equation
 * across each inter-slice cut.  Per problem p, slice n, site s (norb orbitals):
 *   blk[blk_off[p] + ((n W + s) norb + o) norb + o'] = A_L(n s o, n s o')
 *       on-site blocks (complex, [L][W][norb][norb]): Tr / (2 pi) is the
 *       density injected from the left lead per unit energy, A_00 - A_11 the
 *       sigma_z spin density of section 6.2
 *   jlong[ldos_off + n W + s] = current into site s of slice n from slice n-1,
 *       sum over its bonds of 2 Im Tr[H_ab A_ba] (units e/h per unit energy;
 *       0 for n = 0); over any cross-section it sums to the transmission T
 *   jtran[ldos_off + n W + s] = current into site s from the other sites of
 *       its own slice (sums to 0 over each slice)
 * A right-lead injection is the same call on the mirrored strip (slices in
 * reverse order, V replaced by V^+).  blk_off is device int64 [P]; jlong and
 * jtran use the first L W doubles of each problem's [L][M] LDOS slot.  M > 512
 * returns KNIT_E_UNSUPPORTED.  The workspace is
 * knit_local_observables_workspace() bytes.
 */
size_t knit_local_observables_workspace(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                                        int32_t P, int32_t checkpoint_stride);
int knit_local_observables(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                           const knit_problem *probs_dev, int32_t P, const knit_z *onsite, const knit_z *sigmaL,
                           const knit_z *sigmaR, const knit_z *CL, int32_t checkpoint_stride, knit_z *blk,
                           const int64_t *blk_off, double *jlong, double *jtran, int32_t *pstatus, void *ws,
                           size_t ws_bytes, void *stream);

/*
 * A lead attached to one slice of a strip besides the left and right leads
 * (section 6.1: systems with more than two leads).
 *   slice      0-based slice it is attached to (0 <= slice < L of its problem)
 *   sigma_off  offset, in knit_z, of its self-energy [M][M] (acting on that
 *              slice's orbitals) in `sigmaX` and of its broadening factor
 *              (Gamma = C C^+, as written by knit_gamma_factor) in `CX`
 */
typedef struct knit_lead {
  int32_t slice;
  int32_t reserved;
  int64_t sigma_off;
} knit_lead;

#define KNIT_MAX_SIDE_LEADS 6

/*
 * Conductance matrix of strips with several leads (section 2.3:
 * T_kl = Tr[Gamma_k G_kl Gamma_l G_kl^+], the transmission from lead l to lead
 * k; section 6.1: the conductance matrix g_kl = (e^2/h) T_kl), FP64.  Lead 0
 * is the left lead (slice 0: sigmaL, CL at sigma_off), lead 1 the right lead
 * (slice L-1: sigmaR, CR), leads 2 .. n_side+1 the problem's side leads
 * side_host[p * n_side + j] (their self-energies join the slice matrix of
 * their slice).  A forward sweep keeps checkpoints of the left-connected g_n;
 * the reverse sweep forms the right-connected ones, the full diagonal block at
 * every slice hosting a lead, and carries each lead's columns G_{n,s} C and
 * rows C^+ G_{s,n} down the strip by Dyson's equation across every cut; with
 * K = n_side + 2:
 *   T[p * K * K + k * K + l] = || C_k^+ G_{s_k s_l} C_l ||_F^2   (all k, l; the
 *   diagonal is the formula's value, so row and column sums agree).
 * n_side <= KNIT_MAX_SIDE_LEADS; side_host is host [P][n_side] (validated
 * before any device call), side_dev its device copy; sigmaX, CX device.
 * M > 512 returns KNIT_E_UNSUPPORTED.  checkpoint_stride <= 0 picks
 * ceil(sqrt(L)).  The workspace is knit_conductance_matrix_workspace() bytes.
 */
size_t knit_conductance_matrix_workspace(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                                         int32_t P, int32_t n_side, int32_t checkpoint_stride);
int knit_conductance_matrix(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                            const knit_problem *probs_dev, int32_t P, const knit_z *onsite, const knit_z *sigmaL,
                            const knit_z *sigmaR, const knit_z *CL, const knit_z *CR, int32_t n_side,
                            const knit_lead *side_host, const knit_lead *side_dev, const knit_z *sigmaX,
                            const knit_z *CX, int32_t checkpoint_stride, double *T, int32_t *pstatus, void *ws,
                            size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KNIT_H */
