/*
 * knit_graph.h -- C ABI of libknit: knitting of a system of any geometry.
 *
 * What is computed (section 1, section 5.3-D "knitting", FIG. 9; objects of
 * section 2.3): a tight-binding system of N sites with m orbitals per site
 * (Eq. (1)): on-site blocks H_ii and hopping blocks H_ij (m x m) on the edges
 * of a graph of any shape (holes, several arms, magnetic-field phases,
 * electron-hole blocks), connected to K leads.  Lead k is attached to a list
 * of system sites (its interface) and enters as a self-energy Sigma_k acting
 * on those sites.  The retarded Green function is
 * G = (E - H - sum_k Sigma_k)^{-1} (Eq. (2), Im Sigma <= 0), and the output
 * is the transmission between every pair of leads,
 * T_kl = Re Tr[Gamma_k G_kl Gamma_l G_kl^+], Gamma = i (Sigma - Sigma^+)
 * (section 2.3), plus optionally the block of G on the lead sites.
 *
 * Knitting adds the sites one at a time (section 5.3-D).  The sites of lead 0
 * come first, as one block: g = (E - H_00 - Sigma_0)^{-1} over them.  Then
 * each further site i is added by Dyson's equation with its hopping blocks to
 * the sites already added:
 *   g_i  = (E - H_ii - H_{i,S} G_SS H_{S,i})^{-1}
 *   G_Si = G_SS H_{S,i} g_i,  G_iS = g_i H_{i,S} G_SS,  G_ii = g_i
 *   G_SS <- G_SS + G_SS H_{S,i} g_i H_{i,S} G_SS.
 * Only the "interface" is kept: sites that still have a neighbour to add, and
 * every lead site.  The other leads' self-energies are applied at the end on
 * the lead block, G_LL <- (I - G_LL Sigma')^{-1} G_LL with
 * Sigma' = diag(0, Sigma_1, .., Sigma_{K-1}).  The cost is
 * sum over steps of (interface dimension)^2 (section 5.3-D, calculation time).
 *
 * Conventions are those of knit.h (knit_z, return codes, status bits, device
 * and host pointers, streams, caller-supplied workspace).
 */
#ifndef KNIT_GRAPH_H
#define KNIT_GRAPH_H

#include <stddef.h>
#include <stdint.h>

#include "knit.h"

#ifdef __cplusplus
extern "C" {
#endif

#define KNIT_GRAPH_MAX_LEADS 16
#define KNIT_GRAPH_MAX_PAIRS 16     /* added neighbours x orbitals at one step */
#define KNIT_GRAPH_MAX_DIM 2048     /* largest interface dimension (sites held x norb) */

/* Opaque knitting plan (host object): the graph's structure, the leads and
 * the order of the sites, with the interface bookkeeping worked out. */
typedef struct knit_graph_plan knit_graph_plan;

/* A lead: the system sites it is attached to (host array, read during
 * knit_graph_plan_create only).  Site j of the list carries orbitals
 * j*norb .. j*norb+norb-1 of the lead's self-energy. */
typedef struct knit_graph_lead {
  int32_t nsite;
  int32_t reserved;
  const int32_t *sites;
} knit_graph_lead;

/* Sizes a plan needs, for the caller's buffers and for measurement. */
typedef struct knit_graph_info {
  int32_t nsite, norb, n_leads;
  int32_t max_slots;     /* most sites held at once: lead sites plus the interface */
  int32_t dim;           /* max_slots * norb: dimension of the matrix the knitting updates */
  int32_t lead_dim;      /* sum over leads of nsite * norb: dimension of the lead block */
  int32_t max_pairs;     /* largest (added neighbours x norb) at one step */
  int32_t n_steps;       /* sites added one at a time (nsite minus lead 0's sites) */
  int64_t sigma_size;    /* knit_z per problem in the self-energy pack: sum (nsite_k norb)^2 */
  int64_t nnz;           /* hopping blocks (directed edges) */
  double update_flops;   /* sum over steps of 8 norb D_t^2, D_t the dimension updated at step t */
  double update_bytes;   /* sum over steps of 32 D_t^2: one read and one write of the updated block */
  int32_t block;         /* sites added per step (1: site by site; see knit_graph_plan_create_blocked) */
  int32_t reserved;
} knit_graph_info;

/* One problem: an energy, its on-site blocks and its self-energies. */
typedef struct knit_graph_problem {
  double E;
  int64_t onsite_off;    /* knit_z offset of [nsite][norb][norb] on-site blocks in `onsite` */
  int64_t sigma_off;     /* knit_z offset of the self-energy pack in `sigma`: lead k's
                            Sigma_k [n_k norb][n_k norb] (row-major) at
                            sigma_off + sum_{j<k} (n_j norb)^2 */
  int64_t gll_off;       /* knit_z offset of the [lead_dim][lead_dim] output in `GLL` */
} knit_graph_problem;

/*
 * Build a plan (host only; no device call).
 *   nsite, norb   1 <= norb <= KNIT_MAX_NORB
 *   row_ptr, col  host CSR of the directed hopping graph: site i couples to
 *                 col[e], e in [row_ptr[i], row_ptr[i+1]); no self loops, no
 *                 repeated neighbour, structurally symmetric (j in row i
 *                 exactly when i in row j).  Hopping block e (in `hop` of
 *                 knit_graph_transmission) is H_{i, col[e]}.
 *   n_leads       1 .. KNIT_GRAPH_MAX_LEADS; leads[k].sites distinct, and no
 *                 site in two leads
 *   order         host [nsite], a permutation of the sites, or NULL.  Lead 0's
 *                 sites are taken first (as one block, in the lead's own
 *                 order); the other sites follow in `order`'s sequence.  NULL:
 *                 breadth-first from lead 0's sites, neighbours in CSR order
 *                 (a front that sweeps the system like FIG. 9(a)); sites not
 *                 reachable from lead 0 follow, breadth-first from the lowest
 *                 index.
 * Returns KNIT_E_ARG on any violation (nothing is created) and
 * KNIT_E_UNSUPPORTED when the interface dimension would exceed
 * KNIT_GRAPH_MAX_DIM or a step would couple more than KNIT_GRAPH_MAX_PAIRS
 * neighbour orbitals.  *plan is owned by the caller: knit_graph_plan_destroy.
 */
int knit_graph_plan_create(int32_t nsite, int32_t norb, const int32_t *row_ptr, const int32_t *col,
                           int32_t n_leads, const knit_graph_lead *leads, const int32_t *order,
                           knit_graph_plan **plan);
/*
 * The same, adding `block` sites per step (section 1: a group of sites, like a
 * layer, joins the system by the same Dyson equation with the group's block
 * H_bb, its internal hoppings included, in place of H_ii).  The sites are
 * grouped once on the host: each lead's sites `block` at a time in the lead's
 * order, the other sites `block` at a time in the knitting order (the order
 * knit_graph_plan_create would take); a last group with fewer sites is padded
 * with orbitals that couple to nothing and have E - H = 1, which leave every
 * other entry of G unchanged.  The groups are then knitted as the sites of a
 * graph with block * norb orbitals per site.  T and the lead block of G have
 * the same meaning and layout as for knit_graph_plan_create; the work per
 * step is a rank-(block * norb) update, which spreads one step's fixed
 * latency over `block` sites.
 *   block   1 .. KNIT_MAX_NORB / norb, dividing every lead's nsite
 *           (KNIT_E_ARG otherwise); 1 gives knit_graph_plan_create's plan.
 *           0: automatic.  When the site-by-site interface dimension is at
 *           most 128 (the matrix stays in registers): 2 for one orbital per
 *           site if 2 is valid and the grouped dimension stays within the
 *           same register kernel (at most 64 when the site-by-site one is,
 *           else at most 128), otherwise 1.  Above 128, where every step
 *           passes over the matrix in memory: the valid block with
 *           block * norb closest to 3 (the larger of two equally close)
 *           whose plan exists, else 1.
 * info of a blocked plan: nsite, norb and nnz are the system's; max_slots,
 * dim, max_pairs, n_steps, update_flops and update_bytes count groups, the
 * steps and the updates the device makes; block is the one chosen.
 * knit_graph_plan_order returns the site order the groups were taken from.
 * knit_graph_workspace grows by the groups' blocks, (P * n_groups +
 * n_group_edges) * (block * norb)^2 knit_z (on-site blocks for every problem,
 * hopping blocks once), plus the group map and a copy of the problem table.
 */
int knit_graph_plan_create_blocked(int32_t nsite, int32_t norb, const int32_t *row_ptr, const int32_t *col,
                                   int32_t n_leads, const knit_graph_lead *leads, const int32_t *order,
                                   int32_t block, knit_graph_plan **plan);
int knit_graph_plan_info(const knit_graph_plan *plan, knit_graph_info *info);
/* The site order the plan knits in (host [nsite]). */
int knit_graph_plan_order(const knit_graph_plan *plan, int32_t *order);
void knit_graph_plan_destroy(knit_graph_plan *plan);

/* Workspace bytes of knit_graph_transmission for P problems (0 on a bad plan). */
size_t knit_graph_workspace(const knit_graph_plan *plan, int32_t P);

/*
 * Knit P problems of one plan (one workgroup per problem), FP64.
 *   probs     device [P] knit_graph_problem
 *   hop       device [nnz][norb][norb]: H_{i, col[e]} for edge e, shared by
 *             every problem (Peierls phases etc. go in here; H_{j,i} must be
 *             H_{i,j}^+ for a Hermitian H, which is not checked)
 *   onsite    device, addressed by onsite_off
 *   sigma     device, addressed by sigma_off
 *   T         device [P][K][K]: T[p*K*K + k*K + l] = T_kl (the diagonal is the
 *             formula's value)
 *   GLL       device or NULL: G on the lead sites, [lead_dim][lead_dim] at
 *             gll_off, leads in order, each lead's sites in its own order
 *   pstatus   device [P] status bits (KNIT_P_SINGULAR: a zero pivot;
 *             KNIT_P_NONFINITE: a non-finite result; outputs NaN then)
 * P = 0 returns KNIT_OK and enqueues nothing.  The plan's host memory is
 * read by an asynchronous copy into the workspace: destroy the plan only
 * after the stream's work is done.
 */
int knit_graph_transmission(const knit_graph_plan *plan, const knit_graph_problem *probs, int32_t P,
                            const knit_z *hop, const knit_z *onsite, const knit_z *sigma, double *T, knit_z *GLL,
                            int32_t *pstatus, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KNIT_GRAPH_H */
