// knit_rgf_sweep_noalloc (include/knit.h): the slice sweep of knit_rgf_sweep
// without a workspace argument, for callers that cannot allocate device
// memory.  Its work memory is the static device array below, one copy per GPU;
// the sweep runs as many resident workgroups as the array holds slabs.

#include <mutex>

#include "knit_internal.h"

using namespace knit;

namespace {

// Work memory of knit_rgf_sweep_noalloc, held by each GPU for the life of the
// process.  Host code never uses this name as an address: the device address
// of each GPU's copy comes from hipGetSymbolAddress (scratch_address).
static __device__ __align__(256) char scratch[KNIT_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex mu;
void *scratch_of_device[MAX_DEVICES];

// Device address of the current GPU's copy of `scratch`, resolved once per
// device, with that device current, on its first use.
int scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return KNIT_E_DEVICE;
  if (dev < 0 || dev >= MAX_DEVICES) return KNIT_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(mu);
  if (!scratch_of_device[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return KNIT_E_DEVICE;
    scratch_of_device[dev] = p;
  }
  *out = scratch_of_device[dev];
  return KNIT_OK;
}

}  // namespace

extern "C" int knit_rgf_sweep_noalloc(const knit_strip *strips, int32_t n_strips, const knit_problem *probs_host,
                                      const knit_problem *probs_dev, int32_t P, const knit_z *onsite,
                                      const knit_z *sigmaL, const knit_z *sigmaR, int32_t precision, knit_z *G1N,
                                      knit_z *GN1, knit_z *GNN, int32_t *pstatus, void *stream) {
  int Mmax = 0;
  if (!batch_ok(strips, n_strips, probs_host, P, precision, &Mmax)) return KNIT_E_ARG;
  if (P == 0) return KNIT_OK;
  if (!probs_dev || !onsite || !sigmaL || !sigmaR || !G1N || !pstatus) return KNIT_E_ARG;
  if (!sweep_mfma_supports(Mmax)) return KNIT_E_UNSUPPORTED;
  if (P > KNIT_NOALLOC_MAX_PROBLEMS) return KNIT_E_SCRATCH;
  // resident workgroups: as many slabs as the scratch holds after the queue header
  bool dense = false;
  for (int i = 0; i < n_strips; ++i) dense = dense || strips[i].V != nullptr;
  const int grid = sweep_mfma_grid_within(KNIT_NOALLOC_SCRATCH_BYTES, Mmax, precision, P, dense);
  if (grid < 1) return KNIT_E_SCRATCH;
  void *ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc != KNIT_OK) return rc;
  const StripTable tab = strip_table_of(strips, n_strips);
  const hipError_t err = launch_sweep_mfma(tab, probs_dev, P, onsite, sigmaL, sigmaR, precision, G1N, GN1, GNN,
                                           pstatus, ws, Mmax, grid, (hipStream_t)stream);
  return err == hipSuccess ? KNIT_OK : KNIT_E_DEVICE;
}
