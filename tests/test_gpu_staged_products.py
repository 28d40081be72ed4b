"""The outer update's LDS-staged block products at the shapes where their edge cases live.

Each slice inverse is a blocked Gauss-Jordan elimination whose outer-panel products (the
multipliers of the rows outside the panel, the rank-NO update, the new pivot rows) run as
workgroup products staged through LDS and written in place.  These cases hit:
  * slice dim 224 (256 threads, 128-wide panels): the multipliers with the 1 x 4 group
    shape, a 96-wide last panel (a 32-row tail tile in the new pivot rows), and Gamma_L of
    rank 77 (three stacked 32-row blocks: a tail tile in the multipliers);
  * slice dim 96 (64-wide panels): a 32-wide last panel and one stacked block (rank 21);
  * slice dim 512 (512 threads): seven stacked blocks (rank 200).
T of the projected and of the whole-G_1n sweep against the oracle's Re Tr[Gamma_L G_1L
Gamma_R G_1L^+] at 1e-10 (relative to max(1, T)), G_1L elementwise at 1e-10 of its
largest entry, and the LDOS against the oracle's backward recursion at 1e-10, with seeded
synthetic boundary terms.
"""

import numpy as np
import pytest
import torch

from paper_1010_2627_amd import inputs

pytestmark = pytest.mark.gpu
gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")

CASES = [(224, 4, 77), (96, 6, 21), (512, 3, 200)]   # (W of a square strip, L, rank of Gamma_L)


@gpu
@pytest.mark.parametrize("W,L,rank", CASES)
def test_staged_outer_products_match_oracle(W, L, rank):
    from paper_1010_2627_amd import workload
    from oracle import rgf as OR
    b = workload.square_batch(W, L, 1.5, 2, 1)
    st = b.strips[0]
    E = b.energies[0]
    sL = inputs.synthetic_sigma(st.M, len(E), seed=inputs.SEED_SYNTHETIC_SIGMA + 7, rank=rank)
    sR = inputs.synthetic_sigma(st.M, len(E), seed=inputs.SEED_SYNTHETIC_SIGMA + 8)
    b.set_sigmas([sL], [sR])
    b.compute_gamma_factors()
    G1Np, _, status_p = b.sweep_projected()
    Tp = b.transmission_projected(G1Np)
    G1N, _, _, status = b.sweep("fp64", gnn=False)
    T = b.transmission(G1N)[0]
    ld, status_l = b.ldos("fp64")
    torch.cuda.synchronize()
    for s in (status, status_p, status_l):
        assert int(s.abs().sum()) == 0
    assert torch.all(b.rankL == rank)
    on = b.realizations[0].onsite
    res = OR.rgf_forward(st.H0, st.V_dense(), on, E, sL, sR)
    Tref = OR.transmission_lr(sL, sR, res["G1N"])
    for got in (T.cpu().numpy(), Tp.cpu().numpy()):
        assert np.max(np.abs(got - Tref) / np.maximum(1.0, np.abs(Tref))) <= 1e-10, (got, Tref)
    ldref = OR.ldos_rgf(st.H0, st.V_dense(), on, E, sL, sR)
    for p in range(b.P):
        ei = int(b.prob_meta[p][1])
        ref = res["G1N"][ei]
        assert np.max(np.abs(b.block(G1N, p).cpu().numpy() - ref)) <= 1e-10 * max(1.0, np.abs(ref).max()), p
        got_l = b.ldos_block(ld, p).cpu().numpy()
        assert np.max(np.abs(got_l - ldref[ei])) <= 1e-10 * max(1.0, np.abs(ldref[ei]).max()), p
