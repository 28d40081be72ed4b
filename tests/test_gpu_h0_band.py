"""A stated band of H0 (knit_strip.h0_band): the slice assembly then reads only
the site blocks of H0 within it.  Lattice strips with hard walls have band 1,
and every output must be bitwise the same as with the whole of H0 read
(h0_band = 0): the skipped entries are zeros.  Projected and whole-G_1n
sweeps, the LDOS, and a band that covers the nonzero blocks with room to
spare (2) are checked; the results also match the oracle elsewhere."""

import dataclasses

import numpy as np
import pytest
import torch

from paper_1010_2627_amd import knit as K

pytestmark = pytest.mark.gpu
gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def _with_band(b, band):
    b.dstrips = [dataclasses.replace(s, h0_band=band) for s in b.dstrips]


@gpu
@pytest.mark.parametrize("kind", ["square", "rashba"])
def test_banded_assembly_is_bitwise_the_full_read(kind):
    from paper_1010_2627_amd import workload
    if kind == "square":
        b = workload.square_batch(W=40, L=30, w=1.5, n_energies=6, n_seeds=2)
    else:
        b = workload.rashba_batch(W=24, L=20, w=1.0, n_energies=4, n_seeds=2)
    assert all(s.h0_band == 1 for s in b.dstrips)
    b.compute_sigmas()
    b.compute_gamma_factors()
    out = {}
    for band in (1, 2, 0):
        _with_band(b, band)
        G1N, _, GNN, st = b.sweep("fp64", gnn=True)
        G1Np, _, stp = b.sweep_projected()
        T = b.transmission(G1N, GNN=GNN)[0]
        Tp = b.transmission_projected(G1Np)
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0 and int(stp.abs().sum()) == 0
        out[band] = [x.cpu().numpy() for x in (G1N, GNN, G1Np, T, Tp)]
    for band in (1, 2):
        for x, y in zip(out[band], out[0]):
            assert np.array_equal(x, y), band


@gpu
def test_banded_ldos_is_bitwise_the_full_read():
    from paper_1010_2627_amd import workload
    b = workload.square_batch(W=32, L=24, w=1.0, n_energies=4, n_seeds=1)
    b.compute_sigmas()
    res = {}
    for band in (1, 0):
        _with_band(b, band)
        ws = torch.empty(max(K.knit_ldos_workspace(b.dstrips, b.probs, "fp64", 0), 1), dtype=torch.uint8,
                         device="cuda")
        ld, st = K.knit_ldos(b.dstrips, b.probs, b.onsite, b.sigmaL, b.sigmaR, "fp64", workspace=ws)
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0
        res[band] = ld.cpu().numpy()
    assert np.array_equal(res[1], res[0])
