"""Conductance matrix of strips with side leads on the GPU against the oracle.

Side leads attach to single slices through their self-energies (independent
chains on chosen sites, or a seeded lead-like synthetic term); the GPU sweeps
forward and backward and carries every lead's columns and rows across the
cuts, the oracle inverts the whole strip with every self-energy in place.
T_kl agree elementwise at 1e-10 (relative to max(1, |T|)); row and column
sums agree; with no side lead the matrix is the two-terminal T.
"""

import numpy as np
import pytest
import torch

from paper_1010_2627_amd import inputs

pytestmark = pytest.mark.gpu
gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def _probe(M, sites, E, t=1.0):
    from oracle import leads as OL
    S = np.zeros((M, M), dtype=np.complex128)
    for j in sites:
        S[j, j] = t * t * OL.sigma_chain_closed_form(E)
    return S


def _run(b, sL, sR, side_specs, stride=0):
    """side_specs: per side lead j a function (E) -> Sigma_j [M, M] and a slice.  Returns (T gpu, T oracle)."""
    from oracle import multiterminal as OM
    from oracle import rgf as OR
    from paper_1010_2627_amd import knit as K
    st = b.strips[0]
    M = st.M
    E = b.energies[0]
    nE, nS = len(E), len(side_specs)
    sigX = np.zeros((nS, nE, M, M), dtype=np.complex128)
    for j, (sl, f) in enumerate(side_specs):
        for e in range(nE):
            sigX[j, e] = f(E[e])
    b.set_sigmas([sL], [sR])
    b.compute_gamma_factors()
    sX = torch.from_numpy(sigX.reshape(-1)).to("cuda")
    CX, _ = K.knit_gamma_factor(M, sX, nS * nE)
    side = np.zeros((b.P, nS), dtype=K.LEAD_DTYPE)
    for p in range(b.P):
        ri, ei = b.prob_meta[p]
        for j, (sl, _) in enumerate(side_specs):
            side[p, j]["slice"] = sl
            side[p, j]["sigma_off"] = (j * nE + ei) * M * M
    T, status = K.knit_conductance_matrix(b.dstrips, b.probs, b.onsite, b.sigmaL, b.sigmaR, b.CL, b.CR, side, sX, CX,
                                          checkpoint_stride=stride)
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0
    T = T.cpu().numpy()
    ref = np.zeros_like(T)
    for p in range(b.P):
        ri, ei = b.prob_meta[p]
        on = b.realizations[ri].onsite
        Hn = st.H0[None] + on if st.onsite_dense else OR.slice_hamiltonians(st.H0, on)
        ref[p] = OM.conductance_matrix(st.V_dense(), Hn, E[ei], sL[ei], sR[ei],
                                       [(sl, sigX[j, ei]) for j, (sl, _) in enumerate(side_specs)])
    return T, ref


def _sig(st, E):
    from oracle import leads as OL
    V = st.V_dense()
    return (np.stack([OL.sigma_modes(st.H0, V, e, "L") for e in E]),
            np.stack([OL.sigma_modes(st.H0, V, e, "R") for e in E]))


@gpu
@pytest.mark.parametrize("kind", ["square", "rashba", "nnn"])
@pytest.mark.parametrize("stride", [0, 2])
def test_conductance_matrix_matches_oracle(kind, stride):
    from paper_1010_2627_amd import workload
    st = {"square": lambda: inputs.square_strip(10), "rashba": lambda: inputs.rashba_strip(5),
          "nnn": lambda: inputs.square_nnn_strip(8, tp=0.3)}[kind]()
    L = 9
    E = np.array([-1.2, 0.4, 1.55])
    b = workload.Batch([st], [workload.Realization(0, inputs.onsite_disorder(st, L, 2.0, inputs.SEED_BASE))], [E])
    sL, sR = _sig(st, E)
    M = st.M
    specs = [(3, lambda e: _probe(M, [0, 1], e, 0.9)),          # two chains on the first sites of slice 3
             (3, lambda e: _probe(M, [M - 1], e, 1.2)),         # another lead on the same slice
             (0, lambda e: _probe(M, [M // 2], e)),             # a probe on the left interface slice
             (L - 2, lambda e: _probe(M, list(range(M - 3, M)), e, 0.7))]
    T, ref = _run(b, sL, sR, specs, stride)
    scale = np.maximum(1.0, np.abs(ref))
    assert np.max(np.abs(T - ref) / scale) < 1e-10, np.max(np.abs(T - ref))
    assert np.max(np.abs(T.sum(axis=1) - T.sum(axis=2))) < 1e-9


@gpu
def test_y_junction_closed_form_and_two_terminal_reduction():
    """A chain with a side chain on slice 4 of 7 (clean): T_kl = 4 sin^2 k / (cos^2 k + 9 sin^2 k) for
    every k != l; with no side lead the matrix holds the two-terminal T both ways."""
    from paper_1010_2627_amd import workload
    st = inputs.square_strip(1)
    E = np.array([-1.3, 0.0, 0.9])
    b = workload.Batch([st], [workload.Realization(0, inputs.clean_onsite(st, 7))], [E])
    sL, sR = _sig(st, E)
    T, ref = _run(b, sL, sR, [(4, lambda e: _probe(1, [0], e))])
    k = np.arccos(E / 2)
    expect = 4 * np.sin(k) ** 2 / (np.cos(k) ** 2 + 9 * np.sin(k) ** 2)
    off = ~np.eye(3, dtype=bool)
    for p in range(3):
        assert np.max(np.abs(T[p][off] - expect[p])) < 1e-12
    b2 = workload.square_batch(12, 11, 2.0, 4, 1)
    sL2, sR2 = _sig(b2.strips[0], b2.energies[0])
    T2, ref2 = _run(b2, sL2, sR2, [])
    b2.set_sigmas([sL2], [sR2])
    b2.compute_gamma_factors()
    Tp = b2.transmission_projected(b2.sweep_projected()[0]).cpu().numpy()
    assert np.max(np.abs(T2[:, 0, 1] - Tp) / np.maximum(1, Tp)) < 1e-10
    assert np.max(np.abs(T2[:, 1, 0] - Tp) / np.maximum(1, Tp)) < 1e-10
