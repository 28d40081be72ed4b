"""Transmission eigenvalues and the shot-noise Fano factor on the GPU against the oracle.

The GPU forms t~ = (C_L^+ G_1N) C_R from the projected sweep and reduces
tau = t~^+ t~ (or t~ t~^+) to tridiagonal form before bisection; the oracle
takes t = Gamma_R^{1/2} G_N1 Gamma_L^{1/2} from its own recursion and calls a
dense Hermitian eigensolver.  Both must give the same T_n (|dT_n| <= 1e-10),
channel count min(rank Gamma_L, rank Gamma_R), T = sum T_n and Fano factor.
"""

import numpy as np
import pytest
import torch

from paper_1010_2627_amd import inputs

pytestmark = pytest.mark.gpu
gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def _run(b, sL, sR):
    b.set_sigmas([sL], [sR])
    b.compute_gamma_factors()
    G1Np, _, st = b.sweep_projected()
    tn, nch, T, F = b.transmission_eigenvalues(G1Np)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    return tn.cpu().numpy(), nch.cpu().numpy(), T.cpu().numpy(), F.cpu().numpy()


def _oracle(b, sL, sR):
    from oracle import noise as ON
    from oracle import rgf as OR
    st = b.strips[0]
    E = b.energies[0]
    out = []
    for r in b.realizations:
        res = OR.rgf_forward(st.H0, st.V_dense(), r.onsite, E, sL, sR)
        out.append(ON.transmission_eigenvalues(sL, sR, res["GN1"]))
    return np.concatenate(out)


CASES = {
    "square_w24": lambda w: w.square_batch(24, 30, 2.0, 8, 2),
    "rashba_w20": lambda w: w.rashba_batch(20, 25, 2.0, 6, 1),
    "zigzag_nz12": lambda w: w.zigzag_batch(12, 20, 0.6, [-2.3, -1.1, 0.37, 1.55, 2.6], 1),
    "square_w70_ragged": lambda w: w.square_batch(70, 9, 3.0, 4, 1),
}


@gpu
@pytest.mark.parametrize("case", list(CASES))
def test_transmission_eigenvalues_match_oracle(case):
    from oracle import leads as OL
    from oracle import noise as ON
    from paper_1010_2627_amd import workload
    b = CASES[case](workload)
    st = b.strips[0]
    E = b.energies[0]
    V = st.V_dense()
    sL = np.stack([OL.sigma_modes(st.H0, V, e, "L") for e in E])
    sR = np.stack([OL.sigma_modes(st.H0, V, e, "R") for e in E])
    tn, nch, T, F = _run(b, sL, sR)
    ref = _oracle(b, sL, sR)
    nopen = np.tile([(np.linalg.eigvalsh(OL.gamma_of(s)) > 1e-8).sum() for s in sL], len(b.realizations))
    assert np.array_equal(nch, nopen)
    for p in range(b.P):
        k = nch[p]
        assert np.max(np.abs(tn[p, :k] - ref[p, :k]), initial=0.0) < 1e-10, (case, p)
        assert np.all(tn[p, k:] == 0.0)
        assert np.max(np.abs(ref[p, k:]), initial=0.0) < 1e-9      # the oracle's closed channels
    Tref = ref.sum(axis=1)
    assert np.max(np.abs(T - Tref) / np.maximum(1.0, Tref)) < 1e-10
    Fref = ON.fano_factor(ref)
    ok = Tref > 1e-6
    assert np.max(np.abs(F[ok] - Fref[ok])) < 1e-9
    assert tn.min() > -1e-12 and tn.max() < 1 + 1e-12


@gpu
def test_clean_ribbon_has_unit_eigenvalues_and_zero_noise():
    from oracle import leads as OL
    from paper_1010_2627_amd import workload
    st = inputs.square_strip(16)
    E = inputs.midpoint_grid(-3.6, 3.6, 12)
    b = workload.Batch([st], [workload.Realization(0, inputs.clean_onsite(st, 7))], [E])
    b.compute_sigmas()
    b.compute_gamma_factors()
    G1Np, _, _ = b.sweep_projected()
    tn, nch, T, F = [x.cpu().numpy() for x in b.transmission_eigenvalues(G1Np)]
    nopen = OL.n_open_square(16, E)
    assert np.array_equal(nch, nopen)
    for p in range(b.P):
        assert np.max(np.abs(tn[p, :nch[p]] - 1.0), initial=0.0) < 1e-9
    assert np.max(np.abs(F[nopen > 0])) < 1e-8
    assert np.all(np.isnan(F[nopen == 0]))


@gpu
def test_eigenvalues_at_slice_dim_512_sampled_against_oracle():
    """The spinful W=256 strip (slice dim 512) with lead-like synthetic boundary terms of ranks
    300 and 170: channel count 170 on every problem; two sampled problems (end to end, 64 slices)
    against the oracle; sum T_n = the projected trace on all."""
    from oracle import noise as ON
    from oracle import rgf as OR
    from paper_1010_2627_amd import workload
    b = workload.rashba_batch(256, 64, 2.0, 4, 2)
    st = b.strips[0]
    sL = inputs.synthetic_sigma(st.M, 4, rank=300)
    sR = inputs.synthetic_sigma(st.M, 4, seed=inputs.SEED_SYNTHETIC_SIGMA + 1, rank=170)
    tn, nch, T, F = _run(b, sL, sR)
    assert np.all(nch == 170)
    Tp = b.transmission_projected(b.sweep_projected()[0]).cpu().numpy()
    assert np.max(np.abs(T - Tp) / np.maximum(1.0, Tp)) < 1e-10
    assert np.max(np.abs(tn.sum(axis=1) - T) / np.maximum(1.0, T)) < 1e-10
    for ri, ei in [(0, 1), (1, 3)]:
        p = ri * 4 + ei
        res = OR.rgf_forward(st.H0, st.V_dense(), b.realizations[ri].onsite, b.energies[0][ei:ei + 1],
                             sL[ei:ei + 1], sR[ei:ei + 1])
        ref = ON.transmission_eigenvalues(sL[ei:ei + 1], sR[ei:ei + 1], res["GN1"])[0]
        assert np.max(np.abs(tn[p, :170] - ref[:170])) < 1e-10
        assert abs(F[p] - ON.fano_factor(ref[None])[0]) < 1e-9
