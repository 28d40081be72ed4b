"""GPU parity of the projected-propagator path against the FP64 CPU oracle, through the C ABI.

The path factors Gamma_L = C_L C_L^+ (pivoted Cholesky, rank = open channels), carries
P_n = C_L^+ G_1n through the slice recursion and takes T = ||P_L C_R||_F^2.  C is not
unique (pivots among degenerate channels are decided by rounding), so the checks compare
what the factorisation fixes:
  * C C^+ = Gamma of the oracle's self-energy, elementwise within 1e-10 of
    max(max |Gamma|, max |Sigma_ii|) (Gamma's rounding noise is relative to Sigma: where
    every channel is closed Gamma is that noise alone);
  * rank = the lead's open channels (the oracle's clean-strip conductance); columns past
    the rank zero, each column before it with a positive real entry;
  * T against the oracle's Re Tr[Gamma_L G_1L Gamma_R G_1L^+], |dT| <= 1e-10 max(1, |T|)
    (the FP64 path's bar);
  * the Gram matrix P_L^+ P_L = G_1L^+ Gamma_L G_1L, elementwise within 1e-10 of its
    largest entry.
The oracle knows nothing of the projection: its T and Gram matrix are the definitions.
"""

import numpy as np
import pytest
import torch

from paper_1010_2627_amd import inputs

pytestmark = pytest.mark.gpu
gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def _oracle_sigmas(strip, E):
    from oracle import leads as OL
    V = strip.V_dense()
    sL = np.stack([OL.sigma_modes(strip.H0, V, e, "L") for e in E])
    sR = np.stack([OL.sigma_modes(strip.H0, V, e, "R") for e in E])
    return sL, sR


def _oracle_open_channels(strip, E, sL, sR):
    from oracle import rgf as OR
    T = OR.transmission_full(strip.H0, strip.V_dense(), inputs.clean_onsite(strip, 1), E, sL, sR)[0]
    return np.rint(T).astype(np.int64)


def _gamma(s):
    return 1j * (s - np.conj(np.swapaxes(s, -1, -2)))


def _check_factor(C, rank, sigma):
    """C [n, M, M], rank [n] against Gamma [n, M, M] of the self-energies sigma."""
    Gamma = _gamma(sigma)
    for e in range(len(rank)):
        r = int(rank[e])
        assert 0 <= r <= C.shape[1]
        assert np.all(C[e][:, r:] == 0)
        for k in range(r):
            col = C[e][:, k]
            assert np.any((col.imag == 0) & (col.real > 0)), (e, k)
        G = Gamma[e]
        scale = max(np.abs(G).max(), np.abs(np.diagonal(sigma[e])).max(), 1e-300)
        assert np.abs(C[e] @ C[e].conj().T - G).max() <= 1e-10 * scale, e


@gpu
@pytest.mark.parametrize("case", ["square16", "square5", "rashba4", "zigzag4", "chain"])
def test_gamma_factor_rank_is_open_channels(case):
    from paper_1010_2627_amd import knit
    st = {"square16": inputs.square_strip(16), "square5": inputs.square_strip(5),
          "rashba4": inputs.rashba_strip(4), "zigzag4": inputs.zigzag_strip(4),
          "chain": inputs.square_strip(1)}[case]
    E = inputs.midpoint_grid(-3.9, 3.9, 24)
    if case == "zigzag4":
        E = E[np.abs(E) > 1e-3]
    sL, sR = _oracle_sigmas(st, E)
    nopen = _oracle_open_channels(st, E, sL, sR)
    for s in (sL, sR):
        sig = torch.from_numpy(np.ascontiguousarray(s)).cuda()
        C, rank = knit.knit_gamma_factor(st.M, sig, len(E))
        torch.cuda.synchronize()
        rank = rank.cpu().numpy()
        assert np.array_equal(rank, nopen), (rank, nopen)
        _check_factor(C.cpu().numpy(), rank, s)


@gpu
def test_gamma_factor_edge_cases():
    """Outside the band Gamma = 0 (rank 0, C = 0); a full-rank synthetic term keeps every
    column; a NaN term reports rank -1 and a NaN factor; n = 0 is a no-op."""
    from paper_1010_2627_amd import knit
    st = inputs.square_strip(6)
    E = np.array([-4.7, 4.3, 5.5])
    sL, _ = _oracle_sigmas(st, E)
    C, rank = knit.knit_gamma_factor(st.M, torch.from_numpy(sL).cuda(), len(E))
    torch.cuda.synchronize()
    assert np.array_equal(rank.cpu().numpy(), [0, 0, 0])
    assert not C.cpu().numpy().any()
    full = inputs.synthetic_sigma(37, 3)
    C, rank = knit.knit_gamma_factor(37, torch.from_numpy(full).cuda(), 3)
    torch.cuda.synchronize()
    assert np.array_equal(rank.cpu().numpy(), [37, 37, 37])
    _check_factor(C.cpu().numpy(), rank.cpu().numpy(), full)
    low = inputs.synthetic_sigma(70, 2, rank=23)
    C, rank = knit.knit_gamma_factor(70, torch.from_numpy(low).cuda(), 2)
    torch.cuda.synchronize()
    assert np.array_equal(rank.cpu().numpy(), [23, 23])
    _check_factor(C.cpu().numpy(), rank.cpu().numpy(), low)
    bad = full.copy()
    bad[1, 5, 5] = np.nan
    C, rank = knit.knit_gamma_factor(37, torch.from_numpy(bad).cuda(), 3)
    torch.cuda.synchronize()
    assert np.array_equal(rank.cpu().numpy(), [37, -1, 37])
    assert np.all(np.isnan(C[1].cpu().numpy().real))
    C0, r0 = knit.knit_gamma_factor(8, torch.zeros(0, dtype=torch.complex128, device="cuda"), 0)
    assert r0.numel() == 0


def _projected(b):
    b.compute_sigmas()
    b.compute_gamma_factors()
    G1Np, GNN, status = b.sweep_projected(gnn=True)
    T = b.transmission_projected(G1Np)
    torch.cuda.synchronize()
    return G1Np, GNN, status, T


def _oracle_batch(b, sLs, sRs):
    """Oracle T and G_1L of every problem, per strip class."""
    from oracle import rgf as OR
    T = np.zeros(b.P)
    G1N = {}
    for ri, r in enumerate(b.realizations):
        st = b.strips[r.strip]
        E = b.energies[r.strip]
        sL, sR = sLs[r.strip], sRs[r.strip]
        res = OR.rgf_forward(st.H0, st.V_dense(), r.onsite, E, sL, sR)
        Tr = OR.transmission_lr(sL, sR, res["G1N"])
        for ei in range(len(E)):
            p = [i for i, m in enumerate(b.prob_meta) if tuple(m) == (ri, ei)][0]
            T[p] = Tr[ei]
            G1N[p] = res["G1N"][ei]
    return T, G1N


BATCHES = {
    # one class, several tiles of 32 and a ragged tail (M = 40 -> Mp = 64)
    "square40": lambda w: w.square_batch(40, 23, 1.5, 12, 2),
    # spinful, M = 48
    "rashba24": lambda w: w.rashba_batch(24, 17, 1.0, 10, 2),
    # a single slice: P_1 = C_L^+ g_1 with both leads on it
    "square16_L1": lambda w: w.square_batch(16, 1, 1.0, 16, 1),
    # honeycomb, energies away from the E = 0 edge states
    "zigzag6": lambda w: w.zigzag_batch(6, 20, 0.5, np.linspace(-2.6, 2.6, 10) + 0.013, 2),
}


@gpu
@pytest.mark.parametrize("name", list(BATCHES))
def test_projected_transmission_matches_oracle(name):
    from paper_1010_2627_amd import workload
    from oracle import leads as OL
    b = BATCHES[name](workload)
    G1Np, GNN, status, T = _projected(b)
    assert int(status.abs().sum()) == 0
    st = b.strips[0]
    sL, sR = _oracle_sigmas(st, b.energies[0])
    Tref, G1ref = _oracle_batch(b, [sL], [sR])
    T = T.cpu().numpy()
    assert np.max(np.abs(T - Tref) / np.maximum(1.0, np.abs(Tref))) <= 1e-10
    # the ranks are the leads' open channels
    nopen = _oracle_open_channels(st, b.energies[0], sL, sR)
    assert np.array_equal(b.rankL.cpu().numpy(), nopen)
    assert np.array_equal(b.rankR.cpu().numpy(), nopen)
    # Gram matrix of the projected propagator, and its zero rows
    M = st.M
    for p in range(0, b.P, max(1, b.P // 5)):
        Pm = b.block(G1Np, p).cpu().numpy()
        ei = int(b.prob_meta[p][1])
        r = int(nopen[ei])
        assert not Pm[r:].any()
        gram = Pm.conj().T @ Pm
        ref = G1ref[p].conj().T @ OL.gamma_of(sL[ei]) @ G1ref[p]
        assert np.abs(gram - ref).max() <= 1e-10 * max(np.abs(ref).max(), 1e-300), p
        # G_LL is the full path's own output
        assert GNN is not None and b.block(GNN, p).shape == (M, M)


@gpu
def test_projected_path_agrees_with_full_path_on_mixed_classes():
    """Uneven strips (several classes in one launch): the projected T equals the full
    path's T on every problem, and every strip class's energies include out-of-band
    points where T = 0 and the projected propagator is zero."""
    from paper_1010_2627_amd import workload
    strips = [inputs.square_strip(W) for W in (7, 33, 64)]
    E = np.concatenate([inputs.midpoint_grid(-3.9, 3.9, 10), [4.6, -4.9]])
    reals = [workload.Realization(i % 3, inputs.onsite_disorder(strips[i % 3], 5 + 3 * i, 1.0, 1000 + i))
             for i in range(6)]
    b = workload.Batch(strips, reals, [E for _ in strips])
    G1Np, _, status, T = _projected(b)
    G1N, _, _, st_full = b.sweep("fp64", gnn=False)
    Tf = b.transmission(G1N)[0]
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0 and int(st_full.abs().sum()) == 0
    T, Tf = T.cpu().numpy(), Tf.cpu().numpy()
    assert np.max(np.abs(T - Tf) / np.maximum(1.0, np.abs(Tf))) <= 1e-10
    out = np.abs(E[b.prob_meta[:, 1]]) > 4.5
    assert np.all(T[out] == 0.0)
    for p in np.nonzero(out)[0]:
        assert not b.block(G1Np, int(p)).cpu().numpy().any()
    # against the oracle on one problem of each class
    from oracle import rgf as OR
    for c in range(3):
        p = [i for i, (ri, ei) in enumerate(b.prob_meta) if reals[ri].strip == c and ei == 4][0]
        ri = int(b.prob_meta[p][0])
        st = strips[c]
        sL, sR = _oracle_sigmas(st, E[4:5])
        res = OR.rgf_forward(st.H0, st.V_dense(), reals[ri].onsite, E[4:5], sL, sR)
        Tref = OR.transmission_lr(sL, sR, res["G1N"])[0]
        assert abs(T[p] - Tref) <= 1e-10 * max(1.0, abs(Tref))


@gpu
def test_projected_full_size_spinful_w256():
    """The benchmark's spinful W=256 batch (slice dim 512, L=512, 64 energies x 8 seeds) in
    the launch configuration the benchmark times, with seeded synthetic boundary terms of
    rank 300 (left) and 170 (right): rank = 300 and 170 on every energy, 0 <= T <= 170 on
    every problem, sampled problems against the oracle end to end, and bitwise
    reproducibility of the batch."""
    from paper_1010_2627_amd import workload
    from oracle import rgf as OR
    b = workload.rashba_batch(256, 512, 2.0, 64, 8)
    st = b.strips[0]
    nE = len(b.energies[0])
    sL = inputs.synthetic_sigma(st.M, nE, rank=300)
    sR = inputs.synthetic_sigma(st.M, nE, seed=inputs.SEED_SYNTHETIC_SIGMA + 1, rank=170)
    b.set_sigmas([sL], [sR])
    b.compute_gamma_factors()
    G1Np, _, status = b.sweep_projected()
    T = b.transmission_projected(G1Np)
    G1Np2, _, _ = b.sweep_projected()
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0
    assert torch.all(b.rankL == 300) and torch.all(b.rankR == 170)
    assert torch.equal(G1Np, G1Np2)
    T = T.cpu().numpy()
    assert np.all(T >= -1e-9) and np.all(T <= 170 + 1e-9)
    V = st.V_dense()
    for ri, ei in [(0, 9), (6, 41)]:
        p = ri * nE + ei
        assert tuple(b.prob_meta[p]) == (ri, ei)
        E = np.array([b.energies[0][ei]])
        res = OR.rgf_forward(st.H0, V, b.realizations[ri].onsite, E, sL[ei:ei + 1], sR[ei:ei + 1])
        Tref = OR.transmission_lr(sL[ei:ei + 1], sR[ei:ei + 1], res["G1N"])[0]
        assert abs(T[p] - Tref) <= 1e-10 * max(1.0, abs(Tref)), (p, T[p], Tref)


@gpu
def test_mid_size_odd_tile_counts_match_oracle():
    """Slice dim 416 (512 threads, 128-wide outer panels): the whole-G_1n sweep has 13 bottom
    tiles of 32 rows and the projected one, with Gamma_L of rank 77, has 3, so both use 64-row
    tiles next to a single trailing 32-row tile in the outer products.  Both against the
    oracle's T at 1e-10, with seeded synthetic boundary terms."""
    from paper_1010_2627_amd import workload
    from oracle import rgf as OR
    b = workload.square_batch(416, 5, 1.0, 2, 1)
    st = b.strips[0]
    E = b.energies[0]
    sL = inputs.synthetic_sigma(st.M, len(E), rank=77)
    sR = inputs.synthetic_sigma(st.M, len(E), seed=inputs.SEED_SYNTHETIC_SIGMA + 1)
    b.set_sigmas([sL], [sR])
    b.compute_gamma_factors()
    G1Np, _, status_p = b.sweep_projected()
    Tp = b.transmission_projected(G1Np)
    G1N, _, _, status = b.sweep("fp64", gnn=False)
    T = b.transmission(G1N)[0]
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0 and int(status_p.abs().sum()) == 0
    assert torch.all(b.rankL == 77)
    res = OR.rgf_forward(st.H0, st.V_dense(), b.realizations[0].onsite, E, sL, sR)
    Tref = OR.transmission_lr(sL, sR, res["G1N"])
    for got in (T.cpu().numpy(), Tp.cpu().numpy()):
        assert np.max(np.abs(got - Tref) / np.maximum(1.0, np.abs(Tref))) <= 1e-10, (got, Tref)
    for p in range(b.P):
        ref = res["G1N"][p]
        assert np.max(np.abs(b.block(G1N, p).cpu().numpy() - ref)) <= 1e-10 * max(1.0, np.abs(ref).max())
