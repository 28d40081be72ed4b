"""GPU parity of the matrix-core sweep at larger slice sizes, in every precision mode.

Tolerances (checked per energy):
  FP64          |dT| <= 1e-10 * max(1, |T|)
  FP32_REFINE   |dT| <= 1e-6 * max(1, N_open(E))   (N_open: open channels of the lead)
  FP32          |dT| <= 1e-3 * max(1, N_open(E))   (no refinement: loose sanity bound)
Self-energies come from the oracle's Bloch-mode method (or, at slice dimension
512, seeded synthetic boundary terms of a lead-like rank) so that only the sweep
and the trace are compared.  The refined mode is checked on strips as long as
the benchmark's (L = 1024 at slice dimension 128, L = 512 at 512), on the
whole-propagator and the projected sweeps and on the LDOS.
"""

import numpy as np
import pytest
import torch

from paper_1010_2627_amd import inputs

pytestmark = pytest.mark.gpu
gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def _oracle(batch):
    from oracle import leads as OL
    from oracle import rgf as OR
    st = batch.strips[0]
    V = st.V_dense()
    E = batch.energies[0]
    sL = np.stack([OL.sigma_modes(st.H0, V, e, "L") for e in E])
    sR = np.stack([OL.sigma_modes(st.H0, V, e, "R") for e in E])
    T = np.zeros(batch.P)
    for ri, r in enumerate(batch.realizations):
        res = OR.rgf_forward(st.H0, V, r.onsite, E, sL, sR)
        T[ri * len(E):(ri + 1) * len(E)] = OR.transmission_lr(sL, sR, res["G1N"])
    # open channels from Gamma_L's rank: trace of Gamma normalised by its largest eigenvalue is
    # not an integer, so count propagating modes as the number of eigenvalues of Gamma above 1e-8
    nopen = np.array([(np.linalg.eigvalsh(OL.gamma_of(s)) > 1e-8).sum() for s in sL])
    return sL, sR, T, np.tile(nopen, len(batch.realizations))


CASES = {
    "square64": lambda w: w.square_batch(64, 40, 2.0, 8, 2),
    "square100_odd": lambda w: w.square_batch(100, 17, 1.5, 6, 1),
    "rashba24": lambda w: w.rashba_batch(24, 30, 2.0, 6, 2),
    "zigzag20": lambda w: w.zigzag_batch(20, 25, 0.6, [-2.1, -0.8, 0.45, 1.7], 2),
    "square256_short": lambda w: w.square_batch(256, 6, 2.0, 3, 1),
}


@gpu
@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
def test_sweep_precision_modes_match_oracle(case, prec):
    from paper_1010_2627_amd import workload
    b = CASES[case](workload)
    sL, sR, Tref, nopen = _oracle(b)
    b.set_sigmas([sL], [sR])
    G1N, _, GNN, status = b.sweep(prec, gnn=True)
    T, _, Tw = b.transmission(G1N, GNN=GNN)
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0, status
    T = T.cpu().numpy()
    if prec == "fp64":
        err = np.abs(T - Tref) / np.maximum(1.0, np.abs(Tref))
        assert err.max() < 1e-10, (case, err.max())
        assert np.max(np.abs(Tw.cpu().numpy() - T)) < 1e-9
    else:
        tol = 1e-6 if prec == "fp32_refine" else 1e-3
        err = np.abs(T - Tref) / np.maximum(1.0, nopen)
        print(f"{case} {prec}: max |dT|/max(1,N_open) = {err.max():.3e}")
        assert err.max() < tol, (case, prec, err.max())


@gpu
def test_gn1_on_matrix_core_path():
    from paper_1010_2627_amd import workload
    from oracle import rgf as OR
    b = workload.rashba_batch(20, 12, 2.0, 4, 1)
    sL, sR, Tref, _ = _oracle(b)
    b.set_sigmas([sL], [sR])
    G1N, GN1, GNN, status = b.sweep("fp64", gn1=True, gnn=True)
    T, Trl, Tw = b.transmission(G1N, GN1, GNN)
    torch.cuda.synchronize()
    st = b.strips[0]
    res = OR.rgf_forward(st.H0, st.V_dense(), b.realizations[0].onsite, b.energies[0], sL, sR)
    for ei in range(len(b.energies[0])):
        for name, flat in (("G1N", G1N), ("GN1", GN1), ("GNN", GNN)):
            got = b.block(flat, ei).cpu().numpy()
            ref = res[name][ei]
            assert np.max(np.abs(got - ref)) < 1e-10 * max(1.0, np.abs(ref).max()), name
    assert np.max(np.abs(Trl.cpu().numpy() - T.cpu().numpy())) < 1e-9


@gpu
def test_generic_kernel_above_512():
    """M = 520 (> 512) runs on the generic workgroup kernel; FP64 parity on a short strip."""
    from paper_1010_2627_amd import workload
    b = workload.square_batch(520, 2, 2.0, 1, 1, emin=-0.3, emax=0.3)
    sL, sR, Tref, _ = _oracle(b)
    b.set_sigmas([sL], [sR])
    G1N, _, _, status = b.sweep("fp64", gnn=False)
    T = b.transmission(G1N)[0]
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0
    assert abs(float(T.cpu().numpy()[0]) - Tref[0]) < 1e-10 * max(1.0, abs(Tref[0]))


@gpu
def test_refine_fallback_everywhere_equals_fp64_bitwise():
    """Threshold 0: every problem's refinement is refused, so the call's second (FP64) pass
    recomputes all of them; outputs equal the FP64 sweep bit for bit, status says so."""
    from paper_1010_2627_amd import knit as K, workload
    b = workload.square_batch(40, 24, 2.0, 6, 2)
    b.compute_sigmas()
    G64, _, N64, s64 = b.sweep("fp64", gnn=True)
    old = K.knit_get_refine_threshold()
    try:
        K.knit_set_refine_threshold(0.0)
        Gm, _, Nm, sm = b.sweep("fp32_refine", gnn=True)
        torch.cuda.synchronize()
    finally:
        K.knit_set_refine_threshold(old)
    assert int(s64.abs().sum()) == 0
    assert torch.all(sm == K.KNIT_P_FALLBACK)
    assert torch.equal(Gm, G64) and torch.equal(Nm, N64)


@gpu
def test_refine_guard_bounds_the_error_on_strong_disorder():
    """Strong disorder and many energies (slices far from well conditioned): problems the
    guard hands to FP64 equal the FP64 sweep; the others stay within 1e-6 per open channel."""
    from paper_1010_2627_amd import knit as K, workload
    b = workload.square_batch(48, 96, 6.0, 48, 4, emin=-4.5, emax=4.5)
    b.compute_sigmas()
    G64, _, _, s64 = b.sweep("fp64", gnn=False)
    T64 = b.transmission(G64)[0].cpu().numpy()
    Gm, _, _, sm = b.sweep("fp32_refine", gnn=False)
    Tm = b.transmission(Gm)[0].cpu().numpy()
    sm = sm.cpu().numpy()
    assert int(s64.abs().sum()) == 0
    assert np.all((sm & ~K.KNIT_P_FALLBACK) == 0)
    fb = (sm & K.KNIT_P_FALLBACK) != 0
    assert np.array_equal(Tm[fb], T64[fb])
    # channel count of the clean lead at each energy bounds T
    nopen = np.maximum(1.0, np.ceil(np.abs(T64) - 1e-9))
    err = np.abs(Tm - T64) / nopen
    print(f"strong disorder: {int(fb.sum())}/{len(fb)} fallbacks, max |dT|/channel {err.max():.2e}")
    assert err[~fb].max(initial=0.0) <= 1e-6, (err.max(), int(fb.sum()))


@gpu
@pytest.mark.parametrize("case,prec", [("square70", "fp64"), ("rashba20", "fp64"), ("zigzag18", "fp64"),
                                       ("square70", "fp32"), ("square70", "fp32_refine"),
                                       ("rashba20", "fp32_refine"), ("zigzag18", "fp32_refine")])
def test_ldos_on_matrix_cores_matches_oracle(case, prec):
    """Backward (sewing) sweep on the matrix-core path: slices padded to 32 (M = 70, 40, 36),
    spinful and zigzag couplings, checkpoint stride sqrt(L); FP64 at 1e-10, refined FP32 at
    1e-8, plain FP32 at 1e-3."""
    from oracle import rgf as OR
    from paper_1010_2627_amd import workload
    if case == "square70":
        b = workload.square_batch(70, 19, 2.0, 4, 1)
    elif case == "rashba20":
        b = workload.rashba_batch(20, 17, 2.0, 4, 1)
    else:
        b = workload.zigzag_batch(18, 15, 0.6, inputs.midpoint_grid(-2.9, 2.9, 4), 1)
    st = b.strips[0]
    E = b.energies[0]
    sL, sR, _, _ = _oracle(b)
    b.set_sigmas([sL], [sR])
    ld, status = b.ldos(prec)
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0
    ref = OR.ldos_rgf(st.H0, st.V_dense(), b.realizations[0].onsite, E, sL, sR)
    tol = {"fp64": 1e-10, "fp32_refine": 1e-8, "fp32": 1e-3}[prec]
    for ei in range(len(E)):
        got = b.ldos_block(ld, ei).cpu().numpy()
        assert np.max(np.abs(got - ref[ei]) / np.maximum(1, np.abs(ref[ei]))) < tol, (case, prec, ei)


@gpu
@pytest.mark.parametrize("case", ["square64", "square100_odd", "rashba24", "zigzag20"])
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
def test_projected_sweep_precision_modes_match_oracle(case, prec):
    """The projected propagator C_L^+ G_1n in every precision: refined rows are FP64 products of
    the refined inverses; T = ||P_L C_R||^2 against the oracle's Fisher-Lee trace."""
    from paper_1010_2627_amd import workload
    b = CASES[case](workload)
    sL, sR, Tref, nopen = _oracle(b)
    b.set_sigmas([sL], [sR])
    b.compute_gamma_factors()
    G1Np, _, status = b.sweep_projected(precision=prec)
    T = b.transmission_projected(G1Np).cpu().numpy()
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0, status
    if prec == "fp64":
        err = np.abs(T - Tref) / np.maximum(1.0, np.abs(Tref))
        assert err.max() < 1e-10, (case, err.max())
    else:
        tol = 1e-6 if prec == "fp32_refine" else 1e-3
        err = np.abs(T - Tref) / np.maximum(1.0, nopen)
        print(f"{case} projected {prec}: max |dT|/max(1,N_open) = {err.max():.3e}")
        assert err.max() < tol, (case, prec, err.max())


@gpu
def test_refined_sweeps_on_long_square_strip_match_oracle():
    """Slice dimension 128, L = 1024 (the square W=128 workload's strip), 8 energies across the
    band: the refined whole-propagator and projected sweeps against the oracle on every problem,
    |dT| <= 1e-6 per open channel; problems the guard sent to FP64 are reported."""
    from paper_1010_2627_amd import knit as K, workload
    b = workload.square_batch(128, 1024, 2.0, 8, 1)
    sL, sR, Tref, nopen = _oracle(b)
    b.set_sigmas([sL], [sR])
    b.compute_gamma_factors()
    G1N, _, _, st = b.sweep("fp32_refine", gnn=False)
    T = b.transmission(G1N)[0].cpu().numpy()
    G1Np, _, stp = b.sweep_projected(precision="fp32_refine")
    Tp = b.transmission_projected(G1Np).cpu().numpy()
    torch.cuda.synchronize()
    st, stp = st.cpu().numpy(), stp.cpu().numpy()
    assert np.all((st & ~K.KNIT_P_FALLBACK) == 0) and np.all((stp & ~K.KNIT_P_FALLBACK) == 0)
    for name, got, s_ in (("full", T, st), ("projected", Tp, stp)):
        err = np.abs(got - Tref) / np.maximum(1.0, nopen)
        print(f"L=1024 M=128 refined {name}: max |dT|/channel {err.max():.2e}, "
              f"fallbacks {int((s_ != 0).sum())}/{len(s_)}")
        assert err.max() <= 1e-6, (name, err.max())


@gpu
def test_refined_sweeps_at_slice_dim_512_full_length():
    """The spinful W=256 strip (slice dim 512), L = 512, 8 energies with seeded synthetic boundary
    terms of rank 256 (a lead-like number of open channels, the same on both sides): refined
    whole-propagator and projected T within 1e-6 per channel of the FP64 GPU path on all 8
    problems, and of the oracle on two sampled ones (end to end, 512 slices each)."""
    from oracle import rgf as OR
    from paper_1010_2627_amd import inputs, knit as K, workload
    b = workload.rashba_batch(256, 512, 2.0, 8, 1)
    st = b.strips[0]
    r = 256
    sL = inputs.synthetic_sigma(st.M, 8, rank=r)
    sR = inputs.synthetic_sigma(st.M, 8, seed=inputs.SEED_SYNTHETIC_SIGMA + 1, rank=r)
    b.set_sigmas([sL], [sR])
    b.compute_gamma_factors()
    G64, _, _, s64 = b.sweep("fp64", gnn=False)
    T64 = b.transmission(G64)[0].cpu().numpy()
    Gm, _, _, sm = b.sweep("fp32_refine", gnn=False)
    Tm = b.transmission(Gm)[0].cpu().numpy()
    Gp, _, sp = b.sweep_projected(precision="fp32_refine")
    Tp = b.transmission_projected(Gp).cpu().numpy()
    torch.cuda.synchronize()
    assert int(s64.abs().sum()) == 0
    for name, got, s_ in (("full", Tm, sm.cpu().numpy()), ("projected", Tp, sp.cpu().numpy())):
        assert np.all((s_ & ~K.KNIT_P_FALLBACK) == 0)
        err = np.abs(got - T64) / r
        print(f"L=512 M=512 refined {name}: max |dT|/channel vs FP64 {err.max():.2e}, "
              f"fallbacks {int((s_ != 0).sum())}/{len(s_)}")
        assert err.max() <= 1e-6, (name, err.max())
    V = st.V_dense()
    idx = [1, 6]
    res = OR.rgf_forward(st.H0, V, b.realizations[0].onsite, b.energies[0][idx], sL[idx], sR[idx])
    Tref = OR.transmission_lr(sL[idx], sR[idx], res["G1N"])
    assert np.max(np.abs(T64[idx] - Tref) / np.maximum(1.0, np.abs(Tref))) < 1e-10
    assert np.max(np.abs(Tm[idx] - Tref)) / r <= 1e-6
    assert np.max(np.abs(Tp[idx] - Tref)) / r <= 1e-6
