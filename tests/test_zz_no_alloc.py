"""knit_rgf_sweep_noalloc against knit_rgf_sweep, through the C ABI.

The allocation-free entry point runs the same sweep kernels with the library's
static per-GPU scratch as work memory (fewer resident workgroups).  Every
problem is computed by one workgroup in the same order of operations whatever
the grid, so its outputs must equal the workspace entry point's bit for bit.
Two calls in a row, the second on a smaller batch, check that the scratch left
by the first call does not leak into the second.
"""

import numpy as np
import pytest
import torch

gpu_only = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def gpu(f):
    return pytest.mark.gpu(gpu_only(f))


def test_noalloc_host_argument_checks():
    """Validation happens on the host before any device call (no GPU needed): bad arguments,
    slices above 512 and batches above the problem limit are refused without enqueuing."""
    from paper_1010_2627_amd import knit as K
    lib = K._lib
    FAKE = 0x1000
    s = (K.KnitStrip * 1)(K.KnitStrip(16, 1, FAKE, FAKE, FAKE, None, 0, 0))
    probs = np.zeros(2, dtype=K.PROBLEM_DTYPE)
    probs["L"] = 4
    call = lambda strips, host, P, prec=0, G1N=FAKE, st=FAKE: lib.knit_rgf_sweep_noalloc(
        strips, 1, host.ctypes.data, FAKE, P, FAKE, FAKE, FAKE, prec, G1N, None, None, st, None)
    assert call(s, probs, 2, prec=9) == K.KNIT_E_ARG
    assert call(s, probs, 2, G1N=None) == K.KNIT_E_ARG
    assert call(s, probs, 2, st=None) == K.KNIT_E_ARG
    bad = probs.copy()
    bad["L"] = 0
    assert call(s, bad, 2) == K.KNIT_E_ARG
    wide = (K.KnitStrip * 1)(K.KnitStrip(544, 1, FAKE, FAKE, FAKE, None, 0, 0))
    assert call(wide, probs, 2) == K.KNIT_E_UNSUPPORTED
    big = np.zeros(K.KNIT_NOALLOC_MAX_PROBLEMS + 1, dtype=K.PROBLEM_DTYPE)
    big["L"] = 1
    assert call(s, big, big.shape[0]) == K.KNIT_E_SCRATCH
    assert lib.knit_rgf_sweep_noalloc(s, 1, None, None, 0, None, None, None, 0, None, None, None, None,
                                      None) == K.KNIT_OK


def _run_both(b, prec, gn1, gnn):
    from paper_1010_2627_amd import knit as K
    G1, N1, NN, st = b.sweep(prec, gn1=gn1, gnn=gnn)
    n = G1.numel()
    G1s = torch.full((n,), complex("nan"), dtype=torch.complex128, device="cuda")
    N1s = torch.full((n,), complex("nan"), dtype=torch.complex128, device="cuda") if gn1 else None
    NNs = torch.full((n,), complex("nan"), dtype=torch.complex128, device="cuda") if gnn else None
    sts = torch.full((b.P,), -7, dtype=torch.int32, device="cuda")
    K.knit_rgf_sweep_noalloc(b.dstrips, b.probs, b.onsite, b.sigmaL, b.sigmaR, prec, G1N=G1s, GN1=N1s, GNN=NNs,
                             status=sts)
    torch.cuda.synchronize()
    return (G1, N1, NN, st), (G1s, N1s, NNs, sts)


@gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_noalloc_sweep_equals_workspace_sweep_on_two_calls(prec):
    from paper_1010_2627_amd import workload
    first = workload.rashba_batch(20, 17, 2.0, 6, 2)          # slice dim 40, 12 problems
    second = workload.square_batch(24, 9, 1.0, 3, 1)          # smaller: slice dim 24, 3 problems
    for b, gn1 in ((first, True), (second, False)):
        b.compute_sigmas()
        (G1, N1, NN, st), (G1s, N1s, NNs, sts) = _run_both(b, prec, gn1, True)
        print(f"noalloc {prec}: P={b.P} M={b.strips[0].M} status {sts.cpu().numpy().tolist()}")
        assert torch.equal(sts, st[:b.P])
        assert torch.equal(G1s, G1) and torch.equal(NNs, NN)
        if gn1:
            assert torch.equal(N1s, N1)


@gpu
def test_noalloc_sweep_at_slice_dim_512_with_few_resident_workgroups():
    """Slice dimension 512: the scratch holds three slabs, so 8 problems queue through three
    resident workgroups; outputs equal the full-workspace sweep bit for bit."""
    from paper_1010_2627_amd import inputs, workload
    b = workload.rashba_batch(256, 4, 2.0, 4, 2)
    st = b.strips[0]
    b.set_sigmas([inputs.synthetic_sigma(st.M, 4)], [inputs.synthetic_sigma(st.M, 4, seed=inputs.SEED_SYNTHETIC_SIGMA + 1)])
    (G1, _, NN, s), (G1s, _, NNs, ss) = _run_both(b, "fp64", False, True)
    assert int(s.abs().sum()) == 0
    assert torch.equal(ss, s[:b.P]) and torch.equal(G1s, G1) and torch.equal(NNs, NN)


@gpu
def test_noalloc_rejects_what_does_not_fit_without_enqueuing():
    from paper_1010_2627_amd import knit as K, workload
    b = workload.square_batch(8, 3, 1.0, 2, 1)
    b.compute_sigmas()
    G1 = torch.zeros(b.P * 64, dtype=torch.complex128, device="cuda")
    host = np.zeros(K.KNIT_NOALLOC_MAX_PROBLEMS + 1, dtype=K.PROBLEM_DTYPE)
    host["L"] = 1
    code = K._lib.knit_rgf_sweep_noalloc(K.strip_table(b.dstrips), 1, host.ctypes.data, b.probs.dev.data_ptr(),
                                         host.shape[0], b.onsite.data_ptr(), b.sigmaL.data_ptr(),
                                         b.sigmaR.data_ptr(), 0, G1.data_ptr(), None, None, G1.data_ptr(), None)
    assert code == K.KNIT_E_SCRATCH
    torch.cuda.synchronize()
    assert int(G1.abs().sum()) == 0
