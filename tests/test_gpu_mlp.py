"""GPU: the learned sampler's BF16 kernels against the CPU reference (oracle.mlp), a
training run, and what the trained network gains over uniform energy points.

Tolerances: GEMMs of BF16 operands are exact products summed in FP32, so they agree
with the reference to FP32 summation order (relative 1e-5); BF16 outputs agree within
one BF16 unit in the last place; gradients of the whole network satisfy cosine >= 0.999
and relative L2 <= 1e-2 per tensor.
"""

import numpy as np
import pytest
import torch

from oracle import mlp as OM

pytestmark = pytest.mark.gpu
gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def _bf16(a):
    return torch.from_numpy(OM.bf16_round(np.asarray(a, np.float32))).to(torch.bfloat16).cuda()


def _ulp_close(a_bf16, b_exact):
    """|a - b| within one bf16 ulp of b, plus 1e-6 of the array's largest value (where b
    crosses zero, e.g. gelu' near x = -0.75, FP32 rounding exceeds b itself)."""
    a = a_bf16.float().cpu().numpy().astype(np.float64)
    b = np.asarray(b_exact, np.float64)
    tol = np.abs(b) * 2.0 ** -7 + 1e-6 * np.abs(b).max()
    return np.all(np.abs(a - b) <= tol)


@gpu
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (37, 50, 131), (64, 32, 16), (256, 512, 256), (5, 300, 77)])
def test_gemm_three_layouts_match_reference(M, N, K):
    from paper_1010_2627_amd import mlp
    rng = np.random.Generator(np.random.PCG64(M * 1000 + N + K))
    A = OM.bf16_round(rng.normal(size=(M, K)).astype(np.float32))
    Bm = OM.bf16_round(rng.normal(size=(N, K)).astype(np.float32))
    bias = rng.normal(size=N).astype(np.float32)
    ref = (A.astype(np.float64) @ Bm.astype(np.float64).T) + bias
    tol = 1e-5 * np.sqrt(K) * np.abs(A).max() * np.abs(Bm).max() + 1e-6
    # A B^T with row-major operands
    C = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    mlp.knit_mlp_gemm(M, N, K, _bf16(A), K, 1, _bf16(Bm), K, 1, C, N, bias=torch.from_numpy(bias).cuda())
    assert np.abs(C.cpu().numpy() - ref).max() <= tol
    # the same product from the transposed storage of both operands (strides swapped)
    At, Bt = _bf16(A.T.copy()), _bf16(Bm.T.copy())
    C2 = torch.full((M, N), 2.0, dtype=torch.float32, device="cuda")
    mlp.knit_mlp_gemm(M, N, K, At, 1, M, Bt, 1, N, C2, N, beta=0.5)
    assert np.abs(C2.cpu().numpy() - (ref - bias + 1.0)).max() <= tol


@gpu
def test_activations_and_softmax_match_reference():
    from paper_1010_2627_amd import mlp
    rng = np.random.Generator(np.random.PCG64(7))
    Z = (rng.normal(size=(64, 300)) * 3).astype(np.float32)
    dY = rng.normal(size=(64, 300)).astype(np.float32)
    Zt, dYt = torch.from_numpy(Z).cuda(), torch.from_numpy(dY).cuda()
    Y = torch.empty((64, 300), dtype=torch.bfloat16, device="cuda")
    mlp.knit_mlp_act_fwd(Zt, Y, gelu=True)
    assert _ulp_close(Y, OM.gelu(Z.astype(np.float64)))
    mlp.knit_mlp_act_fwd(Zt, Y, gelu=False)
    assert np.array_equal(Y.float().cpu().numpy(), OM.bf16_round(Z))
    dZ = torch.empty_like(Y)
    mlp.knit_mlp_gelu_bwd(dYt, Zt, dZ)
    assert _ulp_close(dZ, dY.astype(np.float64) * OM.gelu_grad(Z.astype(np.float64)))
    q = rng.random(size=(64, 300)).astype(np.float32)
    q /= q.sum(axis=1, keepdims=True)
    loss = torch.empty(64, dtype=torch.float32, device="cuda")
    probs = torch.empty((64, 300), dtype=torch.float32, device="cuda")
    dl = torch.empty((64, 300), dtype=torch.bfloat16, device="cuda")
    mlp.knit_mlp_softmax_xent(Zt, torch.from_numpy(q).cuda(), 1.0 / 64, loss=loss, probs=probs, dlogits=dl)
    p = OM.softmax(Z.astype(np.float64))
    assert np.allclose(probs.cpu().numpy(), p, rtol=1e-5, atol=1e-7)
    ref_loss = -(q * np.log(p)).sum(axis=1)
    assert np.allclose(loss.cpu().numpy(), ref_loss, rtol=1e-5)
    assert _ulp_close(dl, (p - q) / 64)
    cs = torch.empty(300, dtype=torch.float32, device="cuda")
    mlp.knit_mlp_colsum(dl, cs)
    assert np.allclose(cs.cpu().numpy(), dl.float().cpu().numpy().astype(np.float64).sum(axis=0), rtol=1e-5,
                       atol=1e-7)


@gpu
def test_network_gradients_match_reference():
    from paper_1010_2627_amd import mlp, sampler as S
    net = mlp.Network(S.SIZES, seed=3)
    rng = np.random.Generator(np.random.PCG64(9))
    x = rng.normal(size=(96, S.N_FEATURES)).astype(np.float32)
    q = rng.random(size=(96, S.N_BINS)).astype(np.float32) ** 4
    q /= q.sum(axis=1, keepdims=True)
    loss, grads = net.loss_and_grads(torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
    params = net.params_numpy()
    logits, cache = OM.forward(params, x)
    ref = OM.backward(params, cache, q)
    assert abs(float(loss.mean().cpu()) - OM.xent_loss(logits.astype(np.float64), q)) < 1e-3
    for li, ((dW, db), (rW, rb)) in enumerate(zip(grads, ref)):
        for got, want in ((dW.cpu().numpy(), rW), (db.cpu().numpy(), rb)):
            g, w = got.ravel().astype(np.float64), want.ravel().astype(np.float64)
            cos = g @ w / (np.linalg.norm(g) * np.linalg.norm(w))
            rel = np.linalg.norm(g - w) / np.linalg.norm(w)
            assert cos >= 0.999 and rel <= 1e-2, (li, cos, rel)


@gpu
def test_adamw_kernel_matches_reference():
    from paper_1010_2627_amd import mlp
    rng = np.random.Generator(np.random.PCG64(11))
    w0 = rng.normal(size=1000).astype(np.float32)
    w = torch.from_numpy(w0.copy()).cuda()
    w16 = torch.empty(1000, dtype=torch.bfloat16, device="cuda")
    m, v = torch.zeros_like(w), torch.zeros_like(w)
    wr, mr, vr = w0.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for t in range(1, 6):
        g = rng.normal(size=1000).astype(np.float32)
        mlp.knit_mlp_adamw(w, w16, torch.from_numpy(g).cuda(), m, v, 1e-2, 0.9, 0.999, 1e-8, 0.01, t)
        wr, mr, vr = OM.adamw(wr, g.astype(np.float64), mr, vr, t, 1e-2, 0.9, 0.999, 1e-8, 0.01)
    assert np.allclose(w.cpu().numpy(), wr, rtol=1e-5, atol=1e-6)
    assert np.array_equal(w16.float().cpu().numpy(), OM.bf16_round(w.cpu().numpy()))


def _trained(n_curves=1024, steps=1500):
    from paper_1010_2627_amd import mlp, sampler as S
    X, Q, _ = S.generate_training_set(n_curves)
    net = mlp.Network(S.SIZES, seed=1)
    hist = S.train(net, X, Q, steps=steps, batch=256, lr=1e-3, log_every=250)
    return net, hist, X, Q


@gpu
def test_sampler_trains_and_beats_uniform_points():
    """Train on generated curves (own kernels; targets: where the 256-point trapezoid rule
    leaves its error), then place 256 energies on 64 held-out ribbons and compare the
    integrated-conductance error against the 4096-point grid with 256 uniform points (the
    method without the network).  The network must learn (KL to the targets falls), never
    fall back, and its mean error must be below the uniform points' mean error."""
    from paper_1010_2627_amd import sampler as S
    net, hist, X, Q = _trained()
    # cross-entropy = H(q) + KL(q || p): only the KL part can be learned
    H = float(np.mean(-(Q * np.log(np.maximum(Q, 1e-30))).sum(axis=1)))
    kl0, kl1 = hist[0][1] - H, hist[-1][1] - H
    print(f"\nloss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}, target entropy {H:.4f}, KL {kl0:.4f} -> {kl1:.4f}")
    assert kl1 < 0.7 * kl0, hist
    test = S.train_ribbons(64, start=100000)       # held out: seeds beyond the training range
    rows = S.evaluate(net, test)
    eu = np.array([r["err_uniform"] for r in rows])
    el = np.array([r["err_learned"] for r in rows])
    et = np.array([r["err_threshold"] for r in rows])
    print(f"integrated-conductance error: uniform {eu.mean():.3e}, learned {el.mean():.3e} "
          f"(gain {eu.mean() / el.mean():.2f}x, wins {int((el < eu).sum())}/{len(el)}), "
          f"threshold-aware {et.mean():.3e} (gain {eu.mean() / et.mean():.2f}x)")
    assert not any(r["fallback"] for r in rows)
    assert np.all(np.isfinite(el)) and el.mean() < eu.mean()
