"""CPU pins of the learned sampler's reference network and of the sampler's host logic.

The reference (oracle.mlp) is checked against what fixes it independently: torch's own
bfloat16 rounding, central finite differences of the exact (FP64, unrounded) network,
and torch.optim.AdamW.  Where the rounded network rounds is fixed by properties that
the stated rounding places imply (BF16-valued activations and one-row gradients,
invariance under moves inside a BF16 cell).  The sampler's placement and integration
rules are checked on inputs whose answer is known in closed form.
"""

import numpy as np
import pytest
import torch

from oracle import mlp as OM


def test_bf16_rounding_matches_torch():
    rng = np.random.Generator(np.random.PCG64(1))
    x = np.concatenate([rng.normal(size=4000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 4000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 65504.0, 1e-40, -0.0,
                                  np.inf, -np.inf, 3.3895314e38], np.float32)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = OM.bf16_round(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def _tiny(seed=0, sizes=(5, 7, 6, 4)):
    rng = np.random.Generator(np.random.PCG64(seed))
    params = [(rng.normal(size=(o, i)), rng.normal(size=o) * 0.1) for i, o in zip(sizes[:-1], sizes[1:])]
    x = rng.normal(size=(3, sizes[0]))
    q = rng.random(size=(3, sizes[-1]))
    q /= q.sum(axis=1, keepdims=True)
    return params, x, q


def test_backward_matches_finite_differences_fp64():
    params, x, q = _tiny()
    logits, cache = OM.forward(params, x, rounding=False)
    grads = OM.backward(params, cache, q)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            fd = np.zeros_like(arr)
            it = np.nditer(arr, flags=["multi_index"])
            for _ in it:
                i = it.multi_index
                old = arr[i]
                arr[i] = old + h
                lp = OM.xent_loss(OM.forward(params, x, rounding=False)[0], q)
                arr[i] = old - h
                lm = OM.xent_loss(OM.forward(params, x, rounding=False)[0], q)
                arr[i] = old
                fd[i] = (lp - lm) / (2 * h)
            assert np.linalg.norm(fd - g) <= 1e-6 * max(1.0, np.linalg.norm(fd)), (li, np.abs(fd - g).max())


def test_gelu_and_its_derivative():
    x = np.linspace(-6, 6, 2001)
    from math import erf, sqrt, pi, exp
    ref = np.array([0.5 * v * (1 + erf(v / sqrt(2))) for v in x])
    assert np.allclose(OM.gelu(x), ref, atol=1e-15)
    h = 1e-6
    assert np.allclose(OM.gelu_grad(x), (OM.gelu(x + h) - OM.gelu(x - h)) / (2 * h), atol=1e-8)
    assert OM.gelu(np.array([0.0]))[0] == 0.0 and abs(OM.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15


def test_adamw_matches_torch():
    rng = np.random.Generator(np.random.PCG64(2))
    w0 = rng.normal(size=50)
    gs = [rng.normal(size=50) for _ in range(5)]
    p = torch.nn.Parameter(torch.from_numpy(w0.copy()))
    opt = torch.optim.AdamW([p], lr=3e-3, betas=(0.9, 0.99), eps=1e-8, weight_decay=0.05)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(gs, start=1):
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        w, m, v = OM.adamw(w, g, m, v, t, 3e-3, 0.9, 0.99, 1e-8, 0.05)
    assert np.allclose(w, p.detach().numpy(), rtol=0, atol=1e-14)


def test_rounded_network_stays_close_to_exact():
    """BF16 rounding at the stated boundaries perturbs, but does not change, the gradients."""
    params, x, q = _tiny(3, sizes=(16, 32, 32, 8))
    l64, c64 = OM.forward(params, x, rounding=False)
    l16, c16 = OM.forward([(W.astype(np.float32), b.astype(np.float32)) for W, b in params], x.astype(np.float32))
    assert np.abs(l16 - l64).max() < 0.02 * np.abs(l64).max()      # bf16 keeps 8 significant bits
    g64, g16 = OM.backward(params, c64, q), OM.backward(params, c16, q.astype(np.float32))
    for (a, _), (b, _) in zip(g64, g16):
        cos = float((a * b).sum() / np.linalg.norm(a) / np.linalg.norm(b))
        assert cos > 0.99


def _bf16_exact(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return bool(np.all((a.view(np.uint32) & 0xFFFF) == 0))


def _inside_cell(rng, a):
    """A float32 array that rounds to the same BF16 values as a (a moved inside its cells)."""
    a = OM.bf16_round(np.asarray(a, dtype=np.float32))
    step = np.abs(a) * 2.0 ** -9                       # a quarter of a BF16 ulp (ulp = 2^-7 |a| or more)
    return (a + step * rng.uniform(-1, 1, a.shape)).astype(np.float32)


def test_rounding_sits_where_stated_forward():
    """Where the forward pass rounds, fixed by properties rather than by retyping it:
    stored activations are BF16 values; moving x or W inside their BF16 cells leaves the
    logits bit for bit unchanged (so both are rounded before use); moving b inside its
    BF16 cell changes them (so the bias is not rounded), as does moving x to the next BF16
    value."""
    rng = np.random.Generator(np.random.PCG64(11))
    params, x, _ = _tiny(5, sizes=(16, 32, 32, 8))
    p32 = [(W.astype(np.float32), b.astype(np.float32)) for W, b in params]
    x32 = x.astype(np.float32)
    logits, cache = OM.forward(p32, x32)
    assert all(_bf16_exact(X) for X in cache["X"])
    assert not _bf16_exact(cache["Z"][0])               # pre-activations are not rounded
    l2, _ = OM.forward(p32, _inside_cell(rng, x32))
    assert np.array_equal(l2, logits)
    l3, _ = OM.forward([(_inside_cell(rng, W), b) for W, b in p32], x32)
    assert np.array_equal(l3, logits)
    pc = [(W, OM.bf16_round(b)) for W, b in p32]            # biases at BF16 values, then moved
    pb = [(W, (b * np.float32(1.0 + 2.0 ** -12)).astype(np.float32)) for W, b in pc]   # inside their cells
    assert not np.array_equal(OM.forward(pb, x32)[0], OM.forward(pc, x32)[0])
    xn = OM.bf16_round(x32)
    xn[0, 0] = np.nextafter(xn[0, 0], np.float32(np.inf))
    xn = OM.bf16_round(xn + np.sign(xn) * np.abs(xn) * np.float32(2.0 ** -7))
    assert not np.array_equal(OM.forward(p32, xn)[0], logits)


def test_rounding_sits_where_stated_backward():
    """Where the backward pass rounds, from the structure of one-row gradients: with a batch
    of one, db_l is dZ_l and dW_l the outer product dZ_l X_{l-1}, so db_l must be BF16
    values (rounded after the GELU derivative is applied, not before) and dW_l their exact
    products with the stored activations (a BF16 x BF16 product is exact in FP32); and
    moving W inside its BF16 cells leaves every gradient bit for bit
    unchanged (the backward uses the rounded weights)."""
    rng = np.random.Generator(np.random.PCG64(12))
    params, x, q = _tiny(6, sizes=(16, 32, 32, 8))
    p32 = [(W.astype(np.float32), b.astype(np.float32)) for W, b in params]
    x1, q1 = x[:1].astype(np.float32), q[:1].astype(np.float32)
    _, cache = OM.forward(p32, x1)
    grads = OM.backward(p32, cache, q1)
    for li, (dW, db) in enumerate(grads):
        assert _bf16_exact(db), li
        assert np.array_equal(dW, np.outer(db, cache["X"][li]).astype(np.float32)), li
    pw = [(_inside_cell(rng, W), b) for W, b in p32]
    _, c2 = OM.forward(pw, x1)
    for (a, b), (c, d) in zip(grads, OM.backward(pw, c2, q1)):
        assert np.array_equal(a, c) and np.array_equal(b, d)


# ---------------------------------------------------------------- sampler host logic

def test_placement_of_a_uniform_density_completes_an_even_grid():
    """Three points between neighbouring probe energies: probe + placement is the evenly
    spaced 256-point grid away from the two end stretches."""
    from paper_1010_2627_amd import sampler as S
    E = S.place(np.full(S.N_BINS, 1.0 / S.N_BINS))
    assert len(E) == S.N_LEARNED and np.all(np.diff(E) > 0)
    allE = np.sort(np.concatenate([S.midpoints(S.N_PROBE), E]))
    step = (S.EMAX - S.EMIN) / S.N_TOTAL
    inner = (allE > S.midpoints(S.N_PROBE)[0] - 1e-12) & (allE < S.midpoints(S.N_PROBE)[-1] + 1e-12)
    assert np.allclose(np.diff(allE[inner]), step, atol=1.1e-3)   # points move off E = 0, +-1 by 1e-3
    assert np.all((E > S.EMIN) & (E < S.EMAX))


def test_placement_follows_the_density():
    from paper_1010_2627_amd import sampler as S
    p = np.zeros(S.N_BINS)
    p[100] = 1.0
    E = S.place(p)
    # bin 100 lies between probe energies 12 and 13 (probe spacing is 8 bins, probe j at bin 8j + 4):
    # that interval receives 0.8 of the points plus its uniform share 0.2 * 8 / 512
    pr = S.midpoints(S.N_PROBE)
    inside = (E > pr[12]) & (E < pr[13])
    assert abs(inside.sum() - (0.8 + 0.2 * 8 / S.N_BINS) * S.N_LEARNED) <= 1
    assert np.allclose(np.diff(E[inside]), (pr[13] - pr[12]) / (inside.sum() + 1), atol=1e-12)
    # the square root of the density sets the shares: two bins with p 4:1 get points 2:1
    p = np.zeros(S.N_BINS)
    p[100], p[300] = 4.0, 1.0
    E = S.place(p, mix=1.0)
    a = ((E > pr[12]) & (E < pr[13])).sum()
    b = ((E > pr[37]) & (E < pr[38])).sum()
    assert a + b == S.N_LEARNED and abs(a - 2 * b) <= 1
    assert S.place(np.full(S.N_BINS, np.nan)) is None        # unusable density -> caller falls back
    assert S.place(-np.ones(S.N_BINS)) is None
    assert np.all(np.abs(S.place(np.eye(S.N_BINS)[256])) >= 1e-3)   # never on the zigzag flat band
    E = S.place(np.full(S.N_BINS, 1.0 / S.N_BINS))
    assert np.all(np.abs(np.abs(E) - 1.0) >= 1e-3)                  # nor on the zigzag lead's E = +-t


def test_trapezoid_is_exact_for_piecewise_linear_functions():
    from paper_1010_2627_amd import sampler as S
    rng = np.random.Generator(np.random.PCG64(4))
    E = np.concatenate([[S.EMIN, S.EMAX], rng.uniform(S.EMIN, S.EMAX, 50)])
    assert abs(S.integrate(E, 2.0 * E + 1.0) - 6.0) < 1e-12      # int_{-3}^{3} (2E+1) dE = 6


def test_target_density_is_flat_for_linear_and_peaks_at_a_kink():
    """The trapezoid rule is exact on a line (flat target); a kink puts the error, and the
    target's peak, in the interval of the 256-point rule that holds it."""
    from paper_1010_2627_amd import sampler as S
    E = S.midpoints(S.N_DENSE)
    q = S.target_density(3.0 * E + 2.0)
    assert np.allclose(q, 1.0 / S.N_BINS, rtol=1e-6)
    kink = 0.51
    q = S.target_density(np.abs(E - kink))
    k = int((kink - S.EMIN) / (S.EMAX - S.EMIN) * S.N_BINS)
    assert q.argmax() in (k - 1, k, k + 1) and q.max() > 100 * np.median(q)


def test_target_density_is_the_squared_interval_error():
    """Pinned by hand: a parabola's trapezoid error on an interval of width h is -h^3 T''/12
    exactly, the same for every interval, so the target is flat; a bump confined to one
    interval of the 256-point rule gives that interval's two bins all the mass above the floor."""
    from paper_1010_2627_amd import sampler as S
    E = S.midpoints(S.N_DENSE)
    q = S.target_density(E ** 2)
    assert np.allclose(q, 1.0 / S.N_BINS, rtol=1e-3)
    T = np.zeros(S.N_DENSE)
    T[16 * 100 + 8 + 4: 16 * 100 + 8 + 12] = 1.0     # inside the interval between rule points 100 and 101
    q = S.target_density(T)
    top = np.sort(np.argsort(q)[-2:])
    assert list(top) == [200 + 1, 200 + 2] or list(top) == [201, 202]
    assert q[top].sum() > 0.9
