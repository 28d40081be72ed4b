"""Knitting of systems of any shape on the GPU against the oracle.

The GPU adds the sites one at a time (section 5.3-D) and keeps only the
interface; the oracle inverts the whole system with every lead's self-energy
in place (Eq. (2)) and takes T_kl = Tr[Gamma_k G_kl Gamma_l G_kl^+]
(section 2.3).  Cases: the worked example of section 2.2 (FIG. 3, against the
printed values), holes, magnetic flux (Peierls phases), electron-hole and
spin-orbit blocks (norb = 2), a random graph with norb = 3 and 4, three and
four leads, given and default orders, and the three storage modes (interface
dimension <= 64, <= 128, above).  T_kl and the lead block of G agree with the
oracle at 1e-10 relative to max(1, |x|).
"""

import os

import numpy as np
import pytest
import torch

from paper_1010_2627_amd import inputs

pytestmark = pytest.mark.gpu
gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-10


def _orb(sites, m):
    return np.array([s * m + o for s in sites for o in range(m)])


def _oracle(g, leads, E, onsite, sigmas):
    """T [K, K] and G on the lead sites from one dense inverse."""
    from oracle import dense as OD
    H = g.dense()
    m = g.norb
    for i in range(g.N):
        H[i * m:(i + 1) * m, i * m:(i + 1) * m] = onsite[i]
    idx = [_orb(l, m) for l in leads]
    G = OD.dense_green(H, E, [(idx[k], sigmas[k]) for k in range(len(leads))])
    K = len(leads)
    T = np.array([[OD.dense_transmission(G, (idx[k], sigmas[k]), (idx[l], sigmas[l])) for l in range(K)]
                  for k in range(K)])
    allidx = np.concatenate(idx)
    return T, G[np.ix_(allidx, allidx)]


def _check(g, leads, energies, onsites, sigmas, order=None, want_mode=None, block=None):
    from paper_1010_2627_amd import workload
    b = workload.GraphBatch(g, leads, energies, onsites, sigmas, order=order, block=block)
    if block is not None and block > 0:
        assert b.info["block"] == block
    if want_mode is not None:
        D = b.info["dim"]
        mode = 0 if D <= 64 else (1 if D <= 128 else 2)
        assert mode == want_mode, (D, want_mode)
    print(f"\ngraph N={g.N} norb={g.norb} leads={[len(l) for l in leads]} P={b.P} dim={b.info['dim']} "
          f"block={b.info['block']}", flush=True)
    T, GLL, st = b.run(want_gll=True)
    torch.cuda.synchronize()
    T, GLL, st = T.cpu().numpy(), GLL.cpu().numpy(), st.cpu().numpy()
    assert (st == 0).all(), st
    ld = b.info["lead_dim"]
    onsites = np.asarray(onsites).reshape(-1, g.N, g.norb, g.norb)
    worst = 0.0
    for p, E in enumerate(b.E):
        Tr, Gr = _oracle(g, leads, E, onsites[b.real_of[p]], [s[p] for s in sigmas])
        dT = np.abs(T[p] - Tr) / np.maximum(1.0, np.abs(Tr))
        Gp = GLL[p * ld * ld:(p + 1) * ld * ld].reshape(ld, ld)
        dG = np.abs(Gp - Gr) / np.maximum(1.0, np.abs(Gr))
        worst = max(worst, dT.max(), dG.max())
        assert dT.max() < TOL and dG.max() < TOL, (p, E, dT.max(), dG.max())
    return T, worst


def _sides(g, Lx, Ly, which):
    idx = {s: i for i, s in enumerate(g.coords)}
    out = []
    for w in which:
        if w == "left":
            out.append([idx[(0, y)] for y in range(Ly) if (0, y) in idx])
        elif w == "right":
            out.append([idx[(Lx - 1, y)] for y in range(Ly) if (Lx - 1, y) in idx])
        elif w == "bottom":
            out.append([idx[(x, 0)] for x in range(1, Lx - 1) if (x, 0) in idx])
        elif w == "top":
            out.append([idx[(x, Ly - 1)] for x in range(1, Lx - 1) if (x, Ly - 1) in idx])
    return out


def _synthetic(leads, m, P, seed):
    return [inputs.synthetic_sigma(len(l) * m, P, seed=seed + 17 * k, rank=max(1, len(l) * m // 2))
            for k, l in enumerate(leads)]


@gpu
def test_fig3_worked_example_against_printed_values():
    """Section 2.2, FIG. 3: the 41-site L-shape, its two leads from the modal self-energy."""
    from oracle import leads as OL
    sites = set()
    for x in range(8):
        for y in range(3, 7):
            sites.add((x, y))
    for x in range(5, 8):
        for y in range(0, 7):
            sites.add((x, y))
    sites = sorted(sites)
    g = inputs.square_lattice_graph(sites, t=-1.0)      # H_ij = +1, the example's convention
    idx = {s: i for i, s in enumerate(sites)}
    lead1 = [idx[(0, y)] for y in range(3, 7)]
    lead2 = [idx[(x, 0)] for x in range(5, 8)]
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fig3_lshape.txt")) if l.strip() and not l.startswith("#")]
    gold = np.array([[float(a), float(b)] for a, b in rows])
    E = gold[:, 0]
    s1 = [OL.sigma_square_modal(4, e) for e in E]
    s2 = [OL.sigma_square_modal(3, e) for e in E]
    T, _ = _check(g, [lead1, lead2], E, g.onsite, [s1, s2])
    assert np.abs(T[:, 1, 0] - gold[:, 1]).max() < 2e-11
    assert np.abs(T[:, 0, 1] - gold[:, 1]).max() < 2e-11


@gpu
def test_rectangle_with_hole_and_flux_three_leads():
    Lx, Ly = 14, 10
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly, (5, 3, 8, 6)), flux=0.07)
    leads = _sides(g, Lx, Ly, ["left", "right", "top"])
    P = 6
    E = np.linspace(-2.7, 2.3, P)
    ons = inputs.graph_disorder(g, 1.5, seed=4)
    _check(g, leads, E, ons, _synthetic(leads, 1, P, 100), want_mode=0)


@gpu
def test_four_leads_register_mode_128():
    Lx, Ly = 30, 24
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly, (10, 8, 18, 15)), flux=0.03)
    leads = _sides(g, Lx, Ly, ["left", "right", "bottom", "top"])
    P = 4
    ons = np.stack([inputs.graph_disorder(g, 2.0, seed=s) for s in (1, 2)])
    _check(g, leads, np.linspace(-1.9, 1.7, P), ons, _synthetic(leads, 1, P, 200), want_mode=1)


@gpu
def test_wide_interface_slab_mode():
    Lx, Ly = 12, 80
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly))
    leads = _sides(g, Lx, Ly, ["left", "right"])
    P = 3
    _check(g, leads, [-0.7, 0.3, 1.9], inputs.graph_disorder(g, 1.0, seed=9), _synthetic(leads, 1, P, 300),
           want_mode=2)


@gpu
def test_electron_hole_blocks_norb2():
    Lx, Ly = 10, 8
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly, (4, 2, 5, 4)), flux=0.05, kind="bdg",
                                    mu=0.4, delta=0.3)
    leads = _sides(g, Lx, Ly, ["left", "right"])
    P = 4
    _check(g, leads, np.linspace(-1.5, 1.5, P), inputs.graph_disorder(g, 0.8, seed=3), _synthetic(leads, 2, P, 400))


@gpu
def test_spin_orbit_blocks_norb2_slab_mode():
    Lx, Ly = 8, 40
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly), kind="rashba", alpha=0.3, ez=0.2)
    leads = _sides(g, Lx, Ly, ["left", "right", "top"])
    P = 2
    _check(g, leads, [-0.9, 0.6], inputs.graph_disorder(g, 1.0, seed=5), _synthetic(leads, 2, P, 500),
           want_mode=2)


def _random_graph(N, m, seed, extra=0.3):
    """A connected random graph of degree <= 4: a spanning path plus random extra bonds, random blocks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(N)
    bonds = {}
    deg = np.zeros(N, dtype=int)

    def blk():
        return (rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))) * 0.6

    for a, b in zip(perm[:-1], perm[1:]):
        bonds[(int(a), int(b))] = blk()
        deg[a] += 1
        deg[b] += 1
    for _ in range(int(extra * N)):
        a, b = rng.integers(0, N, 2)
        if a == b or deg[a] >= 4 or deg[b] >= 4 or (a, b) in bonds or (b, a) in bonds:
            continue
        bonds[(int(a), int(b))] = blk()
        deg[a] += 1
        deg[b] += 1
    ons = rng.normal(size=(N, m, m)) + 1j * rng.normal(size=(N, m, m))
    ons = 0.5 * (ons + np.conj(np.swapaxes(ons, 1, 2)))
    return inputs.graph_from_blocks(N, m, ons, bonds), perm


@pytest.mark.parametrize("m", [3, 4])
@gpu
def test_random_graph_many_orbitals(m):
    g, perm = _random_graph(40, m, seed=10 + m)
    leads = [[int(x) for x in perm[:3]], [int(x) for x in perm[-3:]], [int(x) for x in perm[18:20]]]
    P = 3
    _check(g, leads, [-0.5, 0.2, 1.1], g.onsite, _synthetic(leads, m, P, 600 + m))


@gpu
def test_given_orders_agree_with_default():
    """Reverse and random orders change the interface, not the result."""
    Lx, Ly = 9, 7
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly, (3, 2, 4, 3)), flux=0.11)
    leads = _sides(g, Lx, Ly, ["left", "right", "bottom"])
    P = 3
    E = [-1.1, 0.4, 2.2]
    ons = inputs.graph_disorder(g, 1.2, seed=6)
    sig = _synthetic(leads, 1, P, 700)
    T0, _ = _check(g, leads, E, ons, sig)
    rng = np.random.Generator(np.random.PCG64(77))
    for order in (np.arange(g.N)[::-1], rng.permutation(g.N)):
        T1, _ = _check(g, leads, E, ons, sig, order=order)
        assert np.abs(T1 - T0).max() < 1e-10


@gpu
def test_many_problems_grid_stride():
    """More problems than resident workgroups (1024): energies x realizations."""
    Lx, Ly = 6, 5
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly))
    leads = _sides(g, Lx, Ly, ["left", "right"])
    P = 1100
    E = inputs.midpoint_grid(-3.5, 3.5, P)
    ons = np.stack([inputs.graph_disorder(g, 1.0, seed=s) for s in range(5)])
    sig = _synthetic(leads, 1, P, 800)
    from paper_1010_2627_amd import workload
    b = workload.GraphBatch(g, leads, E, ons, sig)
    T, _, st = b.run()
    torch.cuda.synchronize()
    T, st = T.cpu().numpy(), st.cpu().numpy()
    assert (st == 0).all()
    for p in list(range(0, P, 97)) + [P - 1]:
        Tr, _ = _oracle(g, leads, E[p], ons[b.real_of[p]], [s[p] for s in sig])
        assert np.abs(T[p] - Tr).max() / max(1.0, np.abs(Tr).max()) < TOL, p


@gpu
def test_strip_agrees_with_slice_sweep():
    """A W x L rectangle with leads on its end columns is a strip: knitting and the
    slice recursion (both on the GPU) give the same T, and both match the oracle."""
    from paper_1010_2627_amd import knit as K, workload
    W, L = 12, 20
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(L, W), t=-1.0)   # sites (x, y), x along the strip
    idx = {s: i for i, s in enumerate(g.coords)}
    left = [idx[(0, y)] for y in range(W)]
    right = [idx[(L - 1, y)] for y in range(W)]
    st = inputs.square_strip(W)
    ons_strip = inputs.onsite_disorder(st, L, 1.3, seed=21)
    ons = np.zeros((g.N, 1, 1), dtype=np.complex128)
    for x in range(L):
        for y in range(W):
            ons[idx[(x, y)], 0, 0] = ons_strip[x, y, 0, 0]
    E = np.array([-1.3, 0.55])
    sL = inputs.synthetic_sigma(W, 2, seed=31, rank=6)
    sR = inputs.synthetic_sigma(W, 2, seed=32, rank=5)
    T, _ = _check(g, [left, right], E, ons, [sL, sR])
    b = workload.Batch([st], [workload.Realization(0, ons_strip)], [E], "cuda")
    b.sigmaL = torch.from_numpy(sL).cuda()
    b.sigmaR = torch.from_numpy(sR).cuda()
    G1N, _, _, status = b.sweep("fp64", gnn=False)
    Ts = b.transmission(G1N)[0].cpu().numpy()
    assert np.abs(Ts - T[:, 1, 0]).max() < 1e-10, (Ts, T[:, 1, 0])


@gpu
def test_single_lead_and_lead_covering_everything():
    """Degenerate plans: one lead (T_00 only), and a lead holding every site (no knitting
    step: G is lead 0's block inverse alone)."""
    Lx, Ly = 7, 5
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly), flux=0.13)
    left = _sides(g, Lx, Ly, ["left"])
    ons = inputs.graph_disorder(g, 1.4, seed=12)
    _check(g, left, [-1.2, 0.9], ons, _synthetic(left, 1, 2, 900))
    every = [list(range(g.N))]
    sig = [inputs.synthetic_sigma(g.N, 2, seed=901, rank=8)]
    _check(g, every, [-0.4, 1.6], ons, sig)


@gpu
def test_mode_boundaries_and_a_detached_cluster():
    """Interface dimensions 64 and 65 (the two register modes' edge) and 128 / 129 (register
    and slab mode), plus a small cluster attached to no lead (a closed part: it must not
    disturb T)."""
    from paper_1010_2627_amd import graph as GR
    for W, Lx, want in ((31, 9, 0), (32, 6, 1), (63, 4, 1), (64, 4, 2)):
        g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, W))
        leads = _sides(g, Lx, W, ["left", "right"])
        D = GR.plan_create(g.N, 1, g.row_ptr, g.col, leads).info()["dim"]
        mode = 0 if D <= 64 else (1 if D <= 128 else 2)
        assert mode == want, (W, D)
        _check(g, leads, [0.37], inputs.graph_disorder(g, 1.0, seed=W), _synthetic(leads, 1, 1, 1000 + W),
               want_mode=want)
    # detached 2 x 2 cluster beside a 6 x 4 sample
    sites = inputs.rectangle_with_hole(6, 4) + [(20, 0), (21, 0), (20, 1), (21, 1)]
    g = inputs.square_lattice_graph(sites)
    leads = _sides(g, 6, 4, ["left", "right"])
    _check(g, leads, [-0.83, 1.21], inputs.graph_disorder(g, 2.0, seed=77), _synthetic(leads, 1, 2, 1100))
