"""Knitting several sites per step (section 1: a group of sites joins by the same
Dyson equation as one site, with the group's own block, internal hoppings
included) against the oracle's dense inverse.

Cases: groups of 2, 3 and 4 sites with one orbital, groups of 2 sites with two
orbitals (electron-hole blocks), a last group padded with decoupled orbitals,
three and four leads with flux and a hole, the interface in registers and in
the workgroup's slab, random graphs with one and two orbitals per site, and
the automatic choice (groups of 3 in slab mode).  T_kl and the lead block of G
agree with the oracle at 1e-10 relative to max(1, |x|), as site by site.
"""

import numpy as np
import pytest
import torch

from paper_1010_2627_amd import inputs
from test_gpu_graph import _check, _sides, _synthetic

pytestmark = pytest.mark.gpu
gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


@gpu
@pytest.mark.parametrize("block", [2, 0])
def test_blocked_rectangle_with_hole_and_flux_three_leads(block):
    Lx, Ly = 14, 10          # leads of 10, 10 and 12 sites: groups of 2 (automatic: 2)
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly, (5, 3, 8, 6)), flux=0.07)
    leads = _sides(g, Lx, Ly, ["left", "right", "top"])
    P = 6
    E = np.linspace(-2.7, 2.3, P)
    ons = inputs.graph_disorder(g, 1.5, seed=4)
    T1, _ = _check(g, leads, E, ons, _synthetic(leads, 1, P, 100))
    Tb, _ = _check(g, leads, E, ons, _synthetic(leads, 1, P, 100), block=block)
    assert np.abs(Tb - T1).max() < 1e-10 * max(1.0, np.abs(T1).max())


@gpu
@pytest.mark.parametrize("block", [2, 0])
def test_blocked_four_leads(block):
    Lx, Ly = 30, 24          # leads of 24, 24, 28, 28 sites (groups of 4 would couple more than 16 orbitals)
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly, (10, 8, 18, 15)), flux=0.03)
    leads = _sides(g, Lx, Ly, ["left", "right", "bottom", "top"])
    P = 4
    ons = np.stack([inputs.graph_disorder(g, 2.0, seed=s) for s in (1, 2)])
    _check(g, leads, np.linspace(-1.9, 1.7, P), ons, _synthetic(leads, 1, P, 200), block=block)


@gpu
def test_blocked_groups_of_three_with_a_padded_last_group():
    Lx, Ly = 9, 6            # 50 sites, leads of 6: 38 other sites, the last group of 3 holds 2
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly, (3, 2, 4, 3)), flux=0.11)
    leads = _sides(g, Lx, Ly, ["left", "right"])
    assert (g.N - 12) % 3 == 2
    P = 5
    _check(g, leads, np.linspace(-3.1, 2.9, P), inputs.graph_disorder(g, 1.2, seed=7), _synthetic(leads, 1, P, 500),
           block=3)


@gpu
def test_blocked_electron_hole_blocks_norb2():
    Lx, Ly = 10, 8
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly, (4, 2, 5, 4)), flux=0.05, kind="bdg",
                                    mu=0.4, delta=0.3)
    leads = _sides(g, Lx, Ly, ["left", "right"])
    P = 4
    _check(g, leads, np.linspace(-1.5, 1.5, P), inputs.graph_disorder(g, 0.8, seed=3), _synthetic(leads, 2, P, 400),
           block=2)


@gpu
@pytest.mark.parametrize("block", [4, 2])
def test_blocked_wide_interface_slab_mode(block):
    Lx, Ly = 12, 80
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly))
    leads = _sides(g, Lx, Ly, ["left", "right"])
    P = 3
    _check(g, leads, [-0.7, 0.3, 1.9], inputs.graph_disorder(g, 1.0, seed=9), _synthetic(leads, 1, P, 300),
           want_mode=2, block=block)


@gpu
def test_automatic_groups_of_three_in_slab_mode():
    Lx, Ly = 10, 81          # interface wider than 128: the automatic plan takes groups of 3
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly, (3, 30, 6, 50)), flux=0.02)
    leads = _sides(g, Lx, Ly, ["left", "right"])
    from paper_1010_2627_amd import graph as GR
    assert GR.plan_create(g.N, 1, g.row_ptr, g.col, leads, block=0).info()["block"] == 3
    P = 3
    T, _ = _check(g, leads, [-1.1, 0.4, 2.2], inputs.graph_disorder(g, 1.0, seed=13), _synthetic(leads, 1, P, 600),
                  want_mode=2, block=0)


@gpu
@pytest.mark.parametrize("m", [1, 2])
def test_blocked_random_graph(m):
    """A random connected graph with random hopping and on-site blocks, three leads of even
    size, groups of 2 sites (2 or 4 orbitals per group)."""
    from test_gpu_graph import _random_graph
    g, perm = _random_graph(40, m, seed=10 + m)
    leads = [[int(x) for x in perm[:4]], [int(x) for x in perm[-4:]], [int(x) for x in perm[18:20]]]
    P = 3
    _check(g, leads, [-0.5, 0.2, 1.1], g.onsite, _synthetic(leads, m, P, 700 + m), block=2)
