"""Pins of the oracle's conductance matrix with side leads (CPU only).

Fixed independently of the oracle's formula:
  * with no side lead it is the two-terminal Fisher-Lee T of the slice
    recursion (T_RL = T_LR);
  * a chain with a second chain attached at any slice is a three-way junction
    of identical chains: T_kl = 4 sin^2 k / (cos^2 k + 9 sin^2 k) at E = 2 cos k
    for every k != l, whatever the length and the slice (the interface slices
    belong to the leads);
  * row sums equal column sums (unitarity of the scattering matrix), and both
    equal Tr[Gamma_k i (G_kk - G_kk^dagger)], a formula without the second G;
  * a real Hamiltonian (no field, no spin-orbit coupling) gives T_kl = T_lk;
    the Rashba + Zeeman strip breaks that while keeping the sum rules.
"""

import numpy as np
import pytest

from oracle import leads as OL
from oracle import multiterminal as OM
from oracle import rgf as OR
from paper_1010_2627_amd import inputs


def _sig(st, E):
    V = st.V_dense()
    return OL.sigma_modes(st.H0, V, E, "L"), OL.sigma_modes(st.H0, V, E, "R")


def _probe(M, sites, E, t=1.0):
    """Self-energy of independent chains attached with hopping t to the given sites of a slice."""
    S = np.zeros((M, M), dtype=np.complex128)
    for j in sites:
        S[j, j] = t * t * OL.sigma_chain_closed_form(E)
    return S


def test_two_leads_reduce_to_fisher_lee():
    st = inputs.rashba_strip(3)
    on = inputs.onsite_disorder(st, 6, 2.0, 9)
    E = 0.7
    sL, sR = _sig(st, E)
    T = OM.conductance_matrix(st.V_dense(), OR.slice_hamiltonians(st.H0, on), E, sL, sR)
    ref = OR.transmission_lr(sL[None], sR[None], OR.rgf_forward(st.H0, st.V_dense(), on, np.array([E]), sL[None],
                                                                 sR[None])["G1N"])[0]
    assert abs(T[1, 0] - ref) < 1e-10 and abs(T[0, 1] - ref) < 1e-10


@pytest.mark.parametrize("L,s", [(1, 0), (5, 0), (5, 2), (7, 6)])
@pytest.mark.parametrize("E", [-1.3, 0.0, 0.9])
def test_chain_with_a_side_chain_is_a_y_junction(L, s, E):
    st = inputs.square_strip(1)
    sL, sR = _sig(st, E)
    Hn = OR.slice_hamiltonians(st.H0, inputs.clean_onsite(st, L))
    T = OM.conductance_matrix(st.V_dense(), Hn, E, sL, sR, [(s, _probe(1, [0], E))])
    k = np.arccos(E / 2)
    expect = 4 * np.sin(k) ** 2 / (np.cos(k) ** 2 + 9 * np.sin(k) ** 2)
    off = T[~np.eye(3, dtype=bool)]
    assert np.max(np.abs(off - expect)) < 1e-12


@pytest.mark.parametrize("kind", ["square", "rashba"])
def test_sum_rules_and_reciprocity(kind):
    st = inputs.square_strip(5) if kind == "square" else inputs.rashba_strip(3)
    L = 6
    on = inputs.onsite_disorder(st, L, 2.0, 31)
    Hn = OR.slice_hamiltonians(st.H0, on)
    V = st.V_dense()
    E = 0.55
    sL, sR = _sig(st, E)
    side = [(2, _probe(st.M, [0, 1], E, 0.8)), (4, _probe(st.M, [st.M - 1], E, 1.1)), (4, _probe(st.M, [2], E))]
    T = OM.conductance_matrix(V, Hn, E, sL, sR, side)
    assert np.max(np.abs(T.sum(axis=0) - T.sum(axis=1))) < 1e-10
    leads = [(0, sL), (L - 1, sR)] + side
    G = OM.green_with_leads(V, Hn, E, leads)
    M = st.M
    for k, (s, sg) in enumerate(leads):
        Gkk = G[s * M:(s + 1) * M, s * M:(s + 1) * M]
        ref = np.real(np.trace(OL.gamma_of(sg) @ (1j * (Gkk - Gkk.conj().T))))
        assert abs(T[k].sum() - ref) < 1e-10
    assert T.min() > -1e-12
    asym = np.max(np.abs(T - T.T))
    if kind == "square":
        assert asym < 1e-10
    else:
        assert asym > 1e-4
