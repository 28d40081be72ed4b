"""Pins of the oracle's lesser-Green-function observables (CPU only).

Fixed independently of the oracle's own formulas:
  * the current through every cross-section between two slices equals the
    Landauer transmission from the injecting lead (Fisher-Lee trace of the slice
    recursion, a different formula);
  * per-site continuity in a steady state: inflow from the previous slice plus
    inflow from the own slice equals the outflow to the next slice;
  * A_L + A_R = i (G - G^dagger) on the diagonal, i.e. 2 pi times the LDOS of
    the backward sweep;
  * a clean chain injects the density A_L,nn = 1 / (2 sin k) at E = 2 cos k on
    every site, with unit current on every bond;
  * a Zeeman-split clean spinful strip carries the spin difference of two
    decoupled spin species: the injected sigma_z density equals the same
    quantity computed from two scalar strips shifted by -/+ E_Z.
"""

import numpy as np
import pytest

from oracle import leads as OL
from oracle import lesser as OX
from oracle import rgf as OR
from paper_1010_2627_amd import inputs


def _sig(st, E):
    V = st.V_dense()
    return OL.sigma_modes(st.H0, V, E, "L"), OL.sigma_modes(st.H0, V, E, "R")


@pytest.mark.parametrize("kind", ["square", "rashba", "zigzag", "nnn"])
def test_cross_section_current_is_transmission_and_sites_conserve(kind):
    st = {"square": lambda: inputs.square_strip(5), "rashba": lambda: inputs.rashba_strip(3),
          "zigzag": lambda: inputs.zigzag_strip(4), "nnn": lambda: inputs.square_nnn_strip(4, tp=0.3)}[kind]()
    L = 7
    on = inputs.onsite_disorder(st, L, 2.0, 23)
    Hn = OR.slice_hamiltonians(st.H0, on)
    V = st.V_dense()
    for E in (-1.3, 0.45, 1.9):
        sL, sR = _sig(st, E)
        ob = OX.local_observables(V, Hn, E, sL, sR, st.norb)
        T = OR.transmission_lr(sL[None], sR[None], OR.rgf_forward(st.H0, V, on, np.array([E]), sL[None],
                                                                 sR[None])["G1N"])[0]
        for n in range(1, L):
            assert abs(ob["j_long"][n].sum() - T) < 1e-10, (kind, E, n)
        if st.vcol is not None:
            # outflow of site b of slice n = inflow of the site of slice n+1 bonded to it (slice 1
            # also receives the current injected by the lead, which j_long does not hold)
            for n in range(1, L - 1):
                out = np.zeros(st.W)
                for a, b in enumerate(st.vcol):
                    if b >= 0:
                        out[b] += ob["j_long"][n + 1, a]
                assert np.max(np.abs(ob["j_long"][n] + ob["j_tran"][n] - out)) < 1e-10, (kind, E, n)
        assert abs(ob["j_tran"].sum()) < 1e-10        # transverse currents cancel within each slice


def test_injected_spectral_functions_add_up_to_the_ldos():
    st = inputs.rashba_strip(3)
    L = 6
    on = inputs.onsite_disorder(st, L, 1.5, 5)
    Hn = OR.slice_hamiltonians(st.H0, on)
    V = st.V_dense()
    E = 0.8
    sL, sR = _sig(st, E)
    aL = OX.local_observables(V, Hn, E, sL, sR, st.norb, "L")["onsite"]
    aR = OX.local_observables(V, Hn, E, sL, sR, st.norb, "R")["onsite"]
    diag = np.real(np.einsum("nsoo->nso", aL + aR)).reshape(L, st.M)
    ldos = OR.ldos_rgf(st.H0, V, on, np.array([E]), sL[None], sR[None])[0]
    assert np.max(np.abs(diag - 2 * np.pi * ldos)) < 1e-10


@pytest.mark.parametrize("E", [-1.5, 0.3, 1.1])
def test_clean_chain_injected_density_and_current(E):
    st = inputs.square_strip(1)
    L = 6
    k = np.arccos(E / 2.0)
    sL, sR = _sig(st, E)
    Hn = OR.slice_hamiltonians(st.H0, inputs.clean_onsite(st, L))
    ob = OX.local_observables(st.V_dense(), Hn, E, sL, sR, 1)
    assert np.max(np.abs(ob["onsite"][:, 0, 0, 0] - 1.0 / (2 * np.sin(k)))) < 1e-12
    assert np.max(np.abs(ob["j_long"][1:, 0] - 1.0)) < 1e-12
    assert np.max(np.abs(ob["j_tran"])) == 0.0


def test_zeeman_split_strip_spin_density_is_two_scalar_copies():
    W, L, ez, E = 4, 5, 0.1, 0.62
    sp = inputs.rashba_strip(W, alpha=0.0, ez=ez)
    on = inputs.onsite_disorder(sp, L, 1.2, 3)
    sL, sR = _sig(sp, E)
    ob = OX.local_observables(sp.V_dense(), OR.slice_hamiltonians(sp.H0, on), E, sL, sR, 2)
    sz = np.real(ob["onsite"][..., 0, 0] - ob["onsite"][..., 1, 1])
    sc = inputs.square_strip(W)
    on1 = on[:, :, 0:1, 0:1]
    dens = []
    for shift in (ez, -ez):              # spin up sits at +ez: a scalar strip at E - ez
        s1, s2 = _sig(sc, E - shift)
        o1 = OX.local_observables(sc.V_dense(), OR.slice_hamiltonians(sc.H0, on1), E - shift, s1, s2, 1)
        dens.append(np.real(o1["onsite"][..., 0, 0]))
    assert np.max(np.abs(sz - (dens[0] - dens[1]))) < 1e-10
