"""Pins of the oracle's transmission eigenvalues and Fano factor (CPU only).

What fixes them independently of the oracle's own formula:
  * unitarity: every T_n lies in [0, 1];
  * a clean ribbon is a set of decoupled perfect channels: exactly N_open(E)
    eigenvalues equal 1 (N_open from the closed-form transverse modes), the rest
    0, and the Fano factor is 0;
  * sum_n T_n equals the Fisher-Lee trace (computed without square roots or
    eigenvalues);
  * one channel with a single impurity of strength u on a chain with hopping 1
    transmits (2 sin k)^2 / ((2 sin k)^2 + u^2) at E = 2 cos k, so T_1 is that
    and F = 1 - T_1;
  * the slice recursion and the dense inverse of the whole system give the same
    eigenvalues;
  * the matrix square root squares back to its argument.
"""

import numpy as np
import pytest

from oracle import dense as OD
from oracle import leads as OL
from oracle import noise as ON
from oracle import rgf as OR
from paper_1010_2627_amd import inputs


def _sig(st, E):
    V = st.V_dense()
    return (np.stack([OL.sigma_modes(st.H0, V, e, "L") for e in E]),
            np.stack([OL.sigma_modes(st.H0, V, e, "R") for e in E]))


def test_psd_sqrt_squares_back():
    rng = np.random.Generator(np.random.PCG64(3))
    B = rng.normal(size=(7, 4)) + 1j * rng.normal(size=(7, 4))
    A = B @ B.conj().T                       # rank 4, positive semidefinite
    S = ON.psd_sqrt(A)
    assert np.max(np.abs(S @ S - A)) < 1e-12 * np.abs(A).max()
    assert np.max(np.abs(S - S.conj().T)) < 1e-13
    assert np.linalg.eigvalsh(S).min() > -1e-12


@pytest.mark.parametrize("W", [5, 8])
def test_clean_ribbon_eigenvalues_are_open_channels(W):
    st = inputs.square_strip(W)
    E = inputs.midpoint_grid(-3.7, 3.7, 9)
    sL, sR = _sig(st, E)
    r = OR.rgf_forward(st.H0, st.V_dense(), inputs.clean_onsite(st, 4), E, sL, sR)
    Tn = ON.transmission_eigenvalues(sL, sR, r["GN1"])
    nopen = OL.n_open_square(W, E)
    for i in range(len(E)):
        k = int(nopen[i])
        assert np.max(np.abs(Tn[i, :k] - 1.0), initial=0.0) < 1e-10, (E[i], Tn[i])
        assert np.max(np.abs(Tn[i, k:]), initial=0.0) < 1e-10
    F = ON.fano_factor(Tn)
    assert np.all(np.abs(F[nopen > 0]) < 1e-9)
    assert np.all(np.isnan(F[nopen == 0]))


@pytest.mark.parametrize("kind", ["square", "rashba", "zigzag"])
def test_eigenvalues_sum_to_fisher_lee_and_lie_in_unit_interval(kind):
    st = {"square": lambda: inputs.square_strip(6), "rashba": lambda: inputs.rashba_strip(4),
          "zigzag": lambda: inputs.zigzag_strip(5)}[kind]()
    on = inputs.onsite_disorder(st, 9, 2.0, 41)
    E = np.array([-1.85, -0.4, 0.75, 1.6])
    sL, sR = _sig(st, E)
    r = OR.rgf_forward(st.H0, st.V_dense(), on, E, sL, sR)
    Tn = ON.transmission_eigenvalues(sL, sR, r["GN1"])
    T = OR.transmission_lr(sL, sR, r["G1N"])
    assert np.max(np.abs(Tn.sum(axis=1) - T)) < 1e-10
    assert Tn.min() > -1e-12 and Tn.max() < 1 + 1e-12
    # not all channels perfect or closed: the disorder mixes them
    assert np.any((Tn > 1e-3) & (Tn < 1 - 1e-3))


@pytest.mark.parametrize("u", [0.3, 1.0, 2.5])
def test_single_impurity_chain_closed_form(u):
    st = inputs.square_strip(1)
    on = inputs.clean_onsite(st, 3)
    on[1, 0, 0, 0] = u
    E = np.array([-1.3, 0.2, 1.7])
    k = np.arccos(E / 2.0)
    expect = (2 * np.sin(k)) ** 2 / ((2 * np.sin(k)) ** 2 + u ** 2)
    sL, sR = _sig(st, E)
    r = OR.rgf_forward(st.H0, st.V_dense(), on, E, sL, sR)
    Tn = ON.transmission_eigenvalues(sL, sR, r["GN1"])
    assert np.max(np.abs(Tn[:, 0] - expect)) < 1e-12
    assert np.max(np.abs(ON.fano_factor(Tn) - (1.0 - expect))) < 1e-12


def test_recursion_and_dense_inverse_give_the_same_eigenvalues():
    st = inputs.rashba_strip(3)
    L = 5
    on = inputs.onsite_disorder(st, L, 1.7, 8)
    E = np.array([-0.9, 1.25])
    sL, sR = _sig(st, E)
    r = OR.rgf_forward(st.H0, st.V_dense(), on, E, sL, sR)
    Tn = ON.transmission_eigenvalues(sL, sR, r["GN1"])
    H = OD.dense_strip_hamiltonian(st.H0, st.V_dense(), on)
    M = st.M
    left, right = np.arange(M), np.arange((L - 1) * M, L * M)
    for i, e in enumerate(E):
        G = OD.dense_green(H, e, [(left, sL[i]), (right, sR[i])])
        GN1 = G[np.ix_(right, left)]
        ref = ON.transmission_eigenvalues(sL[i:i + 1], sR[i:i + 1], GN1[None])[0]
        assert np.max(np.abs(Tn[i] - ref)) < 1e-11
