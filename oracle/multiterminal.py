"""Conductance matrix of a strip with more than two leads (oracle, FP64).  Test infrastructure only.

Section 2.3 defines the transmission between any two leads k, l of a system
from the Green function between their interface sites,
    T_kl = Tr[Gamma_k G_kl Gamma_l G_kl^dagger],
with the conductance g_kl = (e^2 / h) T_kl (Landauer); section 6.1 computes the
conductance matrix of a three-lead system (KNIT's conductance_matrix, whose
entry [to, from] is T_kl with k = to and l = from).

Here the system is a strip of L slices with the left lead on slice 1, the
right lead on slice L and further leads attached to single slices: lead k
contributes its self-energy Sigma_k ([M, M], acting on the sites of slice
s_k).  Plain definition: one dense inverse of the whole strip with every
self-energy in place, then the formula above for every ordered pair (k, l),
k = l included (its row and column sums then agree: both equal
Tr[Gamma_k i (G_kk - G_kk^dagger)]).  Lead order: left, right, then the side
leads in the order given.
"""

from __future__ import annotations

import numpy as np

from .leads import gamma_of


def green_with_leads(V: np.ndarray, Hn: np.ndarray, E: float, leads):
    """Dense retarded G of the strip (slice Hamiltonians Hn [L, M, M], inter-slice hopping V)
    with ``leads`` = list of (slice index, Sigma [M, M]) attached."""
    L, M, _ = Hn.shape
    N = L * M
    A = E * np.eye(N, dtype=np.complex128)
    for n in range(L):
        A[n * M:(n + 1) * M, n * M:(n + 1) * M] -= Hn[n]
        if n > 0:
            A[n * M:(n + 1) * M, (n - 1) * M:n * M] -= V
            A[(n - 1) * M:n * M, n * M:(n + 1) * M] -= V.conj().T
    for s, sig in leads:
        A[s * M:(s + 1) * M, s * M:(s + 1) * M] -= sig
    return np.linalg.inv(A)


def conductance_matrix(V: np.ndarray, Hn: np.ndarray, E: float, sigma_L: np.ndarray, sigma_R: np.ndarray,
                       side=()) -> np.ndarray:
    """T[k, l] = Re Tr[Gamma_k G_{s_k s_l} Gamma_l G_{s_k s_l}^dagger] for the leads
    (left on slice 0, right on slice L-1, then ``side`` = [(slice, Sigma), ...])."""
    L, M, _ = Hn.shape
    leads = [(0, sigma_L), (L - 1, sigma_R)] + list(side)
    G = green_with_leads(V, Hn, E, leads)
    K = len(leads)
    T = np.zeros((K, K))
    for k, (sk, sgk) in enumerate(leads):
        for l, (sl, sgl) in enumerate(leads):
            Gkl = G[sk * M:(sk + 1) * M, sl * M:(sl + 1) * M]
            T[k, l] = np.real(np.trace(gamma_of(sgk) @ Gkl @ gamma_of(sgl) @ Gkl.conj().T))
    return T
