"""Brute force: one dense inverse of the whole finite system (oracle, FP64).

Test infrastructure only.  This is the plain definition the slice recursion
must reproduce: the retarded Green function of the finite system with the
leads integrated out as self-energies on the interface sites,
G = (E - H - sum_l Sigma_l)^{-1} (section 2.3, Eq. (2), with the sign reading
stated in ``oracle.leads``), and from it the transmission between two leads
T_kl = Tr[Gamma_k G_kl Gamma_l G_kl^dagger] (section 2.3) and the local
density of states -Im G_ii / pi.
"""

from __future__ import annotations

import numpy as np

from .leads import gamma_of


def dense_strip_hamiltonian(H0, V, onsite) -> np.ndarray:
    """Full [L*M, L*M] Hamiltonian of a strip: H_n on the diagonal, V below, V^dagger above."""
    L, W, no, _ = onsite.shape
    M = W * no
    H = np.zeros((L * M, L * M), dtype=np.complex128)
    for n in range(L):
        blk = H0.astype(np.complex128).copy()
        for s in range(W):
            blk[s * no:(s + 1) * no, s * no:(s + 1) * no] += onsite[n, s]
        H[n * M:(n + 1) * M, n * M:(n + 1) * M] = blk
        if n > 0:
            H[n * M:(n + 1) * M, (n - 1) * M:n * M] = V
            H[(n - 1) * M:n * M, n * M:(n + 1) * M] = V.conj().T
    return H


def dense_green(H: np.ndarray, E: float, sigmas) -> np.ndarray:
    """G = (E - H - sum_l Sigma_l)^{-1}; ``sigmas`` is a list of (site_indices, Sigma_l)."""
    N = H.shape[0]
    A = E * np.eye(N, dtype=np.complex128) - H
    for idx, s in sigmas:
        idx = np.asarray(idx)
        A[np.ix_(idx, idx)] -= s
    return np.linalg.inv(A)


def dense_transmission(G: np.ndarray, lead_k, lead_l) -> float:
    """T_kl = Re Tr[Gamma_k G_{kl} Gamma_l G_{kl}^dagger] between leads k and l.

    ``lead_k`` and ``lead_l`` are (site_indices, Sigma) pairs.  The paper's
    ``G_MATRIX[to, from]`` is T with k = to and l = from.
    """
    ik, sk = lead_k
    il, sl = lead_l
    Gkl = G[np.ix_(np.asarray(ik), np.asarray(il))]
    return float(np.real(np.trace(gamma_of(sk) @ Gkl @ gamma_of(sl) @ Gkl.conj().T)))


def dense_ldos(G: np.ndarray) -> np.ndarray:
    """-Im G_ii / pi for every orbital of the system."""
    return -np.imag(np.diagonal(G)) / np.pi
