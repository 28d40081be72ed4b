"""Lesser Green function of injection from one lead and its local observables (oracle, FP64).

Test infrastructure only.  Section 2.3: with the distribution f_l of lead l,
G^< = sum_l f_l G_l^<, G_l^< = i G Gamma_l G^dagger, and one element of G_l^<
between sites i and j is i sum over the lead's sites of G_{i a} Gamma_{a b}
conj(G_{j b}).  Section 5.3-D (sewing) and section 6 use it for local
observables: the non-equilibrium particle density, the local current density
between neighbouring sites (section 6.1, Re of V_ji G^<_ij per bond) and the
spin accumulation (section 6.2, the sigma_z components of G^<_ii).

Everything here follows the plain definition: one dense inverse of the whole
finite strip, G = (E - H - Sigma_L - Sigma_R)^{-1}, then
A_l = -i G_l^< = G Gamma_l G^dagger (Hermitian, positive semidefinite), the
injected spectral function of lead l (f_l = 1 for that lead, 0 for the other).
From it, per energy and in units of e/h per unit energy:
  * on-site blocks A_l[n, s] (norb x norb) of every site s of every slice n:
    Tr A_l[n, s] / (2 pi) is the density injected from lead l, and the sigma
    components (e.g. A_00 - A_11) its spin;
  * the particle current into orbital block a of site s from site b,
    I_{b -> a} = 2 Im Tr[H_ab A_ba] (continuity equation of the density
    matrix with the Hermitian H), summed into
      J_long[n, s] = inflow into site s of slice n from slice n - 1 (n >= 1;
                     J_long[0] = 0),
      J_tran[n, s] = inflow into site s of slice n from the other sites of
                     slice n.
With f_l = 1 the current through every cross-section equals the Landauer
transmission T_{l -> other lead}.
"""

from __future__ import annotations

import numpy as np

from .leads import gamma_of


def strip_green_dense(V: np.ndarray, Hn: np.ndarray, E: float, sigma_L: np.ndarray, sigma_R: np.ndarray):
    """Full [L M, L M] retarded G of a strip from its slice Hamiltonians Hn [L, M, M] and the
    inter-slice hopping V = H_{n,n-1}, leads on slices 1 and L.  Returns (G, H)."""
    L, M, _ = Hn.shape
    N = L * M
    H = np.zeros((N, N), dtype=np.complex128)
    for n in range(L):
        H[n * M:(n + 1) * M, n * M:(n + 1) * M] = Hn[n]
        if n > 0:
            H[n * M:(n + 1) * M, (n - 1) * M:n * M] = V
            H[(n - 1) * M:n * M, n * M:(n + 1) * M] = V.conj().T
    A = E * np.eye(N, dtype=np.complex128) - H
    A[:M, :M] -= sigma_L
    A[N - M:, N - M:] -= sigma_R
    return np.linalg.inv(A), H


def injected_spectral(G: np.ndarray, M: int, sigma: np.ndarray, lead: str) -> np.ndarray:
    """A_l = G Gamma_l G^dagger for the lead on the first (lead "L") or last ("R") slice."""
    N = G.shape[0]
    idx = slice(0, M) if lead == "L" else slice(N - M, N)
    Gc = G[:, idx]
    return Gc @ gamma_of(sigma) @ Gc.conj().T


def local_observables(V: np.ndarray, Hn: np.ndarray, E: float, sigma_L: np.ndarray, sigma_R: np.ndarray,
                      norb: int, lead: str = "L"):
    """Local observables of injection from ``lead`` for one strip at one energy.

    Returns dict with
      onsite [L, W, norb, norb] complex : on-site blocks of A_lead,
      j_long [L, W] : current into each site from the previous slice (0 for slice 1),
      j_tran [L, W] : current into each site from the other sites of its slice,
      G, A : the dense Green function and injected spectral function.
    """
    L, M, _ = Hn.shape
    W = M // norb
    G, H = strip_green_dense(V, Hn, E, sigma_L, sigma_R)
    A = injected_spectral(G, M, sigma_L if lead == "L" else sigma_R, lead)
    onsite = np.zeros((L, W, norb, norb), dtype=np.complex128)
    j_long = np.zeros((L, W))
    j_tran = np.zeros((L, W))
    for n in range(L):
        for s in range(W):
            a = slice(n * M + s * norb, n * M + (s + 1) * norb)
            onsite[n, s] = A[a, a]
            # inflow from slice n-1 (all of its sites) and from the other sites of slice n
            if n > 0:
                b = slice((n - 1) * M, n * M)
                j_long[n, s] = 2.0 * np.imag(np.trace(H[a, b] @ A[b, a]))
            for s2 in range(W):
                if s2 == s:
                    continue
                b = slice(n * M + s2 * norb, n * M + (s2 + 1) * norb)
                j_tran[n, s] += 2.0 * np.imag(np.trace(H[a, b] @ A[b, a]))
    return {"onsite": onsite, "j_long": j_long, "j_tran": j_tran, "G": G, "A": A}
