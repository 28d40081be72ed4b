"""Slice recursive Green function, Fisher-Lee transmission and LDOS (oracle, FP64).

Test infrastructure only.  Plain numpy; a stack of B independent problems is
carried along the leading axis so that energies can be batched through
``np.linalg.inv`` and ``np.matmul``; there is no other blocking or fusion.

Method (section 1: the basic recursive Green function algorithm starts at the
left electrode and adds the layers of the system one by one until it reaches
the right electrode; section 2.3 gives the objects it produces).  With slices
n = 1..N (N = L), slice Hamiltonians H_n, inter-slice hopping V = H_{n,n-1}
and the lead self-energies Sigma_L on slice 1 and Sigma_R on slice N (the
interface slices belong to both system and lead, section 5.3-B):

    g_1 = (E - H_1 - Sigma_L - [N = 1] Sigma_R)^{-1}
    g_n = (E - H_n - [n = N] Sigma_R - V g_{n-1} V^dagger)^{-1},     n = 2..N
    G_{1n} = G_{1,n-1} V^dagger g_n,   G_{n1} = g_n V G_{n-1,1},     G_{11} = g_1
    G_{NN} = g_N

g_n is the Green function of slices 1..n with the left lead attached; at
n = N it is the exact G_NN of the whole system.
"""

from __future__ import annotations

import numpy as np

from .leads import gamma_of


def slice_hamiltonians(H0: np.ndarray, onsite: np.ndarray) -> np.ndarray:
    """H_n = H0 + blockdiag(onsite[n]) for every slice; onsite is [..., L, W, norb, norb]."""
    *lead, L, W, no, _ = onsite.shape
    M = W * no
    H = np.broadcast_to(H0, tuple(lead) + (L, M, M)).astype(np.complex128).copy()
    for s in range(W):
        H[..., s * no:(s + 1) * no, s * no:(s + 1) * no] += onsite[..., s, :, :]
    return H


def _eye_stack(B: int, M: int) -> np.ndarray:
    return np.broadcast_to(np.eye(M, dtype=np.complex128), (B, M, M))


def rgf_forward(H0, V, onsite, E, sigma_L, sigma_R, keep_g: bool = False, Hn=None):
    """Left-to-right slice recursion for a stack of B problems.

    H0, V: [M, M]; onsite: [B, L, W, norb, norb] (or [L, W, norb, norb], shared);
    E: [B]; sigma_L, sigma_R: [B, M, M].  ``Hn`` ([B, L, M, M]) may be given
    instead of H0/onsite for slices that are not block-diagonal on site.
    Returns dict with G1N, GN1, GNN ([B, M, M]) and, if keep_g, the list of g_n.
    """
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    B = E.shape[0]
    M = V.shape[0]
    if Hn is None:
        if onsite.ndim == 4:
            onsite = np.broadcast_to(onsite, (B,) + onsite.shape)
        Hn = slice_hamiltonians(H0, onsite)          # [B, L, M, M]
    Hn = np.broadcast_to(Hn, (B,) + Hn.shape[-3:])
    L = Hn.shape[1]
    zI = E[:, None, None] * _eye_stack(B, M)
    Vd = V.conj().T
    gs = []
    g = None
    G1n = Gn1 = None
    for n in range(L):
        A = zI - Hn[:, n]
        if n == 0:
            A = A - sigma_L
        else:
            A = A - V @ g @ Vd
        if n == L - 1:
            A = A - sigma_R
        g = np.linalg.inv(A)
        if n == 0:
            G1n = g.copy()
            Gn1 = g.copy()
        else:
            G1n = G1n @ Vd @ g
            Gn1 = g @ V @ Gn1
        if keep_g:
            gs.append(g)
    out = {"G1N": G1n, "GN1": Gn1, "GNN": g}
    if keep_g:
        out["g"] = gs
    return out


def transmission_lr(sigma_L, sigma_R, G1N):
    """Fisher-Lee T_LR = Re Tr[Gamma_L G_1N Gamma_R G_1N^dagger] (section 2.3, T_kl)."""
    GL = np.stack([gamma_of(s) for s in sigma_L])
    GR = np.stack([gamma_of(s) for s in sigma_R])
    prod = GL @ G1N @ GR @ np.conj(np.swapaxes(G1N, -1, -2))
    return np.real(np.trace(prod, axis1=-2, axis2=-1))


def transmission_rl(sigma_L, sigma_R, GN1):
    """T_RL = Re Tr[Gamma_R G_N1 Gamma_L G_N1^dagger]."""
    GL = np.stack([gamma_of(s) for s in sigma_L])
    GR = np.stack([gamma_of(s) for s in sigma_R])
    prod = GR @ GN1 @ GL @ np.conj(np.swapaxes(GN1, -1, -2))
    return np.real(np.trace(prod, axis1=-2, axis2=-1))


def transmission_ward(sigma_R, GNN):
    """T from G_NN alone: Re{Tr[Gamma_R i(G_NN - G_NN^dagger)] - Tr[Gamma_R G_NN Gamma_R G_NN^dagger]}.

    Block (N, N) of the identity i(G - G^dagger) = G (Gamma_L + Gamma_R) G^dagger
    (no dissipation inside the system) gives
    Tr[Gamma_R i(G_NN - G_NN^dagger)] = T_RL + Tr[Gamma_R G_NN Gamma_R G_NN^dagger].
    """
    GR = np.stack([gamma_of(s) for s in sigma_R])
    GNNd = np.conj(np.swapaxes(GNN, -1, -2))
    a = np.trace(GR @ (1j * (GNN - GNNd)), axis1=-2, axis2=-1)
    b = np.trace(GR @ GNN @ GR @ GNNd, axis1=-2, axis2=-1)
    return np.real(a - b)


def transmission_full(H0, V, onsite, E, sigma_L, sigma_R):
    """Convenience: forward sweep then T_LR, T_RL and the Ward value."""
    r = rgf_forward(H0, V, onsite, E, sigma_L, sigma_R)
    return (transmission_lr(sigma_L, sigma_R, r["G1N"]),
            transmission_rl(sigma_L, sigma_R, r["GN1"]),
            transmission_ward(sigma_R, r["GNN"]))


def ldos_rgf(H0, V, onsite, E, sigma_L, sigma_R):
    """LDOS[b, n, i] = -Im (G_nn)_ii / pi from the backward sweep.

    Second half of the sewing idea of section 5.3-D: after the forward sweep
    has stored the left-connected g_n, the exact diagonal blocks follow from
    the right end back:
        G_NN = g_N,   G_nn = g_n + g_n V^dagger G_{n+1,n+1} V g_n,   n = N-1..1.
    """
    r = rgf_forward(H0, V, onsite, E, sigma_L, sigma_R, keep_g=True)
    gs = r["g"]
    L = len(gs)
    B, M, _ = gs[0].shape
    out = np.zeros((B, L, M), dtype=np.float64)
    Vd = V.conj().T
    Gnn = gs[-1]
    out[:, L - 1] = -np.imag(np.diagonal(Gnn, axis1=-2, axis2=-1)) / np.pi
    for n in range(L - 2, -1, -1):
        g = gs[n]
        Gnn = g + g @ Vd @ Gnn @ V @ g
        out[:, n] = -np.imag(np.diagonal(Gnn, axis1=-2, axis2=-1)) / np.pi
    return out
