"""Lead self-energies (oracle, FP64).  Test infrastructure only.

A lead is the semi-infinite repetition of a clean slice with intra-slice
Hamiltonian H0 and inter-slice hopping V = H_{n,n-1} (section 5.3-B: the lead
repeats its interface layer; the hopping from the lead into the system equals
the hopping inside the lead).  Its effect on the system is a self-energy on the
interface slice (section 2.3, Eq. (2) and item (3)).

Reading of the paper's Eq. (2): the retarded Green function is
G = (E - H - Sigma_L - Sigma_R)^{-1} with Im Sigma <= 0 (the printed
"+ i Sigma" is taken as a typesetting slip).  Gamma = i (Sigma - Sigma^dagger)
(the printed "Gamma = Im Sigma" would make a clean chain transmit 1/4).
"""

from __future__ import annotations

import numpy as np


def surface_gf_decimation(h: np.ndarray, alpha: np.ndarray, beta: np.ndarray, z: complex,
                          tol: float = 1e-15, max_iter: int = 200):
    """Surface Green function of a semi-infinite stack by decimation (renormalised doubling).

    The stack has identical layers with Hamiltonian ``h``; ``alpha`` couples
    the surface layer to the next layer into the bulk and ``beta`` the way
    back.  The surface Green function solves g = (z - h - alpha g beta)^{-1}.
    Decimation (Lopez Sancho, Lopez Sancho and Rubio, J. Phys. F 15, 851
    (1985)) eliminates every other layer at each step, so after k steps the
    effective couplings span 2^k layers; they decay for Im z > 0.

    Returns (g_surface, iterations, converged).
    """
    M = h.shape[0]
    I = np.eye(M, dtype=np.complex128)
    eps_s = h.astype(np.complex128).copy()     # renormalised surface layer
    eps = h.astype(np.complex128).copy()       # renormalised bulk layer
    a = alpha.astype(np.complex128).copy()     # effective coupling towards the bulk
    b = beta.astype(np.complex128).copy()      # effective coupling back to the surface
    scale = max(1.0, np.abs(h).max(), np.abs(alpha).max(), np.abs(beta).max())
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        g = np.linalg.inv(z * I - eps)
        agb = a @ g @ b
        bga = b @ g @ a
        eps_s = eps_s + agb
        eps = eps + agb + bga
        a = a @ g @ a
        b = b @ g @ b
        if max(np.abs(a).max(), np.abs(b).max()) < tol * scale:
            converged = True
            break
    return np.linalg.inv(z * I - eps_s), it, converged


def sigma_left(H0: np.ndarray, V: np.ndarray, E: float, eta: float = 1e-12, **kw):
    """Sigma_L = V g_L V^dagger on slice 1.

    The left lead occupies slices n <= 0; its surface slice 0 couples to the
    bulk slice -1 through H_{0,-1} = V, so g_L = (z - H0 - V g_L V^dagger)^{-1},
    and slice 1 couples to it through H_{1,0} = V.
    """
    g, it, ok = surface_gf_decimation(H0, V, V.conj().T, E + 1j * eta, **kw)
    return V @ g @ V.conj().T, it, ok


def sigma_right(H0: np.ndarray, V: np.ndarray, E: float, eta: float = 1e-12, **kw):
    """Sigma_R = V^dagger g_R V on slice N.

    The right lead occupies slices n >= N+1; its surface slice couples to the
    bulk through H_{N+1,N+2} = V^dagger, so g_R = (z - H0 - V^dagger g_R V)^{-1},
    and slice N couples to it through H_{N,N+1} = V^dagger.
    """
    g, it, ok = surface_gf_decimation(H0, V.conj().T, V, E + 1j * eta, **kw)
    return V.conj().T @ g @ V, it, ok


def sigma_chain_closed_form(x, t: float = 1.0):
    """Self-energy of a semi-infinite 1D chain (on-site 0, hopping t) at real energy x.

    t^2 g solves s^2 - x s + t^2 = 0; the retarded root is
    (x - i sqrt(4t^2 - x^2)) / 2 inside the band |x| < 2|t| and the decaying
    root (x - sign(x) sqrt(x^2 - 4t^2)) / 2 outside it.
    """
    x = np.asarray(x, dtype=np.float64)
    inside = np.abs(x) < 2 * abs(t)
    s_in = 0.5 * (x - 1j * np.sqrt(np.clip(4 * t * t - x * x, 0, None)))
    s_out = 0.5 * (x - np.sign(x) * np.sqrt(np.clip(x * x - 4 * t * t, 0, None)))
    return np.where(inside, s_in, s_out)


def square_modes(W: int, t: float = 1.0, onsite: float = 0.0):
    """Transverse eigenpairs of the scalar square-lattice slice (open boundaries).

    eps_k = onsite + 2 t cos(k pi / (W+1)), phi_k(y) = sqrt(2/(W+1)) sin(k pi y / (W+1)),
    k, y = 1..W.
    """
    k = np.arange(1, W + 1)
    y = np.arange(1, W + 1)
    eps = onsite + 2.0 * t * np.cos(k * np.pi / (W + 1))
    phi = np.sqrt(2.0 / (W + 1)) * np.sin(np.outer(y, k) * np.pi / (W + 1))   # [y, k]
    return eps, phi


def sigma_square_modal(W: int, E: float, t: float = 1.0, onsite: float = 0.0) -> np.ndarray:
    """Exact (eta = 0) self-energy of a scalar square-lattice lead of width W.

    V = t I commutes with H0, so the lead separates into W independent 1D
    chains, one per transverse mode k with on-site energy eps_k:
    Sigma = sum_k phi_k sigma_chain(E - eps_k) phi_k^T.  Left and right leads
    coincide.
    """
    eps, phi = square_modes(W, t, onsite)
    s = sigma_chain_closed_form(E - eps, t)
    return (phi * s[None, :]) @ phi.T


def n_open_square(W: int, E, t: float = 1.0, onsite: float = 0.0):
    """Number of propagating channels of a scalar square-lattice lead: #{k : |E - eps_k| < 2|t|}."""
    eps, _ = square_modes(W, t, onsite)
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    return (np.abs(E[:, None] - eps[None, :]) < 2 * abs(t)).sum(axis=1)


def gamma_of(sigma: np.ndarray) -> np.ndarray:
    """Broadening Gamma = i (Sigma - Sigma^dagger) (positive semidefinite for Im Sigma <= 0)."""
    return 1j * (sigma - sigma.conj().T)


def _select_modes(lam_num, lam_den, Y, V, side, tol_unit=1e-8, tol_deg=1e-7):
    """Pick the M Bloch modes that leave the system into the lead.

    Eigenpairs come from the pencil of the lead's wave equation (see
    ``sigma_modes``).  ``lam = lam_num / lam_den`` may be infinite.  Left lead:
    modes decaying towards -x (|lam| > 1, including lam = inf) or propagating
    with group velocity v < 0.  Right lead: |lam| < 1 (including 0) or v > 0.
    For |lam| = 1, v = -2 Im(phi^dag V^dag lam phi) / phi^dag phi (Hellmann-
    Feynman on E(k) of H0 + V e^{-ik} + V^dag e^{ik}); degenerate propagating
    modes are first rotated to diagonalise the velocity in their subspace.
    """
    M = V.shape[0]
    with np.errstate(divide="ignore", invalid="ignore"):
        absn, absd = np.abs(lam_num), np.abs(lam_den)
        unit = np.abs(absn - absd) <= tol_unit * np.maximum(absn, absd)
        lam = np.where(absd > 0, lam_num / np.where(absd > 0, lam_den, 1), np.inf)
    out_idx = []
    prop = np.where(unit)[0]
    nonprop = np.where(~unit)[0]
    for i in nonprop:
        outside = absn[i] > absd[i]               # |lam| > 1 (or infinite)
        if (side == "L" and outside) or (side == "R" and not outside):
            out_idx.append(("col", i))
    # propagating: cluster degenerate eigenvalues, diagonalise the velocity operator
    Vd = V.conj().T
    done = set()
    newcols = []
    for i in prop:
        if i in done:
            continue
        cl = [j for j in prop if j not in done and abs(lam[j] - lam[i]) < tol_deg]
        done.update(cl)
        l = lam[i] / abs(lam[i])
        Phi = Y[M:, cl]                            # psi_j components
        Vop = 1j * (Vd * l - V / l)                # Hermitian for |l| = 1
        Hv = Phi.conj().T @ Vop @ Phi
        S = Phi.conj().T @ Phi
        if len(cl) == 1:
            vel = np.real(Hv[0, 0] / S[0, 0])
            Yc = Y[:, cl]
            vels = [vel]
        else:
            import scipy.linalg as sla
            w, c = sla.eigh((Hv + Hv.conj().T) / 2, (S + S.conj().T) / 2)
            Yc = Y[:, cl] @ c
            vels = list(w)
        for k, vel in enumerate(vels):
            if (side == "L" and vel < 0) or (side == "R" and vel > 0):
                newcols.append(Yc[:, k])
    cols = [Y[:, i] for _, i in out_idx] + newcols
    if len(cols) != M:
        raise RuntimeError(f"mode selection found {len(cols)} outgoing modes, expected {M}")
    return np.stack(cols, axis=1)


def sigma_modes(H0: np.ndarray, V: np.ndarray, E: complex, side: str):
    """Exact lead self-energy from the lead's Bloch modes (second, independent method).

    The wave equation in the clean lead, (z - H0) psi_j - V psi_{j-1} - V^dag psi_{j+1} = 0,
    written for the pair y_j = (psi_{j-1}, psi_j), is the pencil
        [[0, I], [-V, z - H0]] y = lam [[I, 0], [0, V^dag]] y,
    whose eigenvalue lam is the Bloch factor psi_{j+1} = lam psi_j (it may be
    0 or infinite when V is singular).  With the M outgoing modes Y of the lead:
      left lead:  F = Y_top Y_bot^{-1} maps psi_j -> psi_{j-1};
                  g_L = (z - H0 - V F)^{-1},      Sigma_L = V g_L V^dag
      right lead: F = Y_bot Y_top^{-1} maps psi_{j-1} -> psi_j;
                  g_R = (z - H0 - V^dag F)^{-1},  Sigma_R = V^dag g_R V
    Works at real z (no broadening): propagating modes are split by the sign
    of their group velocity.
    """
    import scipy.linalg as sla
    M = H0.shape[0]
    I = np.eye(M, dtype=np.complex128)
    Z = np.zeros((M, M), dtype=np.complex128)
    zH = complex(E) * I - H0
    A = np.block([[Z, I], [-V, zH]])
    Bm = np.block([[I, Z], [Z, V.conj().T]])
    w, Y = sla.eig(A, Bm, homogeneous_eigvals=True)
    Y = Y / np.linalg.norm(Y, axis=0, keepdims=True)
    Ysel = _select_modes(w[0], w[1], Y, V, side)
    top, bot = Ysel[:M], Ysel[M:]
    if side == "L":
        F = np.linalg.solve(bot.T, top.T).T           # top @ inv(bot)
        g = np.linalg.inv(zH - V @ F)
        return V @ g @ V.conj().T
    F = np.linalg.solve(top.T, bot.T).T               # bot @ inv(top)
    g = np.linalg.inv(zH - V.conj().T @ F)
    return V.conj().T @ g @ V
