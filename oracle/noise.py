"""Transmission eigenvalues and shot noise (oracle, FP64).  Test infrastructure only.

Section 2.1 item (a) lists the conductance and the shot noise among the
quantities the method yields from the retarded Green function between the
leads.  In the scattering description behind the Fisher-Lee formula of
section 2.3 the transmission amplitude matrix from lead L to lead R is, up to
unitary factors on each side that change no eigenvalue,

    t = Gamma_R^{1/2} G_{N1} Gamma_L^{1/2},

the transmission eigenvalues T_n are the eigenvalues of t t^dagger (each in
[0, 1] by unitarity of the scattering matrix), sum_n T_n is the Landauer
transmission, and the zero-temperature shot noise of a two-terminal conductor
relative to the Poisson value is the Fano factor

    F = sum_n T_n (1 - T_n) / sum_n T_n.

This module writes those definitions out directly: matrix square roots from
Hermitian eigendecompositions, one Hermitian eigenvalue problem per energy.
It takes G_{N1} from the slice recursion (``rgf.rgf_forward``) or the dense
inverse (``dense``); it shares no code with the GPU path.
"""

from __future__ import annotations

import numpy as np

from .leads import gamma_of


def psd_sqrt(A: np.ndarray) -> np.ndarray:
    """Hermitian square root of a positive semidefinite matrix (negative rounding noise in the
    spectrum clipped to zero)."""
    A = 0.5 * (A + A.conj().T)
    w, U = np.linalg.eigh(A)
    w = np.sqrt(np.clip(w, 0.0, None))
    return (U * w[None, :]) @ U.conj().T


def transmission_amplitude(sigma_L: np.ndarray, sigma_R: np.ndarray, GN1: np.ndarray) -> np.ndarray:
    """t = Gamma_R^{1/2} G_N1 Gamma_L^{1/2} for one problem ([M, M] each)."""
    return psd_sqrt(gamma_of(sigma_R)) @ GN1 @ psd_sqrt(gamma_of(sigma_L))


def transmission_eigenvalues(sigma_L: np.ndarray, sigma_R: np.ndarray, GN1: np.ndarray) -> np.ndarray:
    """Eigenvalues of t t^dagger, descending, for a stack of B problems ([B, M, M] each).
    Returns [B, M] (the M - rank trailing values are rounding noise around 0)."""
    out = []
    for sL, sR, g in zip(sigma_L, sigma_R, GN1):
        t = transmission_amplitude(sL, sR, g)
        out.append(np.sort(np.linalg.eigvalsh(t @ t.conj().T))[::-1])
    return np.array(out)


def fano_factor(Tn: np.ndarray) -> np.ndarray:
    """F = sum T_n (1 - T_n) / sum T_n along the last axis (NaN where sum T_n = 0)."""
    Tn = np.asarray(Tn, dtype=np.float64)
    s = Tn.sum(axis=-1)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(s > 0, (Tn * (1.0 - Tn)).sum(axis=-1) / np.where(s > 0, s, 1.0), np.nan)
