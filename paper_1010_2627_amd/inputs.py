"""Seeded synthetic inputs: tight-binding strips, on-site disorder, energy grids.

This module only *builds* the Hamiltonian data of a two-lead strip (the input
of the method); it contains none of the transport arithmetic (no self-energy,
no Green function, no trace).  Both the GPU path and the CPU oracle take their
inputs from here and from nowhere else.

Model (tight-binding Hamiltonian of the paper's Eq. (1), section 2.3): every
site carries ``norb`` internal degrees of freedom, the hopping between
neighbouring sites is an ``norb x norb`` matrix and each site has an
``norb x norb`` on-site matrix.  Hoppings use the paper's sign (+t, the
``scalarM(1.)`` of its first example, section 2.2).

Slicing.  A strip is a sequence of identical slices n = 1..L along the
transport direction.  Inside a slice the W sites are numbered along the
transverse direction and the slice-local index of orbital ``o`` of site ``s``
is ``s * norb + o`` (so a slice has dimension M = W * norb).  A strip class is
described by

* ``H0``   [M, M]  clean intra-slice Hamiltonian (hoppings inside the slice and
  any uniform on-site term such as a Zeeman field);
* ``vcol`` [W]     for every site ``a`` of slice n the site of slice n-1 it is
  bonded to, or -1 when it has no bond to the previous slice;
* ``vblk`` [W, norb, norb] the hopping block H_{n,n-1}(a, vcol[a]).

Each site has at most one bond to the previous slice in every lattice built
here (square lattice, spinful square lattice, brick-wall honeycomb), so the
inter-slice hopping V = H_{n,n-1} is a block-monomial matrix.  The leads are
semi-infinite repetitions of the clean slice (H0, V) (section 5.3-B: a lead
repeats its interface layer, and the lead-to-system hopping equals the
intra-lead one).  The per-slice on-site blocks ``onsite`` [L, W, norb, norb]
hold the disorder and are added to H0 on the system slices only.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SIGMA0 = np.eye(2, dtype=np.complex128)
SIGMAX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SIGMAY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SIGMAZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)

# Seed conventions for the synthetic workloads.
SEED_BASE = 10102627        # realization r uses SEED_BASE + r
SEED_UNEVEN_LAYOUT = 10102626  # draws (W, L, w) of the uneven batch
SEED_UNEVEN_STRIP = SEED_BASE + 1000  # strip p of the uneven batch uses this + p
SEED_SYNTHETIC_SIGMA = 10102628     # synthetic boundary self-energies of the full-size sweep checks


@dataclass
class Strip:
    """Clean strip class: slice Hamiltonian H0 and inter-slice coupling V.

    V is block-monomial (``vcol`` / ``vblk``) unless ``V`` holds a dense [M, M]
    inter-slice hopping (then ``vcol`` / ``vblk`` are None).  ``onsite_dense``
    strips take their per-slice on-site terms as full [L, M, M] matrices
    instead of site blocks [L, W, norb, norb]."""

    name: str
    W: int
    norb: int
    H0: np.ndarray            # [M, M] complex128
    vcol: np.ndarray | None   # [W] int32
    vblk: np.ndarray | None   # [W, norb, norb] complex128
    meta: dict = field(default_factory=dict)
    V: np.ndarray | None = None      # [M, M] complex128, dense inter-slice hopping
    onsite_dense: bool = False

    @property
    def M(self) -> int:
        return self.W * self.norb

    def onsite_shape(self, L: int) -> tuple:
        return (L, self.M, self.M) if self.onsite_dense else (L, self.W, self.norb, self.norb)

    def V_dense(self) -> np.ndarray:
        """Assemble V = H_{n,n-1} as a dense [M, M] matrix."""
        if self.V is not None:
            return self.V.copy()
        M, no = self.M, self.norb
        V = np.zeros((M, M), dtype=np.complex128)
        for a in range(self.W):
            c = int(self.vcol[a])
            if c >= 0:
                V[a * no:(a + 1) * no, c * no:(c + 1) * no] = self.vblk[a]
        return V


def _check(strip: Strip) -> Strip:
    M = strip.M
    assert strip.H0.shape == (M, M) and strip.H0.dtype == np.complex128
    assert np.allclose(strip.H0, strip.H0.conj().T), "H0 must be Hermitian"
    if strip.V is not None:
        assert strip.V.shape == (M, M) and strip.V.dtype == np.complex128
        return strip
    assert strip.vcol.shape == (strip.W,) and strip.vcol.dtype == np.int32
    assert strip.vblk.shape == (strip.W, strip.norb, strip.norb)
    used = strip.vcol[strip.vcol >= 0]
    assert len(np.unique(used)) == len(used), "each site of slice n-1 bonds at most once"
    return strip


def square_strip(W: int, t: float = 1.0, onsite: float = 0.0) -> Strip:
    """Scalar (norb=1) square-lattice strip of width W, nearest-neighbour hopping +t."""
    H0 = np.zeros((W, W), dtype=np.complex128)
    for y in range(W - 1):
        H0[y + 1, y] = t
        H0[y, y + 1] = t
    H0 += onsite * np.eye(W)
    vcol = np.arange(W, dtype=np.int32)
    vblk = np.full((W, 1, 1), t, dtype=np.complex128)
    return _check(Strip(f"square_W{W}", W, 1, H0, vcol, vblk, {"t": t}))


def rashba_strip(W: int, t: float = 1.0, alpha: float = 0.2, ez: float = 0.1) -> Strip:
    """Spinful (norb=2) square-lattice strip with lattice Rashba coupling and a Zeeman field.

    Hopping block from site i to its neighbour i+x (along the strip, i.e. the
    inter-slice V) is t*s0 + i*alpha*s_y; from i to i+y (inside a slice) it is
    t*s0 - i*alpha*s_x.  The Zeeman term ez*s_z (out of plane) sits on every
    site, leads included, so it is part of H0.
    """
    no = 2
    M = W * no
    hx = t * SIGMA0 + 1j * alpha * SIGMAY
    hy = t * SIGMA0 - 1j * alpha * SIGMAX
    H0 = np.zeros((M, M), dtype=np.complex128)
    for y in range(W):
        H0[y * no:(y + 1) * no, y * no:(y + 1) * no] = ez * SIGMAZ
    for y in range(W - 1):
        H0[(y + 1) * no:(y + 2) * no, y * no:(y + 1) * no] = hy
        H0[y * no:(y + 1) * no, (y + 1) * no:(y + 2) * no] = hy.conj().T
    vcol = np.arange(W, dtype=np.int32)
    vblk = np.broadcast_to(hx, (W, no, no)).astype(np.complex128).copy()
    return _check(Strip(f"rashba_W{W}", W, no, H0, vcol, vblk,
                        {"t": t, "alpha": alpha, "ez": ez}))


def zigzag_strip(Nz: int, t: float = 1.0) -> Strip:
    """Honeycomb zigzag ribbon as a brick-wall lattice, slice = 2 columns x Nz rows.

    Rows are the zigzag chains (they run along the strip); every site has a
    bond to its left and right neighbour in its row, and the vertical bond
    (x, y)-(x, y+1) exists iff x + y is even.  A slice holds columns x = 2n
    (local column 0) and x = 2n + 1 (local column 1); the slice-local index of
    (c, y) is c * Nz + y, so M = 2 Nz.  The inter-slice bonds join column 1 of
    slice n-1 to column 0 of slice n, row by row: V has rank Nz (singular).
    """
    M = 2 * Nz
    H0 = np.zeros((M, M), dtype=np.complex128)
    for y in range(Nz):
        a, b = y, Nz + y                   # (col0, y) -- (col1, y)
        H0[a, b] = H0[b, a] = t
    for c in range(2):
        for y in range(Nz - 1):
            if (c + y) % 2 == 0:
                a, b = c * Nz + y, c * Nz + y + 1
                H0[a, b] = H0[b, a] = t
    vcol = np.full(M, -1, dtype=np.int32)
    vcol[:Nz] = Nz + np.arange(Nz, dtype=np.int32)
    vblk = np.zeros((M, 1, 1), dtype=np.complex128)
    vblk[:Nz, 0, 0] = t
    return _check(Strip(f"zigzag_Nz{Nz}", M, 1, H0, vcol, vblk, {"t": t}))


def square_nnn_strip(W: int, t: float = 1.0, tp: float = 0.25) -> Strip:
    """Scalar square-lattice strip with next-nearest-neighbour hopping +tp along the
    diagonals.  Site y of slice n bonds to sites y-1, y, y+1 of slice n-1, so V =
    t I + tp (shift up + shift down) is tridiagonal: not block-monomial, a dense
    coupling for the library."""
    H0 = np.zeros((W, W), dtype=np.complex128)
    for y in range(W - 1):
        H0[y + 1, y] = H0[y, y + 1] = t
    V = t * np.eye(W, dtype=np.complex128)
    for y in range(W - 1):
        V[y + 1, y] = V[y, y + 1] = tp
    return _check(Strip(f"square_nnn_W{W}", W, 1, H0, None, None, {"t": t, "tp": tp}, V=V))


def random_unitary(M: int, seed: int) -> np.ndarray:
    """Seeded Haar-distributed unitary [M, M] (QR of a complex Gaussian matrix, phases fixed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Z = (rng.normal(size=(M, M)) + 1j * rng.normal(size=(M, M))) / np.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R)
    return Q * (d / np.abs(d))[None, :]


def rotated_strip(strip: Strip, U: np.ndarray) -> Strip:
    """The same strip written in another slice basis: H0 -> U H0 U^+, V -> U V U^+, the
    same unitary U on every slice and in both leads.  V becomes dense and so do the
    on-site terms (rotate them with rotated_onsite)."""
    Ud = U.conj().T
    H0 = U @ strip.H0 @ Ud
    H0 = 0.5 * (H0 + H0.conj().T)
    V = U @ strip.V_dense() @ Ud
    return _check(Strip(strip.name + "_rotated", strip.W, strip.norb, H0, None, None, dict(strip.meta), V=V,
                        onsite_dense=True))


def rotated_onsite(strip: Strip, onsite: np.ndarray, U: np.ndarray) -> np.ndarray:
    """On-site terms of ``strip`` (site blocks [L, W, norb, norb]) as full matrices in the
    rotated basis: [L, M, M] = U blockdiag(onsite[n]) U^+."""
    L = onsite.shape[0]
    M, no = strip.M, strip.norb
    out = np.zeros((L, M, M), dtype=np.complex128)
    for s_ in range(strip.W):
        out[:, s_ * no:(s_ + 1) * no, s_ * no:(s_ + 1) * no] = onsite[:, s_]
    return U[None] @ out @ U.conj().T[None]


def onsite_disorder(strip: Strip, L: int, w: float, seed: int) -> np.ndarray:
    """On-site blocks [L, W, norb, norb]: eps * identity with eps ~ U[-w/2, w/2].

    The scalar draw follows the paper's disorder recipe W*(random()-0.5)
    (section 5.3-A, "Introducing disorder"), drawn slice by slice then site by
    site from numpy's PCG64 generator (not bit-compatible with Python's
    ``random``).  Spinful strips get spin-independent disorder eps * s0.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = rng.uniform(-0.5 * w, 0.5 * w, size=(L, strip.W)) if w > 0 else np.zeros((L, strip.W))
    out = np.zeros((L, strip.W, strip.norb, strip.norb), dtype=np.complex128)
    for o in range(strip.norb):
        out[:, :, o, o] = eps
    return out


def clean_onsite(strip: Strip, L: int) -> np.ndarray:
    return np.zeros(strip.onsite_shape(L), dtype=np.complex128)


def synthetic_sigma(M: int, n: int, seed: int = SEED_SYNTHETIC_SIGMA, scale: float = 0.5,
                    rank: int | None = None) -> np.ndarray:
    """n seeded matrices [n, M, M] of the form S = H - i G / 2 with H Hermitian and G
    positive definite: valid retarded boundary terms for exercising the slice
    recursion at sizes where the leads' own self-energies are costly to obtain on
    a CPU (the recursion and the trace are defined for any such term).  With
    ``rank`` = r, G = scale * B B^+ / r for a Gaussian B of M x r instead: positive
    semidefinite of rank r, like a lead with r open channels."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n, M, M), dtype=np.complex128)
    for i in range(n):
        A = rng.normal(size=(M, M)) + 1j * rng.normal(size=(M, M))
        if rank is None:
            B = rng.normal(size=(M, M)) + 1j * rng.normal(size=(M, M))
            G = scale * (B @ B.conj().T) / M + 0.05 * np.eye(M)
        else:
            B = rng.normal(size=(M, rank)) + 1j * rng.normal(size=(M, rank))
            G = scale * (B @ B.conj().T) / max(rank, 1)
            G = 0.5 * (G + G.conj().T)
        H = scale * (A + A.conj().T) / (2.0 * np.sqrt(M))
        out[i] = H - 0.5j * G
    return out


def midpoint_grid(a: float, b: float, n: int) -> np.ndarray:
    """n energies uniform in the open interval (a, b): a + (b-a)(j+1/2)/n."""
    j = np.arange(n, dtype=np.float64)
    return a + (b - a) * (j + 0.5) / n


@dataclass
class UnevenLayout:
    widths: np.ndarray   # [S] int
    lengths: np.ndarray  # [S] int
    ws: np.ndarray       # [S] disorder strengths
    seeds: np.ndarray    # [S] per-strip disorder seed


def uneven_layout(n_strips: int = 512, wmin: int = 32, wmax: int = 256, wstep: int = 32,
                  lmin: int = 256, lmax: int = 2048, dmin: float = 0.5, dmax: float = 3.0,
                  seed: int = SEED_UNEVEN_LAYOUT) -> UnevenLayout:
    """Widths ~ U{wmin, wmin+wstep, .., wmax}, lengths ~ U[lmin, lmax], w ~ U[dmin, dmax]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    choices = np.arange(wmin, wmax + 1, wstep)
    widths = rng.choice(choices, size=n_strips)
    lengths = rng.integers(lmin, lmax + 1, size=n_strips)
    ws = rng.uniform(dmin, dmax, size=n_strips)
    seeds = SEED_UNEVEN_STRIP + np.arange(n_strips)
    return UnevenLayout(widths.astype(np.int64), lengths.astype(np.int64), ws, seeds)


def general_square_system(sites, t: float = 1.0):
    """Dense Hamiltonian of an arbitrary set of square-lattice sites (scalar, on-site 0).

    ``sites`` is a list of integer (x, y) pairs; two sites are bonded when
    their distance is one lattice step.  Returns (H [N, N], index dict).
    Used for the non-strip worked example of section 2.2.
    """
    index = {tuple(s): i for i, s in enumerate(sites)}
    N = len(sites)
    H = np.zeros((N, N), dtype=np.complex128)
    for (x, y), i in index.items():
        for dx, dy in ((1, 0), (0, 1)):
            j = index.get((x + dx, y + dy))
            if j is not None:
                H[i, j] = H[j, i] = t
    return H, index


# ---------------------------------------------------------------- systems of any shape (knitting)

@dataclass
class Graph:
    """A tight-binding system of any shape (Eq. (1)): N sites with norb orbitals,
    a CSR hopping graph (row_ptr, col) with the block H_{i, col[e]} per directed
    edge e in ``hop`` [nnz, norb, norb], and on-site blocks ``onsite`` [N, norb, norb]."""
    N: int
    norb: int
    row_ptr: np.ndarray
    col: np.ndarray
    hop: np.ndarray
    onsite: np.ndarray
    coords: list | None = None

    def dense(self) -> np.ndarray:
        """The full [N*norb, N*norb] Hamiltonian."""
        no = self.norb
        H = np.zeros((self.N * no, self.N * no), dtype=np.complex128)
        for i in range(self.N):
            H[i * no:(i + 1) * no, i * no:(i + 1) * no] = self.onsite[i]
            for e in range(self.row_ptr[i], self.row_ptr[i + 1]):
                j = self.col[e]
                H[i * no:(i + 1) * no, j * no:(j + 1) * no] = self.hop[e]
        return H


def graph_from_blocks(N: int, norb: int, onsite: np.ndarray, bonds: dict) -> Graph:
    """``bonds`` maps (i, j) to the block H_{ij}; H_{ji} = H_{ij}^+ is added for every bond."""
    rows = [dict() for _ in range(N)]
    for (i, j), b in bonds.items():
        b = np.asarray(b, dtype=np.complex128).reshape(norb, norb)
        rows[i][j] = b
        rows[j][i] = b.conj().T
    row_ptr = np.zeros(N + 1, dtype=np.int32)
    col, hop = [], []
    for i in range(N):
        for j in sorted(rows[i]):
            col.append(j)
            hop.append(rows[i][j])
        row_ptr[i + 1] = len(col)
    hop = np.array(hop, dtype=np.complex128).reshape(len(col), norb, norb)
    return Graph(N, norb, row_ptr, np.array(col, dtype=np.int32), hop,
                 np.asarray(onsite, dtype=np.complex128).reshape(N, norb, norb))


def square_lattice_graph(sites, t: float = 1.0, flux: float = 0.0, kind: str = "scalar", mu: float = 0.0,
                         delta: float = 0.0, alpha: float = 0.0, ez: float = 0.0) -> Graph:
    """Square-lattice sites (list of integer (x, y)), nearest-neighbour bonds.

    * ``flux``: magnetic flux per plaquette in flux quanta, Landau gauge: the
      x-bond from (x, y) to (x+1, y) carries the Peierls phase exp(2 pi i flux y).
    * ``kind``: "scalar" (one orbital, H_ij = -t), "bdg" (electron-hole blocks
      diag(-t e^{i phi}, +t e^{-i phi}) on bonds, diag(-mu, mu) + delta sigma_x
      on site), "rashba" (spin-1/2: -t on bonds plus the Rashba term
      i alpha (sigma_y for x-bonds, -sigma_x for y-bonds), ez sigma_z on site).
    """
    index = {tuple(s): i for i, s in enumerate(sites)}
    N = len(sites)
    sx = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    sy = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    sz = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    no = 1 if kind == "scalar" else 2
    onsite = np.zeros((N, no, no), dtype=np.complex128)
    if kind == "bdg":
        onsite[:] = np.array([[-mu, delta], [delta, mu]], dtype=np.complex128)
    elif kind == "rashba":
        onsite[:] = ez * sz
    bonds = {}
    for (x, y), i in index.items():
        for dx, dy in ((1, 0), (0, 1)):
            j = index.get((x + dx, y + dy))
            if j is None:
                continue
            ph = np.exp(2j * np.pi * flux * y) if dx == 1 else 1.0
            if kind == "scalar":
                b = np.array([[-t * ph]])
            elif kind == "bdg":
                b = np.array([[-t * ph, 0], [0, t * np.conj(ph)]])
            else:
                b = -t * ph * np.eye(2) + 1j * alpha * ph * (sy if dx == 1 else -sx)
            bonds[(i, j)] = b
    g = graph_from_blocks(N, no, onsite, bonds)
    g.coords = [tuple(s) for s in sites]
    return g


def graph_disorder(g: Graph, w: float, seed: int) -> np.ndarray:
    """On-site blocks [N, norb, norb] of g plus eps * identity, eps ~ U[-w/2, w/2], PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = w * (rng.random(g.N) - 0.5)
    out = g.onsite.copy()
    for i in range(g.N):
        out[i] += eps[i] * np.eye(g.norb)
    return out


def rectangle_with_hole(Lx: int, Ly: int, hole: tuple | None = None):
    """Sites of an Lx x Ly rectangle, minus the rectangle hole = (x0, y0, x1, y1) (inclusive)."""
    sites = []
    for x in range(Lx):
        for y in range(Ly):
            if hole and hole[0] <= x <= hole[2] and hole[1] <= y <= hole[3]:
                continue
            sites.append((x, y))
    return sites
