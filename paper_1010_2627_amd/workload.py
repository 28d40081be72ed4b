"""Batches of transport problems on the GPU: packing and driving the C ABI.

A batch is a set of strip realizations (a strip class plus its seeded on-site
blocks) crossed with the energies of their strip class.  This module packs
the host data into the flat device buffers and the problem table that
``libknit`` expects, and calls the entry points in order (lead self-energies,
sweep, transmission, LDOS).  It holds no transport arithmetic.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import inputs
from . import knit as K


@dataclass
class Realization:
    strip: int               # index into Batch.strips
    onsite: np.ndarray       # [L, W, norb, norb] complex128
    label: str = ""


@dataclass
class Batch:
    strips: list                      # inputs.Strip (host)
    realizations: list                # Realization
    energies: list                    # per strip class: float64 array of energies
    device: str = "cuda"
    dstrips: list = field(default_factory=list)
    probs: K.ProblemTable | None = None
    onsite: torch.Tensor | None = None
    sigmaL: torch.Tensor | None = None
    sigmaR: torch.Tensor | None = None
    sigma_status: torch.Tensor | None = None
    sigma_iters: torch.Tensor | None = None
    CL: torch.Tensor | None = None            # Gamma_L = C_L C_L^+ factors, addressed like sigmaL
    CR: torch.Tensor | None = None
    rankL: torch.Tensor | None = None         # per (strip class, energy) slot, in slot order
    rankR: torch.Tensor | None = None
    prob_meta: np.ndarray | None = None      # [P, 2]: (realization, energy index)

    def __post_init__(self):
        assert len(self.energies) == len(self.strips)
        self.dstrips = [K.DeviceStrip.from_host(s, self.device) for s in self.strips]
        # on-site blocks, concatenated
        offs, chunks, pos = [], [], 0
        for r in self.realizations:
            st = self.strips[r.strip]
            assert r.onsite.shape[1:] == st.onsite_shape(1)[1:]
            offs.append(pos)
            chunks.append(np.ascontiguousarray(r.onsite, dtype=np.complex128).reshape(-1))
            pos += chunks[-1].size
        flat = np.concatenate(chunks) if chunks else np.zeros(1, np.complex128)
        self.onsite = torch.from_numpy(flat).to(self.device)
        # sigma slots: one per (strip class, energy)
        self.sigma_base = []
        spos = 0
        for s, E in zip(self.strips, self.energies):
            self.sigma_base.append(spos)
            spos += len(E) * s.M * s.M
        self.sigma_elems = max(spos, 1)
        # energies on the device (the self-energy call takes device energies; keeping them
        # resident lets a whole step be captured in a graph)
        self.denergies = [torch.as_tensor(np.asarray(E, dtype=np.float64), device=self.device)
                          for E in self.energies]
        # problems: realization x energy of its strip class
        rows, meta = [], []
        out_pos = ldos_pos = 0
        for ri, r in enumerate(self.realizations):
            st = self.strips[r.strip]
            L = r.onsite.shape[0]
            for ei, E in enumerate(self.energies[r.strip]):
                rows.append((r.strip, L, float(E), offs[ri],
                             self.sigma_base[r.strip] + ei * st.M * st.M, out_pos, ldos_pos))
                meta.append((ri, ei))
                out_pos += st.M * st.M
                ldos_pos += L * st.M
        host = np.array(rows, dtype=K.PROBLEM_DTYPE) if rows else np.zeros(0, K.PROBLEM_DTYPE)
        self.probs = K.ProblemTable.from_host(host, self.device)
        self.prob_meta = np.array(meta, dtype=np.int64).reshape(-1, 2)

    @property
    def P(self) -> int:
        return self.probs.P

    def slice_steps(self) -> int:
        return int(self.probs.host["L"].sum())

    def compute_sigmas(self, eta=1e-16, tol=1e-16, max_iter=100, stream=None):
        self.sigmaL = torch.empty(self.sigma_elems, dtype=torch.complex128, device=self.device)
        self.sigmaR = torch.empty(self.sigma_elems, dtype=torch.complex128, device=self.device)
        stats, its = [], []
        for si, (ds, E) in enumerate(zip(self.dstrips, self.energies)):
            if len(E) == 0:
                continue
            Et = self.denergies[si]
            base, n = self.sigma_base[si], len(E) * ds.M * ds.M
            sig, it, st = K.knit_lead_selfenergy(ds, 2, Et, eta, tol, max_iter, stream)
            self.sigmaL[base:base + n].copy_(sig[0].reshape(-1))
            self.sigmaR[base:base + n].copy_(sig[1].reshape(-1))
            stats.append(st)
            its.append(it)
        self.sigma_status = torch.cat(stats) if stats else None
        self.sigma_iters = torch.cat(its) if its else None
        return self.sigmaL, self.sigmaR

    def repair_sigmas(self, eta=1e-16, tol=1e-16, max_iter=100, group=4, nudge=0.0, stream=None):
        """Redo, in calls of at most `group` energies, the self-energies whose status is not
        clean (one call redoes at most four energies at slice eigenvalues with its two-slice
        cell; a batch with more such energies leaves the rest flagged).  With nudge != 0 the
        redone self-energy is taken at E + nudge * max(1, |E|) (for an energy sitting exactly
        on a channel threshold, where the lead's Bloch factors degenerate); the problems keep
        their E.  Returns the number of energies still flagged afterwards."""
        st = self.sigma_status.cpu().numpy()
        left, pos = 0, 0
        for si, (ds, E) in enumerate(zip(self.dstrips, self.energies)):
            n = len(E)
            bad = np.nonzero(st[pos:pos + n] != 0)[0]
            for g0 in range(0, len(bad), group):
                idx = bad[g0:g0 + group]
                Et = self.denergies[si][torch.as_tensor(idx, device=self.device)].contiguous()
                if nudge:
                    Et = Et + nudge * torch.clamp(Et.abs(), min=1.0)
                sig, it, s2 = K.knit_lead_selfenergy(ds, 2, Et, eta, tol, max_iter, stream)
                s2 = s2.cpu().numpy()
                MM = ds.M * ds.M
                for j, e in enumerate(idx):
                    o = self.sigma_base[si] + int(e) * MM
                    self.sigmaL[o:o + MM].copy_(sig[0][j].reshape(-1))
                    self.sigmaR[o:o + MM].copy_(sig[1][j].reshape(-1))
                    self.sigma_status[pos + int(e)] = int(s2[j])
                left += int((s2 != 0).sum())
            pos += n
        return left

    def compute_gamma_factors(self, tol=0.0, stream=None):
        """Factor Gamma = C C^+ of both leads at every (strip class, energy) slot."""
        self.CL = torch.zeros(self.sigma_elems, dtype=torch.complex128, device=self.device)
        self.CR = torch.zeros(self.sigma_elems, dtype=torch.complex128, device=self.device)
        rl, rr = [], []
        for si, (ds, E) in enumerate(zip(self.dstrips, self.energies)):
            if len(E) == 0:
                continue
            base, n = self.sigma_base[si], len(E) * ds.M * ds.M
            rl.append(K.knit_gamma_factor(ds.M, self.sigmaL[base:base + n], len(E), tol, self.CL[base:base + n],
                                          stream)[1])
            rr.append(K.knit_gamma_factor(ds.M, self.sigmaR[base:base + n], len(E), tol, self.CR[base:base + n],
                                          stream)[1])
        self.rankL = torch.cat(rl) if rl else None
        self.rankR = torch.cat(rr) if rr else None
        return self.CL, self.CR

    def problem_ranks(self) -> tuple[np.ndarray, np.ndarray]:
        """(rank of Gamma_L, rank of Gamma_R) of every problem, from its (strip class, energy) slot."""
        slot_base = np.cumsum([0] + [len(E) for E in self.energies])[:-1]
        slot = np.array([slot_base[r.strip] + int(ei) for r, (ri, ei) in
                         ((self.realizations[int(m[0])], m) for m in self.prob_meta)], dtype=np.int64)
        return self.rankL.cpu().numpy()[slot], self.rankR.cpu().numpy()[slot]

    def sweep_projected(self, gnn=False, stream=None, workspace=None, precision="fp64"):
        return K.knit_rgf_sweep_projected(self.dstrips, self.probs, self.onsite, self.sigmaL, self.sigmaR,
                                          self.CL, GNN=gnn, stream=stream, workspace=workspace, precision=precision)

    def transmission_projected(self, G1Np, stream=None):
        return K.knit_transmission_projected(self.dstrips, self.probs, self.CR, G1Np, stream)

    def local_observables(self, checkpoint_stride=0, stream=None):
        """Injection from the left lead (needs compute_gamma_factors): per problem the on-site
        blocks of A_L = G Gamma_L G^+ [L, W, norb, norb] and the currents into every site from
        the previous slice and from its own slice [L, W].  Returns (blk, blk_off, jlong, jtran,
        status); see local_block / current_block."""
        return K.knit_local_observables(self.dstrips, self.probs, self.onsite, self.sigmaL, self.sigmaR, self.CL,
                                        checkpoint_stride, stream)

    def local_block(self, blk, blk_off, p: int) -> torch.Tensor:
        row = self.probs.host[p]
        st = self.strips[int(row["strip"])]
        L = int(row["L"])
        o = int(blk_off[p])
        return blk[o:o + L * st.M * st.norb].view(L, st.W, st.norb, st.norb)

    def current_block(self, flat: torch.Tensor, p: int) -> torch.Tensor:
        row = self.probs.host[p]
        st = self.strips[int(row["strip"])]
        o = int(row["ldos_off"])
        return flat[o:o + int(row["L"]) * st.W].view(int(row["L"]), st.W)

    def transmission_eigenvalues(self, G1Np, stream=None):
        """(T_n [P, ld] descending, channel count [P], T [P], Fano factor [P]) from the projected sweep."""
        return K.knit_transmission_eigenvalues(self.dstrips, self.probs, self.CR, G1Np, stream)

    def set_sigmas(self, sigL_list, sigR_list):
        """Install externally computed self-energies: one [nE, M, M] array per strip class."""
        self.sigmaL = torch.empty(self.sigma_elems, dtype=torch.complex128, device=self.device)
        self.sigmaR = torch.empty(self.sigma_elems, dtype=torch.complex128, device=self.device)
        for si, (sl, sr) in enumerate(zip(sigL_list, sigR_list)):
            base = self.sigma_base[si]
            n = np.asarray(sl).size
            self.sigmaL[base:base + n] = torch.from_numpy(np.ascontiguousarray(sl).reshape(-1)).to(self.device)
            self.sigmaR[base:base + n] = torch.from_numpy(np.ascontiguousarray(sr).reshape(-1)).to(self.device)

    def sigma_of(self, p: int):
        """(Sigma_L, Sigma_R) of problem p as [M, M] device views."""
        row = self.probs.host[p]
        M = self.strips[int(row["strip"])].M
        o = int(row["sigma_off"])
        return self.sigmaL[o:o + M * M].view(M, M), self.sigmaR[o:o + M * M].view(M, M)

    def sweep(self, precision="fp64", gn1=False, gnn=True, stream=None, workspace=None):
        return K.knit_rgf_sweep(self.dstrips, self.probs, self.onsite, self.sigmaL, self.sigmaR,
                                precision, GN1=gn1, GNN=gnn, stream=stream, workspace=workspace)

    def transmission(self, G1N, GN1=None, GNN=None, stream=None):
        return K.knit_transmission(self.dstrips, self.probs, self.sigmaL, self.sigmaR, G1N, GN1, GNN,
                                   stream)

    def ldos(self, precision="fp64", checkpoint_stride=0, stream=None):
        return K.knit_ldos(self.dstrips, self.probs, self.onsite, self.sigmaL, self.sigmaR, precision,
                           checkpoint_stride, stream)

    def block(self, flat: torch.Tensor, p: int) -> torch.Tensor:
        row = self.probs.host[p]
        M = self.strips[int(row["strip"])].M
        o = int(row["out_off"])
        return flat[o:o + M * M].view(M, M)

    def ldos_block(self, flat: torch.Tensor, p: int) -> torch.Tensor:
        row = self.probs.host[p]
        M = self.strips[int(row["strip"])].M
        o = int(row["ldos_off"])
        return flat[o:o + int(row["L"]) * M].view(int(row["L"]), M)


# ---------------------------------------------------------------- the synthetic workloads

def square_batch(W, L, w, n_energies, n_seeds, emin=-3.9, emax=3.9, device="cuda", seed0=None):
    """Square-lattice strip, Anderson disorder U[-w/2, w/2], midpoint energies, n_seeds realizations."""
    st = inputs.square_strip(W)
    seed0 = inputs.SEED_BASE if seed0 is None else seed0
    reals = [Realization(0, inputs.onsite_disorder(st, L, w, seed0 + r), f"seed{seed0 + r}")
             for r in range(n_seeds)]
    return Batch([st], reals, [inputs.midpoint_grid(emin, emax, n_energies)], device)


def rashba_batch(W, L, w, n_energies, n_seeds, alpha=0.2, ez=0.1, emin=-3.9, emax=3.9,
                 device="cuda", seed0=None):
    st = inputs.rashba_strip(W, alpha=alpha, ez=ez)
    seed0 = inputs.SEED_BASE if seed0 is None else seed0
    reals = [Realization(0, inputs.onsite_disorder(st, L, w, seed0 + r), f"seed{seed0 + r}")
             for r in range(n_seeds)]
    return Batch([st], reals, [inputs.midpoint_grid(emin, emax, n_energies)], device)


def zigzag_batch(Nz, L, w, energies, n_seeds, device="cuda", seed0=None):
    st = inputs.zigzag_strip(Nz)
    seed0 = inputs.SEED_BASE if seed0 is None else seed0
    reals = [Realization(0, inputs.onsite_disorder(st, L, w, seed0 + r), f"seed{seed0 + r}")
             for r in range(n_seeds)]
    return Batch([st], reals, [np.asarray(energies, dtype=np.float64)], device)


def uneven_batch(n_strips=512, n_energies=32, emin=-3.9, emax=3.9, device="cuda", **layout_kw):
    """Strips of uneven width and length (one strip class per width), 32 energies each."""
    lay = inputs.uneven_layout(n_strips, **layout_kw)
    widths = sorted(set(int(x) for x in lay.widths))
    classes = {W: i for i, W in enumerate(widths)}
    strips = [inputs.square_strip(W) for W in widths]
    reals = []
    for i in range(n_strips):
        st = strips[classes[int(lay.widths[i])]]
        reals.append(Realization(classes[int(lay.widths[i])],
                                 inputs.onsite_disorder(st, int(lay.lengths[i]), float(lay.ws[i]),
                                                        int(lay.seeds[i])), f"strip{i}"))
    E = inputs.midpoint_grid(emin, emax, n_energies)
    return Batch(strips, reals, [E for _ in strips], device)


# ---------------------------------------------------------------- systems of any shape

class GraphBatch:
    """Problems of one system of any shape (``inputs.Graph``) and its leads, resident
    on the GPU: energies, per-realization on-site blocks and per-problem self-energy
    packs (lead k's Sigma_k [n_k norb]^2 after the earlier leads').  Arranges arrays
    only; the knitting runs in ``knit_graph_transmission``."""

    def __init__(self, g, leads, energies, onsites, sigmas, device="cuda", order=None, block=None):
        from . import graph as GR
        self.g, self.leads = g, [np.asarray(l, dtype=np.int32) for l in leads]
        self.plan = GR.plan_create(g.N, g.norb, g.row_ptr, g.col, self.leads, order, block)
        self.info = self.plan.info()
        E = np.atleast_1d(np.asarray(energies, dtype=np.float64))
        P = len(E)
        onsites = np.asarray(onsites, dtype=np.complex128).reshape(-1, g.N, g.norb, g.norb)
        real_of = np.arange(P) % onsites.shape[0] if onsites.shape[0] > 1 else np.zeros(P, dtype=np.int64)
        ss = self.info["sigma_size"]
        packs = np.zeros((P, ss), dtype=np.complex128)
        for p in range(P):
            o = 0
            for k in range(len(self.leads)):
                s = np.asarray(sigmas[k][p], dtype=np.complex128)
                packs[p, o:o + s.size] = s.ravel()
                o += s.size
            assert o == ss
        ld = self.info["lead_dim"]
        tab = GR.problem_table(E, real_of * g.N * g.norb * g.norb, np.arange(P) * ss, np.arange(P) * ld * ld)
        self.P, self.E, self.real_of = P, E, real_of
        self.device = device
        self.hop = torch.from_numpy(np.ascontiguousarray(g.hop)).to(device) if len(g.col) else None
        self.onsite = torch.from_numpy(np.ascontiguousarray(onsites)).to(device)
        self.sigma = torch.from_numpy(packs).to(device)
        self.probs = torch.from_numpy(tab.view(np.uint8).copy()).to(device)

    def run(self, want_gll=False, ws=None, stream=None):
        from . import graph as GR
        return GR.knit_graph_transmission(self.plan, self.probs, self.P, self.hop, self.onsite, self.sigma,
                                          want_gll=want_gll, ws=ws, stream=stream)
