"""Learned energy sampling for T(E) curves.

The transmission of a disordered ribbon has channel steps at the lead's
thresholds and sharp resonances in between, so a uniform energy grid wastes
points on smooth stretches. A small network (``mlp.Network``, trained and run
by the library's BF16 kernels) reads a coarse uniform probe of the curve and
proposes where to spend the remaining points. The transport path evaluates
every proposed point; nothing is interpolated from the network.

**Per curve.** Ribbon cross-section M, length L, disorder w.
1. **Probe.** T at 64 midpoint energies in (EMIN, EMAX), plus the lead's
   open-channel count at the same energies (the clean strip's T).
2. **Features.** Probe T / Nmax, the lead's N_open / Nmax at the 512 bin
   centres (a clean-lead property that locates the channel thresholds), log L / 8,
   w and M / 256 (579 numbers; Nmax = max(1, max N_open)).
3. **Density.** The network outputs a softmax density p over 512 equal bins:
   its estimate of where the 256-point trapezoid rule leaves its error.
4. **Placement.** The placement density is d = 0.8·norm(√p) + 0.2·uniform.
   The 192 further energies are shared among the 65 intervals that the probe
   points cut (EMIN, the 64 probe energies, EMAX) in proportion to each
   interval's mass of d (largest remainders), and sit evenly spaced inside
   their interval.  A uniform p gives back the evenly spaced 256-point grid
   (three points between neighbouring probe points), so the probe is never
   wasted on an uneven grid.
5. **Integration.** The integrated conductance uses the trapezoid over the
   sorted 256 points, with the interval's end points (T evaluated there too).
6. **Fallback.** A dense uniform grid is the fallback when p is not finite,
   and a 4096-point one is the reference the error is measured against.

**Training target.** A disordered ribbon's T(E) fluctuates on energy scales
below the 256-point spacing, so the trapezoid error of each interval behaves
like a random term whose variance depends on where the interval sits (channel
thresholds, the edge-state band, resonance-rich stretches).  The error of the
sum is smallest when the sampling density follows the square root of that
variance (Neyman's allocation: with n_i points in a stretch of error variance
s_i² per point, sum s_i²/n_i under sum n_i = n is minimal at n_i ∝ s_i).  So
the target q of a training curve, computed on a dense grid, is the squared
signed error of each interval of the uniform 256-point rule, spread over the
bins it covers, plus a floor of 1e-3 of its mean, normalised; the network's
softmax fitted by cross-entropy estimates the expected profile given the
features, and the placement takes its square root.  (Equidistributing the
curvature, |T''|^{1/3}, is the rule for smooth integrands and loses here.)
The loss is minimised with AdamW.

**Seeds.** Training curve i uses seed 20101010 + i for its (Nz, L, w) draw and
its disorder. Evaluation ribbons use 10102627 + r.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import inputs, workload

EMIN, EMAX = -3.0, 3.0
N_PROBE = 64
N_BINS = 512
N_LEARNED = 192
N_TOTAL = N_PROBE + N_LEARNED
N_JUDGE = 4096
N_DENSE = 4096      # dense grid of the training curves (a multiple of N_TOTAL and N_BINS)
SEED_TRAIN = 20101010
N_FEATURES = N_PROBE + N_BINS + 3
SIZES = [N_FEATURES, 256, 256, 256, N_BINS]


@dataclass
class Ribbon:
    Nz: int
    L: int
    w: float
    seed: int

    @property
    def M(self) -> int:
        return 2 * self.Nz


def midpoints(n, a=EMIN, b=EMAX):
    return inputs.midpoint_grid(a, b, n)


def train_ribbons(n, Nz_choices=(6, 8, 10, 12, 14, 16), L_choices=(32, 64), w_range=(0.2, 0.8), start=0):
    out = []
    for i in range(start, start + n):
        rng = np.random.Generator(np.random.PCG64(SEED_TRAIN + i))
        out.append(Ribbon(int(rng.choice(Nz_choices)), int(rng.choice(L_choices)), float(rng.uniform(*w_range)),
                          SEED_TRAIN + i))
    return out


def transmission_curves(ribbons, energies_list, chunk=64, device="cuda", progress=None):
    """T(E) on the GPU path for every ribbon at its own energies (list of arrays).
    Ribbons are grouped by cross-section so each strip class shares its self-energies.
    progress(msg), if given, is called after every chunk."""
    out = [None] * len(ribbons)
    for c0 in range(0, len(ribbons), chunk):
        idx = list(range(c0, min(len(ribbons), c0 + chunk)))
        classes = sorted(set(ribbons[i].Nz for i in idx))
        cls_of = {nz: k for k, nz in enumerate(classes)}
        strips = [inputs.zigzag_strip(nz) for nz in classes]
        # one energy list per class: the union of its ribbons' energies
        E_cls = [np.unique(np.concatenate([np.asarray(energies_list[i]) for i in idx if ribbons[i].Nz == nz]))
                 for nz in classes]
        reals = []
        for i in idx:
            r = ribbons[i]
            st = strips[cls_of[r.Nz]]
            reals.append(workload.Realization(cls_of[r.Nz], inputs.onsite_disorder(st, r.L, r.w, r.seed)))
        b = workload.Batch(strips, reals, E_cls, device)
        b.compute_sigmas()
        if int((b.sigma_status.cpu().numpy() != 0).sum()):
            if b.repair_sigmas():
                b.repair_sigmas(nudge=1e-6)     # energies exactly on a threshold
        G1N, _, _, status = b.sweep("fp64", gnn=False)
        T = b.transmission(G1N)[0].cpu().numpy()
        st_sig, st_sw = b.sigma_status.cpu().numpy(), status.cpu().numpy()
        if int((st_sw != 0).sum()) or int((st_sig != 0).sum()):
            bad = np.nonzero(st_sig != 0)[0]
            Eall = np.concatenate([np.asarray(e) for e in E_cls])
            Nall = np.concatenate([np.full(len(e), nz) for e, nz in zip(E_cls, classes)])
            raise RuntimeError(f"transport path reported a problem status while sampling: {len(bad)} self-energies "
                               f"at (E, Nz) {[(float(Eall[k]), int(Nall[k])) for k in bad[:8]]} "
                               f"(status {sorted(set(st_sig[bad].tolist()))}), "
                               f"{int((st_sw != 0).sum())} sweeps (status {sorted(set(st_sw[st_sw != 0].tolist()))})")
        for ri, i in enumerate(idx):
            E_c = E_cls[cls_of[ribbons[i].Nz]]
            sel = np.searchsorted(E_c, np.asarray(energies_list[i]))
            rows = np.nonzero(b.prob_meta[:, 0] == ri)[0]
            out[i] = T[rows][sel]
        del b, G1N
        if progress:
            progress(f"transport: {idx[-1] + 1}/{len(ribbons)} ribbons")
    return out


def open_channels(Nz_list, energies, device="cuda"):
    """N_open(E) of the clean zigzag lead of each cross-section (T of one clean slice)."""
    classes = sorted(set(Nz_list))
    strips = [inputs.zigzag_strip(nz) for nz in classes]
    reals = [workload.Realization(k, inputs.clean_onsite(st, 1)) for k, st in enumerate(strips)]
    b = workload.Batch(strips, reals, [np.asarray(energies) for _ in strips], device)
    b.compute_sigmas()
    G1N, _, _, _ = b.sweep("fp64", gnn=False)
    T = np.rint(b.transmission(G1N)[0].cpu().numpy()).astype(np.int64)
    res = {}
    for k, nz in enumerate(classes):
        res[nz] = T[b.prob_meta[:, 0] == k]
    return res


def features(ribbons, T_probe, nopen_dense):
    """[n, N_FEATURES] float32 (see the module docstring); nopen_dense: {Nz: N_open at the
    N_BINS bin centres}."""
    X = np.zeros((len(ribbons), N_FEATURES), np.float32)
    for i, r in enumerate(ribbons):
        no = nopen_dense[r.Nz].astype(np.float64)
        nmax = max(1.0, float(no.max()))
        X[i, :N_PROBE] = np.asarray(T_probe[i]) / nmax
        X[i, N_PROBE:N_PROBE + N_BINS] = no / nmax
        X[i, N_PROBE + N_BINS:] = [np.log(r.L) / 8.0, r.w, r.M / 256.0]
    return X


def target_density(T_dense, floor_rel=1e-3):
    """q over the N_BINS bins from a curve on a dense midpoint grid of n points (n a multiple
    of N_TOTAL and N_BINS): the squared trapezoid error of each interval of the uniform
    N_TOTAL-point rule, spread over the dense points it covers, averaged per bin, plus a floor
    of floor_rel times its mean, normalised."""
    T = np.asarray(T_dense, dtype=np.float64)
    n = T.shape[0]
    assert n % N_TOTAL == 0 and n % N_BINS == 0
    E = midpoints(n)
    s = n // N_TOTAL
    k = np.arange(N_TOTAL) * s + s // 2           # dense points nearest the uniform rule's energies
    e2 = np.zeros(n)
    for a, b in zip(k[:-1], k[1:]):
        x, y = E[a:b + 1], T[a:b + 1]
        lin = y[0] + (y[-1] - y[0]) * (x - x[0]) / (x[-1] - x[0])
        r = y - lin
        e = float(np.sum(0.5 * (r[1:] + r[:-1]) * np.diff(x)))
        e2[a:b] = e * e
    e2[:k[0]] = e2[k[0]]                          # the end stretches take their neighbour's value
    e2[k[-1]:] = e2[k[-1] - 1]
    q = e2.reshape(N_BINS, -1).mean(axis=1)
    q = q + floor_rel * q.mean() + 1e-300
    return (q / q.sum()).astype(np.float32)


def place(p, n=N_LEARNED, mix=0.8):
    """n energies: the density d = mix * norm(sqrt(p)) + (1 - mix) * uniform over the bins is
    integrated over the intervals the probe energies cut, the n points are shared among them in
    proportion (largest remainders) and sit evenly spaced inside each interval."""
    p = np.asarray(p, dtype=np.float64)
    if p.shape != (N_BINS,) or not np.all(np.isfinite(p)) or p.sum() <= 0 or np.any(p < 0):
        return None
    r = np.sqrt(p)
    d = mix * r / r.sum() + (1.0 - mix) / N_BINS
    cdf = np.concatenate([[0.0], np.cumsum(d)])
    width = (EMAX - EMIN) / N_BINS
    edges = np.concatenate([[EMIN], midpoints(N_PROBE), [EMAX]])
    mass = np.diff(np.interp(edges, EMIN + width * np.arange(N_BINS + 1), cdf))
    share = mass / mass.sum() * n
    cnt = np.floor(share).astype(int)
    cnt[np.argsort(-(share - cnt), kind="stable")[:n - cnt.sum()]] += 1
    E = np.concatenate([edges[k] + (edges[k + 1] - edges[k]) * np.arange(1, c + 1) / (c + 1)
                        for k, c in enumerate(cnt)])
    # the zigzag lead is singular at E = 0 (its flat edge band) and at E = +-t (every subband
    # meets there at the zone boundary), where its decimation does not converge: keep points
    # at least 1e-3 away (the 4096-point reference grid's nearest points are 7.3e-4 away)
    for e0 in (0.0, -1.0, 1.0):
        near = np.abs(E - e0) < 1e-3
        E[near] = np.where(E[near] < e0, e0 - 1e-3, e0 + 1e-3)
    return np.sort(E)


def threshold_density(nopen_dense, weight=20.0):
    """Non-learned placement density: uniform plus a bump on every bin next to a change of
    the lead's open-channel count (reported beside the network for comparison)."""
    no = np.asarray(nopen_dense, dtype=np.float64)
    jump = np.zeros(N_BINS)
    d = np.abs(np.diff(no))
    jump[:-1] += d
    jump[1:] += d
    p = 1.0 + weight * jump
    return p / p.sum()


def integrate(E, T):
    """Trapezoid of T over the sorted points (the interval's end points included by the caller)."""
    o = np.argsort(E)
    E, T = np.asarray(E)[o], np.asarray(T)[o]
    return float(np.sum(0.5 * (T[1:] + T[:-1]) * np.diff(E)))


def learned_points(net, ribbons, T_probe, nopen_dense, device="cuda"):
    """Per ribbon: the 192 proposed energies, or the uniform fallback when the density is unusable."""
    X = torch.from_numpy(features(ribbons, T_probe, nopen_dense)).to(device)
    P = net.probs(X).cpu().numpy()
    pts, fell_back = [], []
    for i in range(len(ribbons)):
        e = place(P[i])
        fell_back.append(e is None)
        pts.append(midpoints(N_LEARNED) if e is None else e)
    return pts, fell_back


def generate_training_set(n_curves, device="cuda", progress=None, chunk=64, n_dense=N_DENSE, **kw):
    """Features and target densities of n_curves seeded ribbons (targets from n_dense points)."""
    rib = train_ribbons(n_curves, **kw)
    Ep, Ed = midpoints(N_PROBE), midpoints(n_dense)
    curves = transmission_curves(rib, [np.concatenate([Ep, Ed])] * len(rib), chunk=chunk, device=device,
                                 progress=progress)
    nopen = open_channels([r.Nz for r in rib], midpoints(N_BINS), device)
    T_probe = [c[:N_PROBE] for c in curves]
    T_dense = [c[N_PROBE:] for c in curves]
    X = features(rib, T_probe, nopen)
    Q = np.stack([target_density(t) for t in T_dense])
    return X, Q, rib


def train(net, X, Q, steps=300, batch=256, lr=2e-3, wd=1e-4, seed=0, device="cuda", log_every=0):
    """Minibatch AdamW on the mean cross-entropy; returns the loss history."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Xt = torch.from_numpy(np.asarray(X, np.float32)).to(device)
    Qt = torch.from_numpy(np.asarray(Q, np.float32)).to(device)
    hist = []
    for s in range(steps):
        idx = torch.from_numpy(rng.choice(len(X), size=min(batch, len(X)), replace=False)).to(device)
        loss, grads = net.loss_and_grads(Xt[idx].contiguous(), Qt[idx].contiguous())
        net.adamw_step(grads, lr=lr, wd=wd)
        if log_every and (s % log_every == 0 or s == steps - 1):
            hist.append((s, float(loss.mean().cpu())))
    return hist


def evaluate(net, ribbons, device="cuda", progress=None, chunk=16):
    """Integrated-conductance error of the learned 256 points and of 256 uniform points
    against the 4096-point reference, per ribbon."""
    Ep, Eu, Ej = midpoints(N_PROBE), midpoints(N_TOTAL), midpoints(N_JUDGE)
    ends = np.array([EMIN, EMAX])
    nopen = open_channels([r.Nz for r in ribbons], midpoints(N_BINS), device)
    base = transmission_curves(ribbons, [np.concatenate([Ep, Eu, Ej, ends])] * len(ribbons), chunk=chunk,
                               device=device, progress=progress)
    n1, n2, n3 = N_PROBE, N_PROBE + N_TOTAL, N_PROBE + N_TOTAL + N_JUDGE
    T_probe = [c[:n1] for c in base]
    pts, fb = learned_points(net, ribbons, T_probe, nopen, device)
    learned_T = transmission_curves(ribbons, pts, chunk=chunk, device=device, progress=progress)
    thr_pts = [place(threshold_density(nopen[r.Nz])) for r in ribbons]
    thr_T = transmission_curves(ribbons, thr_pts, chunk=chunk, device=device, progress=progress)
    rows = []
    for i in range(len(ribbons)):
        c = base[i]
        Te = c[n3:]
        I_ref = integrate(np.concatenate([Ej, ends]), np.concatenate([c[n2:n3], Te]))
        I_uni = integrate(np.concatenate([Eu, ends]), np.concatenate([c[n1:n2], Te]))
        I_l = integrate(np.concatenate([Ep, pts[i], ends]), np.concatenate([T_probe[i], learned_T[i], Te]))
        I_t = integrate(np.concatenate([Ep, thr_pts[i], ends]), np.concatenate([T_probe[i], thr_T[i], Te]))
        den = max(abs(I_ref), 1e-12)
        rows.append({"err_uniform": abs(I_uni - I_ref) / den, "err_learned": abs(I_l - I_ref) / den,
                     "err_threshold": abs(I_t - I_ref) / den, "fallback": bool(fb[i]), "I_ref": I_ref})
    return rows
