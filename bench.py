"""Benchmark of the two-lead strip transport path on one MI355X.

One step = the whole T(E) path over the batch, with the inputs resident in HBM:
  * the lead self-energies of both leads for every energy (double-double
    decimation);
  * the broadening factors Gamma = C C^+ of both leads (pivoted Cholesky; the
    rank is the lead's open channels);
  * the slice sweep of every (energy, realization) problem, carrying the
    projected propagator C_L^+ G_1n;
  * the Fisher-Lee trace T = ||C_L^+ G_1L C_R||^2.

Beside the headline, full steps of three other paths are timed:
  * the FP64 sweep carrying the whole G_1n (and the full trace);
  * the refined paths, projected and whole G_1n: FP32 matrix-core elimination
    of each slice with FP64-residual Newton steps on its inverse and the
    propagator as an FP64 product of the refined inverse.
Their T(E) is compared with the FP64 one of the same path, per open channel,
with the count of problems the refinement handed to FP64.  The headline
`value` is the step throughput of the projected FP64 path, which meets the
tolerance at every point; the others' figures sit beside it.

Also timed, each once after an untimed call: the LDOS backward sweep, the
transmission eigenvalues and Fano factor from the headline propagator, the
injected densities and site currents, the conductance matrix with a side lead
(the last three on every strip cut to 64 slices except the eigenvalues), and
the knitting of a system with a hole and three leads.

Prints one JSON line. --gpus above 1 is refused: the benchmark runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RGF slice-steps/s at W=256, FP32-MFMA+refine vs FP64; T(E) points/s at |ΔT|≤1e-6"

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "fp32_refine": 157.3}
TOL_PER_CHANNEL = 1e-6

# HBM bytes per launch of the projected FP64 sweep kernel (the headline step) from the calibrated FETCH_SIZE /
# WRITE_SIZE counter runs, per workload, valid for the sweep source whose sha256
# prefix is given; any other source reports null.
MEASURED_TRAFFIC = {
    "c4": {"sha": "61f785c6138b6adf", "bytes": 4.1383e+13,
           "profile": "profiles/sweep_fp64_c4_hbm_traffic.md",
           # executed matrix work and L2 behaviour of the same launch (same counter runs)
           "counters": {"mfma_f64_flops_executed": 4.3128e+14, "mfma_busy_fraction": 0.496,
                        "l2_hit_rate": 0.473}},
}


def sweep_source_sha():
    import hashlib
    path = os.path.join(ROOT, "paper_1010_2627_amd", "csrc", "sweep_mfma.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]

WORKLOADS = {
    # name: builder kwargs and description
    "c4": dict(kind="rashba", W=256, L=512, w=2.0, n_energies=64, n_seeds=8,
               desc="spinful square lattice W=256 (slice dim M=512), Rashba 0.2t, Zeeman 0.1t (sigma_z), "
                    "L=512, disorder U[-1,1] sigma0, 64 midpoint energies in (-3.9,3.9) x 8 seeds "
                    "= 512 problems"),
    "c2": dict(kind="square", W=128, L=1024, w=2.0, n_energies=256, n_seeds=16,
               desc="square-lattice strip W=128 (M=128), L=1024, disorder U[-1,1], "
                    "256 midpoint energies in (-3.9,3.9) x 16 seeds = 4096 problems"),
    "c2w256": dict(kind="square", W=256, L=1024, w=2.0, n_energies=64, n_seeds=8,
                   desc="square-lattice strip W=256 (M=256), L=1024, disorder U[-1,1], "
                        "64 energies x 8 seeds = 512 problems"),
    "c1": dict(kind="square", W=16, L=64, w=1.0, n_energies=64, n_seeds=1,
               desc="square-lattice strip W=16, L=64, disorder U[-0.5,0.5], 64 energies"),
    "c5": dict(kind="sampler", Nz=100, L=1024, w=0.6, n_test=8, n_train=128, train_L=(64, 128, 256),
               train_w=(0.2, 0.8), steps=1500, n_dense=1024,
               desc="learned energy sampling on a zigzag ribbon (slice dim 200, L=1024, disorder U[-0.3,0.3]): "
                    "network trained by the library's BF16 kernels on 128 ribbons of the same width "
                    "(L in {64,128,256}, w in [0.2,0.8], targets from 1024 points per curve); 256 points vs 256 "
                    "uniform on 8 held-out ribbons, measured against 4096 points"),
    "c3": dict(kind="uneven", n_strips=512, n_energies=32,
               desc="uneven batch in one persistent launch: 512 square-lattice strips, W ~ U{32,64,..,256}, "
                    "L ~ U[256,2048], disorder U[-w/2,w/2] with w ~ U[0.5,3], 32 midpoint energies in "
                    "(-3.9,3.9) each = 16384 problems"),
}


def progress(msg):
    """One line per finished phase on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def build_batch(cfg):
    from paper_1010_2627_amd import workload
    if cfg["kind"] == "uneven":
        return workload.uneven_batch(n_strips=cfg["n_strips"], n_energies=cfg["n_energies"])
    if cfg["kind"] == "square":
        return workload.square_batch(cfg["W"], cfg["L"], cfg["w"], cfg["n_energies"], cfg["n_seeds"])
    return workload.rashba_batch(cfg["W"], cfg["L"], cfg["w"], cfg["n_energies"], cfg["n_seeds"])


def open_channels(b):
    """N_open(E) of every problem's lead: T of the clean strip (one slice between the two
    leads) of its strip class, on the GPU path, with the batch's own self-energies."""
    import torch
    from paper_1010_2627_amd import inputs, workload
    reals = [workload.Realization(i, inputs.clean_onsite(st, 1)) for i, st in enumerate(b.strips)]
    c = workload.Batch(b.strips, reals, [np.asarray(E) for E in b.energies])
    c.sigmaL, c.sigmaR = b.sigmaL, b.sigmaR
    G1N, _, _, _ = c.sweep("fp64", gnn=False)
    T = np.rint(c.transmission(G1N)[0].cpu().numpy()).astype(np.int64)
    torch.cuda.synchronize()
    per_class = {}
    for p, (ri, ei) in enumerate(c.prob_meta):
        per_class[(int(ri), int(ei))] = T[p]
    return np.array([per_class[(b.realizations[int(ri)].strip, int(ei))] for ri, ei in b.prob_meta])


def sampler_bench(args, cfg):
    """Learned energy sampling at the ribbon size of the learned-sampling workload: train, then
    place 256 points per held-out ribbon and measure the integrated conductance against the
    4096-point FP64 grid.  `value` is the transport throughput of the evaluation (T points/s)."""
    import torch
    from paper_1010_2627_amd import inputs, mlp, sampler as S
    t0 = time.perf_counter()
    X, Q, _ = S.generate_training_set(cfg["n_train"], Nz_choices=(cfg["Nz"],), L_choices=cfg["train_L"],
                                      w_range=cfg["train_w"], chunk=16, progress=progress,
                                      n_dense=cfg.get("n_dense", S.N_DENSE))
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    progress(f"training set: {cfg['n_train']} curves in {t_data:.1f} s")
    net = mlp.Network(S.SIZES, seed=1)
    t1 = time.perf_counter()
    hist = S.train(net, X, Q, steps=cfg["steps"], batch=256, lr=1e-3, log_every=250)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    H = float(np.mean(-(Q * np.log(np.maximum(Q, 1e-30))).sum(axis=1)))
    progress(f"trained: KL {hist[0][1] - H:.4f} -> {hist[-1][1] - H:.4f} in {t_train:.1f} s")
    test = [S.Ribbon(cfg["Nz"], cfg["L"], cfg["w"], inputs.SEED_BASE + r) for r in range(cfg["n_test"])]
    t2 = time.perf_counter()
    rows = S.evaluate(net, test, progress=progress, chunk=2)
    torch.cuda.synchronize()
    t_eval = time.perf_counter() - t2
    n_points = cfg["n_test"] * (S.N_PROBE + S.N_TOTAL + S.N_JUDGE + 2 + 2 * S.N_LEARNED)
    eu = np.array([r["err_uniform"] for r in rows])
    el = np.array([r["err_learned"] for r in rows])
    et = np.array([r["err_threshold"] for r in rows])
    M = 2 * cfg["Nz"]
    out = {
        "metric": METRIC, "value": n_points / t_eval, "unit": "T(E) points/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": t_eval * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (transport), bf16/f32 (network)", "data": "synthetic",
        "config": {"workload": args.workload, "description": cfg["desc"], "slice_dim_M": M,
                   "test_ribbons": cfg["n_test"], "points_per_ribbon": n_points // cfg["n_test"]},
        "sampler": {"integrated_conductance_rel_error": {
                        "uniform_256": float(eu.mean()), "learned_256": float(el.mean()),
                        "threshold_aware_256": float(et.mean())},
                    "gain_learned_over_uniform": float(eu.mean() / el.mean()),
                    "wins": f"{int((el < eu).sum())}/{len(el)}",
                    "fallbacks": int(sum(r["fallback"] for r in rows)),
                    "kl_start_end": [hist[0][1] - H, hist[-1][1] - H],
                    "train_data_s": round(t_data, 2), "train_s": round(t_train, 2),
                    "eval_s": round(t_eval, 2)},
    }
    print(json.dumps(out))


def cpu_baseline(cfg, b, budget_s=20.0, single_thread_s=8.0):
    """The oracle on a bounded sample, with all host threads, then again with one thread
    (threadpoolctl) on a smaller sample; both rates in slice-steps/s."""
    out = _cpu_baseline(cfg, b, budget_s)
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            one = _cpu_baseline(cfg, b, single_thread_s, n_energies=1)
        out["single_thread"] = {"value": one["value"], "unit": one["unit"], "cores": 1, "sample": one["sample"]}
    except ImportError:                                                 # pragma: no cover
        out["single_thread"] = None
    return out


def _cpu_baseline(cfg, b, budget_s=20.0, n_energies=None):
    """The CPU oracle on a bounded sample of the same workload (oracle untuned).

    Up to M = 256 the sample includes the oracle's own lead self-energies (Bloch-mode
    method).  Above that one such solve takes about a minute per energy, so the sample
    times the oracle's sweep and trace only, fed with the batch's self-energies, and the
    rate is compared with the GPU sweep rate."""
    from paper_1010_2627_amd import inputs
    from oracle import leads as OL
    from oracle import rgf as OR
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] + [1])
    except Exception:                                                  # pragma: no cover
        threads = os.cpu_count() or 1
    r0 = b.realizations[0]
    st = b.strips[r0.strip]
    V = st.V_dense()
    E_all = np.asarray(b.energies[r0.strip])
    nE = n_energies or (4 if st.M <= 256 else 2)
    idx = np.linspace(0, len(E_all) - 1, nE).astype(int)
    E = E_all[idx]
    on = r0.onsite
    L = on.shape[0]
    with_sigma = st.M <= 256
    t0 = time.perf_counter()
    if with_sigma:
        sL = np.stack([OL.sigma_modes(st.H0, V, e, "L") for e in E])
        sR = np.stack([OL.sigma_modes(st.H0, V, e, "R") for e in E])
    else:
        M, base = st.M, b.sigma_base[r0.strip]
        sl = [slice(base + int(i) * M * M, base + (int(i) + 1) * M * M) for i in idx]
        sL = np.stack([b.sigmaL[k].view(M, M).cpu().numpy() for k in sl])
        sR = np.stack([b.sigmaR[k].view(M, M).cpu().numpy() for k in sl])
    t_sigma = time.perf_counter() - t0 if with_sigma else 0.0
    # a bounded number of slices keeps the sample inside the time budget
    t1 = time.perf_counter()
    probe = max(4, min(L, 16))
    OR.rgf_forward(st.H0, V, on[:probe], E, sL, sR)
    per_slice = (time.perf_counter() - t1) / probe
    Ls = int(max(probe, min(L, (budget_s - t_sigma) / max(per_slice, 1e-9))))
    t2 = time.perf_counter()
    r = OR.rgf_forward(st.H0, V, on[:Ls], E, sL, sR)
    OR.transmission_lr(sL, sR, r["G1N"])
    t_sweep = time.perf_counter() - t2
    steps = nE * Ls
    what = (f"lead self-energies by the oracle's Bloch-mode method ({t_sigma:.1f} s, pro-rated to "
            f"{Ls}/{L} of the strip), sweep and trace {t_sweep:.1f} s" if with_sigma else
            f"sweep and trace only ({t_sweep:.1f} s; compare with sweep_slice_steps_per_s): one "
            f"Bloch-mode self-energy at M={st.M} takes about a minute per energy on the host")
    return {"value": steps / (t_sigma * Ls / L + t_sweep), "unit": "slice-steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{nE} energies x 1 seed of this workload, first {Ls} of {L} slices; {what}"}


# Knitting of a system of any shape (site by site): a 56 x 256 square-lattice sample with a
# 64 x 16 hole, magnetic flux 0.01 per plaquette, disorder U[-0.5, 0.5], two end leads and a
# 12-site lead on the top edge; 512 energies.  The interface matrix (dimension <= 128) lives in
# registers; the kernel's work is the rank-1 update of that matrix per added site.
GRAPH_WORKLOAD = dict(W=56, L=256, hole=(96, 20, 159, 35), flux=0.01, w=1.0, top=(120, 132), P=512,
                      desc="square-lattice sample 56 x 256 with a 64 x 16 hole, flux 0.01 per plaquette, "
                           "disorder U[-0.5,0.5], leads on both ends and 12 top-edge sites, 512 energies, "
                           "seeded synthetic lead self-energies")


def graph_leg(steps=3):
    import torch
    from paper_1010_2627_amd import inputs, workload
    c = GRAPH_WORKLOAD
    W, L = c["W"], c["L"]
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(L, W, c["hole"]), flux=c["flux"])
    idx = {s: i for i, s in enumerate(g.coords)}
    leads = [[idx[(0, y)] for y in range(W)], [idx[(L - 1, y)] for y in range(W)],
             [idx[(x, W - 1)] for x in range(*c["top"])]]
    P = c["P"]
    E = inputs.midpoint_grid(-3.5, 3.5, P)
    sig = [inputs.synthetic_sigma(len(l), P, seed=2101 + k, rank=max(1, len(l) // 2)) for k, l in enumerate(leads)]
    b = workload.GraphBatch(g, leads, E, inputs.graph_disorder(g, c["w"], seed=10102627), sig)
    inf = b.info
    ws = torch.empty(b.plan.workspace(P), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    T, _, st = b.run(ws=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        T, _, st = b.run(ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / steps
    flops = inf["update_flops"] * P
    Tn = T.cpu().numpy()
    # the automatic plan (groups of sites per step where they pay) beside it
    ba = workload.GraphBatch(g, leads, E, inputs.graph_disorder(g, c["w"], seed=10102627), sig, block=0)
    wsa = torch.empty(ba.plan.workspace(P), dtype=torch.uint8, device="cuda")
    ta, (Ta, _, sta) = _timed_call(lambda: ba.run(ws=wsa), stream, steps)
    auto = {"sites_per_step": ba.info["block"], "interface_dim_max": ba.info["dim"], "steps": ba.info["n_steps"],
            "seconds_per_launch": round(ta, 5), "site_steps_per_s": inf["n_steps"] * P / ta,
            "speedup": t / ta, "problems_with_status": int((sta.cpu().numpy() != 0).sum()),
            "max_dT_vs_site_by_site": float(np.abs(Ta.cpu().numpy() - Tn).max())}
    return {"workload": c["desc"], "sites": inf["nsite"], "norb": inf["norb"], "leads": len(leads),
            "interface_dim_max": inf["dim"], "site_steps_per_launch": inf["n_steps"] * P,
            "seconds_per_launch": round(t, 5), "site_steps_per_s": inf["n_steps"] * P / t,
            "t_matrices_per_s": P / t, "problems_with_status": int((st.cpu().numpy() != 0).sum()),
            "row_sum_check_max": float(np.abs(Tn[:, 0, 1:].sum(axis=1) - Tn[:, 1:, 0].sum(axis=1)).max()),
            "automatic_groups": auto,
            "roofline": {"bound": "alu", "achieved": flops / t / 1e12, "peak": PEAK_TFLOPS["fp64"],
                         "unit": "TFLOP/s", "frac": flops / t / 1e12 / PEAK_TFLOPS["fp64"],
                         "kernel": "graph_knit_kernel<512, 8, 4, true, 1> (interface matrix in registers)",
                         "flops_per_launch": flops,
                         "flops_per_site_step": "8 norb D_t^2 (rank-norb update of the interface matrix)"}}


# Knitting with an interface wider than the register mode holds (the matrix in the workgroup's
# slab): a 96 x 96 sample with a 30 x 16 hole, flux 0.01, disorder U[-0.5, 0.5], leads on both
# ends, 256 energies; site by site against the automatic groups of sites per step.
GRAPH_WIDE_WORKLOAD = dict(W=96, L=96, hole=(30, 40, 60, 56), flux=0.01, w=1.0, P=256,
                           desc="square-lattice sample 96 x 96 with a 30 x 16 hole, flux 0.01 per plaquette, "
                                "disorder U[-0.5,0.5], leads on both ends, 256 energies, seeded synthetic lead "
                                "self-energies")


def graph_wide_leg(steps=2):
    import torch
    from paper_1010_2627_amd import inputs, workload
    c = GRAPH_WIDE_WORKLOAD
    W, L, P = c["W"], c["L"], c["P"]
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(L, W, c["hole"]), flux=c["flux"])
    idx = {s: i for i, s in enumerate(g.coords)}
    leads = [[idx[(0, y)] for y in range(W) if (0, y) in idx], [idx[(L - 1, y)] for y in range(W) if (L - 1, y) in idx]]
    E = inputs.midpoint_grid(-3.5, 3.5, P)
    sig = [inputs.synthetic_sigma(len(l), P, seed=3101 + k, rank=max(1, len(l) // 2)) for k, l in enumerate(leads)]
    ons = inputs.graph_disorder(g, c["w"], seed=20102627)
    stream = torch.cuda.current_stream()
    out, Ts = {"workload": c["desc"], "sites": g.N}, []
    for name, block in (("site_by_site", None), ("automatic_groups", 0)):
        b = workload.GraphBatch(g, leads, E, ons, sig, block=block)
        inf = b.info
        ws = torch.empty(b.plan.workspace(P), dtype=torch.uint8, device="cuda")
        t, (T, _, st) = _timed_call(lambda: b.run(ws=ws), stream, steps)
        Ts.append(T.cpu().numpy())
        out[name] = {"sites_per_step": inf["block"], "interface_dim_max": inf["dim"], "steps": inf["n_steps"],
                     "seconds_per_launch": round(t, 5), "site_steps_per_s": (g.N - len(leads[0])) * P / t,
                     "problems_with_status": int((st.cpu().numpy() != 0).sum())}
    out["speedup"] = out["site_by_site"]["seconds_per_launch"] / out["automatic_groups"]["seconds_per_launch"]
    out["max_dT_groups_vs_site_by_site"] = float(np.abs(Ts[1] - Ts[0]).max())
    return out


def _timed_call(fn, stream, reps=1):
    """Run fn once untimed, then `reps` times between two events on `stream`; (seconds per call, result)."""
    import torch
    out = fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        out = fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps, out


def _cut_table(b, knit, n_slices, ldos_width):
    """The batch's problem table with every strip cut to its first n_slices slices; ldos_off packs
    [L][ldos_width(strip)] per problem."""
    host = b.probs.host.copy()
    host["L"] = np.minimum(host["L"], n_slices)
    w = np.array([ldos_width(b.strips[int(x)]) for x in host["strip"]], dtype=np.int64)
    sizes = host["L"].astype(np.int64) * w
    host["ldos_off"] = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    return knit.ProblemTable.from_host(host), host


def next_rows(b, knit, G1Np, Tp, rankL, rankR, stream, n_slices=64):
    """Timing of the three observables built on the sweep: transmission eigenvalues and the Fano
    factor from the headline projected propagator (every problem), injected densities and site
    currents, and the conductance matrix with one side lead (every problem cut to its first
    n_slices slices).  Each carries its algorithmic flop count, the fraction of the FP64 peak
    it reaches and a check that holds at any size."""
    import torch
    res = {}
    Ms = np.array([b.strips[int(s)].M for s in b.probs.host["strip"]], dtype=np.float64)
    P = b.P
    rl, rr = rankL.astype(np.float64), rankR.astype(np.float64)

    # transmission eigenvalues: t~ = P_N C_R (r_L x M x r_R), tau = t~^+ t~ on the smaller side,
    # Householder tridiagonalisation (16/3 n^3), bisection not counted
    n, m = np.minimum(rl, rr), np.maximum(rl, rr)
    fl = float(np.sum(8.0 * rl * Ms * rr + 8.0 * n * n * m + 16.0 / 3.0 * n ** 3))
    t, (tn, nch, T, fano) = _timed_call(lambda: b.transmission_eigenvalues(G1Np, stream), stream)
    tn_h, T_h = tn.cpu().numpy(), T.cpu().numpy()
    res["transmission_eigenvalues"] = {
        "problems": P, "seconds": round(t, 4), "problems_per_s": P / t,
        "tflops": fl / t / 1e12, "frac_of_fp64_peak": fl / t / 1e12 / PEAK_TFLOPS["fp64"],
        "flops_per_problem": "8 r_L M r_R + 8 n^2 max(r_L, r_R) + 16/3 n^3, n = min(r_L, r_R)",
        "kernel": "transmission_eigs_kernel (vector FP64, one workgroup per problem)",
        "max_rel_dT_sum_Tn_vs_trace": float((np.abs(tn_h.sum(axis=1) - Tp) / np.maximum(1.0, Tp)).max()),
        "max_rel_dT_trace_vs_headline": float((np.abs(T_h - Tp) / np.maximum(1.0, Tp)).max()),
        "Tn_range": [float(tn_h.min()), float(tn_h.max())],
        "fano_range": [float(fano.min()), float(fano.max())]}
    del tn, nch, T, fano
    progress(f"transmission eigenvalues: {t:.3f} s for {P} problems")

    # injected densities and currents: forward inverse (8 M^3) and two rank-r propagations (16 M^2 r)
    # per slice
    sub, host = _cut_table(b, knit, n_slices, lambda s: s.W)
    Lc = host["L"].astype(np.float64)
    fl = float(np.sum((8.0 * Ms ** 3 + 16.0 * Ms ** 2 * rl) * Lc))
    ws = torch.empty(max(knit._lib.knit_local_observables_workspace(
        knit.strip_table(b.dstrips), len(b.dstrips), knit._ptr(sub.host), sub.P, 0), 1),
        dtype=torch.uint8, device="cuda")
    t, (blk, blk_off, jl, jt, st) = _timed_call(
        lambda: knit.knit_local_observables(b.dstrips, sub, b.onsite, b.sigmaL, b.sigmaR, b.CL, 0, stream,
                                            workspace=ws), stream)
    del ws
    # current conservation: the same current crosses every cut of a strip; the transverse inflows
    # of a slice cancel
    jl_h, jt_h = jl.cpu().numpy(), jt.cpu().numpy()
    spread, tsum = 0.0, 0.0
    for p in range(P):
        o, L, W = int(host["ldos_off"][p]), int(host["L"][p]), b.strips[int(host["strip"][p])].W
        cur = jl_h[o:o + L * W].reshape(L, W)[1:].sum(axis=1)
        spread = max(spread, float((cur.max() - cur.min()) / max(1.0, abs(cur).max())))
        tsum = max(tsum, float(np.abs(jt_h[o:o + L * W].reshape(L, W).sum(axis=1)).max() / max(1.0, abs(cur).max())))
    res["local_observables"] = {
        "slices_per_problem": f"min(L, {n_slices})", "problems": P, "slice_steps": int(Lc.sum()),
        "seconds": round(t, 4), "slice_steps_per_s": float(Lc.sum()) / t,
        "tflops": fl / t / 1e12, "frac_of_fp64_peak": fl / t / 1e12 / PEAK_TFLOPS["fp64"],
        "flops_per_slice_step": "8 M^3 + 16 M^2 r (slice inverse, forward and reverse rank-r "
                                "propagation; checkpoint recomputation not counted)",
        "kernel": "lesser_mfma_kernel (FP64 MFMA)",
        "problems_with_status": int((st.cpu().numpy() != 0).sum()),
        "max_rel_spread_of_cut_currents": spread, "max_rel_transverse_inflow_sum": tsum}
    del blk, jl, jt, st
    progress(f"local observables: {t:.3f} s for {int(Lc.sum())} slice-steps")

    # conductance matrix with one side lead on the middle slice of every cut strip (a lead of the
    # strip's own cross section: Sigma_L and C_L of the same energy attached there)
    sub, host = _cut_table(b, knit, n_slices, lambda s: s.M)
    side = np.zeros((P, 1), dtype=knit.LEAD_DTYPE)
    side["slice"][:, 0] = host["L"] // 2
    side["sigma_off"][:, 0] = host["sigma_off"]
    Lc = host["L"].astype(np.float64)
    s_mid = (host["L"] // 2).astype(np.float64)
    # forward and reverse inverses (16 M^3 per slice), one full-block inverse per lead slice (3),
    # columns and rows of each lead carried from its slice to slice 0 (16 M^2 r each per slice)
    fl = float(np.sum(16.0 * Ms ** 3 * Lc + 3 * 8.0 * Ms ** 3
                      + 16.0 * Ms ** 2 * (rr * (Lc - 1) + rl * s_mid)))
    ws = torch.empty(max(knit._lib.knit_conductance_matrix_workspace(
        knit.strip_table(b.dstrips), len(b.dstrips), knit._ptr(sub.host), sub.P, 1, 0), 1),
        dtype=torch.uint8, device="cuda")
    t, (Tm, st) = _timed_call(
        lambda: knit.knit_conductance_matrix(b.dstrips, sub, b.onsite, b.sigmaL, b.sigmaR, b.CL, b.CR, side,
                                             b.sigmaL, b.CL, 0, stream, workspace=ws), stream)
    del ws
    Tm_h = Tm.cpu().numpy()
    rs = np.abs(Tm_h.sum(axis=2) - Tm_h.sum(axis=1)).max(axis=1) / np.maximum(1.0, np.abs(Tm_h).max(axis=(1, 2)))
    res["conductance_matrix"] = {
        "slices_per_problem": f"min(L, {n_slices})", "leads": 3, "problems": P, "slice_steps": int(Lc.sum()),
        "seconds": round(t, 4), "slice_steps_per_s": float(Lc.sum()) / t, "matrices_per_s": P / t,
        "tflops": fl / t / 1e12, "frac_of_fp64_peak": fl / t / 1e12 / PEAK_TFLOPS["fp64"],
        "flops_per_problem": "16 M^3 L + 24 M^3 + 16 M^2 (r_R (L-1) + r_X s_X)",
        "kernel": "multiterminal_mfma_kernel (FP64 MFMA)",
        "problems_with_status": int((st.cpu().numpy() != 0).sum()),
        "max_rel_row_minus_column_sum": float(rs.max())}
    del Tm, st
    progress(f"conductance matrix: {t:.3f} s for {int(Lc.sum())} slice-steps")
    return res


def stated_form(b, knit, G1Np, ws_for, T64, wall64, nopen, steps, autotuned):
    """The uneven batch in its stated form: FP32 elimination with FP64 refinement on the projected
    path, the whole step (self-energies, broadening factors, projected sweep with its FP64 second
    launch, trace) captured in one graph and replayed; compared with the eager FP64 step."""
    import torch
    prec = "fp32_refine"
    ws_for(prec)

    def body():
        b.compute_sigmas()
        b.compute_gamma_factors()
        _, _, status = knit.knit_rgf_sweep_projected(b.dstrips, b.probs, b.onsite, b.sigmaL, b.sigmaR, b.CL,
                                                     G1Np=G1Np, workspace=ws_for(prec), precision=prec)
        return b.transmission_projected(G1Np), status

    s2 = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s2):
        T_e, st_e = body()
        T_e, st_e = T_e.clone(), st_e.clone()
    torch.cuda.synchronize()
    progress("stated form: eager refined step done")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s2):
        T_g, st_g = body()
    torch.cuda.synchronize()
    progress("stated form: step captured")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(steps):
        with torch.cuda.stream(s2):
            e0.record(s2)
            g.replay()
            e1.record(s2)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
        progress(f"stated form: replay {len(ts)}/{steps}: {ts[-1]:.2f} s")
    t = float(np.mean(ts))
    Tg, Te, st = T_g.cpu().numpy(), T_e.cpu().numpy(), st_g.cpu().numpy()
    d = np.abs(Tg - T64) / np.maximum(1, nopen)
    return {"precision": prec, "graph_captured": True, "autotuned": bool(autotuned),
            "seconds_per_step": round(t, 4), "slice_steps_per_s": b.slice_steps() / t,
            "speed_vs_fp64_projected_eager_step": wall64 / t,
            "replay_equals_eager": bool(np.array_equal(Tg, Te)),
            "max_dT_per_open_channel_vs_fp64": float(d.max()),
            "points_within_1e-6_per_channel": f"{int((d <= TOL_PER_CHANNEL).sum())}/{len(d)}",
            "problems_recomputed_in_fp64": int(((st & knit.KNIT_P_FALLBACK) != 0).sum()),
            "problems_with_status": int(((st & ~knit.KNIT_P_FALLBACK) != 0).sum())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32+refinement step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ldos", action="store_true", help="skip the LDOS (backward sweep) timing")
    ap.add_argument("--no-observables", action="store_true",
                    help="skip the timing of transmission eigenvalues, local observables and the conductance "
                         "matrix")
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline (projected FP64) step only: no other paths, no CPU baseline "
                         "(for profiler runs)")
    ap.add_argument("--autotune", action="store_true",
                    help="time the sweep's launch shapes on a sample of the batch first and use the best")
    ap.add_argument("--graph-only", action="store_true",
                    help="time only the knitting of a system of any shape (its JSON object alone)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device copy of this size (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.headline_only:
        args.no_mixed = args.no_ldos = args.no_cpu_baseline = args.no_observables = True
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (multi-GPU sharding "
                                   "is described, not run)"}))
        sys.exit(2)

    import torch
    from paper_1010_2627_amd import knit

    cfg = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    if args.graph_only:
        leg = graph_leg()
        leg["wide_interface"] = graph_wide_leg()
        print(json.dumps(leg))
        return
    if cfg["kind"] == "sampler":
        sampler_bench(args, cfg)
        return
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    b = build_batch(cfg)
    Ms = np.array([b.strips[int(s)].M for s in b.probs.host["strip"]], dtype=np.float64)
    M = int(Ms.max())
    steps_per_pass = b.slice_steps()
    flops_full = float(np.sum(16.0 * Ms ** 3 * b.probs.host["L"]))
    G1N = torch.empty(int(np.sum(Ms ** 2)), dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()
    wss = {}

    def ws_for(prec):
        if prec not in wss:
            wss[prec] = torch.empty(max(knit.knit_rgf_sweep_workspace(b.dstrips, b.probs, prec), 1),
                                    dtype=torch.uint8, device="cuda")
        return wss[prec]

    def one_step(prec, events=None):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record(stream)
        b.compute_sigmas()
        e[1].record(stream)
        _, _, _, status = knit.knit_rgf_sweep(b.dstrips, b.probs, b.onsite, b.sigmaL, b.sigmaR, prec,
                                              G1N=G1N, workspace=ws_for(prec))
        e[2].record(stream)
        T = b.transmission(G1N)[0]
        e[3].record(stream)
        if events is not None:
            events.append(e)
        return T, status

    G1Np = torch.empty_like(G1N)

    def one_step_projected(events=None, prec="fp64"):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record(stream)
        b.compute_sigmas()
        b.compute_gamma_factors()
        e[1].record(stream)
        _, _, status = knit.knit_rgf_sweep_projected(b.dstrips, b.probs, b.onsite, b.sigmaL, b.sigmaR, b.CL,
                                                     G1Np=G1Np, workspace=ws_for(prec), precision=prec)
        e[2].record(stream)
        T = b.transmission_projected(G1Np)
        e[3].record(stream)
        if events is not None:
            events.append(e)
        return T, status

    def timed(prec, steps):
        evs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            if prec.startswith("projected"):
                T, status = one_step_projected(evs, "fp32_refine" if prec == "projected_refine" else "fp64")
            else:
                T, status = one_step(prec, evs)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        ph = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])]
                       for e in evs]) / 1e3
        st = status.cpu().numpy()
        bad = int(((st & ~knit.KNIT_P_FALLBACK) != 0).sum()) + int((b.sigma_status.cpu().numpy() != 0).sum())
        timed.fallbacks = int(((st & knit.KNIT_P_FALLBACK) != 0).sum())
        return T.cpu().numpy(), wall, ph.mean(axis=0), bad

    progress(f"workload {args.workload}: {b.P} problems, M<={M}, {steps_per_pass} slice-steps per step")
    tuning = None
    if args.autotune:
        from paper_1010_2627_amd import autotune
        b.compute_sigmas()
        tuning = {}
        for prec in ("fp64",) if args.no_mixed else ("fp64", "fp32_refine"):
            r = autotune.tune_batch(b, prec, sample_slices=32, max_problems=2048)
            tuning[prec] = {"Mp": r["Mp"], "best": r["best"],
                            "candidates_ms": [[c, round(t * 1e3, 2)] for c, t in r["results"]]}
            progress(f"autotune {prec}: {r['best']}")
    for i in range(args.warmup):
        one_step_projected()
        torch.cuda.synchronize()
        progress(f"warmup step {i + 1}/{args.warmup} done")
    Tp, wallp, (tsp, twp, ttp), badp = timed("projected", args.steps)
    progress(f"fp64 projected: {args.steps} timed step(s), {wallp:.2f} s/step (self-energies and "
             f"broadening factors {tsp:.2f} s, sweep {twp:.2f} s, trace {ttp:.3f} s)")
    rankL, _ = b.problem_ranks()
    # algorithmic flops of the projected sweep per slice: the slice inverse (8 M^3) and the
    # product P_{n-1} V^+ g_n with r = rank(Gamma_L) rows (8 M^2 r)
    flops_proj = float(np.sum((8.0 * Ms ** 3 + 8.0 * Ms ** 2 * rankL) * b.probs.host["L"]))
    if not args.headline_only:
        T64, wall64, (ts64, tw64, tt64), bad64 = timed("fp64", 1)
        progress(f"fp64 full propagator: {wall64:.2f} s/step (sweep {tw64:.2f} s)")
    nopen = open_channels(b)
    ldos_info = None
    if not args.no_ldos:
        # local density of states (backward sweep with checkpoints): the whole batch with every
        # strip cut to its first 64 slices
        host = b.probs.host.copy()
        host["L"] = np.minimum(host["L"], 64)
        # LDOS blocks of the cut strips, packed: every value of the output is written
        Ms_sub = np.array([b.strips[int(x)].M for x in host["strip"]], dtype=np.int64)
        sizes = host["L"].astype(np.int64) * Ms_sub
        host["ldos_off"] = np.concatenate([[0], np.cumsum(sizes)[:-1]])
        sub = knit.ProblemTable.from_host(host)
        wsl = torch.empty(max(knit.knit_ldos_workspace(b.dstrips, sub, "fp64", 0), 1), dtype=torch.uint8,
                          device="cuda")
        knit.knit_ldos(b.dstrips, sub, b.onsite, b.sigmaL, b.sigmaR, "fp64", workspace=wsl)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ld, lst = knit.knit_ldos(b.dstrips, sub, b.onsite, b.sigmaL, b.sigmaR, "fp64", workspace=wsl)
        e1.record(stream)
        torch.cuda.synchronize()
        tl = e0.elapsed_time(e1) / 1e3
        steps_l = int(host["L"].sum())
        Ms_l = np.array([b.strips[int(x)].M for x in host["strip"]], dtype=np.float64)
        fl = float(np.sum(32.0 * Ms_l ** 3 * host["L"]))
        ldos_info = {"slices_per_problem": "min(L, 64)", "seconds": round(tl, 4),
                     "slice_steps_per_s": steps_l / tl,
                     "tflops_at_32M3": fl / tl / 1e12,
                     "frac_of_fp64_peak": fl / tl / 1e12 / PEAK_TFLOPS["fp64"],
                     "flops_per_slice_step": "32*M^3 (forward inverse, checkpoint recompute, two products)",
                     "problems_with_status": int((lst.cpu().numpy() != 0).sum()),
                     "min_ldos": float(ld[:int(sizes.sum())].min())}
        del wsl, ld
        progress(f"ldos: {tl:.2f} s for {steps_l} slice-steps")

    observables = None
    if not args.no_observables:
        rankR = b.problem_ranks()[1]
        observables = next_rows(b, knit, G1Np, Tp, rankL, rankR, stream)

    achieved = flops_proj / twp / 1e12
    sweep_threads = knit.knit_sweep_tuning_get("fp64", knit.tuning_class((M + 31) // 32 * 32))["threads"]
    tr = MEASURED_TRAFFIC.get(args.workload)
    traffic = tr["bytes"] if tr and tr["sha"] == sweep_source_sha() else None
    out = {
        "metric": METRIC,
        "value": steps_per_pass / wallp,
        "unit": "slice-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wallp * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": cfg["desc"], "slice_dim_M_max": M,
                   "problems": b.P, "slice_steps_per_step": steps_per_pass,
                   "headline_precision": "fp64, projected propagator C_L^+ G_1n (meets the T tolerance "
                                         "at every point)"},
        "phases_s": {"lead_selfenergy_dd_and_gamma_factors": round(float(tsp), 4), "sweep": round(float(twp), 4),
                     "trace": round(float(ttp), 4)},
        "sweep_slice_steps_per_s": steps_per_pass / twp,
        "t_points_per_s": b.P / wallp,
        "problems_with_status": badp,
        "gamma_rank_range": [int(rankL.min()), int(rankL.max())],
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["fp64"], "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (calibrated counters)",
                     "traffic_source": tr["profile"] if traffic else None,
                     "counters": tr["counters"] if traffic else None,
                     "kernel": f"sweep_mfma_kernel<double, double, false, {sweep_threads}, true> (FP64 MFMA, "
                               f"projected)",
                     "flops_per_slice_step": "8*M^3 + 8*M^2*r (inverse + projected propagator, r = rank "
                                             "Gamma_L)",
                     "flops_per_step": flops_proj},
        "fp64_full_propagator": None if args.headline_only else {
            "slice_steps_per_s": steps_per_pass / wall64,
            "sweep_s": round(float(tw64), 4),
            "sweep_slice_steps_per_s": steps_per_pass / tw64,
            "tflops_at_16M3": flops_full / tw64 / 1e12,
            "frac_of_fp64_peak": flops_full / tw64 / 1e12 / PEAK_TFLOPS["fp64"],
            "projected_sweep_speedup": tw64 / twp,
            "max_dT_per_open_channel_projected_vs_full": float((np.abs(Tp - T64) / np.maximum(1, nopen)).max()),
            "problems_with_status": bad64,
        },
    }
    if not args.no_mixed:
        # FP32 elimination with FP64-residual Newton steps on each slice inverse; the propagator
        # (whole G_1n, or the projected rows) is an FP64 product of the refined inverse
        mixed = {}
        for name, prec, ref_T, ref_sweep, flops in (("projected", "projected_refine", Tp, twp, flops_proj),
                                                    ("full", "fp32_refine", T64, tw64, flops_full)):
            Tm, wallm, (tsm, twm, ttm), badm = timed(prec, 1)
            fb = timed.fallbacks
            progress(f"fp32_refine {name}: {wallm:.2f} s/step (sweep {twm:.2f} s, {fb} problems recomputed in FP64)")
            dT = np.abs(Tm - ref_T)
            rel = dT / np.maximum(1, nopen)
            ok = rel <= TOL_PER_CHANNEL
            am = flops / twm / 1e12
            mixed[name] = {
                "slice_steps_per_s": steps_per_pass / wallm,
                "sweep_s": round(float(twm), 4),
                "sweep_slice_steps_per_s": steps_per_pass / twm,
                "algorithmic_tflops": am,
                "frac_of_fp32_peak": am / PEAK_TFLOPS["fp32_refine"],
                "sweep_speedup_vs_fp64_same_path": ref_sweep / twm,
                "max_dT_per_open_channel_vs_fp64": float(rel.max()),
                "median_dT_per_open_channel_vs_fp64": float(np.median(rel)),
                "max_abs_dT_vs_fp64": float(dT.max()),
                "points_within_1e-6_per_channel": f"{int(ok.sum())}/{b.P}",
                "t_points_per_s_within_tol": float(ok.sum()) / wallm,
                "problems_recomputed_in_fp64": fb,
                "problems_with_status": badm,
            }
        out["fp32_refine"] = mixed
    out["n_open_range"] = [int(nopen.min()), int(nopen.max())]
    if ldos_info is not None:
        out["ldos"] = ldos_info
    if observables is not None:
        out["observables"] = observables
    if tuning is not None:
        out["autotune"] = tuning
    if args.workload == "c3" and not args.headline_only:
        out["c3_stated_form"] = stated_form(b, knit, G1Np, ws_for, Tp, wallp, nopen, args.steps,
                                            autotuned=tuning is not None)
        progress("c3 stated form done")
    if not args.headline_only:
        out["graph_knitting"] = graph_leg()
        out["graph_knitting"]["wide_interface"] = graph_wide_leg()
        progress("graph knitting done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, b)
        progress("cpu baseline done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
