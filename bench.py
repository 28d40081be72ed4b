"""Benchmark of the two-lead strip transport path on one MI355X.

One step = the whole T(E) path over the batch, inputs resident in HBM:
lead self-energies of both leads for every energy (double-double decimation),
the slice sweep of every (energy, realization) problem, and the Fisher-Lee
trace.  The headline precision is the FP32 matrix-core sweep with one
FP64-residual refinement per slice inverse; the FP64 sweep is timed beside it
on the same batch, and every mixed-precision T(E) is compared with the FP64
one per open channel.

Prints one JSON line (see the fields below).  --gpus above 1 is refused: this
build runs on one GPU.
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

WORKLOADS = {
    # name: (builder kwargs, description)
    "c2": dict(kind="square", W=128, L=1024, w=2.0, n_energies=256, n_seeds=16,
               desc="square-lattice strip W=128 (M=128), L=1024, disorder U[-1,1], "
                    "256 midpoint energies in (-3.9,3.9) x 16 seeds = 4096 problems"),
    "c2w256": dict(kind="square", W=256, L=1024, w=2.0, n_energies=64, n_seeds=8,
                   desc="square-lattice strip W=256 (M=256), L=1024, disorder U[-1,1], "
                        "64 energies x 8 seeds = 512 problems"),
    "c4": dict(kind="rashba", W=256, L=512, w=2.0, n_energies=64, n_seeds=8,
               desc="spinful square lattice W=256 (M=512), Rashba 0.2t, Zeeman 0.1t, L=512, "
                    "disorder U[-1,1], 64 energies x 8 seeds = 512 problems"),
    "c1": dict(kind="square", W=16, L=64, w=1.0, n_energies=64, n_seeds=1,
               desc="square-lattice strip W=16, L=64, disorder U[-0.5,0.5], 64 energies"),
}


def build_batch(cfg):
    from paper_1010_2627_amd import workload
    if cfg["kind"] == "square":
        return workload.square_batch(cfg["W"], cfg["L"], cfg["w"], cfg["n_energies"], cfg["n_seeds"])
    return workload.rashba_batch(cfg["W"], cfg["L"], cfg["w"], cfg["n_energies"], cfg["n_seeds"])


def open_channels(cfg, energies):
    """N_open(E) of the lead = transmission of the clean strip (one slice), on the GPU path."""
    import torch
    from paper_1010_2627_amd import workload
    if cfg["kind"] == "square":
        b = workload.square_batch(cfg["W"], 1, 0.0, 1, 1)
    else:
        b = workload.rashba_batch(cfg["W"], 1, 0.0, 1, 1)
    b = workload.Batch(b.strips, b.realizations, [np.asarray(energies)])
    b.compute_sigmas()
    G1N, _, _, st = b.sweep("fp64", gnn=False)
    T = b.transmission(G1N)[0]
    torch.cuda.synchronize()
    return np.rint(T.cpu().numpy()).astype(np.int64)


def cpu_baseline(cfg, budget_s=20.0):
    """The CPU oracle on a bounded sample of the same workload (oracle untuned)."""
    from paper_1010_2627_amd import inputs
    from oracle import leads as OL
    from oracle import rgf as OR
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:                                                  # pragma: no cover
        threads = os.cpu_count() or 1
    st = inputs.square_strip(cfg["W"]) if cfg["kind"] == "square" else inputs.rashba_strip(cfg["W"])
    V = st.V_dense()
    E_all = inputs.midpoint_grid(-3.9, 3.9, cfg["n_energies"])
    nE = 4
    E = E_all[np.linspace(0, len(E_all) - 1, nE).astype(int)]
    on = inputs.onsite_disorder(st, cfg["L"], cfg["w"], inputs.SEED_BASE)
    # bounded number of slices so the sample stays within the time budget
    t0 = time.perf_counter()
    sL = np.stack([OL.sigma_modes(st.H0, V, e, "L") for e in E])
    sR = np.stack([OL.sigma_modes(st.H0, V, e, "R") for e in E])
    t_sigma = time.perf_counter() - t0
    L = cfg["L"]
    t1 = time.perf_counter()
    probe = max(4, min(L, 32))
    OR.rgf_forward(st.H0, V, on[:probe], E, sL, sR)
    per_slice = (time.perf_counter() - t1) / probe
    Ls = int(max(probe, min(L, (budget_s - t_sigma) / max(per_slice, 1e-9))))
    t2 = time.perf_counter()
    r = OR.rgf_forward(st.H0, V, on[:Ls], E, sL, sR)
    OR.transmission_lr(sL, sR, r["G1N"])
    t_sweep = time.perf_counter() - t2
    steps = nE * Ls
    return {"value": steps / (t_sigma * Ls / L + t_sweep), "unit": "slice-steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{nE} energies x 1 seed of this workload, first {Ls} of {L} slices; "
                      f"lead self-energies by the Bloch-mode method ({t_sigma:.1f} s, pro-rated to "
                      f"{Ls}/{L} of the strip), sweep {t_sweep:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32_refine", choices=["fp32_refine", "fp32", "fp64"])
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_1010_2627_amd import knit

    cfg = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    b = build_batch(cfg)
    M = b.strips[0].M
    steps_per_pass = b.slice_steps()
    flops_per_pass = 16.0 * M ** 3 * steps_per_pass
    ws = torch.empty(max(knit.knit_rgf_sweep_workspace(b.dstrips, b.probs, args.precision), 1),
                     dtype=torch.uint8, device="cuda")
    G1N = torch.empty(b.P * M * M, dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()

    def one_step(prec=args.precision, events=None):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record(stream)
        b.compute_sigmas()
        e[1].record(stream)
        _, _, _, status = knit.knit_rgf_sweep(b.dstrips, b.probs, b.onsite, b.sigmaL, b.sigmaR, prec,
                                              G1N=G1N, workspace=ws)
        e[2].record(stream)
        T = b.transmission(G1N)[0]
        e[3].record(stream)
        if events is not None:
            events.append(e)
        return T, status

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        T, status = one_step(events=evs)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    ph = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])] for e in evs]) / 1e3
    t_sigma, t_sweep, t_trace = ph.mean(axis=0)
    T_mixed = T.cpu().numpy()
    bad_status = int((status.cpu().numpy() != 0).sum()) + int((b.sigma_status.cpu().numpy() != 0).sum())

    extra = {}
    if not args.no_fp64_compare and args.precision != "fp64":
        ws64 = torch.empty(max(knit.knit_rgf_sweep_workspace(b.dstrips, b.probs, "fp64"), 1),
                           dtype=torch.uint8, device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        knit.knit_rgf_sweep(b.dstrips, b.probs, b.onsite, b.sigmaL, b.sigmaR, "fp64", G1N=G1N, workspace=ws64)
        e0.record(stream)
        knit.knit_rgf_sweep(b.dstrips, b.probs, b.onsite, b.sigmaL, b.sigmaR, "fp64", G1N=G1N, workspace=ws64)
        e1.record(stream)
        T64 = b.transmission(G1N)[0].cpu().numpy()
        t64 = e0.elapsed_time(e1) / 1e3
        del ws64
        nopen = open_channels(cfg, b.energies[0])
        nopen_p = np.tile(nopen, len(b.realizations))
        dT = np.abs(T_mixed - T64)
        rel = dT / np.maximum(1, nopen_p)
        ok = rel <= 1e-6
        extra = {
            "fp64_sweep_s": round(t64, 4),
            "fp64_slice_steps_per_s": steps_per_pass / t64,
            "fp64_frac_of_fp64_peak": flops_per_pass / t64 / 1e12 / PEAK_TFLOPS["fp64"],
            "mixed_over_fp64_sweep_speedup": t64 / t_sweep,
            "max_dT_per_open_channel_vs_fp64": float(rel.max()),
            "max_abs_dT_vs_fp64": float(dT.max()),
            "points_within_1e-6_per_channel": int(ok.sum()),
            "t_points_per_s": float(ok.sum()) / wall,
        }
    achieved = flops_per_pass / t_sweep / 1e12
    peak = PEAK_TFLOPS[args.precision]
    out = {
        "metric": METRIC,
        "value": steps_per_pass / wall,
        "unit": "slice-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32_refine": "f32+f64", "fp32": "f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "description": cfg["desc"], "slice_dim_M": M,
                   "problems": b.P, "slice_steps_per_step": steps_per_pass,
                   "precision": args.precision},
        "phases_s": {"lead_selfenergy_dd": round(float(t_sigma), 4), "sweep": round(float(t_sweep), 4),
                     "trace": round(float(t_trace), 4)},
        "sweep_slice_steps_per_s": steps_per_pass / t_sweep,
        "problems_with_status": bad_status,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "sweep_mfma_kernel", "flops_per_slice_step": "16*M^3"},
    }
    out.update(extra)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
