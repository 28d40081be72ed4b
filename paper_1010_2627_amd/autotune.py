"""Autotuner for the batched matrix-core sweep's launch shape.

The persistent sweep kernel has four launch knobs, kept per precision and
padded-slice class in the library's tuning table (``knit_sweep_tuning_set``):

* threads per workgroup, 256 or 512. One panel row per thread, so at least
  the padded slice size Mp.
* workgroups per compute unit the grid is sized for, 1 or 2. With two, two
  problems share a compute unit and hide each other's barrier latency.
* queue order: the problem table's order, or longest-processing-time first
  on the cost Mp³·L.
* outer panel width of the blocked elimination, 64 or 128. Each outer panel
  is one pass over the slice matrix in memory; wider panels make fewer passes
  but a longer restricted elimination inside each.

``tune_batch`` times every valid candidate on a sample of a batch and
installs the fastest. The sample is the batch's own problems with each strip
cut to its first ``sample_slices`` slices, which keeps the per-slice cost and
the mix of slice sizes. ``save`` and ``load`` keep the table as JSON, keyed
by precision and class.
"""

from __future__ import annotations

import itertools
import json
import time

import numpy as np
import torch

from . import knit as K


def candidates(Mp: int):
    """Every valid tuning entry for padded slice size Mp."""
    out = []
    for threads, wg, order, outer in itertools.product((256, 512), (1, 2), (0, 1), (64, 128)):
        if threads < Mp or outer > Mp:
            continue
        out.append({"threads": threads, "wg_per_cu": wg, "order": order, "outer": outer})
    return out


def _sample_table(batch, sample_slices: int, max_problems: int | None):
    host = batch.probs.host.copy()
    if max_problems is not None and len(host) > max_problems:
        # keep the cost mix: every k-th problem
        idx = np.linspace(0, len(host) - 1, max_problems).astype(np.int64)
        host = host[idx]
    host["L"] = np.minimum(host["L"], sample_slices)
    return K.ProblemTable.from_host(host, batch.device)


def tune_batch(batch, precision: str = "fp64", sample_slices: int = 32, max_problems: int | None = None,
               repeats: int = 2, install: bool = True, verbose: bool = False) -> dict:
    """Time every candidate launch shape on a sample of ``batch``.

    Returns {"precision", "cls", "Mp", "best", "results": [(entry, seconds), ...]}.
    The sample's outputs go to scratch buffers; the batch is not modified.
    """
    Mmax = max(int(s.M) for s in batch.strips)
    Mp = (Mmax + 31) // 32 * 32
    cls = K.tuning_class(Mp)
    probs = _sample_table(batch, sample_slices, max_problems)
    if batch.sigmaL is None:
        raise ValueError("compute or set the batch's self-energies first")
    ws = torch.empty(max(K.knit_rgf_sweep_workspace(batch.dstrips, probs, precision), 1), dtype=torch.uint8,
                     device=batch.device)
    before = K.knit_sweep_tuning_get(precision, cls)
    results = []
    try:
        for cand in candidates(Mp):
            K.knit_sweep_tuning_set(precision, cls, **cand)
            K.knit_rgf_sweep(batch.dstrips, probs, batch.onsite, batch.sigmaL, batch.sigmaR, precision,
                             workspace=ws)          # first launch of this shape, untimed
            torch.cuda.synchronize()
            best = float("inf")
            for _ in range(repeats):
                t0 = time.perf_counter()
                K.knit_rgf_sweep(batch.dstrips, probs, batch.onsite, batch.sigmaL, batch.sigmaR, precision,
                                 workspace=ws)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            results.append((cand, best))
            if verbose:
                print(f"  {precision} Mp={Mp} {cand}: {best * 1e3:.2f} ms", flush=True)
    finally:
        K.knit_sweep_tuning_set(precision, cls, **before)
    best_cand = min(results, key=lambda r: r[1])[0]
    if install:
        K.knit_sweep_tuning_set(precision, cls, **best_cand)
    return {"precision": precision, "cls": cls, "Mp": Mp, "best": best_cand, "results": results}


def save(path: str, tuned: list):
    """Write tune_batch results (a list of them) as a JSON tuning table."""
    table = {}
    for r in tuned:
        table.setdefault(r["precision"], {})[str(r["cls"])] = dict(r["best"], Mp=r["Mp"],
                                                                    seconds=min(t for _, t in r["results"]))
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def load(path: str) -> int:
    """Install the entries of a JSON tuning table; returns how many were set."""
    with open(path) as f:
        table = json.load(f)
    n = 0
    for prec, entries in table.items():
        for cls, e in entries.items():
            K.knit_sweep_tuning_set(prec, int(cls), int(e["threads"]), int(e["wg_per_cu"]), int(e["order"]),
                                    int(e.get("outer", 64)))
            n += 1
    return n
