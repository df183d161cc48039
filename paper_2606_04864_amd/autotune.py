"""Autotuner for the batched form: times candidate schedules on a sample of
the problems and picks the fastest time to solution (setup + batched PCG to
rtol, inputs resident on the device).

Host orchestration over the C ABI only: every candidate runs the library's
own setup and amsp_pcg_batched; nothing here computes any part of the method.

A candidate is a dict with
  * problem parameters passed to the caller's make_problem (for instance the
    subdomain size, which changes the partition, and nev): the paper's
    trade-off between the number of subdomains and the number of local
    eigenvectors (Section 5, parameter test);
  * "precision"      "fp64" | "fp32" | "bf16";
  * "coarse_solver"  "auto" | "dense" | "sparse";
  * "columns"        right-hand sides per batched PCG pass (1 .. 16).
make_problem(**params) returns a dict with A (row_ptr, col_idx, val), part,
nparts, nev, overlap, F (n x k host array) and prob_ptr (nprob + 1).
"""
from __future__ import annotations

import itertools
import time

import numpy as np

PROBLEM_KEYS_RESERVED = ("precision", "coarse_solver", "columns")


def grid(**axes):
    """Cartesian product of candidate axes as a list of dicts."""
    keys = list(axes)
    return [dict(zip(keys, vals)) for vals in itertools.product(*(axes[k] for k in keys))]


def run_candidate(make_problem, cand, rtol=1e-8, maxit=2000, repeats=1):
    """Median time to solution of one candidate (one untimed run first);
    returns a record with the phases and the step counts."""
    import torch
    from . import Preconditioner
    params = {k: v for k, v in cand.items() if k not in PROBLEM_KEYS_RESERVED}
    prob = make_problem(**params)
    A = prob["A"]
    F = torch.tensor(prob["F"], device="cuda")
    k = F.shape[1]
    cols = int(cand.get("columns", k))
    recs = []
    for rep in range(repeats + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pc = Preconditioner(A.row_ptr, A.col_idx, A.val, prob["part"], prob["nparts"], prob["nev"],
                            overlap=prob["overlap"], precision=cand.get("precision", "fp32"),
                            coarse_solver=cand.get("coarse_solver", "auto"))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        steps, conv, worst = [], True, 0.0
        for c0 in range(0, k, cols):
            _, info, its, rel = pc.pcg_batched(F[:, c0:c0 + cols].contiguous(), prob["prob_ptr"],
                                               rtol, maxit, raise_on_noconv=False)
            steps.append(its)
            conv = conv and info["converged"] == 1
            worst = max(worst, float(rel.max()))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        upload = pc.info["phase_ms"][1]
        pc.close()
        if rep > 0:
            its = np.concatenate(steps, axis=1)
            recs.append(dict(setup_ms=(t1 - t0) * 1e3 - upload, pcg_ms=(t2 - t1) * 1e3,
                             total_ms=(t2 - t0) * 1e3 - upload, steps_max=int(its.max()),
                             steps_mean=float(its.mean()), converged=conv, worst_relres=worst))
    best = min(recs, key=lambda r: r["total_ms"])
    return dict(cand, **{k: (float(f"{v:.4g}") if isinstance(v, float) else v)
                         for k, v in best.items()})


def autotune(make_problem, candidates, rtol=1e-8, maxit=2000, repeats=1, log=None):
    """Runs every candidate; returns (the fastest converged candidate's
    record, all records)."""
    table = []
    for cand in candidates:
        rec = run_candidate(make_problem, cand, rtol, maxit, repeats)
        table.append(rec)
        if log:
            log(f"autotune {rec}")
    ok = [r for r in table if r["converged"]]
    if not ok:
        raise RuntimeError("autotune: no candidate converged")
    return min(ok, key=lambda r: r["total_ms"]), table
