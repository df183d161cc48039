"""Benchmark: time to relative residual 1e-8 (setup + PCG) at n ~ 1M on one MI355X.

One step = one pass of the whole hot path on the gauss1024 workload (2D
1024x1024 two-point-flux Darcy matrix, n = 1,048,576; kappa = exp(GRF, var 4,
corr 0.05) times 1e6 in 200 disks; 1024 parts, 2 overlap layers, 6
eigenvectors): host index planning, device extraction, local Cholesky
factorisations, batched local eigensolves, coarse basis, A0 and its factor,
then preconditioned CG to ||f - A u|| <= 1e-8 ||f||.  Both the FP64 form and
the mixed form (float32 local factors/basis/coarse inverse factor inside the
float64 CG) run; `value` is the mixed form's time with the input matrix
already resident in HBM: the host-to-device transfer of the input CSR inside
setup is excluded (and reported); host planning and the upload of its index
arrays are included.

Prints one JSON line (rank 0, N = 1 only).  Besides the contract fields it
carries `roofline` (the dominant PCG kernel), `spmv` (amsp_spmv alone, warm and
with the MALL flushed between calls, outside the timed steps), `rtol_1e-6`
(the paper's own solver setting: GMRES(30) with the preconditioner to a 1e-6
reduction, and PCG to the same, outside the timed steps),
`multiplicative_cycle` (the symmetric two-grid cycle as the preconditioner,
setup + PCG to 1e-8, outside the timed steps), `multi_rhs` (16 columns per
apply and 8 CG recurrences sharing each operator application, against one
column at a time, outside the timed steps), `adjoint256` (forward and backward
pass of dJ/dtheta on the adjoint configuration), `batch64` (64 independent
problems with 8 right-hand sides in one batched solve, default and autotuned
schedules), `sweep_layered64` (subdomain size against eigenvectors per
subdomain in 3D) and `cpu_baseline` (the oracle on
a bounded sample, on the host cores) and `oracle_full_run` (the recorded run of
the oracle on the whole workload against the GPU forms, from `--oracle-full`).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
TIMING_STRIDE = 8  # local-apply launches per timed launch


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(P, torch, w, f, prec, steps, warmup, timing, coarse="auto"):
    rec = []
    for k in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision=prec,
                     timing=timing, timing_stride=TIMING_STRIDE, coarse_solver=coarse)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u, info = pc.pcg(f, 1e-8, 2000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        si = pc.info
        pc.close()
        del pc
        if k >= warmup:
            rec.append(dict(setup_ms=(t1 - t0) * 1e3, pcg_ms=(t2 - t1) * 1e3,
                            input_upload_ms=si["phase_ms"][1], plan_ms=si["phase_ms"][0],
                            phase_ms=si["phase_ms"], eig_sweeps=si["eig_sweeps"],
                            coupling_ms=si["coupling_ms"], coupling_wait_ms=si["coupling_wait_ms"],
                            plan_host_ms=si["plan_host_ms"], plan_upload_ms=si["plan_upload_ms"],
                            iterations=info["iterations"], relres_true=info["relres_true"],
                            relres_floor=info["relres_floor"], restarts=info["restarts"],
                            first_segment=info["first_segment"],
                            coarse_solver=si["coarse_solver"],
                            kernel_ms=info["kernel_ms"], kernel_launches=info["kernel_launches"],
                            local_apply_bytes=info["local_apply_bytes"],
                            bytes_per_iter=info["bytes_per_iter"], u=u))
        log(f"[{prec}] step {k}: setup {(t1 - t0) * 1e3:.1f} ms, pcg {(t2 - t1) * 1e3:.1f} ms, "
            f"its {info['iterations']}, relres {info['relres_true']:.2e}")
    return rec


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(w, gpu_fp64_iterations):
    """The oracle as it stands (oracle.setup, then oracle.pcg to 1e-8: plain
    numpy/scipy FP64, serial loop over subdomains, LAPACK on the host's
    threads) on a bounded sample of the workload: the same recipe at 1/16 of
    the area (gauss256: 256 x 256, 64 parts of ~1024 dofs, overlap 2, nev 6,
    12 disks), setup and PCG timed separately with its own iteration count.
    Scaled to the benchmark workload: setup and the cost of one PCG iteration
    grow with the number of subdomains (x N / 64); the iteration count is the
    one measured at full size for the FP64 form (equal to the oracle's to
    within one step in the parity tests, and 113 against 113 in the full
    oracle run recorded in profiles/oracle_gauss1024_full.md)."""
    import oracle as O
    from workloads import configs
    s = configs.gauss_inclusions(nx=256, nparts=64, overlap=w.overlap, nev=w.nev)
    A = s.A.to_scipy()
    t0 = time.perf_counter()
    st = O.setup(A, s.part, s.nparts, s.nev, s.overlap)
    t1 = time.perf_counter()
    res = O.pcg(A, s.b, st.apply, 1e-8, 2000)
    t2 = time.perf_counter()
    scale = w.nparts / s.nparts
    setup_s = (t1 - t0) * scale
    per_it_s = (t2 - t1) / max(res.iterations, 1) * scale
    total_s = setup_s + per_it_s * gpu_fp64_iterations
    threads = len(os.sched_getaffinity(0))
    return {"value": round(total_s * 1e3, 1), "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": (f"oracle.setup + oracle.pcg(1e-8) on {s.name} with {s.nparts} parts (the "
                       f"benchmark recipe at 1/16 of the area): setup {t1 - t0:.2f} s, PCG "
                       f"{t2 - t1:.2f} s for {res.iterations} iterations (true relres "
                       f"{res.relres_true:.2e}); scaled x{scale:.0f} in subdomains and to "
                       f"{gpu_fp64_iterations} iterations; CPU: {_cpu_model()}"),
            "setup_ms": round(setup_s * 1e3, 1), "pcg_ms_per_iteration": round(per_it_s * 1e3, 1),
            "sample_measured_s": round(t2 - t0, 2)}


def oracle_full_run(P, torch, w, f):
    """The oracle on the whole benchmark workload (no sampling): setup and
    PCG to 1e-8 timed separately on the host cores, against the GPU's FP64
    and mixed forms on the same inputs (solution errors, iteration counts,
    true residuals and their attainable floors).  Minutes of CPU time: run
    on request only (--oracle-full)."""
    import oracle as O
    A = w.A.to_scipy()
    gpu = {}
    # the bfloat16 basis both ways: A0 from the stored (rounded) basis, the
    # default, and from the float64 basis before rounding
    for name, prec, cb in (("fp64", "fp64", "stored"), ("fp32", "fp32", "stored"),
                           ("bf16", "bf16", "stored"), ("bf16_a0_fp64_basis", "bf16", "fp64")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision=prec,
                     coarse_basis=cb)
        u, info = pc.pcg(f, 1e-8, 2000, raise_on_noconv=False)
        torch.cuda.synchronize()
        gpu[name] = (u.cpu().numpy(), info, (time.perf_counter() - t0) * 1e3)
        pc.close()
        log(f"[{name}] GPU: {info['iterations']} its, converged {info['converged']}, "
            f"relres {info['relres_true']:.3e}")
    t0 = time.perf_counter()

    def progress(i, N):
        if (i + 1) % 64 == 0:
            log(f"oracle setup: {i + 1}/{N} subdomains, {time.perf_counter() - t0:.0f} s")

    st = O.setup(A, w.part, w.nparts, w.nev, w.overlap, progress=progress)
    t1 = time.perf_counter()
    log(f"oracle setup {t1 - t0:.1f} s")
    napply = [0]

    def apply_logged(r):  # the oracle's own apply; a line every 8 applications
        napply[0] += 1
        if napply[0] % 8 == 0:
            log(f"oracle pcg: {napply[0]} preconditioner applications, "
                f"{time.perf_counter() - t1:.0f} s")
        return st.apply(r)

    res = O.pcg(A, w.b, apply_logged, 1e-8, 2000)
    t2 = time.perf_counter()
    log(f"oracle pcg {t2 - t1:.1f} s, {res.iterations} its")
    floor_o = np.finfo(float).eps * np.linalg.norm(abs(A) @ abs(res.x)) / np.linalg.norm(w.b)
    out = {"oracle": {"setup_s": round(t1 - t0, 2), "pcg_s": round(t2 - t1, 2),
                      "iterations": res.iterations, "relres_true": float(f"{res.relres_true:.4g}"),
                      "relres_floor": float(f"{floor_o:.4g}"),
                      "threads": len(os.sched_getaffinity(0)), "cpu": _cpu_model()}}
    for prec, (u, info, ms) in gpu.items():
        out[prec] = {"iterations": int(info["iterations"]), "converged": int(info["converged"]),
                     "first_segment": int(info["first_segment"]), "restarts": int(info["restarts"]),
                     "u_relerr_vs_oracle": float(f"{np.linalg.norm(u - res.x) / np.linalg.norm(res.x):.4g}"),
                     "relres_true": float(f"{info['relres_true']:.4g}"),
                     "relres_floor": float(f"{info['relres_floor']:.4g}"),
                     "host_clock_ms": round(ms, 1)}
    return out


def oracle_record():
    """The recorded full oracle run at the benchmark workload, if present."""
    path = os.path.join(ROOT, "profiles", "oracle_gauss1024_full.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    import re
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    return json.loads(m.group(1)) if m else None


COPY_BYTES = 256 << 20


def spmv_measure(P, torch, w, reps=30):
    """amsp_spmv alone on the workload's matrix (the sliced copy the CG
    kernels read), median of `reps` calls after 5 untimed ones: warm (the
    previous call's data may sit in the 256 MB MALL) and flushed (a read-only
    pass over 512 MiB between calls).  Algorithmic bytes: 12 per stored entry
    plus x read and y written once."""
    pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision="fp32")
    x = torch.randn(w.n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    flush = torch.ones(512 * 2**20 // 8, dtype=torch.float64, device="cuda")
    alg = w.A.nnz * 12 + w.n * 16
    out = {"bytes": int(alg)}
    for mode in ("warm", "flushed"):
        ts = []
        for k in range(reps + 5):
            if mode == "flushed":
                flush.sum()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            pc.spmv(x, out=y)
            e1.record()
            torch.cuda.synchronize()
            if k >= 5:
                ts.append(e0.elapsed_time(e1))
        med = float(np.median(ts))
        gbs = alg / (med * 1e-3) / 1e9
        out[mode] = {"us": round(med * 1e3, 2), "gbs": round(gbs, 1),
                     "frac": round(gbs / PEAK_HBM_GBS, 4)}
    pc.close()
    return out


def copy_calibration(torch):
    """Five device-to-device copies of COPY_BYTES each (read COPY_BYTES, write
    COPY_BYTES per launch): the reference that turns the FETCH_SIZE and
    WRITE_SIZE counters of a profiled run into HBM bytes."""
    src = torch.rand(COPY_BYTES // 4, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: 5 copies of {COPY_BYTES} bytes")


def traffic_from_profile():
    """HBM bytes per local-apply launch from the committed counter summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "local_apply_traffic_gauss1024.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    import hashlib
    import re
    m = re.search(r"kernel sources sha256: ([0-9a-f]{64})", text)
    b = re.search(r"HBM bytes per launch: (\d+)", text)
    if not m or not b:
        return None
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2606_04864_amd", "csrc", name), "rb").read())
    return int(b.group(1)) if h.hexdigest() == m.group(1) else None


# sources that define the local-apply kernel (a change invalidates its counters)
TRAFFIC_SOURCES = ("k_apply.hip", "k_common.h", "amsp_consts.h", "amsp_internal.h")


def cycle_measure(P, torch, w, f, forms):
    """The multiplicative two-grid cycle (twice the local solves, two more
    SpMVs per application) against the additive operator: setup and PCG to
    1e-8, one untimed run then one timed, host clock around synchronised
    calls."""
    out = {}
    for prec in forms:
        rec = {}
        for k in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision=prec,
                         cycle="multiplicative")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, info = pc.pcg(f, 1e-8, 2000)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            upload = pc.info["phase_ms"][1]
            pc.close()
            rec = {"iterations": int(info["iterations"]), "pcg_ms": round((t2 - t1) * 1e3, 3),
                   "time_to_solution_ms": round((t2 - t0) * 1e3 - upload, 3),
                   "relres_true": float(f"{info['relres_true']:.4g}")}
        out[prec] = rec
        log(f"[{prec}] multiplicative cycle: {rec}")
    return out


def multi_rhs_measure(P, torch, w, f, forms, ncols=8):
    """Several right-hand sides (the batched reading: 8 columns): the block
    apply of 16 columns against 16 one-column applies (median of 5 after one
    untimed), and PCG to 1e-8 on 8 columns together against the same 8 one
    after another; the first column is the workload's f, the others seeded
    N(0, 1).  Host clock around synchronised calls."""
    out = {}
    g = torch.Generator(device="cuda")
    g.manual_seed(2606)
    F = torch.randn((ncols, w.n), dtype=torch.float64, device="cuda", generator=g)
    F[0] = f
    R16 = torch.randn((16, w.n), dtype=torch.float64, device="cuda", generator=g)
    cols = [R16[j].contiguous() for j in range(16)]
    fcols = [F[j].contiguous() for j in range(ncols)]

    def clock(fn, reps=5):
        fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(ts))

    for prec in forms:
        pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision=prec)
        block_ms = clock(lambda: pc.apply_columns(R16))
        single_ms = clock(lambda: [pc.apply(c) for c in cols])
        info = {}

        def block_pcg():
            info["b"] = pc.pcg_columns(F, 1e-8, 2000)[1]

        def seq_pcg():
            info["s"] = sum(pc.pcg(c, 1e-8, 2000)[1]["iterations"] for c in fcols)

        bp = clock(block_pcg, reps=1)
        sp = clock(seq_pcg, reps=1)
        pc.close()
        out[prec] = {"apply_16_columns_ms": round(block_ms, 3),
                     "apply_16_single_ms": round(single_ms, 3),
                     "pcg_columns": ncols, "block_pcg_ms": round(bp, 3),
                     "sequential_pcg_ms": round(sp, 3),
                     "block_pcg_iterations": int(info["b"]["iterations"]),
                     "sequential_pcg_iterations": int(info["s"]),
                     "block_relres_true_max": float(f"{info['b']['relres_true']:.4g}")}
        log(f"[{prec}] several right-hand sides: {out[prec]}")
    return out


def adjoint_measure(P, torch, forms):
    """The adjoint configuration (adjoint256: theta = log kappa on 256 x 256,
    J = 0.5 ||u - u_obs||^2): the forward pass (torch two-point-flux assembly,
    setup, PCG to 1e-10) and the backward pass (adjoint PCG on the same
    handle, gradient of the stored values, chain to theta through the
    assembly), one untimed run then one timed, host clock around
    synchronised calls."""
    import workloads as W
    from workloads.tpfa_torch import TpfaAssembly
    w = W.get("adjoint256")
    asm = TpfaAssembly(w.grid, w.A.row_ptr, w.A.col_idx)
    ft = torch.tensor(w.b, device="cuda")
    ut = torch.tensor(w.u_obs, device="cuda")
    out = {}
    for prec in forms:
        rec = {}
        for k in range(2):
            theta = torch.tensor(w.theta, device="cuda", requires_grad=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u = P.solve(asm.values(theta), ft, w.A.row_ptr, w.A.col_idx, w.part, w.nparts, w.nev,
                        rtol=1e-10, overlap=w.overlap, precision=prec)
            J = 0.5 * ((u - ut) ** 2).sum()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            J.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            rec = {"forward_ms": round((t1 - t0) * 1e3, 3), "backward_ms": round((t2 - t1) * 1e3, 3),
                   "J": float(f"{float(J.detach()):.10g}"),
                   "grad_norm": float(f"{float(torch.linalg.norm(theta.grad)):.6g}")}
        out[prec] = rec
        log(f"[{prec}] adjoint256: {rec}")
    return out


def batch_measure(P, torch, forms):
    """The batched configuration (batch64: 64 independent 2D problems of side
    U{128..512}, lognormal kappa, 8 right-hand sides each; 512 CG recurrences
    in one amsp_pcg_batched call on one block-diagonal setup).  The
    autotuner first picks the subdomain size, nev and the columns per pass on
    the batch's first 16 problems (mixed form); then the full
    batch runs with the default schedule and with the tuned one.  One untimed
    run, then one timed, host clock around synchronised calls; inputs
    resident (the input transfer inside setup excluded)."""
    from workloads import configs
    from paper_2606_04864_amd import autotune

    def make(box=32, nev=6):
        s = configs.batch(box=box, nev=nev, first=16)
        return dict(A=s.A, part=s.part, nparts=s.nparts, nev=s.nev, overlap=s.overlap, F=s.B,
                    prob_ptr=s.seg_ptr)

    cands = autotune.grid(box=[24, 32, 48], nev=[4, 6, 8], precision=["fp32"], columns=[8, 4])
    best, table = autotune.autotune(make, cands, repeats=2, log=log)
    out = {"autotune": {"sample": "the first 16 problems of the batch, mixed form, best of 2",
                        "best": best, "candidates": table}}
    for sched, box, nev, cols in (("default", 32, 6, 8),
                                  ("tuned", best["box"], best["nev"], best["columns"])):
        w = configs.batch(box=box, nev=nev)
        prob = dict(A=w.A, part=w.part, nparts=w.nparts, nev=w.nev, overlap=w.overlap, F=w.B,
                    prob_ptr=w.seg_ptr)
        rec = {"box": box, "nev": nev, "columns": cols, "n": w.n, "problems": w.nprob,
               "parts": w.nparts}
        for prec in forms:
            r = autotune.run_candidate(lambda **_: prob, {"precision": prec, "columns": cols})
            rec[prec] = {k: r[k] for k in ("setup_ms", "pcg_ms", "total_ms", "steps_max",
                                           "steps_mean", "converged", "worst_relres")}
            log(f"[{prec}] batch64 {sched}: {rec[prec]}")
        out[sched] = rec
    return out


def sweep_3d(P, torch):
    """The subdomain-count / eigenvector-count trade-off (Section 5, parameter
    test) on the 3D layered recipe at 64^3 (n = 262,144, one overlap layer,
    mixed form): parts of ~2048, ~1024 and ~512 dofs (the 128^3 benchmark
    configuration uses ~512) and nev 4, 8, 12; setup + PCG to 1e-8."""
    from workloads import configs
    out = []
    for nparts in (128, 256, 512):
        base = configs.layered(n=64, nparts=nparts, nev=8)
        for nev in (4, 8, 12):
            f = torch.tensor(base.b, device="cuda")
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pc = P.setup(base.A, base.part, nparts, nev, overlap=1, precision="fp32")
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                _, info = pc.pcg(f, 1e-8, 3000, raise_on_noconv=False)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                upload = pc.info["phase_ms"][1]
                nc = pc.info["nc"]
                pc.close()
            rec = {"parts": nparts, "dofs_per_part": base.n // nparts, "nev": nev, "nc": nc,
                   "iterations": int(info["iterations"]),
                   "setup_ms": round((t1 - t0) * 1e3 - upload, 2),
                   "pcg_ms": round((t2 - t1) * 1e3, 2),
                   "total_ms": round((t2 - t0) * 1e3 - upload, 2)}
            out.append(rec)
            log(f"sweep layered64: {rec}")
    return out


def gmres_measure(P, torch, w, f, forms, sums):
    """The paper's own solver configuration (Section 5): GMRES with the
    preconditioner, restarted every 30 steps, until the residual has dropped
    by 1e-6; PCG to the same 1e-6 on the same handle for comparison.  One
    untimed solve first; solve times by host clock around synchronised calls.
    time_to_solution_ms adds the form's median setup with inputs resident."""
    out = {}
    for prec in forms:
        pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision=prec)
        rec = {}
        for name, call in (("gmres", lambda: pc.gmres(f, rtol=1e-6, restart=30, maxit=2000)),
                           ("pcg", lambda: pc.pcg(f, 1e-6, 2000))):
            call()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = call()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            rec[name] = {"iterations": int(info["iterations"]), "restarts": int(info["restarts"]),
                         "solve_ms": round(ms, 3), "relres_true": float(f"{info['relres_true']:.4g}"),
                         "time_to_solution_ms": round(sums[prec]["setup_ms"]
                                                      - sums[prec]["input_upload_ms"] + ms, 3)}
        pc.close()
        out[prec] = rec
        log(f"[{prec}] rtol 1e-6: gmres {rec['gmres']}, pcg {rec['pcg']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gauss1024")
    ap.add_argument("--forms", default="fp64,fp32")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--coarse", default="auto", choices=["auto", "dense", "sparse"],
                    help="coarse factorisation of the timed steps (default: the library's choice)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed steps (no SpMV, GMRES, cycle, several-column, adjoint "
                         "or CPU-baseline sections)")
    ap.add_argument("--oracle-full", action="store_true",
                    help="run the oracle on the whole workload against the GPU forms and print "
                         "that record only (minutes of CPU time)")
    ap.add_argument("--setup-only", action="store_true",
                    help="only one setup per form (no timing line): the run profiled for the "
                         "matrix-core counters of the setup kernels")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies of known size (reference for the HBM "
                         "byte counters FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the preconditioner runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    import paper_2606_04864_amd as P
    import workloads as W
    t = time.perf_counter()
    w = W.get(args.workload)
    log(f"workload {w.name}: n={w.n} nnz={w.A.nnz} parts={w.nparts} overlap={w.overlap} "
        f"nev={w.nev} (generated in {time.perf_counter() - t:.1f} s, partition sha256 "
        f"{w.part_sha256()[:16]})")
    f = torch.tensor(w.b, device="cuda")
    forms = args.forms.split(",")
    if args.oracle_full:
        print(json.dumps({"workload": w.name, "oracle_full_run": oracle_full_run(P, torch, w, f)}),
              flush=True)
        return
    if args.setup_only:
        for prec in forms:
            pc = P.setup(w.A, w.part, w.nparts, w.nev, overlap=w.overlap, precision=prec)
            torch.cuda.synchronize()
            log(f"[{prec}] setup phases (ms): {[round(x, 2) for x in pc.info['phase_ms']]}")
            pc.close()
        return
    res = {}
    for prec in forms:
        # HIP events around every TIMING_STRIDE-th launch of the local-apply
        # kernel only: each timed launch adds two event records to the stream
        res[prec] = run_form(P, torch, w, f, prec, args.steps, args.warmup,
                             timing=1 << P.KERNEL_CLASS["local"], coarse=args.coarse)

    def summary(rec):
        med = lambda k: float(np.median([r[k] for r in rec]))
        tot = [r["setup_ms"] + r["pcg_ms"] for r in rec]
        resident = [r["setup_ms"] - r["input_upload_ms"] + r["pcg_ms"] for r in rec]
        return dict(ms_per_step=float(np.mean(tot)), time_to_solution_ms=float(np.median(resident)),
                    pcie_inclusive_ms=float(np.median(tot)), setup_ms=med("setup_ms"),
                    input_upload_ms=med("input_upload_ms"), plan_ms=med("plan_ms"), pcg_ms=med("pcg_ms"),
                    iterations=int(rec[-1]["iterations"]), relres_true=float(rec[-1]["relres_true"]),
                    relres_floor=float(rec[-1]["relres_floor"]),
                    first_segment=int(rec[-1]["first_segment"]), restarts=int(rec[-1]["restarts"]),
                    coarse_solver={1: "dense", 2: "sparse"}[int(rec[-1]["coarse_solver"])],
                    eig_sweeps=int(rec[-1]["eig_sweeps"]),
                    setup_phase_ms=[round(x, 3) for x in rec[-1]["phase_ms"]],
                    coupling_plan_ms=med("coupling_ms"), coupling_wait_ms=med("coupling_wait_ms"),
                    plan_host_ms=med("plan_host_ms"), plan_upload_ms=med("plan_upload_ms"),
                    pcg_gbs=float(rec[-1]["bytes_per_iter"] * rec[-1]["iterations"]
                                  / (np.median([r["pcg_ms"] for r in rec]) * 1e-3) / 1e9))

    sums = {p: summary(res[p]) for p in forms}
    head = "fp32" if "fp32" in forms else forms[0]
    # roofline of the dominant PCG kernel (local apply), from HIP events on the
    # library's stream over the timed steps
    rec = res[head]
    kms = sum(r["kernel_ms"][1] for r in rec)
    kl = sum(r["kernel_launches"][1] for r in rec)
    avg_ms = kms / max(kl, 1)
    achieved = rec[-1]["local_apply_bytes"] / (avg_ms * 1e-3) / 1e9 if kl else 0.0
    # solution agreement between forms
    agree = None
    if "fp64" in res and head != "fp64":
        a, b = res["fp64"][-1]["u"], res[head][-1]["u"]
        agree = float(torch.linalg.norm(a - b) / torch.linalg.norm(a))
    fp64_t = sums.get("fp64", {}).get("time_to_solution_ms")
    line = {
        "metric": "time-to-rel-res 1e-8 at n=1M, mixed/batched vs FP64 form; PCG HBM GB/s",
        "value": round(sums[head]["time_to_solution_ms"], 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sums[head]["ms_per_step"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if head != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": (f"{w.name}: 2D {w.grid[0]}x{w.grid[1]} TPFA Darcy, n={w.n}, "
                                f"kappa=exp(GRF var4 corr0.05) x1e6 in 200 disks, f~N(0,1), "
                                f"{w.nparts} parts, overlap {w.overlap}, nev {w.nev}, rtol 1e-8"
                                if len(w.grid) == 2 else
                                f"{w.name}: 3D {'x'.join(map(str, w.grid))} TPFA Darcy, n={w.n}, "
                                f"32 layers of exp(GRF var3) with x1e6 channels, kz=0.1kx, "
                                f"f~N(0,1), {w.nparts} parts, overlap {w.overlap}, nev {w.nev}, "
                                f"rtol 1e-8"),
                   "form": {"fp32": "mixed: f32 local factors/basis/coarse inverse factor, f64 CG",
                            "bf16": "mixed: f32 factors, bf16 basis, f64 CG",
                            "fp64": "fp64"}[head],
                   "parallelism": "single GPU"},
        "forms": {p: {k: (float(f"{v:.5g}") if isinstance(v, float) else v) for k, v in s.items()}
                  for p, s in sums.items()},
        "mixed_vs_fp64_speedup": (round(fp64_t / sums[head]["time_to_solution_ms"], 3)
                                  if fp64_t and head != "fp64" else None),
        "mixed_vs_fp64_u_relerr": agree,
        "roofline": {"bound": "hbm", "kernel": "k_local_apply_stream (gather, streamed "
                                               "forward/backward solves, prolongation)",
                     "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic_from_profile(),
                     "avg_launch_ms": round(avg_ms, 5), "launches": kl,
                     "timed_every_nth_launch": TIMING_STRIDE,
                     "bytes_per_launch": rec[-1]["local_apply_bytes"]},
    }
    if args.no_extras:
        print(json.dumps(line), flush=True)
        return
    log("spmv alone ...")
    line["spmv"] = spmv_measure(P, torch, w)
    log("paper's stopping rule (GMRES(30) and PCG to 1e-6) ...")
    line["rtol_1e-6"] = gmres_measure(P, torch, w, f, forms, sums)
    log("multiplicative two-grid cycle ...")
    line["multiplicative_cycle"] = cycle_measure(P, torch, w, f, forms)
    log("several right-hand sides ...")
    line["multi_rhs"] = multi_rhs_measure(P, torch, w, f, forms)
    log("adjoint configuration ...")
    line["adjoint256"] = adjoint_measure(P, torch, forms)
    log("batched configuration ...")
    line["batch64"] = batch_measure(P, torch, forms)
    log("3D subdomain / eigenvector sweep ...")
    line["sweep_layered64"] = sweep_3d(P, torch)
    if not args.no_cpu:
        log("cpu baseline (oracle, bounded sample) ...")
        its64 = sums["fp64"]["iterations"] if "fp64" in sums else sums[head]["iterations"]
        line["cpu_baseline"] = cpu_baseline(w, its64)
    orec = oracle_record()
    if orec is not None and orec.get("workload") == w.name:
        line["oracle_full_run"] = dict(orec["oracle_full_run"],
                                       recorded_in="profiles/oracle_gauss1024_full.md")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
