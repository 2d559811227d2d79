#!/usr/bin/env python3
"""Benchmark: Nystrom-preconditioned NGD steps per second on one MI355X, against plain CG.

Workload (default): 2D Poisson -Laplace u = f on [0,1]^2, u* = sin(pi x) sin(pi y), tanh MLP
2-64-64-64-1 (P = 8,577), 4,096 uniform interior + 512 boundary points, FP32 residuals / Jacobian /
matvecs with FP64 CG scalars, sketch size ell = 400, PCG to relative residual 1e-6, damping
mu = max(10 eps lam1_hat, 1e-4 L^2). One step = residuals + Jacobian + gradient, Gaussian sketch
and FP64 Nystrom core, damping, PCG, Armijo line search and update: the whole hot path.

Both solvers run the same trajectory length from the same start (default 2 warm-up + 48 timed NGD
steps each, the 50-step comparison of the workload). Prints one JSON line with the steps/s of the
Nystrom-PCG loop (`value`), plain-CG steps/s, the one-pass Gramian-matvec bandwidth with its roofline,
the sketch contractions against the MFMA peak, and the FP64 CPU oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# dense MFMA peaks (TFLOP/s) by the sketch's compute type
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}

WORKLOADS = {
    "c1": "2D Poisson 2-32-32-1 tanh (P=1,185), 30x30 grid + 120 boundary points, FP64, ell=100, "
          "lambda=1e-6, PCG rtol 1e-8",
    "c2": "2D Poisson 2-64-64-64-1 tanh (P=8,577), 4,096 + 512 random points, FP32 (FP64 CG scalars), "
          "ell=400, PCG rtol 1e-6",
    "c3": "5D Poisson 5-128-128-128-1 tanh (P=33,921), 16,384 + 2,048 points, FP32 Jacobian, BF16 sketch, "
          "FP64 core, ell=800, PCG rtol 1e-6",
    "c4": "2+1D heat 3-64-64-64-64-1 tanh (P=12,801), 8,192 + 1,024 lateral + 1,024 initial points, FP32, "
          "J recomputed by the JVP / adjoint kernels (never stored), ell=400, PCG rtol 1e-6",
}
WORKLOADS["c5"] = ("32 independent 2D/3D Poisson PINNs, hidden widths from {32,48,64,96}, depth 2-4 (P 1,185-28,417), "
                    "N_int 1,024-8,192 + N_int/8 boundary points, ell from {50,100,200,400}, FP32; batched residual/"
                    "Jacobian launch, per-problem Nystrom sketch with batched eigensolver stages, batched graph-replayed "
                    "PCG, batched Armijo line search")
WORKLOADS["paper3d"] = ("the paper's 3D Poisson PINN: 3-64-64-64-1 tanh (P=8,641), 10,000 + 1,000 random points, FP64, "
                         "u* = sin(pi x) sin(pi y) sin(pi z); Nystrom NGD with adaptive sketch size (ell from 20 in "
                         "steps of 20 up to 500), at most 20 PCG iterations at rtol 1e-6, mu = max(10 eps lam1_hat, "
                         "1e-4 L^2), Armijo; relative H1 error on 100,000 random points")
WORKLOADS["paper_heat"] = ("the paper's heat equation in 3+1D: 4-64-64-64-1 tanh (P=8,705), 10,000 + 1,000 random "
                            "points, FP64, u* = (cos(pi x) + cos(pi y) + cos(pi z)) exp(-pi^2 t / 4); the paper3d "
                            "solver settings; relative H1 error (space-time gradient) on 100,000 random points")
WORKLOADS["paper_ns"] = ("the paper's Kovasznay flow (steady Navier-Stokes, Re = 40): velocity 2-45-45-45-2 and pressure "
                          "2-45-45-45-1 tanh networks (P=8,688), 10,000 + 1,000 random points (32,000 rows: two momentum "
                          "and one continuity row per interior point, two Dirichlet rows per boundary point), FP64, "
                          "Gauss-Newton metric, Levenberg-Marquardt damping, the paper3d sketch-size settings; relative "
                          "H1 error of the velocity on 100,000 random points")
# The paper's methods on its setups (one RTX 4090, FP64): time to the plateau error over at most 1,000 NGD
# iterations (2,000 for the Kovasznay flow), so seconds / iterations bounds its time per step from below
# (a derived upper bound on its rate).
PAPER_BASELINE_S = {"paper3d": ({"gaussian": 66.8, "sampling": 81.2, "rpchol": 74.1, "direct": 317.7}, 1000),
                    "paper_heat": ({"gaussian": 106.1, "sampling": 59.0, "rpchol": 111.9, "direct": 279.2}, 1000),
                    "paper_ns": ({"gaussian": 878.5, "sampling": 548.0, "rpchol": 654.4, "direct": 5708.3}, 2000)}
_VARIANT_NAME = {"rpchol": "RPCholNGD", "direct": "NGD full (direct Cholesky)"}
# FP32 vector peak without packed FP32 instructions (the library is compiled without them): 256 CUs x 128 FLOP
# per clock (4 SIMDs x 16 lanes x an FMA) x 2.4 GHz = 78.6 TFLOP/s; the 157.3 of the data sheet counts
# packed FP32
FP32_VECTOR_PEAK_TFLOPS = 78.6


def bench_paper(a):
    """The paper's own 3D Poisson setup with the full Nystrom NGD of Alg. 1 + Alg. 4 (adaptive rank)."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_2505_11638_amd.driver import NGD

    prob = wl.config(a.config, seed=a.seed)
    ns = prob.pde == wl.PDE_NAVIER_STOKES
    theta0 = wl.ns_glorot_theta(prob.widths, a.seed) if ns else wl.glorot_theta(prob.widths, a.seed)
    P, N = prob.n_params, prob.n_rows
    variant = a.solver if a.solver in ("rpchol", "direct") else a.test_matrix
    if a.solver == "rpchol":  # RPCholNGD (Alg. 5): block size 20, rank up to 500
        ngd = NGD(prob, theta0, solver="rpchol", rtol=1e-6, seed=a.seed, ell_max=prob.ell_max,
                  rpchol_form=a.rpchol_form)
    elif a.solver == "direct":  # NGD full (Alg. 2): explicit FP64 Gramian and its Cholesky factor
        ngd = NGD(prob, theta0, solver="direct", seed=a.seed)
    else:
        ngd = NGD(prob, theta0, solver="nystrom", rtol=1e-6, seed=a.seed, test_matrix=a.test_matrix)
    gp = ngd.gp
    if ns:  # the velocity's error (Section 5.1.3)
        Xe, ue, ge = wl.kovasznay_evaluation_set(prob.nu, 100_000, seed=a.seed)
    else:
        Xe, ue, ge = wl.evaluation_set(prob, 100_000, seed=a.seed)
    _, h1_start, sums = gp.solution_error(ngd.theta, Xe, ue, ge)
    for _ in range(a.warmup):
        ngd.step()
    gp.timing(True, only=["matvec_rows"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = [ngd.step() for _ in range(a.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_mv, ms_mv = gp.timers()["matvec_rows"]
    gp.timing(False)
    l2_end, h1_end, _ = gp.solution_error(ngd.theta, Xe, ue, ge, sums=sums)
    avg_ms = ms_mv / max(n_mv, 1)
    alg_bytes = N * P * 8 + 2 * P * 8
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    sps = a.steps / dt
    ranks = [r.rank for r in reps]
    base_s, base_iters = PAPER_BASELINE_S[a.config]
    base_sps = base_iters / base_s[variant]
    line = {
        "metric": "NGD steps/s at PCG rtol 1e-6 (Nystrom vs plain CG); Gramian-matvec GB/s",
        "value": sps, "unit": "NGD steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1000.0 * dt / a.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": sps / base_sps,
        "baseline": {"value": base_sps, "unit": "NGD steps/s",
                     "kind": f"the paper's {_VARIANT_NAME.get(variant, 'Nystrom NGD (' + variant + ' test matrix)')}"
                             f" on this problem, RTX 4090, FP64: {base_s[variant]} s to its plateau over at most "
                             f"{base_iters:,} iterations (an upper bound on its rate)"},
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{a.config}: {WORKLOADS[a.config]}; {a.warmup} + {a.steps} NGD steps from a "
                               f"Glorot start (the last {a.steps} timed)", "P": P, "N": N,
                   "ell0": prob.ell, "ell_max": prob.ell_max, "dell": prob.dell, "maxit": prob.maxit,
                   "preconditioner": variant if variant != "rpchol" else f"rpchol ({a.rpchol_form})",
                   "damping": prob.damping},
        "ell_first_last_max": [ranks[0], ranks[-1], max(ranks)],
        "ell_trajectory": ranks,
        "mean_pcg_iters": float(np.mean([r.iters for r in reps])),
        "mu_trajectory": [r.mu for r in reps],
        "loss_first_last": [reps[0].loss, reps[-1].loss_new],
        "rel_h1_error_start_end": [h1_start, h1_end], "rel_l2_error_end": l2_end,
        "roofline": {"bound": "hbm", "kernel": "pcg_rows_kernel (one-pass J^T(J v)), FP64", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": avg_ms, "launches": n_mv},
    }
    torch.cuda.synchronize()
    gp.close()
    print(json.dumps(line), flush=True)
    return 0


def bench_batch(a):
    """The batched workload: NGD steps of all problems together; `value` counts problem-steps/s."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_2505_11638_amd.driver import BatchNGD

    probs = wl.batch_instances(seed=a.seed)
    thetas = [wl.glorot_theta(p.widths, a.seed + i) for i, p in enumerate(probs)]
    ngd = BatchNGD(probs, thetas, solver="nystrom", seed=a.seed)
    for _ in range(a.warmup):
        ngd.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, conv = [], True
    for _ in range(a.steps):
        L0, L1, outs = ngd.step()
        iters.append(np.mean([o.iters for o in outs]))
        conv = conv and all(o.converged for o in outs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = len(probs)
    # roofline of the batched one-pass matvec (every member's J_w read once per PCG iteration), timed
    # with HIP events on the stream it runs on, on the directions of the last solve
    mv_ms = ngd.batch.matvec_time(20)
    alg_bytes = sum(p.n_rows * p.n_params * 4 + 2 * p.n_params * 8 for p in probs)
    achieved = alg_bytes / (mv_ms * 1e-3) / 1e9
    line = {
        "metric": "NGD steps/s at PCG rtol 1e-6 (Nystrom vs plain CG); Gramian-matvec GB/s",
        "value": n * a.steps / dt, "unit": "problem NGD steps/s (sum over the batch)", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1000.0 * dt / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c5: {WORKLOADS['c5']}", "problems": n,
                   "P": [p.n_params for p in probs], "N": [p.n_rows for p in probs], "ell": [p.ell for p in probs],
                   },
        "nystrom_mean_pcg_iters": float(np.mean(iters)), "nystrom_converged": conv,
        "roofline": {"bound": "hbm", "kernel": "pcg_batch_rows_kernel (one pass over all 32 J_w)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": mv_ms, "launches": 20},
    }
    ngd.batch.close()
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batch(probs, thetas, a.seed, max(1, min(a.cpu_steps, 4)))
    print(json.dumps(line), flush=True)
    return 0


def cpu_baseline_batch(probs, thetas, seed: int, members: int):
    """The FP64 NumPy oracle's NGD step on the first `members` problems of the batch (bounded sample)."""
    import numpy as np

    from oracle import ngd as ongd
    import workloads as wl

    t0 = time.perf_counter()
    for i in range(members):
        p = probs[i]
        p64 = p.cast(p.dtype)
        th = thetas[i].astype(np.float32).astype(np.float64)
        Om = wl.gaussian_omega(p.n_params, p.ell, seed=seed, counter=i)
        ongd.ngd_step(th, p64, solver="nystrom", Omega=Om, rtol=1e-6, maxit=1000)
    dt = time.perf_counter() - t0
    return {"value": members / dt, "unit": "problem NGD steps/s", "cores": _cpu_threads(), "kind": "oracle",
            "sample": f"one Nystrom-PCG NGD step of each of the first {members} problems of workload c5 (same data, "
                      f"their own ell, rtol 1e-6) in the FP64 NumPy oracle, {dt:.1f} s"}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "pcg_rows_kernel_c2_c3_hbm_traffic.md")
MATVEC_SOURCE = os.path.join(ROOT, "paper_2505_11638_amd", "csrc", "matvec.hip")


def measured_traffic(config: str):
    """HBM bytes per matvec launch from the committed counter summary, or None when the kernel source
    has changed since the counters were taken (or none were taken for this workload)."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        src = hashlib.sha256(open(MATVEC_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    vals, sha = {}, None
    for line in text.splitlines():
        parts = line.split()
        if len(parts) == 3 and parts[0] == "traffic_bytes_per_launch":
            vals[parts[1]] = float(parts[2])
        if len(parts) == 2 and parts[0] == "source_sha256":
            sha = parts[1]
    return vals.get(config) if sha == src else None


def recompute_matvec_flops(prob) -> float:
    """Floating-point operations of one recompute-mode Gramian matvec (tangent pass + adjoint pass),
    counted from the implemented recurrences: per point and channel, the tangent pass does the primal
    and two tangent layer products (3 W multiply-adds, W = sum of n_in n_out over the layers), the
    adjoint pass the primal and the adjoint products (2 W) plus the parameter derivative (P)."""
    widths = prob.widths
    W = sum(widths[i] * widths[i + 1] for i in range(len(widths) - 1))
    C = 1 + (prob.d if prob.pde == 0 else prob.d - 1) + 1 + (0 if prob.pde == 0 else 1)
    return 2.0 * prob.n_rows * C * (5 * W + prob.n_params)


def _cpu_threads():
    try:
        from threadpoolctl import threadpool_info
        n = max((i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"), default=0)
        if n:
            return int(n)
    except Exception:
        pass
    return len(os.sched_getaffinity(0))


def cpu_baseline(cfg: str, seed: int, steps: int = 1):
    """The FP64 NumPy oracle's NGD step on the same workload (bounded sample)."""
    import numpy as np

    import workloads as wl
    from oracle import ngd as ongd

    prob = wl.config(cfg, seed=seed)
    theta = wl.glorot_theta(prob.widths, seed)
    prob64 = prob.cast(prob.dtype)
    th = theta.astype(np.float32).astype(np.float64) if prob.dtype == "f32" else theta
    rtol = 1e-8 if cfg == "c1" else 1e-6
    t0 = time.perf_counter()
    for k in range(steps):
        Om = wl.gaussian_omega(prob.n_params, prob.ell, seed=seed, counter=k)
        th, _ = ongd.ngd_step(th, prob64, solver="nystrom", Omega=Om, rtol=rtol, maxit=1000)
    dt = time.perf_counter() - t0
    return {"value": steps / dt, "unit": "NGD steps/s", "cores": _cpu_threads(), "kind": "oracle",
            "sample": f"{steps} Nystrom-PCG NGD step(s) of workload {cfg} (same data, ell={prob.ell}, "
                      f"rtol {rtol:g}) in the FP64 NumPy oracle, {dt:.1f} s"}


def time_to_rtol(cfg: str, seed: int, at_steps=(0, 10, 49), reps: int = 3, cg_maxit: int = 2000):
    """Single solves to rtol 1e-6 at fixed theta (the iterates after `at_steps` Nystrom NGD steps from the
    Glorot start) and fixed lambda (the damping rule's value there): Nystrom = sketch + FP64 core + PCG,
    plain CG = CG alone (capped at `cg_maxit` iterations). Median wall time of `reps` runs each."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_2505_11638_amd.driver import EPS, NGD

    prob = wl.config(cfg, seed=seed)
    ngd = NGD(prob, wl.glorot_theta(prob.widths, seed), solver="nystrom", rtol=1e-6, seed=seed)
    gp = ngd.gp
    out = []
    for k in range(max(at_steps) + 1):
        if k in at_steps:
            theta = ngd.theta.clone()
            r, J, grad, loss = gp.residual_jacobian(theta, ngd.J)
            pc = gp.nystrom_sketch(J, ngd.ell, seed=seed, counter=10_000 + k, sketch_dtype=ngd.sketch_dtype)
            _, mu = gp.damping(pc.lam_hat[:1], loss, 10.0 * EPS[gp.dtype_name], 1e-4)
            row = {"step": k, "lambda": mu}
            for name in ("nystrom", "cg"):
                times, its, conv = [], 0, True
                for rep in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    if name == "nystrom":
                        pc = gp.nystrom_sketch(J, ngd.ell, seed=seed, counter=20_000 + 10 * k + rep,
                                               sketch_dtype=ngd.sketch_dtype, want_info=False, out=pc)
                        o = gp.pcg_solve(J, grad, mu, precond=pc, rtol=1e-6, maxit=1000)
                    else:
                        o = gp.pcg_solve(J, grad, mu, rtol=1e-6, maxit=cg_maxit)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                    its, conv = o.iters, o.converged
                row[name] = {"ms": 1000.0 * float(np.median(times)), "iters": its, "converged": conv}
            row["speedup_nystrom_vs_cg"] = row["cg"]["ms"] / row["nystrom"]["ms"]
            out.append(row)
        if k < max(at_steps):
            ngd.step()
    torch.cuda.synchronize()
    gp.close()
    return {"workload": cfg, "rtol": 1e-6, "ell": prob.ell, "sketch_dtype": prob.sketch_dtype,
            "cg_maxit": cg_maxit, "reps": reps, "solves": out}


def c3_subrun(seed: int, steps: int = 3):
    """A short run of the 5D workload (BF16 sketch, ell = 800): the one-pass matvec's HBM roofline and the
    sketch contractions' MFMA roofline, timed with HIP events over `steps` Nystrom NGD steps."""
    import torch

    import workloads as wl
    from paper_2505_11638_amd.driver import NGD

    prob = wl.config("c3", seed=seed)
    ngd = NGD(prob, wl.glorot_theta(prob.widths, seed), solver="nystrom", rtol=1e-6, seed=seed)
    gp = ngd.gp
    ngd.step()
    gp.timing(True, only=["matvec_rows", "sketch_z", "sketch_w"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ngd.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t = gp.timers()
    gp.timing(False)
    gp.close()
    P, N = prob.n_params, prob.n_rows
    n_mv, ms_mv = t["matvec_rows"]
    mv_ms = ms_mv / max(n_mv, 1)
    mv_bytes = N * P * 4 + 2 * P * 8
    mv_gbs = mv_bytes / (mv_ms * 1e-3) / 1e9
    n_sk = t["sketch_z"][0] + t["sketch_w"][0]
    sk_ms = (t["sketch_z"][1] + t["sketch_w"][1]) / max(n_sk, 1)
    sk_flops = 2.0 * N * P * prob.ell
    sk_tf = sk_flops / (sk_ms * 1e-3) / 1e12
    return {"workload": f"c3: {WORKLOADS['c3']}; 1 + {steps} NGD steps", "steps_per_s": steps / dt,
            "roofline_matvec": {"bound": "hbm", "kernel": "pcg_rows_kernel (one-pass J^T(J v))", "achieved": mv_gbs,
                                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": mv_gbs / HBM_PEAK_GBS,
                                "alg_bytes_per_launch": mv_bytes, "avg_launch_ms": mv_ms, "launches": n_mv},
            "roofline_sketch": {"bound": "mfma", "kernel": "nt_gemm_kernel (Z = J Omega and B^T = Q^T J), BF16",
                                "achieved": sk_tf, "peak": MFMA_PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                                "frac": sk_tf / MFMA_PEAK_TFLOPS["bf16"], "alg_flops_per_launch": sk_flops,
                                "avg_launch_ms": sk_ms, "launches": n_sk}}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=48)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--cg-steps", type=int, default=None,
                    help="timed plain-CG steps after the same warm-up (default: --steps, the same trajectory length)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--no-cg", action="store_true", help="skip the plain-CG comparison loop")
    ap.add_argument("--phase-steps", type=int, default=5,
                    help="further Nystrom steps, after the timed ones, with every phase timer on")
    ap.add_argument("--rpchol-form", default="woodbury", choices=["woodbury", "svd"],
                    help="RPCholNGD's preconditioner: Woodbury-Cholesky (eq. rpchol_precond) or from the eigenpairs "
                         "of F^T F")
    ap.add_argument("--solver", default="nystrom", choices=["nystrom", "rpchol", "direct"],
                    help="paper3d: Nystrom NGD, RPCholNGD or NGD full")
    ap.add_argument("--test-matrix", default="gaussian", choices=["gaussian", "sampling"],
                    help="paper3d: Gaussian test matrix or identity columns sampled proportionally to diag(G)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB device copy (known bytes) to calibrate the HBM traffic counters")
    ap.add_argument("--no-extras", action="store_true",
                    help="c2: skip the time-to-rtol solves and the 5D sub-run")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        return 2

    if a.config == "c5":
        return bench_batch(a)
    if a.config in ("paper3d", "paper_heat", "paper_ns"):
        return bench_paper(a)

    import numpy as np
    import torch

    import workloads as wl
    from paper_2505_11638_amd.driver import NGD

    prob = wl.config(a.config, seed=a.seed)
    theta0 = wl.glorot_theta(prob.widths, a.seed)
    P, N = prob.n_params, prob.n_rows
    rtol = 1e-8 if a.config == "c1" else 1e-6

    # ---- Nystrom-PCG NGD ----
    nys = NGD(prob, theta0, solver="nystrom", rtol=rtol, seed=a.seed)
    for _ in range(a.warmup):
        nys.step()
    gp = nys.gp
    # in the timed steps only the matvec kernel is timed: its events are stamped by the kernel's own
    # dispatch and add nothing to the stream
    gp.timing(True, only=["matvec_rows"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = [nys.step() for _ in range(a.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mv_timer = gp.timers()["matvec_rows"]
    nys_sps = a.steps / (t1 - t0)
    # per-phase breakdown (event records around kernel sequences) over further, untimed steps
    n_phase = max(a.phase_steps, 0)
    gp.timing(True)
    for _ in range(n_phase):
        nys.step()
    torch.cuda.synchronize()
    timers = gp.timers()
    gp.timing(False)

    # ---- plain CG NGD: the same start, warm-up and number of steps (power-method damping, maxit = P) ----
    cg = None
    creps, cg_sps = [], float("nan")
    cg_steps = a.steps if a.cg_steps is None else a.cg_steps
    if not a.no_cg and cg_steps > 0:
        cg = NGD(prob, theta0, solver="cg", rtol=rtol, seed=a.seed)
        for _ in range(a.warmup):
            cg.step()
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        creps = [cg.step() for _ in range(cg_steps)]
        torch.cuda.synchronize()
        c1 = time.perf_counter()
        cg_sps = cg_steps / (c1 - c0)

    if a.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- roofline of the one-pass Gramian matvec kernel ----
    n_mv, ms_mv = mv_timer
    avg_ms = ms_mv / max(n_mv, 1)
    elem = 8 if prob.dtype == "f64" else 4
    alg_bytes = N * P * elem + 2 * P * 8
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    if prob.recompute:  # no stored J: the matvec is bound by the vector ALUs, not HBM
        mv_flops = recompute_matvec_flops(prob)
        achieved_tf = mv_flops / (avg_ms * 1e-3) / 1e12
    phases = {k: {"launches": n, "avg_ms": (ms / n if n else 0.0), "ms_per_step": ms / max(n_phase, 1)}
              for k, (n, ms) in timers.items()}
    phases["steps"] = n_phase
    # ---- MFMA roofline of the two sketch contractions (Z = J Omega, B^T = Q^T J) ----
    sk_n = timers["sketch_z"][0] + timers["sketch_w"][0]
    sk_ms = timers["sketch_z"][1] + timers["sketch_w"][1]
    sk_flops = 2.0 * N * P * prob.ell
    sk_achieved = sk_flops / (sk_ms / max(sk_n, 1) * 1e-3) / 1e12 if sk_n else 0.0
    sk_peak = MFMA_PEAK_TFLOPS[prob.sketch_dtype]

    line = {
        "metric": "NGD steps/s at PCG rtol 1e-6 (Nystrom vs plain CG); Gramian-matvec GB/s",
        "value": nys_sps,
        "unit": "NGD steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1000.0 / nys_sps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prob.dtype == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{a.config}: {WORKLOADS[a.config]}; {a.warmup} + {a.steps} NGD steps per solver "
                               f"from the same Glorot start (the last {a.steps} timed)",
                   "P": P, "N": N, "ell": prob.ell, "sketch_dtype": prob.sketch_dtype,
                   "recompute": bool(prob.recompute)},
        "plain_cg": ({"value": cg_sps, "unit": "NGD steps/s", "steps": cg_steps, "warmup": a.warmup,
                      "mean_cg_iters": float(np.mean([r.iters for r in creps])),
                      "cg_iters": [r.iters for r in creps],
                      "converged": all(r.converged for r in creps),
                      "loss_first_last": [creps[0].loss, creps[-1].loss_new]} if creps else None),
        "nystrom_mean_pcg_iters": float(np.mean([r.iters for r in reps])),
        "nystrom_pcg_iters": [r.iters for r in reps],
        "nystrom_converged": all(r.converged for r in reps),
        "speedup_vs_plain_cg": (nys_sps / cg_sps) if creps else None,
        "matvec_gbs": None if prob.recompute else achieved,
        "loss_first_last": [reps[0].loss, reps[-1].loss_new],
        "phases": phases,
        "roofline": ({"bound": "hbm", "kernel": "pcg_rows_kernel (one-pass J^T(J v))", "achieved": achieved,
                      "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                      "traffic": measured_traffic(a.config),
                      "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": avg_ms, "launches": n_mv}
                     if not prob.recompute else
                     {"bound": "alu", "kernel": "jvp_kernel + residual_jacobian_kernel<VJP> (J v, J^T t)",
                      "achieved": achieved_tf, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": achieved_tf / FP32_VECTOR_PEAK_TFLOPS, "traffic": None,
                      "alg_flops_per_launch": mv_flops, "avg_launch_ms": avg_ms, "launches": n_mv}),
        "roofline_sketch": {"bound": "mfma", "kernel": "nt_gemm_kernel (Z = J Omega and B^T = Q^T J)",
                            "achieved": sk_achieved, "peak": sk_peak, "unit": "TFLOP/s",
                            "frac": sk_achieved / sk_peak, "compute_dtype": prob.sketch_dtype,
                            "alg_flops_per_launch": sk_flops, "avg_launch_ms": sk_ms / max(sk_n, 1),
                            "launches": sk_n},
    }
    # release the library handles while the runtime is alive
    torch.cuda.synchronize()
    nys.gp.close()
    if cg is not None:
        cg.gp.close()
    # time-to-rtol 1e-6 at fixed theta and lambda (Nystrom: sketch + core + PCG; plain CG: CG alone) for
    # this workload and the 5D one, and the 5D workload's matvec and BF16-sketch rooflines
    if a.config == "c2" and not a.no_extras:
        line["time_to_rtol"] = [time_to_rtol("c2", a.seed), time_to_rtol("c3", a.seed, at_steps=(0, 10, 49), reps=2)]
        line["c3_subrun"] = c3_subrun(a.seed)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(a.config, a.seed, a.cpu_steps)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
