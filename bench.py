"""Benchmark: full-spectrum eigensolve + spectral application at n = 16384.

One step = the whole hot path on one batch of synthetic input that is already
resident in HBM:
  * the FP64 generalized eigensolve K phi = theta M phi (Cholesky, standard
    form, band reduction, bulge chasing, divide and conquer, both
    back-transforms, V = L^-T Z) of bilinear elements on the 128 x 128
    interior-node unit-square grid (n = 16384);
  * the fractional solutions v(alpha_i, f_j) for 1024 seeded random cubic
    polynomial forcings x 32 orders alpha ~ U(0, 2) (32768 solutions).
value = solutions per second of the whole step (eigensolve included).

Extra fields: eigensolve seconds and TFLOP/s (nominal 9 n^3), the apply alone
(solves/s, TFLOP/s), per-stage times, a live roofline of the dominant
kernel, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "eigensolve s & TFLOP/s at n=16384, mixed vs FP64; fractional solves/sec"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--m", type=int, default=128, help="interior grid side (n = m^2)")
    p.add_argument("--nf", type=int, default=1024)
    p.add_argument("--na", type=int, default=32)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work")
    return p.parse_args()


def cpu_baseline(m: int, nf: int, na: int, budget: float):
    """Time the oracle (never tuned) on a bounded sample of the same workload:
    the Jacobi eigensolve at the largest n_s that fits the budget (its time
    is scaled by (n/n_s)^3, the eigensolve's cost law), and the oracle's
    spectral application at the full n on a few (f, alpha) pairs with the
    exact discrete basis (scaled linearly to the full batch)."""
    import numpy as np

    import oracle
    from oracle.closed_form import Q1Rectangle
    from paper_1911_11906_amd import inputs

    threads = oracle.num_threads()
    # eigensolve sample
    ms = 12
    t_eig = None
    while True:
        mesh = inputs.q1_rectangle(ms, ms)
        K, M = oracle.assemble(mesh)
        t0 = time.perf_counter()
        oracle.eigensolve(K, M)
        dt = time.perf_counter() - t0
        t_eig = (ms * ms, dt)
        if dt > budget / 8 or ms >= 40:
            break
        ms = int(ms * 1.4) + 1
    n = m * m
    t_eig_full = t_eig[1] * (n / t_eig[0]) ** 3
    # apply sample at full n with the exact basis (dense V built from the closed form)
    mesh = inputs.q1_rectangle(m, m)
    cf = Q1Rectangle(m, m)
    th = np.add.outer(cf.ty, cf.tx).ravel()
    V = np.asfortranarray(np.kron(cf.Ny, cf.Nx))
    _, M = oracle.assemble(mesh) if n <= 4096 else (None, None)
    if M is None:
        # mass matrix of the full grid (dense) from the oracle's assembly
        K, M = oracle.assemble(mesh)
    F = inputs.polynomial_forcings(mesh, 1, tag=4)
    al = inputs.alphas_uniform(2, tag=4)
    t0 = time.perf_counter()
    oracle.apply_fractional(th, V, M, F, al)
    dt_apply = (time.perf_counter() - t0) / 2.0
    total = t_eig_full + dt_apply * nf * na
    return {"value": nf * na / total, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": (f"Jacobi eigensolve at n={t_eig[0]} ({t_eig[1]:.2f} s) scaled by (n/{t_eig[0]})^3 to "
                       f"{t_eig_full:.0f} s; oracle apply at n={n} on 2 (f, alpha) pairs "
                       f"({dt_apply:.2f} s each) scaled to {nf * na} solutions")}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: only --gpus 1 is supported"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1911_11906_amd import inputs
    from paper_1911_11906_amd.api import Context, Operator, colmajor, empty_colmajor

    dev = torch.device("cuda", 0)
    ctx = Context(0)
    mesh = inputs.q1_rectangle(args.m, args.m)
    n = mesh.n_dof
    op = Operator.assemble(ctx, mesh)
    F = colmajor(inputs.polynomial_forcings(mesh, args.nf, tag=4), dev)
    alpha = inputs.alphas_uniform(args.na, tag=4)
    U = empty_colmajor(n, args.nf * args.na, dev)
    torch.cuda.synchronize()

    def step():
        info = op.eigensolve("fp64")
        s = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        op.apply(F, alpha, out=U)
        e1.record(s)
        return info, e0, e1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos, apply_ms = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info, e0, e1 = step()
        infos.append(info)
        apply_ms.append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    apply_ms = [a.elapsed_time(b) for a, b in apply_ms]
    eig_ms = [i["total_ms"] for i in infos]
    step_s = wall / args.steps
    nsol = args.nf * args.na
    flops_eig = 9.0 * n ** 3
    flops_apply = 2.0 * n * n * args.nf * (1 + args.na)
    eig_s = float(np.median(eig_ms)) / 1e3
    app_s = float(np.median(apply_ms)) / 1e3
    stages = {k: float(np.median([i["stage_ms"][k] for i in infos])) for k in infos[0]["stage_ms"]}
    out = {
        "metric": METRIC,
        "value": nsol / step_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"Q1 unit square {args.m}x{args.m} (n={n}): FP64 full eigensolve + "
                               f"{args.nf} cubic forcings x {args.na} alpha", "n": n, "nf": args.nf,
                   "na": args.na, "precision": "fp64"},
        "eigensolve_s": eig_s,
        "eigensolve_tflops_nominal": flops_eig / eig_s / 1e12,
        "eigensolve_stage_ms": stages,
        "apply_s": app_s,
        "apply_solves_per_s": nsol / app_s,
        "apply_tflops": flops_apply / app_s / 1e12,
        "roofline": {"bound": "mfma", "achieved": flops_apply / app_s / 1e12, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": flops_apply / app_s / 1e12 / PEAK_FP64_TFLOPS, "traffic": None,
                     "kernel": "spectral apply (scaled GEMM)"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.m, args.nf, args.na, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
