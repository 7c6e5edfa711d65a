"""Benchmark: full-spectrum eigensolve + spectral application at n = 16384.

One step = the whole hot path on one batch of synthetic input that is already
resident in HBM:
  * the generalized eigensolve K phi = theta M phi of bilinear elements on the
    128 x 128 interior-node unit-square grid (n = 16384): Cholesky, standard
    form, band reduction, bulge chasing, divide and conquer, both
    back-transforms, V = L^-T Z, and in mixed mode (the default) FP32
    back-transforms followed by two FP64 refinement steps;
  * the fractional solutions v(alpha_i, f_j) for 1024 seeded random cubic
    polynomial forcings x 32 orders alpha ~ U(0, 2) (32768 solutions), as a
    replay of the captured application graph;
  * the batched FP64 eigensolve of 256 seeded Q1 rectangles / L-shapes with
    n ~ U[64, 1024] (one persistent launch).
value = solutions per second of the whole step (both eigensolves included).

Outside the timed region: the launch shapes of the application's products
(tuned on the device, or read from the tuning file for this architecture);
the measured FP64 / FP32 matrix-core and copy ceilings; the eigensolve in
both precisions on the Q1 square and on the P1 polygon mesh with two holes
(n = 16384), one warm-up then the median of 3 each, with nominal TFLOP/s
(9 n^3) and the fraction of the stage-wise roofline; the application alone
(3 warm-ups, median of 10 graph replays): fractional solves/s =
nf na / T_apply; live per-kernel rooflines (HIP events on each kernel's
launch stream) with the dominant kernel as `roofline`; and the CPU oracle
timed on a bounded sample.
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
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
KERNELS = ("q2_apply", "sb2st", "scaled_gemm", "batched_eig")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--m", type=int, default=128, help="interior grid side (n = m^2)")
    p.add_argument("--nf", type=int, default=1024)
    p.add_argument("--na", type=int, default=32)
    p.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    p.add_argument("--nbatch", type=int, default=256, help="problems of the batched eigensolve (0 = skip)")
    p.add_argument("--no-compare", action="store_true", help="skip the other precision's eigensolve")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="run one plain device copy of this many MiB before the timed region "
                        "(reference reading for HBM byte counters)")
    p.add_argument("--no-extra", action="store_true",
                   help="skip the untimed measurements (P1 mesh, medians, apply alone, peaks)")
    p.add_argument("--tuning", default=None, help="tuning file (default: the package's file for this "
                                                   "architecture; tuned on the device when missing)")
    p.add_argument("--retune", action="store_true", help="tune the application's products again")
    return p.parse_args()


def host_cpu():
    """CPU model and physical core count of the host (lscpu)."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = dict(line.split(":", 1) for line in out.splitlines() if ":" in line)
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        info["cpu_model"] = kv.get("Model name")
        info["physical_cores"] = int(kv.get("Core(s) per socket", 0)) * int(kv.get("Socket(s)", 0)) or None
        info["logical_cpus"] = int(kv.get("CPU(s)", 0)) or None
    except Exception:
        pass
    return info


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
    host = host_cpu()
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
    return {"value": nf * na / total, "unit": "solves/s", "cores": threads, "kind": "oracle", **host,
            "sample": (f"Jacobi eigensolve at n={t_eig[0]} ({t_eig[1]:.2f} s) scaled by (n/{t_eig[0]})^3 to "
                       f"{t_eig_full:.0f} s; oracle apply at n={n} on 2 (f, alpha) pairs "
                       f"({dt_apply:.2f} s each) scaled to {nf * na} solutions")}


def q2_flops(n: int, b: int) -> float:
    """Algorithmic flops of applying the bulge-chasing reflectors to n
    columns: a reflector of length L costs 4 L n (w = v^T Z, Z -= tau v w^T).
    Sweep i has tasks j = 0 .. 1 + (n-3-i)//b - 1 with L = min(b, n-1-i-j b)."""
    import numpy as np
    tot = 0
    for i in range(max(n - 2, 0)):
        nt = 1 + (n - 3 - i) // b
        j = np.arange(nt)
        tot += int(np.minimum(b, n - 1 - i - j * b).sum())
    return 4.0 * n * tot


def sb2st_flops(n: int, b: int) -> float:
    """Algorithmic flops of the bulge chase: per task with reflector length L
    (next block L'): the left update of the annihilated block 4 L b, the
    two-sided update of the diagonal block 4 L^2, the right update of the
    block below 4 L L'."""
    import numpy as np
    tot = 0.0
    for i in range(max(n - 2, 0)):
        nt = 1 + (n - 3 - i) // b
        j = np.arange(nt)
        L = np.minimum(b, n - 1 - i - j * b).astype(float)
        Ln = np.concatenate([L[1:], [0.0]])
        tot += float((4 * L * b + 4 * L * L + 4 * L * Ln).sum())
    return tot


def traffic_for(kernel: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current source of the kernel (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        f = line.split()
        if len(f) == 4 and f[0] == kernel:
            # f[1]: the kernel's source files joined by '+', hashed in that order
            h = hashlib.sha256()
            for name in f[1].split("+"):
                src = os.path.join(ROOT, "paper_1911_11906_amd", "csrc", name)
                if not os.path.exists(src):
                    return None
                h.update(open(src, "rb").read())
            return float(f[3]) if h.hexdigest()[:16] == f[2] else None
    return None


def half_bandwidth(mesh) -> int:
    """max |i - j| over the stored entries of the mesh's pencil (the
    element couplings of the degrees of freedom, in their own numbering)."""
    import numpy as np
    d = np.asarray(mesh.dof_of_node())[np.asarray(mesh.conn)]
    d = np.where(d >= 0, d, np.nan)
    d = d[~np.all(np.isnan(d), axis=1)]   # elements with every node constrained
    return int(np.nanmax(np.nanmax(d, axis=1) - np.nanmin(d, axis=1)))


def eig_roofline_ms(n: int, prec: str, refine_steps: int, bw: int = -1) -> float:
    """Stage-wise roofline time of the eigensolve: each stage's algorithmic
    flops at the datasheet peak of its arithmetic (FP64: Cholesky n^3/3,
    standard form n^3, band reduction 4/3 n^3, divide and conquer 4/3 n^3,
    back-substitution n^3; both back-transforms 2 n^3 each, FP32 in mixed
    mode; refinement 4 n^3 per step in FP64).  A mass matrix of
    half-bandwidth bw that the library takes on its band (q = ceil(bw/128),
    (q + 1) 128 <= n/4) counts the banded algorithms instead: Cholesky
    n (128 q)^2, and 2 n^2 128 (q + 1) for each of the three block
    substitutions (two for the standard form, one for the back-substitution)."""
    n3 = float(n) ** 3
    q = -(-max(bw, 1) // 128) if bw >= 0 else -1
    if q > 0 and (q + 1) * 128 <= n // 4:
        chol_sygst_trsm = n * (128.0 * q) ** 2 + 3 * 2.0 * n * n * 128 * (q + 1)
    else:
        chol_sygst_trsm = (1 / 3 + 1 + 1) * n3
    f64 = chol_sygst_trsm + (4 / 3 + 4 / 3) * n3 + 4.0 * n3 * refine_steps
    bt = 4.0 * n3
    t = f64 / (PEAK_FP64_TFLOPS * 1e12)
    t += bt / ((PEAK_FP32_TFLOPS if prec == "mixed" else PEAK_FP64_TFLOPS) * 1e12)
    return t * 1e3


def time_eigensolves(op, prec: str, reps: int = 3, bw: int = -1):
    import numpy as np
    op.eigensolve(prec)  # warm-up
    infos = [op.eigensolve(prec) for _ in range(reps)]
    ms = float(np.median([i["total_ms"] for i in infos]))
    n = op.n
    return {"s": ms / 1e3, "tflops_nominal": 9.0 * n ** 3 / (ms / 1e3) / 1e12,
            "roofline_frac": eig_roofline_ms(n, prec, infos[0]["refine_iters"], bw) / ms,
            "refine_iters": infos[0]["refine_iters"],
            "stage_ms": {k: float(np.median([i["stage_ms"][k] for i in infos])) for k in infos[0]["stage_ms"]}}


def setup_tuning(ctx, args, n: int, nf: int, na: int):
    """Launch shapes of the application's two products: read from the tuning
    file for this architecture, or measured on the device (and written)."""
    import torch
    arch = torch.cuda.get_device_properties(ctx.device).gcnArchName.split(":")[0]
    path = args.tuning or os.path.join(ROOT, "paper_1911_11906_amd", "tuning", f"{arch}.json")
    shapes = [("f64", n, nf, n, True, False), ("scaled", n, nf * na, n, False, False)]
    if os.path.exists(path) and not args.retune:
        ctx.load_tuning(path)
        have = {(e["kind"], e["m"], e["n"]) for e in ctx.tuning_table()}
        kinds = {"f64": 0, "scaled": 2}
        if all((kinds[k], m, nn) in have for k, m, nn, _, _, _ in shapes):
            return {"source": os.path.relpath(path, ROOT), "entries": ctx.tuning_table()}
    for kind, m, nn, k, ta, tb in shapes:
        ctx.gemm_tune(kind, m, nn, k, ta=ta, tb=tb, reps=3)
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        ctx.save_tuning(path)
    except OSError:
        pass
    return {"source": "tuned on the device", "entries": ctx.tuning_table()}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: this benchmark runs on one GPU only (--gpus 1)"}))
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
    bmeshes = inputs.batched_problem_meshes(args.nbatch, tag=4) if args.nbatch > 0 else []
    bops = [Operator.assemble(ctx, m) for m in bmeshes]
    bflops = sum(9.0 * m.n_dof ** 3 for m in bmeshes)
    torch.cuda.synchronize()
    tuning = setup_tuning(ctx, args, n, args.nf, args.na)
    prec = args.precision
    other = "mixed" if prec == "fp64" else "fp64"
    binfos = []

    def step():
        info = op.eigensolve(prec)
        op.apply_graph(F, alpha, out=U)
        if bops:
            binfos.append(ctx.eigensolve_batched(bops)[0])
        return info

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # one elementwise kernel: reads and writes MIB MiB
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    extra = {}
    if not args.no_extra:
        extra["peaks_measured"] = ctx.measure_peaks()
        # the eigensolve alone: both precisions on both n = 16384 meshes
        eig = {"q1_square": {p: time_eigensolves(op, p, bw=half_bandwidth(mesh)) for p in ("fp64", "mixed")}}
        op.eigensolve(prec)  # leave the timed precision's basis in place
        pm = inputs.p1_polygon_with_holes(16384)
        op3 = Operator.assemble(ctx, pm)
        eig["p1_polygon"] = {p: time_eigensolves(op3, p, bw=half_bandwidth(pm)) for p in ("fp64", "mixed")}
        op3.close()
        for mk in eig:
            eig[mk]["mixed_speedup_over_fp64"] = eig[mk]["fp64"]["s"] / eig[mk]["mixed"]["s"]
        extra["eigensolve_n16384"] = eig
        # the application alone: graph replays timed with events on the caller's stream
        st = torch.cuda.current_stream(dev)
        for _ in range(3):
            op.apply_graph(F, alpha, out=U)
        times = []
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            op.apply_graph(F, alpha, out=U)
            e1.record(st)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        t_apply = float(np.median(times))
        nsol = args.nf * args.na
        extra["apply"] = {"ms": t_apply, "apply_solves_per_s": nsol / (t_apply / 1e3),
                          "tflops": 2.0 * n * n * args.nf * (1 + args.na) / (t_apply / 1e3) / 1e12,
                          "bound_solves_per_s": nsol / (2.0 * n * n * args.nf * (1 + args.na)
                                                        / (PEAK_FP64_TFLOPS * 1e12))}
    # the fused scaled product timed live on its launch stream (eager launches)
    if args.warmup == 0 and args.no_extra:
        op.eigensolve(prec)  # the application needs a basis
    ctx.kernel_timing(True)
    for k in KERNELS:
        ctx.kernel_time(k)
    for _ in range(3):
        op.apply(F, alpha, out=U)
    torch.cuda.synchronize()
    sg_cnt, sg_ms = ctx.kernel_time("scaled_gemm")
    info_other = op.eigensolve(other) if not args.no_compare else None
    op.eigensolve(prec)
    torch.cuda.synchronize()
    for k in KERNELS:
        ctx.kernel_time(k)  # drop anything recorded before
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ktime = {k: ctx.kernel_time(k) for k in KERNELS}
    ctx.kernel_timing(False)
    ktime["scaled_gemm"] = (sg_cnt, sg_ms)

    step_s = wall / args.steps
    nsol = args.nf * args.na
    flops_eig = 9.0 * n ** 3
    eig_s = float(np.median([i["total_ms"] for i in infos])) / 1e3
    stages = {k: float(np.median([i["stage_ms"][k] for i in infos])) for k in infos[0]["stage_ms"]}
    b = 64
    peak_mm = PEAK_FP32_TFLOPS if prec == "mixed" else PEAK_FP64_TFLOPS
    per_launch_flops = {
        "q2_apply": q2_flops(n, b),
        "sb2st": sb2st_flops(n, b),
        "scaled_gemm": 2.0 * n * n * nsol,
        "batched_eig": bflops,
    }
    kernels = {}
    for k, (cnt, ms) in ktime.items():
        if cnt == 0:
            continue
        fl = per_launch_flops[k] * cnt
        ach = fl / (ms / 1e3) / 1e12
        bound, peak = ("alu", PEAK_FP64_TFLOPS) if k in ("sb2st", "batched_eig") else (
            "mfma", peak_mm if k == "q2_apply" else PEAK_FP64_TFLOPS)
        kernels[k] = {"launches": cnt, "total_ms": ms, "avg_ms": ms / cnt, "flops_per_launch": fl / cnt,
                      "bound": bound, "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak}
    # dominant kernel: largest time per step (the scaled product was timed
    # on its own launches; each step launches every kernel once)
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    d = kernels[dom]
    traffic = traffic_for(dom)
    roofline = {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": "TFLOP/s",
                "frac": d["frac"], "traffic": traffic, "kernel": dom, "avg_launch_ms": d["avg_ms"],
                "flops_per_launch": d["flops_per_launch"]}
    apply_ms = kernels.get("scaled_gemm", {}).get("avg_ms")
    bms = [bi["total_ms"] for bi in binfos[-args.steps:]]
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
        "dtype": "f64" if prec == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"Q1 unit square {args.m}x{args.m} (n={n}): {prec} full generalized eigensolve + "
                               f"{args.nf} cubic forcings x {args.na} alpha (graph replay) + batched FP64 "
                               f"eigensolve of {args.nbatch} seeded rectangles/L-shapes (n in [64, 1024])", "n": n,
                   "nf": args.nf, "na": args.na, "precision": prec, "nbatch": args.nbatch},
        "eigensolve_s": eig_s,
        "eigensolve_tflops_nominal": flops_eig / eig_s / 1e12,
        "eigensolve_stage_ms": stages,
        "refine_iters": infos[0]["refine_iters"],
        "scaled_gemm_tflops": (2.0 * n * n * nsol) / (apply_ms / 1e3) / 1e12 if apply_ms else None,
        "roofline": roofline,
        "batched_eigensolve": None if not bops else {
            "problems": len(bops), "n_min": min(m.n_dof for m in bmeshes), "n_max": max(m.n_dof for m in bmeshes),
            "launch_ms": float(np.median(bms)), "problems_per_s": len(bops) / (float(np.median(bms)) / 1e3),
            "tflops_nominal": bflops / (float(np.median(bms)) / 1e3) / 1e12},
        "kernels": kernels,
        "tuning": tuning,
        **extra,
    }
    if info_other is not None:
        t_other = info_other["total_ms"] / 1e3
        out[f"eigensolve_{other}_s"] = t_other
        t64, tmx = (eig_s, t_other) if prec == "fp64" else (t_other, eig_s)
        out["mixed_speedup_over_fp64"] = t64 / tmx
    # release every library object before the process exits
    for o in bops:
        o.close()
    op.close()
    torch.cuda.synchronize()
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.m, args.nf, args.na, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
