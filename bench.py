"""Benchmark: determinant-updates/s of the sigma build H.c on one MI355X.

Workload: complex spinor FCI, 24 spinors, 8 electrons (735,471 determinants),
integrals seeded as (pq|rs) = sum_P L^P_pq L^P_rs with a rank-32 Hermitian
factor (entries N(0, 0.03)); 2 roots, so one step is the sigma build of the
2 new Davidson directions (n_vec = 2), inputs resident in HBM.
Metric: det-updates/s = nnz(H) * n_vec / t_step (nonzero couplings applied
per second).  Also reported: the dominant kernel against its roofline, the
Davidson solve latency (p50/p99) at the 1e-8 Eh certificate, and the CPU
oracle on a bounded sample of rows.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-solve]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (and matrix) peak
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--partition", default="24", help="subspace sizes, e.g. 24 or 8,8,8")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--solves", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calib-mb", type=float, default=0.0,
                    help="only run a plain device copy of this many MB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calib_mb > 0:
        # a plain copy kernel of known size: reads and writes exactly n bytes per launch
        n = int(args.copy_calib_mb * 2 ** 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(args.steps, 1)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8, "launches": max(args.steps, 1)}))
        return

    import synth
    import paper_2505_20375_amd as stpci

    torch.cuda.set_device(0)
    cfg = synth.CONFIGS["c2"]
    ints, sp, roots = synth.config("c2")
    sub = [int(x) for x in args.partition.split(",")]
    assert sum(sub) == sp.n_spin_orb
    space = synth.SpaceSpec(sp.n_elec, sub)
    ctx = stpci.Context(0)
    ctx.set_integrals(ints.h, ints.g)
    ctx.set_space(space.n_elec, space.sub, space.lo, space.hi)
    info = ctx.space_info()
    n = info.n_dets
    n_vec = roots
    log("space: %d determinants, %d categories, nnz(H) %.4g, W1+W2 %.4g" % (n, info.n_cat, info.nnz_h,
                                                                         info.w_sigma_macs))
    g = torch.Generator(device="cuda").manual_seed(2102)
    c = torch.randn(n_vec * n, dtype=torch.complex128, device="cuda", generator=g)
    c /= torch.linalg.vector_norm(c)
    out = torch.empty_like(c)

    for _ in range(args.warmup):
        ctx.sigma(c, out, n_vec=n_vec)
    torch.cuda.synchronize()
    ctx.profile(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for i in range(args.steps):
        ctx.sigma(c, out, n_vec=n_vec)
        log("step %d issued" % i)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_ev = ev0.elapsed_time(ev1)
    n2, t2 = ctx.kernel_time("sigma2e")
    n1, t1 = ctx.kernel_time("sigma1e")
    ctx.profile(False)
    ms_per_step = ms_ev / args.steps
    value = info.nnz_h * n_vec / (ms_per_step * 1e-3)
    log("sigma step: %.3f ms (events), %.3f ms (wall)" % (ms_per_step, wall * 1e3 / args.steps))

    # roofline of the dominant kernel: algorithmic FP64 flops per launch
    W1, W2, n_inter, max_deg = ctx.work_counts()
    flops_2e = 8.0 * W2 * n_vec
    avg2 = t2 / max(n2, 1)
    achieved = flops_2e / (avg2 * 1e-3) / 1e12
    roof = {"kernel": "sigma2e", "bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None,
            "avg_launch_ms": round(avg2, 4), "flops_per_launch": flops_2e,
            "sigma1e_avg_ms": round(t1 / max(n1, 1), 4)}

    res = {
        "metric": "determinant-updates/s in H.c sigma",
        "value": value,
        "unit": "det-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "complex spinor FCI sigma, 24 spinors, 8 electrons, %d determinants, "
                               "n_vec=%d" % (n, n_vec),
                   "n_dets": n, "partition": sub, "n_vec": n_vec, "nnz_h": info.nnz_h,
                   "w1_macs": W1, "w2_macs": W2, "dets_per_s": n * n_vec / (ms_per_step * 1e-3)},
        "roofline": roof,
    }

    # precision form: FP32 contraction of the same step
    for _ in range(max(1, args.warmup)):
        ctx.sigma(c, out, n_vec=n_vec, precision=stpci.FP32)
    out64 = torch.empty_like(out)
    ctx.sigma(c, out64, n_vec=n_vec)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        ctx.sigma(c, out, n_vec=n_vec, precision=stpci.FP32)
    e1.record()
    torch.cuda.synchronize()
    ms32 = e0.elapsed_time(e1) / args.steps
    rel = float(torch.linalg.vector_norm(out - out64) / torch.linalg.vector_norm(out64))
    res["precision"] = {"sigma_fp32_ms": ms32, "sigma_fp64_ms": ms_per_step, "sigma_speedup": ms_per_step / ms32,
                        "sigma_fp32_rel_err": rel,
                        "contraction": "FP32 integrals, coefficients and accumulation; FP64 sigma, residual, "
                                       "orthogonalisation and subspace solve"}
    if not args.no_solve:
        res["solve"] = _solve(ctx, roots, args.solves, stpci.FP64)
        mixed = _solve(ctx, roots, args.solves, stpci.FP32)
        res["precision"]["solve_mixed"] = mixed
        res["precision"]["solve_speedup"] = res["solve"]["p50_ms"] / mixed["p50_ms"]
        res["precision"]["energy_diff_eh"] = max(abs(a - b) for a, b in zip(mixed["energies"],
                                                                            res["solve"]["energies"]))
    if not args.no_cpu:
        res["cpu_baseline"] = _cpu_baseline(ints, sp, info.nnz_h / n, args.cpu_seconds)
    print(json.dumps(res))


def _solve(ctx, roots, nsolve, precision):
    """Davidson time-to-solution at residual tolerance 1e-5; the lowest energy
    is then within ||r0||^2 / gamma^- (gap theorem with the rigorous gap
    bound from the second root), reported as energy_bound_eh (<= 1e-8 Eh)."""
    import numpy as np
    import torch
    times, its = [], []
    e = r = None
    for i in range(nsolve):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, r, it, st = ctx.davidson(k=roots, tol=1e-5, max_iter=400, precision=precision)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        its.append(it)
        log("solve %d (%s): %.1f ms, %d iterations" % (i, "fp32+fp64" if precision else "fp64", times[-1], it))
    gamma = (e[1] - r[1]) - e[0] if len(e) > 1 else None
    cert = (r[0] ** 2 / gamma) if gamma and gamma > 0 else None
    n64, n32 = ctx.dav_stats()
    return {"p50_ms": float(np.percentile(times, 50)), "p99_ms": float(np.percentile(times, 99)),
            "n": nsolve, "iterations": its[-1], "energies": [float(x) for x in e],
            "resid": [float(x) for x in r], "energy_bound_eh": cert, "tol_residual": 1e-5,
            "sigma_vectors_fp64": n64, "sigma_vectors_fp32": n32}


def _cpu_baseline(ints, sp, nnz_per_row, seconds):
    """The CPU oracle (row-driven Slater-Condon sigma) on a bounded sample of
    rows of the same workload, extrapolated to det-updates/s."""
    import numpy as np
    import synth
    from oracle import csc, space as ospace
    nthreads = os.cpu_count() or 1
    dets = ospace.enumerate_dets(sp.n_elec, sp.sub, sp.lo, sp.hi)
    c = synth.test_vector(len(dets), 2002)
    rng = np.random.default_rng(0)
    rows = rng.choice(len(dets), 2000, replace=False)
    t0 = time.perf_counter()
    csc.sigma_rows(dets, ints.h, ints.g, c, rows, nthreads=nthreads)
    t = time.perf_counter() - t0
    nrows = int(min(len(dets), max(2000, 2000 * seconds / max(t, 1e-3))))
    rows = rng.choice(len(dets), nrows, replace=False)
    t0 = time.perf_counter()
    csc.sigma_rows(dets, ints.h, ints.g, c, rows, nthreads=nthreads)
    t = time.perf_counter() - t0
    return {"value": nnz_per_row * nrows / t, "unit": "det-updates/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d random rows of the 24-spinor/8-electron sigma (row-driven Slater-Condon, "
                      "%.1f s)" % (nrows, t)}


if __name__ == "__main__":
    main()
