"""Benchmark: determinant-updates/s of the sigma build H.c on one MI355X.

Headline workload: the STP-DAS categorical space of 40 complex spinors split
12 | 16 | 12 with occupation windows [2..6] | [4..10] | [2..6] and 11
electrons (1,365,867,360 determinants in 10 categories, 21.9 GB per vector),
integrals seeded as (pq|rs) = sum_P L^P_pq L^P_rs with a rank-16 Hermitian
factor (entries N(0, 0.05)); lowest root, so one step is the sigma build of
one Davidson direction (n_vec = 1), inputs resident in HBM.
Metric: det-updates/s = nnz(H) * n_vec / t_step (nonzero couplings applied
per second).  Also reported: the dominant kernel against its roofline (HIP
events recorded by the library around that kernel), the BF16 form of the
same step, the 24-spinor / 8-electron complex FCI problem (sigma, precision
forms, Davidson solve latency p50/p99 with the library's gap certificate),
a continuous-batching serving run, and the CPU oracle on a bounded sample
of rows of the headline space.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-solve] [--serve N]
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
BF16_PEAK_TFLOPS = 2500.0   # MI355X dense bfloat16 matrix-core peak
FP32_PEAK_TFLOPS = 157.3   # MI355X dense FP32 matrix-core peak
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3p", choices=["c3p", "c2"],
                    help="headline: c3p (40 spinors, 12|16|12, 11 electrons) or c2 (24 spinors, 8 electrons)")
    ap.add_argument("--partition", default="24", help="config-2 subspace sizes, e.g. 24 or 8,8,8")
    ap.add_argument("--no-c2", action="store_true", help="skip the config-2 section")
    ap.add_argument("--no-bf16", action="store_true", help="skip the FP32 and BF16 steps of the headline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--solves", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--serve", type=int, default=512, help="requests in the serving run (0: skip)")
    ap.add_argument("--no-sparse", action="store_true", help="skip the sparse-vector sigma timings")
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured GEMM and copy reference rates")
    ap.add_argument("--serve-max-dets", type=int, default=300000)
    ap.add_argument("--serve-rate", type=float, default=40.0, help="Poisson arrival rate (requests/s)")
    ap.add_argument("--copy-calib-mb", type=float, default=0.0,
                    help="only run a plain device copy of this many MB (counter calibration)")
    ap.add_argument("--precision-study", type=int, default=0, metavar="ITERS",
                    help="only run the precision-form study (Davidson solves in FP64, FP32 + FP64 and BF16 + "
                         "FP64 on a 24,190,320-determinant space of the headline integrals, then ITERS "
                         "iterations of the FP64 and of the FP32 solve on the headline space) and print its JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
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
    if args.precision_study > 0:
        print(json.dumps(_precision_study(args.precision_study)))
        return
    if args.workload == "c3p":
        res = _headline_c3p(args)
        ctx = None
        if not args.no_c2:
            sec, ctx = _config2(args)
            sec.pop("n_gpus", None)
            for key in ("metric", "unit", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline",
                        "data"):
                sec.pop(key, None)
            res["config2"] = sec
    else:
        res, ctx = _config2(args)
    if not args.no_peaks:
        # reference rates only: an error here is reported, not fatal to the line
        try:
            res["measured_peaks"] = _measured_peaks(res["roofline"])
        except RuntimeError as exc:
            res["measured_peaks"] = {"error": str(exc)[:200]}
    if args.serve > 0:
        del ctx
        res["serving"] = _serve(args.serve, args.serve_max_dets, args.serve_rate)
    if not args.no_cpu:
        if args.workload == "c3p":
            res["cpu_baseline"] = _cpu_baseline_c3p(args.cpu_seconds)
        else:
            ints, sp, _ = synth.config("c2")
            res["cpu_baseline"] = _cpu_baseline(ints, sp, res["config"]["nnz_h"] / res["config"]["n_dets"],
                                                args.cpu_seconds)
    print(json.dumps(res))


def _headline_c3p(args):
    """The headline step: FP64 sigma of one vector on the 40-spinor,
    12|16|12, 11-electron STP-DAS space, and the FP32 and BF16 forms of the
    same step."""
    import numpy as np
    import torch
    import synth
    import paper_2505_20375_amd as stpci

    ints, sp, roots = synth.config("c3p")
    ctx = stpci.Context(0)
    ctx.set_integrals(ints.h, ints.g)
    ctx.set_space(sp.n_elec, sp.sub, sp.lo, sp.hi)
    info = ctx.space_info()
    n = info.n_dets
    n_vec = roots
    log("space: %d determinants, %d categories, nnz(H) %.4g" % (n, info.n_cat, info.nnz_h))
    g = torch.Generator(device="cuda").manual_seed(3103)
    c = torch.randn(n_vec * n, dtype=torch.complex128, device="cuda", generator=g)
    c /= torch.linalg.vector_norm(c)
    out = torch.empty_like(c)
    for i in range(args.warmup):
        ctx.sigma(c, out, n_vec=n_vec)
        torch.cuda.synchronize()
        log("warmup %d done" % i)
    ctx.profile(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for i in range(args.steps):
        ctx.sigma(c, out, n_vec=n_vec)
        if i + 1 < args.steps:
            torch.cuda.synchronize()   # progress line per step (the steps run back to back on the device)
        log("step %d done" % i)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    nk, tk = ctx.kernel_time("sigma")
    ctx.profile(False)
    value = info.nnz_h * n_vec / (ms_per_step * 1e-3)
    log("sigma step: %.1f ms (events), %.1f ms (wall)" % (ms_per_step, wall * 1e3 / args.steps))
    W1, W2, _, _ = ctx.work_counts()
    Wp, n_pair, max_pdeg = ctx.pair_counts()
    kname = ctx.sigma_kernel()
    avg = tk / max(nk, 1)   # the kernel launches of one step, summed per step
    flops = 8.0 * Wp * n_vec
    flops_paper = 8.0 * (W1 + W2) * n_vec
    ex_flops, items = ctx.sb_counts(n_vec) if kname == "pair_sb" else (None, None)
    achieved = flops / (avg * 1e-3) / 1e12
    roof = {"kernel": "k_sigma_pair_sb (one pass: pair-resolved 1e + 2e sigma, the pair intermediates of a "
                      "category sharing their leading-subspace strings contracted as one product, FP64 matrix "
                      "cores, v_mfma_f64_16x16x4f64; one launch per column-group count)",
            "bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": _traffic(n_vec, kname, "c3p"),
            "avg_launch_ms": round(avg, 2), "launches": nk, "flops_per_launch": flops,
            "flops_definition": "8 Wp n_vec: Wp = sum over the (N-2)-electron intermediates of deg^2 complex "
                                "multiply-adds (one- and two-electron parts together)",
            "algorithmic_bytes_per_launch": 2 * n_vec * n * 16,
            "paper_formulation_flops_per_launch": flops_paper,
            "paper_formulation_equiv_tflops": round(flops_paper / (avg * 1e-3) / 1e12, 3),
            "paper_formulation_equiv_over_peak": round(flops_paper / (avg * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)}
    if ex_flops:
        roof["executed_flops_per_launch"] = ex_flops
        roof["executed_tflops"] = round(ex_flops / (avg * 1e-3) / 1e12, 3)
        roof["frac_executed"] = round(ex_flops / (avg * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)
        roof["items"] = items
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
        "config": {"workload": "STP-DAS categorical sigma, 40 complex spinors as 12|16|12, windows "
                               "[2..6]|[4..10]|[2..6], 11 electrons, %d determinants in %d categories, n_vec=%d"
                               % (n, info.n_cat, n_vec),
                   "n_dets": n, "n_categories": info.n_cat, "partition": sp.sub, "windows": [sp.lo, sp.hi],
                   "n_elec": sp.n_elec, "n_vec": n_vec, "nnz_h": info.nnz_h, "w1_macs": W1, "w2_macs": W2,
                   "wp_macs": Wp, "dets_per_s": n * n_vec / (ms_per_step * 1e-3)},
        "roofline": roof,
    }
    if not args.no_bf16:
        # the reduced-precision forms of the same step, error against FP64:
        # FP32 (the same spectator-batched kernel with the FP32 table and B
        # tiles on v_mfma_f32_16x16x4f32) and BF16 (bfloat16 integrals and
        # coefficients on the matrix cores); FP32 accumulation, FP64 sums
        out2 = torch.empty_like(out)
        prec = {"sigma_fp64_ms": ms_per_step}
        for pname, pcode, kdesc in (
                ("fp32", stpci.FP32, "k_sigma_pair_sb FP32 instance (v_mfma_f32_16x16x4f32, FP32 accumulation)"),
                ("bf16", stpci.BF16, "k_sigma_pair_mfma (v_mfma_f32_16x16x32_bf16, FP32 accumulation)")):
            ctx.sigma(c, out2, n_vec=n_vec, precision=pcode)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.sigma(c, out2, n_vec=n_vec, precision=pcode)
            e1.record()
            torch.cuda.synchronize()
            ms_p = e0.elapsed_time(e1)
            err = float(torch.linalg.vector_norm(out2 - out) / torch.linalg.vector_norm(out))
            log("%s sigma: %.1f ms, relative error %.2e" % (pname.upper(), ms_p, err))
            prec.update({"sigma_%s_ms" % pname: ms_p, "sigma_%s_speedup" % pname: ms_per_step / ms_p,
                         "sigma_%s_rel_err" % pname: err, "%s_kernel" % pname: kdesc})
        res["precision"] = prec
        del out2
    if not args.no_sparse:
        del c, out
        torch.cuda.empty_cache()
        # categorically compressed vectors of 1e-6 .. 1e-4 of the space
        res["compressed"] = _compressed(ctx, n, torch.complex128, ms_per_step / n_vec, (1e-6, 1e-5, 1e-4), 3104)
        del ctx
    else:
        del c, out, ctx
    torch.cuda.empty_cache()
    return res


def _precision_study(iters):
    """The precision form (FP32 or BF16 contractions, then FP64 refinement)
    against plain FP64 on the headline integrals: (1) whole Davidson solves
    to residual 1e-5 on the 8-electron space of the same 12|16|12 partition
    with windows [2..3]|[3..4]|[2..3] (24,190,320 determinants), median of 3
    after a warm-up; (2) on the headline space itself, whose solve to 1e-5
    takes longer than one run should, the first `iters` iterations of the
    FP64 solve and of the FP32 phase, timed per iteration, with their
    energies and residual norms side by side."""
    import numpy as np
    import torch
    import synth
    import paper_2505_20375_amd as stpci
    ints, sp3, _ = synth.config("c3p")
    out = {"study": "precision form vs FP64, Davidson, 1 root"}
    sp = synth.SpaceSpec(8, [12, 16, 12], [2, 3, 2], [3, 4, 3])
    ctx = stpci.Context(0)
    ctx.set_integrals(ints.h, ints.g)
    ctx.set_space(sp.n_elec, sp.sub, sp.lo, sp.hi)
    small = {"n_dets": ctx.space_info().n_dets, "partition": sp.sub, "windows": [sp.lo, sp.hi],
             "n_elec": sp.n_elec, "tol_residual": 1e-5}
    ctx.davidson(k=1, tol=1e-5, max_iter=300)
    for name, prec in (("fp64", stpci.FP64), ("fp32+fp64", stpci.FP32), ("bf16+fp64", stpci.BF16)):
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, r, it, st = ctx.davidson(k=1, tol=1e-5, max_iter=300, precision=prec)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        small[name] = {"s": float(np.median(ts)), "energy": float(e[0]), "resid": float(r[0]),
                       "iterations": int(it), "sigma_vectors_fp64": ctx.dav_sigma_count(stpci.FP64),
                       "sigma_vectors_fp32": ctx.dav_sigma_count(stpci.FP32),
                       "sigma_vectors_bf16": ctx.dav_sigma_count(stpci.BF16)}
        log("%d-determinant solve (%s): %.2f s, %d iterations, E %.12f" % (small["n_dets"], name, small[name]["s"],
                                                                          it, e[0]))
    for name in ("fp32+fp64", "bf16+fp64"):
        small[name]["speedup"] = small["fp64"]["s"] / small[name]["s"]
        small[name]["energy_diff_eh"] = abs(small[name]["energy"] - small["fp64"]["energy"])
    out["space_24M"] = small
    del ctx
    torch.cuda.empty_cache()
    ctx = stpci.Context(0)
    ctx.set_integrals(ints.h, ints.g)
    ctx.set_space(sp3.n_elec, sp3.sub, sp3.lo, sp3.hi)
    big = {"n_dets": ctx.space_info().n_dets, "iterations": iters}
    for name, prec in (("fp64", stpci.FP64), ("fp32", stpci.FP32)):
        ctx.dav_begin(k=1, tol=1e-5, max_iter=iters, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ts = []
        for i in range(iters):
            stpci.dav_sigma_batched([ctx])
            done = ctx.dav_finish_step()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            log("headline space, %s iteration %d: %.1f s" % (name, i + 1, ts[-1]))
            if done:
                break
        h = ctx.history(full=True)
        big[name] = {"seconds": ts[-1], "s_per_iteration": ts[-1] / len(ts),
                     "energy": [float(x) for x in h["energies"][:len(ts), 0]],
                     "resid": [float(x) for x in h["resid"][:len(ts), 0]]}
    n = min(len(big["fp64"]["energy"]), len(big["fp32"]["energy"]))
    big["per_iteration_speedup"] = big["fp64"]["s_per_iteration"] / big["fp32"]["s_per_iteration"]
    big["max_energy_diff_eh"] = max(abs(a - b) for a, b in zip(big["fp64"]["energy"][:n], big["fp32"]["energy"][:n]))
    big["max_resid_rel_diff"] = max(abs(a - b) / b for a, b in zip(big["fp32"]["resid"][:n], big["fp64"]["resid"][:n]))
    out["headline_space"] = big
    del ctx
    torch.cuda.empty_cache()
    return out


def _cpu_baseline_c3p(seconds):
    """The CPU oracle (list-free Slater-Condon rows of the windowed space) on
    bounded samples of rows of the headline space, about `seconds` of wall
    time each on 1, 4 and all host threads of the GPU's share (at most 16),
    extrapolated to det-updates/s; the best rate is reported with the thread
    count that gave it.  The rows' determinants are drawn beforehand (not
    timed): the oracle's work is forming and applying each row's nonzero
    couplings.  Threads share the integrals (a process per core would hold
    41 MB of them each); the oracle's C routine runs outside the interpreter
    lock, but each call allocates and clears its row buffers, so threads
    scale poorly (the oracle is timed as it stands)."""
    import numpy as np
    import synth
    from concurrent.futures import ThreadPoolExecutor
    from oracle import csc
    import paper_2505_20375_amd as stpci
    ints, sp, _ = synth.config("c3p")
    ctx = stpci.Context(-1)
    ctx.set_space(sp.n_elec, sp.sub, sp.lo, sp.hi)
    info = ctx.space_info()
    ncores = max(1, min(16, len(os.sched_getaffinity(0))))
    rng = np.random.default_rng(0)

    def rows_work(bits_list):
        tot = 0
        acc = 0j
        for b in bits_list:
            kb, vals = csc.h_row_window(sp.sub, sp.lo, sp.hi, ints.h, ints.g, int(b))
            acc += np.dot(vals, np.ones(len(kb)))   # stand-in coefficients
            tot += len(kb)
        return tot

    def run(nrows, nth):
        addrs = rng.choice(info.n_dets, nrows, replace=False)
        bits = [ctx.address_to_det(int(a)) for a in addrs]
        parts = [bits[i::nth] for i in range(nth)]
        t0 = time.perf_counter()
        with ThreadPoolExecutor(nth) as ex:
            tot = sum(ex.map(rows_work, parts))
        return tot, time.perf_counter() - t0

    run(4, 1)   # untimed: the first call loads the oracle's library
    scan = []
    for nth in sorted({1, min(4, ncores), ncores}):
        # a short run sizes the timed one at about `seconds` of wall time
        est_rows = max(nth * 16, 32)
        tot, t = run(est_rows, nth)
        nrows = int(max(est_rows, est_rows * seconds / max(t, 1e-3)))
        tot, t = run(nrows, nth)
        if t < 0.5 * seconds:   # the short run overestimated the time per row
            nrows = int(nrows * seconds / max(t, 1e-3))
            tot, t = run(nrows, nth)
        scan.append({"threads": nth, "rows": nrows, "couplings": int(tot), "seconds": round(t, 2),
                     "det_updates_per_s": tot / t})
    best = max(scan, key=lambda r: r["det_updates_per_s"])
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": best["det_updates_per_s"], "unit": "det-updates/s", "cores": best["threads"], "kind": "oracle",
            "cpu_model": model, "scan": scan,
            "sample": "random rows of the 40-spinor 12|16|12 11-electron space, list-free row-driven "
                      "Slater-Condon, %d rows (%d couplings) in %.1f s on %d threads; best of 1, 4 and %d threads"
                      % (best["rows"], best["couplings"], best["seconds"], best["threads"], ncores)}


def _compressed(ctx, n, dtype, dense_ms, densities, seed):
    """sigma of categorically compressed vectors (stpci_sigma_csc): a seeded
    vector with the given fraction of nonzero coefficients at random
    addresses, compressed (stpci_csc_compress), then one timed sigma of the
    compressed vector after an untimed one; dense_ms: the dense sigma of one
    vector on the same space, for comparison."""
    import numpy as np
    import torch
    out = {}
    rng = np.random.default_rng(seed)
    for dens in densities:
        nnz = max(1, int(round(dens * n)))
        idx = torch.from_numpy(np.unique(rng.integers(0, n, nnz))).cuda()
        x = torch.zeros(n, dtype=dtype, device="cuda")
        x[idx] = torch.randn(len(idx), dtype=dtype, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cat_ptr, a, v = ctx.csc_compress(x)
        torch.cuda.synchronize()
        ms_c = (time.perf_counter() - t0) * 1e3
        del x
        y = torch.empty(n, dtype=dtype, device="cuda")
        ctx.sigma_csc(cat_ptr, a, v, y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.sigma_csc(cat_ptr, a, v, y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        log("compressed sigma, %d nonzeros: %.3f ms (dense %.3f ms)" % (len(idx), ms, dense_ms))
        out["density_%g" % dens] = {"nonzeros": int(len(idx)), "compress_ms": round(ms_c, 3),
                                    "sigma_csc_ms": round(ms, 3), "dense_sigma_ms": round(dense_ms, 3),
                                    "speedup_vs_dense": round(dense_ms / ms, 2),
                                    "ms_per_nonzero": ms / len(idx)}
        del y, cat_ptr, a, v
    torch.cuda.empty_cache()
    return out


def _eps_study(ctx, roots, n):
    """Davidson with the eps drop of Eq. sparsePreconditioner for several eps
    (residual tolerance 1e-5): iterations, sigma vectors and the energy
    difference to the eps = 0 solve (the paper's eps <~ 10 / sqrt(N) rule
    included)."""
    import numpy as np
    import torch
    res = []
    e_ref = None
    for eps in (0.0, 1e-5, 1e-4, 1e-3, 10.0 / np.sqrt(n), 3e-2, 1e-1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, r, it, st = ctx.davidson(k=roots, tol=1e-5, max_iter=400, eps_drop=float(eps), allow_noconv=True)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if e_ref is None:
            e_ref = e
        nsig = ctx.dav_sigma_count(0)
        res.append({"eps": float(eps), "iterations": int(it), "converged": int(st) == 0, "sigma_vectors": nsig,
                    "max_energy_diff_vs_eps0_eh": float(np.max(np.abs(e - e_ref))), "max_resid": float(np.max(r)),
                    "solve_ms": round(ms, 1)})
        log("eps %.3g: %d iterations, dE %.2e" % (eps, it, res[-1]["max_energy_diff_vs_eps0_eh"]))
    return {"rule_10_over_sqrt_n": 10.0 / float(np.sqrt(n)), "runs": res}


def _config2(args):
    """The 24-spinor / 8-electron complex FCI problem (735,471 determinants,
    2 roots): sigma of the 2 new directions per step, its kernel against the
    roofline, the FP32 and BF16 forms, sparse vectors and the Davidson solve
    latency of each precision form.  Returns (result dict, context)."""
    import numpy as np
    import torch
    import synth
    import paper_2505_20375_amd as stpci

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
    n2, t2 = ctx.kernel_time("sigma")
    n3, t3 = ctx.kernel_time("sigma_reduce")
    ctx.profile(False)
    ms_per_step = ms_ev / args.steps
    value = info.nnz_h * n_vec / (ms_per_step * 1e-3)
    log("sigma step: %.3f ms (events), %.3f ms (wall)" % (ms_per_step, wall * 1e3 / args.steps))

    # roofline of the dominant kernel, the one-pass sigma kernel in use.  Pair
    # kernel: 8 Wp n_vec flop per launch (Wp = sum over the (N-2)-electron
    # intermediates of deg^2 complex multiply-adds, one- and two-electron
    # parts together); the one-move form of Eq. sigmaL1e/2e needs
    # 8 (W1 + W2) n_vec for the same sigma, reported beside it.
    W1, W2, n_inter, max_deg = ctx.work_counts()
    Wp, n_pair, max_pdeg = ctx.pair_counts()
    kname = ctx.sigma_kernel()
    flops_paper = 8.0 * (W1 + W2) * n_vec
    pair = kname.startswith("pair")
    flops = 8.0 * Wp * n_vec if pair else flops_paper
    avg2 = t2 / max(n2, 1)
    achieved = flops / (avg2 * 1e-3) / 1e12
    achieved_paper = flops_paper / (avg2 * 1e-3) / 1e12
    unit = ctx.test_pair_groups()[2] if kname.startswith("pair_grp") else 0
    kdesc = {"pair_grp": "k_sigma_pair_grp (one pass: pair-resolved 1e + 2e sigma, %d intermediates per "
                         "(N-3)-electron core, FP64 matrix cores, v_mfma_f64_16x16x4f64)" % unit,
             "pair_mf64": "k_sigma_pair_mf64 (one pass: pair-resolved 1e + 2e sigma, FP64 matrix cores, "
                          "v_mfma_f64_4x4x4f64)",
             "pair_valu": "k_sigma_pair (one pass: pair-resolved 1e + 2e sigma, FP64 vector ALUs)"}
    roof = {"kernel": kdesc.get(kname.replace("_atomic", ""), "k_sigma_symtile (fused 1e + 2e sigma, FP64)"),
            "bound": "mfma" if kname.startswith(("pair_mf64", "pair_grp")) else "alu",
            "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": _traffic(n_vec, kname),
            "avg_launch_ms": round(avg2, 4), "launches": n2, "flops_per_launch": flops,
            "algorithmic_bytes_per_launch": 2 * n_vec * n * 16,
            "reduce_avg_ms": round(t3 / n3, 4) if n3 else None,
            "paper_formulation_flops_per_launch": flops_paper,
            "paper_formulation_equiv_tflops": round(achieved_paper, 3),
            "paper_formulation_equiv_over_peak": round(achieved_paper / FP64_PEAK_TFLOPS, 4)}
    if kname.startswith("pair_mf64"):
        # executed matrix-core flops: 16-row tiles x 4-column steps over the
        # pair degree rounded up to 32, two real products of 4 columns each
        roof["executed_flops_per_launch"] = ctx_pair_mf64_flops(ctx, n_vec)
    if kname.startswith("pair_grp"):
        # executed matrix-core flops: per item, the core pairs rounded up to 16
        # as rows and columns, 16 right-hand columns, two real products
        roof["executed_flops_per_launch"] = ctx_pair_grp_flops(ctx, sp, n_vec)
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

    # precision forms of the same step: FP32 contraction (VALU) and BF16
    # contraction (matrix cores, FP32 accumulation; executed matrix-core flops
    # include the padding of each batch's dense product over all pairs)
    out64 = torch.empty_like(out)
    ctx.sigma(c, out64, n_vec=n_vec)
    torch.cuda.synchronize()
    prec = {"sigma_fp64_ms": ms_per_step,
            "contraction": "FP32: integrals, coefficients and accumulation in FP32 (spaces of one subspace: "
                           "grouped intermediates on the matrix cores, v_mfma_f32_16x16x4f32; otherwise the "
                           "vector ALUs); "
                           "BF16: bfloat16 integrals and coefficients on the matrix cores "
                           "(v_mfma_f32_16x16x32_bf16), FP32 accumulation; both: FP64 sigma sums, residual, "
                           "orthogonalisation and subspace solve"}
    for pname, pcode in (("fp32", stpci.FP32), ("bf16", stpci.BF16)):
        for _ in range(max(1, args.warmup)):
            ctx.sigma(c, out, n_vec=n_vec, precision=pcode)
        torch.cuda.synchronize()
        ctx.profile(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            ctx.sigma(c, out, n_vec=n_vec, precision=pcode)
        e1.record()
        torch.cuda.synchronize()
        ms_p = e0.elapsed_time(e1) / args.steps
        prec["sigma_%s_ms" % pname] = ms_p
        prec["sigma_%s_speedup" % pname] = ms_per_step / ms_p
        prec["sigma_%s_rel_err" % pname] = float(torch.linalg.vector_norm(out - out64) /
                                                 torch.linalg.vector_norm(out64))
        if pname == "fp32" and kname.startswith("pair_grp"):
            nf, tf = ctx.kernel_time("sigma_fp32")
            ctx.profile(False)
            kms = tf / max(nf, 1)
            ex = ctx_pair_grp_flops(ctx, sp, n_vec)
            prec["fp32_matrix_core"] = {
                "kernel": "k_sigma_pair_grp (FP32 table, products and accumulation, v_mfma_f32_16x16x4f32)",
                "avg_launch_ms": round(kms, 4), "executed_tflops": round(ex / (kms * 1e-3) / 1e12, 3),
                "useful_tflops": round(flops / (kms * 1e-3) / 1e12, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac_executed": round(ex / (kms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4),
                "executed_flops_per_launch": ex, "useful_flops_per_launch": flops}
        if pname == "bf16":
            nb, tb = ctx.kernel_time("sigma_bf16")
            ctx.profile(False)
            npp = (sp.n_spin_orb * (sp.n_spin_orb - 1) // 2 + 31) // 32 * 32
            nbatch = -(-n_pair // (16 // n_vec))
            mf_flops = nbatch * npp * npp * 16 * 2 * 4   # four real products per complex batch
            kms = tb / max(nb, 1)
            prec["bf16_matrix_core"] = {
                "kernel": "k_sigma_pair_mfma", "avg_launch_ms": round(kms, 4),
                "executed_tflops": round(mf_flops / (kms * 1e-3) / 1e12, 3),
                "useful_tflops": round(flops / (kms * 1e-3) / 1e12, 3),
                "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac_executed": round(mf_flops / (kms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, 4),
                "executed_flops_per_launch": mf_flops, "useful_flops_per_launch": flops}
    prec["sigma_speedup"] = prec["sigma_fp32_speedup"]   # FP32 over FP64
    # intermediates whose gathered coefficients are all zero are skipped:
    # FP64 sigma of vectors with a random 1 % and 0.1 % of their entries nonzero
    sparse = {}
    gs = torch.Generator(device="cuda").manual_seed(2103)
    for dens in (() if args.no_sparse else (1e-2, 1e-3)):
        cs = c * (torch.rand(c.shape, generator=gs, device="cuda") < dens)
        for _ in range(max(1, args.warmup)):
            ctx.sigma(cs, out, n_vec=n_vec)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            ctx.sigma(cs, out, n_vec=n_vec)
        e1.record()
        torch.cuda.synchronize()
        ms_s = e0.elapsed_time(e1) / args.steps
        sparse["density_%g" % dens] = {"sigma_fp64_ms": ms_s, "speedup_vs_dense": ms_per_step / ms_s}
    if sparse:
        res["sparse_vectors"] = sparse
    if not args.no_sparse:
        # one vector, dense and compressed
        c1 = c[:n].contiguous()
        o1 = torch.empty_like(c1)
        ctx.sigma(c1, o1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.sigma(c1, o1)
        e1.record()
        torch.cuda.synchronize()
        res["compressed"] = _compressed(ctx, n, c.dtype, e0.elapsed_time(e1), (1e-4, 1e-3, 1e-2, 1e-1), 2104)
        del c1, o1
    res["precision"] = prec
    if not args.no_solve:
        res["eps_study"] = _eps_study(ctx, roots, n)
        res["solve"] = _solve(ctx, roots, args.solves, stpci.FP64)
        for pname, pcode in (("mixed", stpci.FP32), ("mixed_bf16", stpci.BF16)):
            sol = _solve(ctx, roots, args.solves, pcode)
            prec["solve_" + pname] = sol
            prec["solve_speedup" + ("" if pname == "mixed" else "_bf16")] = res["solve"]["p50_ms"] / sol["p50_ms"]
            prec["energy_diff_eh" + ("" if pname == "mixed" else "_bf16")] = max(
                abs(a - b) for a, b in zip(sol["energies"], res["solve"]["energies"]))
    return res, ctx


def ctx_pair_mf64_flops(ctx, n_vec):
    """Matrix-core flops of one launch of the FP64 matrix-core pair kernel:
    per intermediate, cap = degree rounded up to 32 rows and steps, two real
    4-column products (512 flop per v_mfma_f64_4x4x4f64, one per 16 rows x
    4 steps): 16 cap^2 flop per intermediate and pass of at most two vectors.
    Exact when every intermediate has the largest degree (the FCI workload),
    an upper bound otherwise."""
    _, n_pair, max_pdeg = ctx.pair_counts()
    cap = (max_pdeg + 31) // 32 * 32
    return float(n_pair * 16 * cap * cap * ((n_vec + 1) // 2))


def ctx_pair_grp_flops(ctx, sp, n_vec):
    """Matrix-core flops of one launch of the grouped FP64 pair kernel: per
    item of `unit` intermediates, cap = core pairs C(M - N + 3, 2) rounded up
    to 16, cap/16 row tiles x cap/4 steps x unit/4 column groups of
    v_mfma_f64_16x16x4f64 (2048 flop) for each of the two real products (real
    and imaginary part of the table), i.e. 16 unit cap^2 flop per item and
    pass of at most two vectors.  Items and unit are the host grouping's."""
    items, _, unit = ctx.test_pair_groups()
    e = sp.n_spin_orb - sp.n_elec + 3
    cap = (e * (e - 1) // 2 + 15) // 16 * 16
    return float(items * 16 * unit * cap * cap * ((n_vec + 1) // 2))


TRAFFIC_FILES = {("pair_sb", "c3p"): os.path.join(ROOT, "profiles", "sigma_pair_sb_c3p_traffic.txt"),
                 "pair_grp": os.path.join(ROOT, "profiles", "sigma_pair_grp_c2_traffic.txt"),
                 "pair_valu": os.path.join(ROOT, "profiles", "sigma_pair_c2_traffic.txt"),
                 "pair_mf64": os.path.join(ROOT, "profiles", "sigma_pair_mf64_c2_traffic.txt"),
                 "tile": os.path.join(ROOT, "profiles", "sigma_symtile_c2_traffic.txt")}
KERNEL_SOURCES = {"pair_sb": ["sigma_sb.hip", "stp_device.hpp", "stp_internal.hpp"],
                  "pair_grp": ["sigma_grp.hip", "stp_device.hpp", "stp_internal.hpp"],
                  "pair_valu": ["sigma_pair.hip", "pair_arith.hpp", "symtile.hpp", "stp_device.hpp", "stp_internal.hpp"],
                  "pair_mf64": ["sigma_mf64.hip", "pair_arith.hpp", "stp_device.hpp", "stp_internal.hpp"],
                  "tile": ["sigma_sym.hip", "stp_device.hpp", "stp_internal.hpp"]}


def kernel_source_hash(kname="pair_mf64"):
    import hashlib
    hsh = hashlib.sha256()
    for f in KERNEL_SOURCES[kname]:
        with open(os.path.join(ROOT, "paper_2505_20375_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()[:16]


def _traffic(n_vec, kname="pair_mf64", workload="c2"):
    """HBM bytes per launch of the sigma kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by the factor the
    same counter reads on a plain copy of known size), or None when the kernel
    sources changed after the counters were taken."""
    if kname not in KERNEL_SOURCES:   # atomic scatter or another kernel: no counter summary
        return None
    path = TRAFFIC_FILES.get((kname, workload)) or TRAFFIC_FILES.get(kname)
    if path is None or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash(kname) or int(kv.get("n_vec", 0)) != n_vec:
        return None
    return float(kv["traffic_bytes_per_launch"])


def _solve(ctx, roots, nsolve, precision):
    """Davidson time-to-solution at residual tolerance 1e-5; the lowest energy
    is then within ||r0||^2 / gamma^- (gap theorem with the rigorous gap
    bound from the second root, computed by the library:
    stpci_dav_certificate), reported as energy_bound_eh (<= 1e-8 Eh)."""
    import numpy as np
    import torch
    import paper_2505_20375_amd as stpci
    label = {stpci.FP64: "fp64", stpci.FP32: "fp32+fp64", stpci.BF16: "bf16+fp64"}[precision]
    times, its = [], []
    e = r = None
    for i in range(nsolve):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, r, it, st = ctx.davidson(k=roots, tol=1e-5, max_iter=400, precision=precision)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        its.append(it)
        log("solve %d (%s): %.1f ms, %d iterations" % (i, label, times[-1], it))
    # the library's gap certificate of the lowest root (from the second root)
    gam, bnd = ctx.certificate()
    cert = float(bnd[0]) if np.isfinite(bnd[0]) else None
    n64, n32 = ctx.dav_stats()
    nbf = ctx.dav_sigma_count(stpci.BF16)
    # one more solve (not in the percentiles) with the library's HIP events
    # around every sigma launch: the share of the solve's wall time that the
    # sigma kernels take; the rest is the Davidson vector algebra, its round
    # trips and the host's projected problem
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.davidson(k=roots, tol=1e-5, max_iter=400, precision=precision)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    sig_ms = sum(ctx.kernel_time(nm)[1] for nm in ("sigma1e", "sigma", "sigma_fp32", "sigma_reduce", "sigma_bf16"))
    ctx.profile(False)
    return {"p50_ms": float(np.percentile(times, 50)), "p99_ms": float(np.percentile(times, 99)),
            "n": nsolve, "iterations": its[-1], "energies": [float(x) for x in e],
            "resid": [float(x) for x in r], "energy_bound_eh": cert, "tol_residual": 1e-5,
            "sigma_vectors_fp64": n64, "sigma_vectors_fp32": n32 - nbf, "sigma_vectors_bf16": nbf,
            "sigma_share_of_wall": round(sig_ms / wall, 4)}


def _serve(nreq, max_dets, rate):
    """Continuous batching of CI solves with Poisson arrivals.  Requests draw
    16-32 complex spinors in 1-3 subspaces, 6-12 electrons and 1-4 roots from
    their seeds, as in the 512-request serving workload but with at most
    max_dets determinants each; every request is solved to residual 1e-5.
    The same requests are also served with every request present at the
    start, batched (16 active) and one at a time (one active): the ratio of
    their throughputs is the batching speedup."""
    import numpy as np
    import torch
    import synth
    import paper_2505_20375_amd as stpci
    from paper_2505_20375_amd import serve
    descs = synth.serving_requests(nreq, max_dets=max_dets)
    reqs = []
    for d in descs:
        ints = synth.complex_integrals(d["M"], d["seed"], rank=16, sigma_f=0.05)
        sp = d["space"]
        reqs.append(dict(h=ints.h, g=ints.g, n_elec=sp.n_elec, sub=sp.sub, lo=sp.lo, hi=sp.hi, k=d["roots"],
                         tol=1e-5, max_iter=400))
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.6 * free)
    out, energies = {}, {}
    # batched with Poisson arrivals (latency under load), batched with every
    # request present at the start (throughput), and one at a time with
    # every request present at the start (the throughput it is compared with)
    for mode, active, arr in (("batched", 16, serve.arrival_times(nreq, rate, 5000)),
                              ("batched_all_present", 16, None),
                              ("one_at_a_time", 1, None)):
        srv = stpci.Server(0, mem_budget_bytes=budget, max_active=active)
        served, wall = serve.run(srv, reqs, arr)
        st = srv.stats()
        info = [srv.request_info(r.rid) for r in served]
        srv.close()
        updates = sum(nz * sv for (_, nz, _, sv) in info)
        s = serve.summary(served, wall)
        s.update(det_updates_per_s=updates / wall, max_active=active, peak_active=st["peak_active"],
                 peak_footprint_gb=st["peak"] / 1e9, ticks=st["ticks"], sigma_launches=st["sigma_launches"],
                 tick_phase_s={"admission": round(st["admit_s"], 3), "sigma": round(st["sigma_s"], 3),
                               "davidson_step": round(st["step_s"], 3)})
        out[mode] = s
        energies[mode] = [r.energies for r in served]
        log("serving (%s): %d requests, wall %.2f s, p50 %.3f s, p99 %.3f s" % (mode, nreq, wall, s["p50_s"],
                                                                              s["p99_s"]))
    # each request alone versus in the mix
    out["max_energy_diff_mix_vs_alone_eh"] = float(max(np.max(np.abs(a - b)) for a, b in
                                                       zip(energies["batched"], energies["one_at_a_time"])))
    out["batched_vs_one_at_a_time_throughput"] = (out["batched_all_present"]["det_updates_per_s"] /
                                                   out["one_at_a_time"]["det_updates_per_s"])
    out["poisson_batched_vs_one_at_a_time_throughput"] = (out["batched"]["det_updates_per_s"] /
                                                          out["one_at_a_time"]["det_updates_per_s"])
    out["workload"] = ("%d requests, Poisson arrivals at %.0f/s, 16-32 complex spinors, 1-3 subspaces, 6-12 "
                       "electrons, 1-4 roots, %d-%d determinants (scaled down from 512 requests of up to 1e8)"
                       % (nreq, rate, min(d["n_dets"] for d in descs), max(d["n_dets"] for d in descs)))
    out["tol_residual"] = 1e-5
    return out


def _measured_peaks(roof):
    """Reference rates measured on this device beside the published peaks
    the roofline uses: FP64 and complex FP64 library GEMMs (torch.matmul,
    which calls the ROCm BLAS) and a 1 GiB device-to-device copy."""
    import torch

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    g = torch.Generator(device="cuda").manual_seed(7)
    out = {}
    for name, dt, n, fl in (("dgemm", torch.float64, 8192, 2.0), ("zgemm", torch.complex128, 4096, 8.0)):
        a = torch.randn(n, n, dtype=dt, device="cuda", generator=g)
        b = torch.randn(n, n, dtype=dt, device="cuda", generator=g)
        c = torch.empty_like(a)
        t = timed(lambda: torch.matmul(a, b, out=c), 5)
        out[name + "_tflops"] = round(fl * n ** 3 / t / 1e12, 3)
        out[name + "_size"] = n
        del a, b, c
    nb = 1 << 30
    src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    t = timed(lambda: dst.copy_(src), 10)
    out["copy_gbs"] = round(2.0 * nb / t / 1e9, 1)
    del src, dst
    out["sigma_frac_of_dgemm"] = round(roof["achieved"] / out["dgemm_tflops"], 4)
    out["sigma_frac_of_zgemm"] = round(roof["achieved"] / out["zgemm_tflops"], 4)
    return out


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
