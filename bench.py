"""Benchmark: factor + refined solve of the 2D type-II inverse NUDFT at
n = 512 x 512 (N = 262144), M = 1024^2 jittered points, FP32 HSS factors with
FP64 iterative refinement, ir_tol = 1e-10 (an update, or the contraction bound
on the error, below it; relative error vs the true coefficients reported), on
one MI355X.  The refinement's FP64 residual
comes from the exact face-split apply (the FP64 direct sums; --nufft-tol
1e-13 takes Section 4.1's NUFFT operator instead), and both operators'
refined solves are reported.

A step = plan (binning + upload of the points) + factorization (1D HSS
compression with fADI factors, face-splitting assembly, recompression, URV) +
refined solve of one right-hand side, inputs resident in device memory before
timing.  The
FP64-factor path is timed beside it (same refinement target).  The CPU
baseline leg times the oracle's direct-sum apply on a bounded sample of rows.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

WORKLOADS = {
    # name: (nx, ny, mx, my, delta, seed) -- jittered grids (M = 4N)
    "n512": (512, 512, 1024, 1024, 0.4, 3),
    "n256": (256, 256, 512, 512, 0.4, 3),
    "fp64_128": (128, 128, 256, 256, 0.3, 2),
    "small": (32, 32, 64, 64, 0.25, 1),
}
# the paper's grid families (Section 5): name -> (kind, n, seed)
GRID_WORKLOADS = {
    "random512": ("random", 512, 3),   # M = 1.5 N uniform points
    "polar512": ("polar", 512, 3),     # beta = 0.6, M = 1122019
    "random256": ("random", 256, 3),
    "polar256": ("polar", 256, 3),
}

FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0
# FP32 products on the bf16 matrix cores (fp32_products "bf16x3"): six bf16
# products per real FP32 product, so the class's algorithmic FP32 flops run
# against a sixth of the bf16 peak
SPLIT_PEAK_TFLOPS = BF16_PEAK_TFLOPS / 6
# kernel classes of the library's per-launch timing (nudft2_info.kernel_ms)
NCLASS = 6
TIMED_CLASSES = (1,)
HBM_PEAK_GBPS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n512", choices=sorted(WORKLOADS) + sorted(GRID_WORKLOADS))
    ap.add_argument("--refine", type=int, default=0, choices=[0, 1, 2],
                    help="0 iterative refinement, 1 PCG on the normal equations, 2 plsqr")
    ap.add_argument("--eps", type=float, default=1e-2)
    ap.add_argument("--fp32-products", default="bf16x3", choices=["bf16x3", "fp32"],
                    help="matrix instructions of the FP32 factorization's products")
    ap.add_argument("--construct-1d", default="fadi", choices=["fadi", "gram"],
                    help="1D HSS stage: leaf row bases from fADI factors (default) or from "
                         "explicit Gram matrices")
    ap.add_argument("--nufft-tol", type=float, default=0.0,
                    help="operator of the refinement: 0 (default) the exact FP64 face-split "
                         "direct sums; > 0 A and A^* by the NUFFT to this relative accuracy "
                         "(Section 4.1)")
    ap.add_argument("--ir-tol", type=float, default=1e-10)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-factor comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-nrhs16", action="store_true",
                    help="skip the 16-right-hand-side solve timings")
    ap.add_argument("--profile-only", action="store_true",
                    help="only the timed steps (no sweep, apply, FP64 or CPU extras): the "
                         "command the rocprofv3 summaries are taken on")
    ap.add_argument("--profile-sweep", action="store_true",
                    help="factor once (untimed), then --steps direct solves (no refinement): "
                         "the command the sweep's rocprofv3 summaries are taken on")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU (asked for --gpus {args.gpus}); the sharded "
              "multi-GPU path is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.profile_only:
        args.no_fp64 = args.no_cpu_baseline = True
        args.no_nrhs16 = True

    import torch
    from nudft_inputs import make_problem, make_grid_problem
    import paper_2607_00928_amd as nd

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.workload in GRID_WORKLOADS:
        kind, nx, seed = GRID_WORKLOADS[args.workload]
        ny = nx
        pr = make_grid_problem(kind, nx, seed)
        wl_desc = (f"{args.workload}: {kind} grid, nx=ny={nx}, M={pr.M}, eps={args.eps}")
    else:
        nx, ny, mx, my, delta, seed = WORKLOADS[args.workload]
        pr = make_problem(nx, ny, mx, my, delta, seed)
        wl_desc = f"{args.workload}: nx=ny={nx}, M={pr.M}, jitter {delta}, eps={args.eps}"
    M, N = pr.M, nx * ny
    c_true = torch.from_numpy(pr.c_true).to(dev)
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)

    # right-hand side f = A c_true from the library's exact FP64 apply
    p0 = nd.Plan(pr.points, nx, ny, precision="fp32", eps=args.eps)
    f = p0.apply(c_true)
    torch.cuda.synchronize()
    p0.close()

    if args.profile_sweep:
        plan = nd.Plan(pr.points, nx, ny, precision="fp32", eps=args.eps, ir_maxit=0,
                       fp32_products=args.fp32_products, fadi_1d=args.construct_1d == "fadi")
        plan.factor()
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            plan.solve(f)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        sb = plan.info()["sweep_bytes"]
        plan.close()
        med = float(np.median(ts))
        print(json.dumps({"metric": "direct solve (profile run)", "ms": 1e3 * med,
                          "sweep_bytes": sb, "gbps": sb / med / 1e9}))
        return

    def step(precision, profile=False):
        t0 = time.perf_counter()
        plan = nd.Plan(pr.points, nx, ny, precision=precision, eps=args.eps, ir_maxit=200,
                       ir_tol=args.ir_tol, refine=args.refine, fp32_products=args.fp32_products,
                       nufft_tol=args.nufft_tol, fadi_1d=args.construct_1d == "fadi")
        if profile:
            # per-launch events for the dominant class only (the FP32
            # matrix-core GEMMs: about three quarters of the step's kernel
            # time in the rocprofv3 trace); other launches record none
            plan.set_profiling(True, classes=TIMED_CLASSES)
        t1 = time.perf_counter()
        plan.factor()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        c, si = plan.solve(f, return_info=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        err = ((c - c_true).norm() / c_true.norm()).item()
        return plan, dict(plan_s=t1 - t0, factor_s=t2 - t1, solve_s=t3 - t2, total_s=t3 - t0,
                          its=si["iterations"], rel_err=err, rel_update=si["rel_update"],
                          rel_residual=si["rel_residual"])

    for w in range(args.warmup):
        plan, r = step("fp32")
        log(f"warmup {w}: {r}")
        plan.close()
    torch.cuda.synchronize()
    recs = []
    kms, kfl, kn = [0.0] * NCLASS, [0.0] * NCLASS, [0] * NCLASS

    def fold(pl):
        # read back a plan's per-launch HIP events (recorded during its step)
        inf_k = pl.info()
        for i in range(NCLASS):
            kms[i] += inf_k["kernel_ms"][i]
            kfl[i] += inf_k["kernel_flops"][i]
            kn[i] += inf_k["kernel_launches"][i]

    # the steps' plans stay alive until the timed region ends, so reading back
    # their events and freeing them happen outside it (at most two n512 plans,
    # about 100 GB, are held; with more steps the oldest is folded and freed)
    live = []
    t_start = time.perf_counter()
    # plans held at once: two at eps >= 1e-3 (about 60 GB each at n = 512),
    # one below (about 145 GB at eps = 1e-4)
    max_live = 2 if args.eps >= 1e-3 else 1
    for k in range(args.steps):
        if len(live) == max_live:
            fold(live[0])
            live.pop(0).close()
        plan, r = step("fp32", profile=True)
        recs.append(r)
        live.append(plan)
        log(f"step {k}: {r}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    for pl in live:
        fold(pl)
    for pl in live[:-1]:
        pl.close()
    last_plan = live[-1]
    info = last_plan.info()
    # kernel classes timed with HIP events on the plan's stream over the timed steps
    names = ["apply_fp64", "gemm_fp32_mfma", "gemm_fp64_mfma", "qr_panel", "gemv_fp32",
             "gemv_fp64"]
    dominant = max(range(NCLASS), key=lambda i: kms[i])
    split = args.fp32_products == "bf16x3"
    peaks = [FP64_PEAK_TFLOPS, SPLIT_PEAK_TFLOPS if split else FP32_PEAK_TFLOPS,
             FP64_PEAK_TFLOPS, None, None, None]
    avg_ms = kms[dominant] / max(kn[dominant], 1)
    per_launch = kfl[dominant] / max(kn[dominant], 1)
    ach = per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 and per_launch > 0 else None
    pk = peaks[dominant]
    rec = gemm_record(args.fp32_products) if dominant == 1 else None
    roof = dict(bound="mfma", achieved=ach, peak=pk, unit="TFLOP/s",
                frac=(ach / pk if ach is not None and pk else None),
                traffic=rec["hbm_bytes_per_launch"] if rec else None,
                kernel=names[dominant], avg_launch_ms=avg_ms, launches=kn[dominant],
                flops_per_launch=per_launch)
    if dominant == 1:
        roof.update(mfma_dtype="bf16" if split else "fp32",
                    peak_basis=("bf16 dense matrix peak 2500 TFLOP/s / 6 (six bf16 products "
                                "of split FP32 operands per real FP32 product)" if split
                                else "fp32 dense matrix peak"))
    if rec and ach is not None:
        # achieved counts 8 algorithmic flops per complex multiply-add; the
        # matrix cores execute a different count (six bf16 products per real
        # product on the split, Gauss's three real products on the FP32
        # instructions), as the committed PMC record measures: executed rate
        # over each instruction kind's peak, and the busy counter's fraction
        # of the class's time
        t = rec["flops_per_launch"] / (ach * 1e12)   # seconds per launch at this rate
        ex = (rec.get("executed_bf16_flops_per_launch", 0.0) / t / 1e12 / BF16_PEAK_TFLOPS +
              rec.get("executed_f32_flops_per_launch", 0.0) / t / 1e12 / FP32_PEAK_TFLOPS)
        roof.update(executed_frac=ex, mfma_busy_frac=rec["mfma_busy_frac"],
                    algorithmic_flop_per_hbm_byte=rec["flops_per_launch"] / rec["hbm_bytes_per_launch"])
    kernels = {names[i]: dict(ms=kms[i], launches=kn[i],
                              tflops=(kfl[i] / (kms[i] * 1e-3) / 1e12 if kms[i] > 0 and kfl[i] > 0 else None))
               for i in range(NCLASS) if i in TIMED_CLASSES}

    extra = {}
    if args.profile_only:
        last_plan.close()
        out = {"metric": "factor+solve/s (profile-only run)", "value": 1000.0 / ms_per_step,
               "ms_per_step": ms_per_step, "roofline": roof, "kernels": kernels}
        print(json.dumps(out))
        return
    if not args.no_nrhs16:
        # 16 right-hand sides in one call (one refined solve each, the
        # distinct right-hand sides being scaled copies of f), with the exact
        # apply and with the NUFFT operator
        last_plan.set_profiling(False)
        F16 = (f.unsqueeze(0) * torch.arange(1, 17, device=dev, dtype=torch.float64)
               .to(torch.complex128).unsqueeze(1)).contiguous()
        for tol, key in ((0.0, "exact_apply"), (1e-13, "nufft_operator")):
            last_plan.set_nufft_tol(tol)
            last_plan.solve(F16[:2].contiguous())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c16, s16 = last_plan.solve(F16, return_info=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            e16 = ((c16[15] / 16 - c_true).norm() / c_true.norm()).item()
            extra.setdefault("nrhs16", {})[key] = {"s": dt, "solves_per_s": 16 / dt,
                                                   "its": s16["iterations"], "rel_err_rhs16": e16}
        last_plan.set_nufft_tol(args.nufft_tol)
        log(f"nrhs16: {extra['nrhs16']}")
    # direct solve (no refinement): the sweep reads every URV factor once, so
    # its rate against the factor bytes it reads is its HBM roofline (timed
    # without the per-launch events of the steps)
    last_plan.set_profiling(False)
    last_plan.set_solve_opts(ir_maxit=0)
    last_plan.solve(f)
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        last_plan.solve(f)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    sweep_s = float(np.median(ts))
    sb = info["sweep_bytes"]
    sweep = {"ms": 1e3 * sweep_s, "bytes": sb, "gbps": sb / sweep_s / 1e9,
             "frac_hbm": sb / sweep_s / (HBM_PEAK_GBPS * 1e9)}
    last_plan.set_solve_opts(ir_maxit=200)
    # the refined solve with each operator (the exact FP64 direct sums, and
    # the NUFFT's spreading + FFT at tol 1e-13) on the same factors, and the
    # NUFFT alone
    operators = {}
    for tol, key in ((0.0, "exact_apply"), (1e-13, "nufft")):
        try:
            last_plan.set_nufft_tol(tol)
            last_plan.solve(f)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cn, sn = last_plan.solve(f, return_info=True)
            torch.cuda.synchronize()
            t_sn = time.perf_counter() - t0
            en = ((cn - c_true).norm() / c_true.norm()).item()
            operators[key] = {"tol": tol, "refined_solve_s": t_sn, "its": sn["iterations"],
                              "rel_err": en, "solves_per_s": 1.0 / t_sn}
        except Exception as e:   # report, do not hide
            operators[key] = dict(error=str(e))
        log(f"operator {key}: {operators[key]}")
    last_plan.set_nufft_tol(args.nufft_tol)
    try:
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        last_plan.nufft(c_true, 1e-13)
        ev0.record()
        for _ in range(5):
            last_plan.nufft(c_true, 1e-13)
        ev1.record()
        torch.cuda.synchronize()
        operators["nufft"]["type2_ms"] = ev0.elapsed_time(ev1) / 5
    except Exception as e:   # report, do not hide
        operators["nufft_type2_error"] = str(e)
    # exact FP64 apply alone (its own kernel-class timing)
    last_plan.set_profiling(True)
    for _ in range(5):
        last_plan.apply(c_true)
    torch.cuda.synchronize()
    ai = last_plan.info()
    apply_ms = ai["kernel_ms"][0] / max(ai["kernel_launches"][0], 1)
    apply_tf = 8.0 * M * N / (apply_ms * 1e-3) / 1e12
    last_plan.close()

    fp64 = None
    if not args.no_fp64:
        try:
            p64, r64 = step("fp64")
            p64.close()
            fp64 = r64
            log(f"fp64: {r64}")
        except Exception as e:   # report, do not hide
            fp64 = dict(error=str(e))
            log(f"fp64 path failed: {e}")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(pr, nx, ny, log)

    med = sorted(r["total_s"] for r in recs)[len(recs) // 2]
    out = {
        "metric": "factor+solve time & solves/s at N=512^2, rel err <= 1e-10; FP32+IR vs FP64",
        "value": 1000.0 / ms_per_step,
        "unit": "factor+solve/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 factors + f64 refinement",
        "data": ("synthetic (seeded %s grid, complex Gaussian coefficients)"
                 % ("jittered" if args.workload in WORKLOADS else GRID_WORKLOADS[args.workload][0])),
        "config": {"workload": wl_desc, "precision": "fp32+ir", "ir_tol": args.ir_tol,
                   "fp32_products": args.fp32_products,
                   "construct_1d": args.construct_1d,
                   "operator": (f"nufft tol {args.nufft_tol:g}" if args.nufft_tol > 0
                                else "exact FP64 direct sums"),
                   "refine": ["iterative refinement", "pcg-ne", "plsqr"][args.refine]},
        "factor_s": float(np.median([r["factor_s"] for r in recs])),
        "solve_s": float(np.median([r["solve_s"] for r in recs])),
        "plan_s": float(np.median([r["plan_s"] for r in recs])),
        "median_step_s": med,
        "ir_iterations": recs[-1]["its"],
        "rel_err_vs_c_true": max(r["rel_err"] for r in recs),
        "solves_per_s": 1.0 / float(np.median([r["solve_s"] for r in recs])),
        "phases_ms": {k: info[k] for k in ("t_compress_ms", "t_facesplit_ms", "t_recompress_ms", "t_urv_ms")},
        "ranks_u": info["max_rank_u"], "ranks_v": info["max_rank_v"],
        "factor_bytes": info["factor_bytes"],
        "peak_bytes": info["peak_bytes"],
        "kernels": kernels,
        "sweep": sweep,
        "apply": {"ms": apply_ms, "tflops": apply_tf, "frac_fp64_peak": apply_tf / FP64_PEAK_TFLOPS},
        "refinement_operators": operators,
        "fp64_path": fp64,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out))


def gemm_record(products):
    """The FP32 GEMM class's committed rocprofv3 PMC record (HBM bytes per
    launch from FETCH_SIZE / WRITE_SIZE scaled by a plain copy of known size;
    executed matrix-core flops and busy fraction); None when the kernel source
    changed since the counters were taken or they were taken on the other
    kind of FP32 product."""
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "gemm_fp32_traffic_n512.md")
    src = os.path.join(root, "paper_2607_00928_amd", "csrc", "la.hip")
    try:
        rec = json.loads(open(path).read().split("```json")[1].split("```")[0])
        with open(src, "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != rec["la_hip_sha256"]:
                return None
        if rec.get("fp32_products", "fp32") != products:
            return None
        return rec
    except Exception:
        return None


def cpu_baseline(pr, nx, ny, log):
    """The oracle's direct-sum apply (exact FP64) on a bounded row sample,
    scaled to the full problem; plus the dense least-squares oracle is
    infeasible at this size (A would be M x N = 4.4 TB)."""
    try:
        from oracle import nudft as onu
    except Exception as e:
        return {"error": str(e)}
    rows = 4096
    sel = np.arange(rows)
    t0 = time.perf_counter()
    onu.apply(pr.points[sel], pr.c_true)
    dt = time.perf_counter() - t0
    reps = 1
    while dt * reps < 10.0 and reps < 8:
        t0 = time.perf_counter()
        onu.apply(pr.points[sel], pr.c_true)
        dt = min(dt, time.perf_counter() - t0)
        reps += 1
    full_apply_s = dt * pr.M / rows
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    log(f"cpu baseline: {rows} rows in {dt:.3f} s -> full apply {full_apply_s:.1f} s")
    return {"value": 1.0 / full_apply_s, "unit": "exact applies/s (A c, FP64)",
            "cores": cores, "kind": "oracle",
            "sample": f"{rows} of {pr.M} rows of the direct-sum apply, scaled by M/{rows}; "
                      "dense LS oracle infeasible at this size (4.4 TB)"}


if __name__ == "__main__":
    main()
