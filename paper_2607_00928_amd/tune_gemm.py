"""Autotuner of the batched complex GEMM: picks the output tile shape and the
k split per launch shape class by measurement and writes
csrc/gemm_tuning.inc (rebuild afterwards).

    python -m paper_2607_00928_amd.tune_gemm [--workload n512,batch64] [--top 48]

1. Runs each workload (factor + refined solve of one problem; the batch of 64
   uneven problems: factor) with per-launch kernel logging (NUDFT2_PROF_LOG)
   to collect the shapes of the GEMM launches.
2. Buckets the launches into classes (precision, op(A), op(B), ceil(log2) of
   the largest m, n, k and of the descriptor count) and keeps, per workload,
   the classes that took the most time.
3. Times, for each class, a synthetic batch at the class's largest shape with
   every candidate: the 64 x 64 output tiles with each k split, and for A^H B
   with m <= 32 the 32 x 128 and the 16/32-square output tiles of the
   small-output kernels; and the library's heuristic without the table
   (nudft2_test_gemm_cfg: HIP events around the launch).
4. Writes the classes where a candidate beats the heuristic by more than 5%,
   as {..., splits, tile} with tile 0 (64 x 64, splits), 1 (32 x 128) or 2
   (square).  Entries of the existing table are kept for classes this run
   did not measure, and for measured classes whose best candidate is still
   the entry's and still beats the heuristic (merge_entries).
"""
from __future__ import annotations

import argparse
import ctypes as C
import os
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
INC = os.path.join(HERE, "csrc", "gemm_tuning.inc")
SPLITS = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096]
MEM_CAP = 24 << 30   # bytes of synthetic operands per class


def clog2(x: int) -> int:
    l = 0
    while (1 << l) < x:
        l += 1
    return l


TILE_CODES = {1: -5, 2: -6}   # tile -> nudft2_test_gemm_cfg's forcing code


def small_tiles(opa: int, opb: int, m: int, n: int):
    """Small-output tile shapes the library accepts for this shape."""
    if opa != 1 or opb != 0 or m > 32 or n <= 8:
        return []
    return [t for t, nmax in ((1, 128), (2, 32)) if n <= nmax]


def read_table(path: str) -> dict:
    """{class key: (splits, tile)} of a gemm_tuning.inc (8-field entries of
    older tables have tile 0)."""
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        line = line.strip()
        if not (line.startswith("{") and line[1:2].isdigit()):
            continue
        v = [int(x) for x in line.strip("{},").split(",")]
        out[tuple(v[:7])] = (v[7], v[8] if len(v) > 8 else 0)
    return out


def merge_entries(old: dict, measured: dict, threshold: float = 1.05) -> dict:
    """measured: {key: ((splits, tile) of the best candidate, heuristic time /
    best time)}.  A measured class gets its best candidate when it wins by
    more than `threshold`, keeps its old entry when that is still the best
    and still wins, and has no entry otherwise; classes not measured keep
    theirs."""
    out = {k: v for k, v in old.items() if k not in measured}
    for k, (best, gain) in measured.items():
        if gain > threshold:
            out[k] = best
        elif k in old and old[k] == best and gain > 1.0:
            out[k] = old[k]
    return out


def decode(var: int):
    """(opA, opB, skinny) from the launch log's variant code."""
    if var in (2011, 2012, 2021, 2022, 3000):   # small-output tiles: A^H B
        return 1, 0, False
    if var >= 1000:
        v = var - 1000
        return (v % 10) // 2, 0, True
    return (var % 10) // 2, var % 2, False


def collect(workload: str, log_path: str):
    """Run the workload once with launch logging; return the log rows."""
    os.environ["NUDFT2_PROF_LOG"] = log_path
    import torch
    sys.path.insert(0, ROOT)
    import paper_2607_00928_amd as nd
    from nudft_inputs import batch_problems, config_problem, make_problem

    if workload == "batch64":
        probs = batch_problems()
        bp = nd.BatchPlan([p.points for p in probs], [p.c_true.shape[0] for p in probs],
                          [p.c_true.shape[1] for p in probs], precision="fp32", eps=1e-2)
        bp.set_profiling(True)
        bp.factor()
        bp.info()          # folds the recorded launches into the log
        bp.close()
        return np.loadtxt(log_path, ndmin=2)
    if workload == "n512":
        pr = config_problem("n512")
        nx = ny = 512
        eps = 1e-2
    else:
        nx = ny = 128
        pr = make_problem(nx, ny, 256, 256, 0.3, 2)
        eps = 1e-2
    dev = torch.device("cuda", 0)
    plan = nd.Plan(pr.points, nx, ny, precision="fp32", eps=eps, ir_maxit=60, ir_tol=1e-12)
    plan.set_profiling(True)
    f = plan.apply(torch.from_numpy(pr.c_true).to(dev))
    plan.factor()
    plan.solve(f)
    plan.info()          # folds the recorded launches into the log
    plan.close()
    rows = np.loadtxt(log_path, ndmin=2)
    return rows


def classes(rows, top: int):
    out = {}
    for row in rows:
        # class, ms, flops, descriptors, m, n, k, variant (then the algorithm step)
        cls, ms, _fl, ndesc, m, n, k, var = row[:8]
        # matrix-core GEMMs (classes 1, 2) and skinny products (4, 5)
        if int(cls) not in (1, 2, 4, 5) or m <= 0 or n <= 0 or k <= 0:
            continue
        prec = 1 if int(cls) in (1, 4) else 0
        opa, opb, _sk = decode(int(var))
        key = (prec, opa, opb, clog2(int(m)), clog2(int(n)), clog2(int(k)), clog2(int(ndesc)))
        c = out.setdefault(key, dict(ms=0.0, count=0, m=0, n=0, k=0, nd=0))
        c["ms"] += ms
        c["count"] += 1
        c["m"] = max(c["m"], int(m))
        c["n"] = max(c["n"], int(n))
        c["k"] = max(c["k"], int(k))
        c["nd"] = max(c["nd"], int(ndesc))
    return sorted(out.items(), key=lambda kv: -kv[1]["ms"])[:top]


def time_class(lib, key, c, reps=3):
    import torch
    prec, opa, opb = key[0], key[1], key[2]
    m, n, k, ndesc = c["m"], c["n"], c["k"], c["nd"]
    esz = 16 if prec == 0 else 8
    if ndesc * (m * k + k * n + m * n) * esz > MEM_CAP:
        return None
    ct = torch.complex128 if prec == 0 else torch.complex64
    dev = torch.device("cuda", 0)
    # distinct operands per descriptor, as in the factorization's batches
    A = torch.randn((ndesc, m * k), dtype=ct, device=dev)
    B = torch.randn((ndesc, k * n), dtype=ct, device=dev)
    Cs = torch.zeros((ndesc, m * n), dtype=ct, device=dev)
    lda = m if opa == 0 else k
    ldb = k if opb == 0 else n
    mnk = np.tile(np.array([m, n, k], np.int32), ndesc)
    ld = np.tile(np.array([lda, ldb, m], np.int32), ndesc)
    ptr = np.empty(3 * ndesc, np.int64)
    idx = np.arange(ndesc, dtype=np.int64)
    ptr[0::3] = A.data_ptr() + idx * m * k * esz
    ptr[1::3] = B.data_ptr() + idx * k * n * esz
    ptr[2::3] = Cs.data_ptr() + idx * m * n * esz
    p32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
    ms = C.c_float(0)

    def run(s):
        best = float("inf")
        for _ in range(reps + 1):
            # FP32 classes are timed on the bf16 split, the plans' default
            # kind of FP32 product (the table does not tell the kinds apart)
            st = lib.nudft2_test_gemm_cfg(2 if prec == 1 else prec, opa, opb, ndesc, p32(mnk),
                                          p32(ld),
                                          ptr.ctypes.data_as(C.POINTER(C.c_int64)),
                                          1.0, 0.0, 0.0, s, C.byref(ms))
            if st != 0:
                raise RuntimeError(lib.nudft2_last_error())
            best = min(best, ms.value)
        return best

    auto = run(-2)
    res = {}
    kmin = 64 if n <= 8 and opb == 0 else 16
    for s in SPLITS:
        if k // s < kmin and s > 1:
            break
        res[(s, 0)] = run(s)
    for t in small_tiles(opa, opb, m, n):
        res[(0, t)] = run(TILE_CODES[t])
    # the first configuration of a class can run before the clocks settle:
    # time the baseline again once the candidates have run
    auto = min(auto, run(-2))
    del A, B, Cs
    torch.cuda.empty_cache()
    return auto, res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="n512,batch64",
                    help="comma-separated: n512, n128, batch64")
    ap.add_argument("--top", type=int, default=48)
    ap.add_argument("--out", default=INC)
    ap.add_argument("--no-merge", action="store_true",
                    help="write only this run's entries (default: merge with --out's table)")
    args = ap.parse_args()
    workloads = args.workload.split(",")
    for w in workloads:
        if w not in ("n512", "n128", "batch64"):
            raise SystemExit(f"unknown workload {w}")
    picked = {}
    # the library takes the log's path once per process: one file, each
    # workload's rows are the ones it appended
    log_path = os.path.join(tempfile.mkdtemp(prefix="nudft2_tune_"), "launches.txt")
    seen = 0
    for w in workloads:
        t0 = time.time()
        allrows = collect(w, log_path)
        rows = allrows[seen:]
        seen = len(allrows)
        print(f"[tune] {w}: {len(rows)} launches logged in {time.time() - t0:.1f} s", flush=True)
        for key, c in classes(rows, args.top):
            if key in picked:
                o = picked[key]
                o["ms"] += c["ms"]
                o["count"] += c["count"]
                for f in ("m", "n", "k", "nd"):
                    o[f] = max(o[f], c[f])
            else:
                picked[key] = dict(c)
    sys.path.insert(0, ROOT)
    from paper_2607_00928_amd import _lib
    lib = _lib.lib
    measured = {}
    for key, c in sorted(picked.items(), key=lambda kv: -kv[1]["ms"]):
        r = time_class(lib, key, c)
        if r is None:
            print(f"[tune] {key} skipped (operands above the memory cap)", flush=True)
            continue
        auto, res = r
        best = min(res, key=res.get)
        gain = auto / res[best] if res[best] > 0 else 1.0
        what = f"split {best[0]}" if best[1] == 0 else ("32x128 tiles", "square tiles")[best[1] - 1]
        print(f"[tune] {key} m={c['m']} n={c['n']} k={c['k']} nd={c['nd']} "
              f"({c['ms']:.1f} ms in the run): heuristic {auto:.3f} ms, best {what} "
              f"{res[best]:.3f} ms (x{gain:.2f})", flush=True)
        measured[key] = (best, gain)
    old = {} if args.no_merge else read_table(args.out)
    table = merge_entries(old, measured)
    lines = sorted("{%d, %d, %d, %d, %d, %d, %d, %d, %d}," % (*k, *v) for k, v in table.items())
    with open(args.out, "w") as fh:
        fh.write("// Autotuned tile shapes and k splits (written by tune_gemm.py from %s runs):\n"
                 % args.workload)
        fh.write("// {prec, opA, opB, log2 m, log2 n, log2 k, log2 descriptors, splits, tile},\n")
        for l in lines:
            fh.write(l + "\n")
    print(f"[tune] wrote {len(lines)} entries to {args.out} ({len(measured)} classes measured, "
          f"{len(old)} entries before)", flush=True)


if __name__ == "__main__":
    main()
