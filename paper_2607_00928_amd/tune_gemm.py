"""Autotuner of the batched complex GEMM: picks the k split per launch shape
class by measurement and writes csrc/gemm_tuning.inc (rebuild afterwards).

    python -m paper_2607_00928_amd.tune_gemm [--workload n512] [--top 48]

1. Runs factor + refined solve of a workload with per-launch kernel logging
   (NUDFT2_PROF_LOG) to collect the shapes of the GEMM launches.
2. Buckets the launches into classes (precision, op(A), op(B), ceil(log2) of
   the largest m, n, k and of the descriptor count) and keeps the classes that
   took the most time.
3. Times, for each class, a synthetic batch at the class's largest shape with
   every candidate split and with the library's heuristic without the table
   (nudft2_test_gemm_cfg: HIP events around the launch).
4. Writes the classes where a forced split beats the heuristic by more than
   5% (so a rerun keeps the entries that still hold).
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


def decode(var: int):
    """(opA, opB, skinny) from the launch log's variant code."""
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
    from nudft_inputs import config_problem, make_problem

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
        res[s] = run(s)
    # the first configuration of a class can run before the clocks settle:
    # time the baseline again once the candidates have run
    auto = min(auto, run(-2))
    del A, B, Cs
    torch.cuda.empty_cache()
    return auto, res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="n512", choices=["n512", "n128"])
    ap.add_argument("--top", type=int, default=48)
    ap.add_argument("--out", default=INC)
    args = ap.parse_args()
    log_path = os.path.join(tempfile.mkdtemp(prefix="nudft2_tune_"), "launches.txt")
    t0 = time.time()
    rows = collect(args.workload, log_path)
    print(f"[tune] {len(rows)} launches logged in {time.time() - t0:.1f} s", flush=True)
    sys.path.insert(0, ROOT)
    from paper_2607_00928_amd import _lib
    lib = _lib.lib
    lines = []
    for key, c in classes(rows, args.top):
        r = time_class(lib, key, c)
        if r is None:
            print(f"[tune] {key} skipped (operands above the memory cap)", flush=True)
            continue
        auto, res = r
        best_s = min(res, key=res.get)
        gain = auto / res[best_s] if res[best_s] > 0 else 1.0
        print(f"[tune] {key} m={c['m']} n={c['n']} k={c['k']} nd={c['nd']} "
              f"({c['ms']:.1f} ms in the run): heuristic {auto:.3f} ms, best split {best_s} "
              f"{res[best_s]:.3f} ms (x{gain:.2f})", flush=True)
        if gain > 1.05:
            lines.append("{%d, %d, %d, %d, %d, %d, %d, %d}," % (*key, best_s))
    with open(args.out, "w") as fh:
        fh.write("// Autotuned k splits (written by tune_gemm.py from a %s run):\n" % args.workload)
        fh.write("// {prec, opA, opB, log2 m, log2 n, log2 k, log2 descriptors, splits},\n")
        for l in sorted(lines):
            fh.write(l + "\n")
    print(f"[tune] wrote {len(lines)} entries to {args.out}", flush=True)


if __name__ == "__main__":
    main()
