"""ctypes binding of libnudft2.so (argument marshalling only).

The library is loaded from this package's directory; there is no fallback:
if the shared object is missing the import fails with an error that says how
to build it.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnudft2.so")

STATUS = {
    0: "OK", 1: "E_INVAL", 2: "E_STATE", 3: "E_DEVICE", 4: "E_NOMEM",
    5: "E_SINGULAR", 6: "E_NOCONV", 7: "E_INTERNAL",
}


class Opts(C.Structure):
    _fields_ = [
        ("precision", C.c_int32),
        ("eps", C.c_double),
        ("leaf", C.c_int32),
        ("ir_tol", C.c_double),
        ("ir_maxit", C.c_int32),
        ("refine", C.c_int32),
        ("stream", C.c_void_p),
        ("mem_cap", C.c_size_t),
        ("graph", C.c_int32),
        ("nufft_tol", C.c_double),
        ("fp32_products", C.c_int32),
        ("fadi_1d", C.c_int32),
    ]


class SolveInfo(C.Structure):
    _fields_ = [
        ("iterations", C.c_int32),
        ("rel_update", C.c_double),
        ("rel_residual", C.c_double),
    ]


class Info(C.Structure):
    _fields_ = [
        ("nprob", C.c_int32),
        ("levels", C.c_int32),
        ("max_rank_u", C.c_int32 * 16),
        ("max_rank_v", C.c_int32 * 16),
        ("factor_bytes", C.c_int64),
        ("factor_flops", C.c_double),
        ("sweep_bytes", C.c_int64),
        ("t_plan_ms", C.c_double),
        ("t_compress_ms", C.c_double),
        ("t_facesplit_ms", C.c_double),
        ("t_recompress_ms", C.c_double),
        ("t_urv_ms", C.c_double),
        ("kernel_ms", C.c_double * 6),
        ("kernel_flops", C.c_double * 6),
        ("kernel_launches", C.c_int64 * 6),
        ("peak_bytes", C.c_int64),
    ]


class NudftError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        self.code = STATUS.get(status, str(status))
        super().__init__(f"{where}: {self.code}: {msg}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` "
            "(or python paper_2607_00928_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    DP = C.POINTER(C.c_double)
    I64P = C.POINTER(C.c_int64)
    I32P = C.POINTER(C.c_int32)
    FP = C.POINTER(C.c_float)
    sig = {
        "nudft2_default_opts": (None, [C.POINTER(Opts)]),
        "nudft2_plan": (C.c_int, [C.POINTER(P), P, C.c_int64, C.c_int32, C.c_int32,
                                  C.POINTER(Opts)]),
        "nudft2_plan_batch": (C.c_int, [C.POINTER(P), C.c_int32, P, I64P, I32P, I32P,
                                        C.POINTER(Opts)]),
        "nudft2_factor": (C.c_int, [P]),
        "nudft2_solve": (C.c_int, [P, P, P, C.c_int32, C.POINTER(SolveInfo)]),
        "nudft2_solve_adj": (C.c_int, [P, P, P, C.c_int32, C.POINTER(SolveInfo)]),
        "nudft2_lsq_backward": (C.c_int, [P, P, P, P, P, P, C.c_int32, C.POINTER(SolveInfo)]),
        "nudft2_apply": (C.c_int, [P, P, P, C.c_int32]),
        "nudft2_apply_adj": (C.c_int, [P, P, P, C.c_int32]),
        "nudft2_apply_adj_noalloc": (C.c_int, [P, P, P, C.c_int32]),
        "nudft2_nufft": (C.c_int, [P, P, P, C.c_int32, C.c_double]),
        "nudft2_nufft_adj": (C.c_int, [P, P, P, C.c_int32, C.c_double]),
        "nudft2_get_info": (C.c_int, [P, C.POINTER(Info)]),
        "nudft2_destroy": (C.c_int, [P]),
        "nudft2_set_profiling": (C.c_int, [P, C.c_int32]),
        "nudft2_set_profiling_classes": (C.c_int, [P, C.c_uint32]),
        "nudft2_set_nufft_tol": (C.c_int, [P, C.c_double]),
        "nudft2_set_solve_opts": (C.c_int, [P, C.c_double, C.c_int32, C.c_int32]),
        "nudft2_strerror": (C.c_char_p, [C.c_int]),
        "nudft2_last_error": (C.c_char_p, []),
        "nudft2_test_binning": (C.c_int, [DP, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                          I64P, I64P, I64P, I32P]),
        "nudft2_test_mfma_layout": (C.c_int, [DP, DP, DP]),
        "nudft2_test_mfma_layout32": (C.c_int, [FP, FP, FP]),
        "nudft2_test_gemm": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, I32P, I32P,
                                       I64P, C.c_double, C.c_double, C.c_double]),
        "nudft2_test_gemm_cfg": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, I32P,
                                           I32P, I64P, C.c_double, C.c_double, C.c_double,
                                           C.c_int32, C.POINTER(C.c_float)]),
        "nudft2_test_geqrf": (C.c_int, [C.c_int32, C.c_int32, I32P, I32P, I64P]),
        "nudft2_test_ormqr": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, I32P, I32P, I64P]),
        "nudft2_test_pchol": (C.c_int, [C.c_int32, I32P, I32P, I64P, C.c_double, I32P, I32P]),
        "nudft2_test_trsv": (C.c_int, [C.c_int32, C.c_int32, I32P, I32P, I64P, C.c_int32]),
        "nudft2_test_trtri": (C.c_int, [C.c_int32, C.c_int32, I32P, I32P, I64P]),
        "nudft2_test_copy": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, I32P, I32P, I64P, I32P]),
        "nudft2_test_fadi_block": (C.c_int, [P, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                             C.c_double, I32P, DP, DP, C.c_int32, P, P]),
        "nudft2_test_hss1d_matvec": (C.c_int, [P, C.c_int32, C.c_double, P, P, I32P, C.c_int32]),
        "nudft2_test_hss_matvec": (C.c_int, [P, P, P, C.c_int32, C.c_int32, C.c_int32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(status: int, where: str):
    if status != 0:
        msg = lib.nudft2_last_error().decode(errors="replace")
        raise NudftError(status, where, msg)


def default_opts() -> Opts:
    o = Opts()
    lib.nudft2_default_opts(C.byref(o))
    return o


def dptr(arr) -> C.POINTER(C.c_double):
    """Pointer to the data of a C-contiguous float64 numpy array."""
    return arr.ctypes.data_as(C.POINTER(C.c_double))
