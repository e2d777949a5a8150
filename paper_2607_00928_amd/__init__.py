"""MI355X-native direct solver for the 2D type-II inverse NUDFT.

Python binding of libnudft2 (include/nudft2.h).  The binding only marshals
arguments: every step of the factorization, the solve and the transforms
runs in the library's HIP kernels.  PyTorch supplies device memory and the
stream.

    plan = Plan(points, nx, ny, precision="fp32", eps=1e-4)
    plan.factor()
    c = plan.solve(f)          # f: complex128 CUDA tensor (M,) or (nrhs, M)
    f2 = plan.apply(c)         # exact FP64 A c
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import NudftError, check, lib

__all__ = ["Plan", "BatchPlan", "NudftError", "lsq_solve"]

_PREC = {"fp64": 0, "fp32": 1, 0: 0, 1: 1}


_FP32_PRODUCTS = {"bf16x3": 0, "fp32": 1}


def _opts(precision, eps, leaf, ir_tol, ir_maxit, refine, stream, mem_cap, graph=False,
          nufft_tol=0.0, fp32_products="bf16x3", fadi_1d=True):
    o = _lib.default_opts()
    o.fp32_products = _FP32_PRODUCTS[fp32_products]
    o.fadi_1d = 1 if fadi_1d else 0
    o.graph = 1 if graph else 0
    o.nufft_tol = float(nufft_tol)
    o.precision = _PREC[precision]
    o.eps = float(eps)
    o.leaf = int(leaf)
    o.ir_tol = float(ir_tol)
    o.ir_maxit = int(ir_maxit)
    o.refine = int(refine)
    o.stream = C.c_void_p(stream) if stream else None
    o.mem_cap = int(mem_cap)
    return o


def _device_points(points, dev) -> torch.Tensor:
    """The points as a contiguous float64 (M, 2) tensor on dev (the library
    takes a device pointer and copies the points itself)."""
    if isinstance(points, torch.Tensor):
        t = points.detach()
    else:
        t = torch.from_numpy(np.ascontiguousarray(points, dtype=np.float64))
    if t.dim() != 2 or t.shape[1] != 2:
        raise ValueError("points must have shape (M, 2)")
    t = t.to(device=dev, dtype=torch.float64).contiguous()
    # the library reads the points on the plan's stream, which may differ
    # from the one this copy ran on
    torch.cuda.current_stream(dev).synchronize()
    return t


def _current_stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class _PlanBase:
    _handle = None

    def _check_dev(self, t: torch.Tensor, name: str):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
            raise TypeError(f"{name} must be a complex128 CUDA tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def factor(self):
        check(lib.nudft2_factor(self._handle), "nudft2_factor")
        return self

    def info(self) -> dict:
        inf = _lib.Info()
        check(lib.nudft2_get_info(self._handle, C.byref(inf)), "nudft2_get_info")
        L = inf.levels
        return dict(nprob=inf.nprob, levels=L,
                    max_rank_u=list(inf.max_rank_u)[:L + 1],
                    max_rank_v=list(inf.max_rank_v)[:L + 1],
                    factor_bytes=inf.factor_bytes, peak_bytes=inf.peak_bytes,
                    factor_flops=inf.factor_flops,
                    sweep_bytes=inf.sweep_bytes,
                    t_plan_ms=inf.t_plan_ms, t_compress_ms=inf.t_compress_ms,
                    t_facesplit_ms=inf.t_facesplit_ms,
                    t_recompress_ms=inf.t_recompress_ms, t_urv_ms=inf.t_urv_ms,
                    kernel_ms=list(inf.kernel_ms), kernel_flops=list(inf.kernel_flops),
                    kernel_launches=list(inf.kernel_launches))

    def set_solve_opts(self, ir_tol: float | None = None, ir_maxit: int | None = None,
                       refine: int | None = None):
        """Change the refinement options of this plan (factored or not)."""
        tol = self.ir_tol if ir_tol is None else float(ir_tol)
        maxit = self.ir_maxit if ir_maxit is None else int(ir_maxit)
        ref = self.refine if refine is None else int(refine)
        check(lib.nudft2_set_solve_opts(self._handle, tol, maxit, ref), "nudft2_set_solve_opts")
        self.ir_tol, self.ir_maxit, self.refine = tol, maxit, ref
        return self

    def set_nufft_tol(self, tol: float):
        """Refinement operator: 0 the exact direct sums, > 0 the NUFFT."""
        check(lib.nudft2_set_nufft_tol(self._handle, float(tol)), "nudft2_set_nufft_tol")
        return self

    def set_profiling(self, on: bool = True, classes=None):
        """Per-launch event timing of the kernel classes (info()["kernel_ms"]):
        every class when on, or only the class indices listed in classes."""
        if classes is None:
            check(lib.nudft2_set_profiling(self._handle, 1 if on else 0), "nudft2_set_profiling")
        else:
            mask = 0
            for c in classes:
                mask |= 1 << int(c)
            check(lib.nudft2_set_profiling_classes(self._handle, mask if on else 0),
                  "nudft2_set_profiling_classes")

    def _rhs(self, f: torch.Tensor):
        self._check_dev(f, "f")
        if f.dim() == 1:
            if f.numel() != self.M:
                raise ValueError("f has the wrong length")
            return 1, (self.N_shape)
        if f.dim() != 2 or f.shape[1] != self.M:
            raise ValueError("f must be (M,) or (nrhs, M)")
        return f.shape[0], (f.shape[0],) + self.N_shape

    def solve(self, f: torch.Tensor, out: torch.Tensor | None = None,
              return_info: bool = False):
        nrhs, shape = self._rhs(f)
        c = out if out is not None else torch.empty(shape, dtype=torch.complex128,
                                                    device=f.device)
        self._check_dev(c, "out")
        si = _lib.SolveInfo()
        st = lib.nudft2_solve(self._handle, C.c_void_p(f.data_ptr()),
                              C.c_void_p(c.data_ptr()), nrhs, C.byref(si))
        check(st, "nudft2_solve")
        if return_info:
            return c, dict(iterations=si.iterations, rel_update=si.rel_update,
                           rel_residual=si.rel_residual)
        return c

    def solve_adj(self, g: torch.Tensor, return_info: bool = False):
        self._check_dev(g, "g")
        nrhs = 1 if g.dim() == len(self.N_shape) else g.shape[0]
        shape = (self.M,) if nrhs == 1 and g.dim() == len(self.N_shape) else (nrhs, self.M)
        w = torch.empty(shape, dtype=torch.complex128, device=g.device)
        si = _lib.SolveInfo()
        st = lib.nudft2_solve_adj(self._handle, C.c_void_p(g.data_ptr()),
                                  C.c_void_p(w.data_ptr()), nrhs, C.byref(si))
        check(st, "nudft2_solve_adj")
        if return_info:
            return w, dict(iterations=si.iterations, rel_update=si.rel_update,
                           rel_residual=si.rel_residual)
        return w

    def lsq_backward(self, f: torch.Tensor, c: torch.Tensor, g: torch.Tensor,
                     points_grad: bool = True, return_info: bool = False):
        """Backward pass of c = A^+ f for the upstream gradient g = dL/dc:
        returns (dL/df, dL/dpoints or None) (see nudft2_lsq_backward)."""
        nrhs, _ = self._rhs(f)
        self._check_dev(c, "c")
        self._check_dev(g, "g")
        if c.numel() != g.numel() or c.numel() != nrhs * int(np.prod(self.N_shape)):
            raise ValueError("c and g must match the solution shape")
        gf = torch.empty_like(f)
        gp = (torch.empty((self.M, 2), dtype=torch.float64, device=f.device)
              if points_grad else None)
        si = _lib.SolveInfo()
        st = lib.nudft2_lsq_backward(self._handle, C.c_void_p(f.data_ptr()),
                                     C.c_void_p(c.data_ptr()), C.c_void_p(g.data_ptr()),
                                     C.c_void_p(gf.data_ptr()),
                                     C.c_void_p(gp.data_ptr()) if gp is not None else None,
                                     nrhs, C.byref(si))
        check(st, "nudft2_lsq_backward")
        if return_info:
            return gf, gp, dict(iterations=si.iterations, rel_update=si.rel_update)
        return gf, gp

    def apply(self, c: torch.Tensor) -> torch.Tensor:
        self._check_dev(c, "c")
        nrhs = 1 if c.dim() == len(self.N_shape) else c.shape[0]
        shape = (self.M,) if c.dim() == len(self.N_shape) else (nrhs, self.M)
        f = torch.empty(shape, dtype=torch.complex128, device=c.device)
        check(lib.nudft2_apply(self._handle, C.c_void_p(c.data_ptr()),
                               C.c_void_p(f.data_ptr()), nrhs), "nudft2_apply")
        return f

    def nufft(self, c: torch.Tensor, tol: float = 1e-12) -> torch.Tensor:
        """f ~= A c by spreading and FFT (nudft2_nufft)."""
        self._check_dev(c, "c")
        nrhs = 1 if c.dim() == len(self.N_shape) else c.shape[0]
        shape = (self.M,) if c.dim() == len(self.N_shape) else (nrhs, self.M)
        f = torch.empty(shape, dtype=torch.complex128, device=c.device)
        check(lib.nudft2_nufft(self._handle, C.c_void_p(c.data_ptr()), C.c_void_p(f.data_ptr()),
                               nrhs, float(tol)), "nudft2_nufft")
        return f

    def nufft_adj(self, f: torch.Tensor, tol: float = 1e-12) -> torch.Tensor:
        """c ~= A^* f by spreading and FFT (nudft2_nufft_adj)."""
        nrhs, shape = self._rhs(f)
        c = torch.empty(shape, dtype=torch.complex128, device=f.device)
        check(lib.nudft2_nufft_adj(self._handle, C.c_void_p(f.data_ptr()),
                                   C.c_void_p(c.data_ptr()), nrhs, float(tol)),
              "nudft2_nufft_adj")
        return c

    def apply_adj(self, f: torch.Tensor) -> torch.Tensor:
        nrhs, shape = self._rhs(f)
        c = torch.empty(shape, dtype=torch.complex128, device=f.device)
        check(lib.nudft2_apply_adj(self._handle, C.c_void_p(f.data_ptr()),
                                   C.c_void_p(c.data_ptr()), nrhs), "nudft2_apply_adj")
        return c

    def close(self):
        if self._handle is not None:
            lib.nudft2_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan(_PlanBase):
    """One problem: points (M, 2) float64 (array or tensor; handed to the
    library in device memory), nx x ny centred frequencies.
    fp32_products ("bf16x3" or "fp32"): matrix instructions of the FP32
    factorization's products (nudft2_opts.fp32_products).
    fadi_1d: 1D construction from fADI factors (True) or explicit Gram
    matrices (nudft2_opts.fadi_1d)."""

    def __init__(self, points, nx: int, ny: int, *, precision="fp32", eps=1e-4,
                 leaf=16, ir_tol=1e-12, ir_maxit=30, refine=0, stream=None,
                 mem_cap=0, device=None, graph=False, nufft_tol=0.0,
                 fp32_products="bf16x3", fadi_1d=True):
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        pts = _device_points(points, dev)
        self.M = pts.shape[0]
        self.nx, self.ny = int(nx), int(ny)
        self.N_shape = (self.nx, self.ny)
        if stream is None:
            stream = _current_stream(dev)
        o = _opts(precision, eps, leaf, ir_tol, ir_maxit, refine, stream, mem_cap, graph,
                  nufft_tol, fp32_products, fadi_1d)
        self.ir_tol, self.ir_maxit, self.refine = float(ir_tol), int(ir_maxit), int(refine)
        h = C.c_void_p()
        with torch.cuda.device(dev):
            st = lib.nudft2_plan(C.byref(h), C.c_void_p(pts.data_ptr()), self.M, self.nx,
                                 self.ny, C.byref(o))
        check(st, "nudft2_plan")
        self._handle = h
        self.points = pts


class BatchPlan(_PlanBase):
    """Many independent problems; right-hand sides and solutions are flat
    concatenations (see nudft2_plan_batch)."""

    def __init__(self, points_list, nx_list, ny_list, *, precision="fp32",
                 eps=1e-4, leaf=16, ir_tol=1e-12, ir_maxit=30, refine=0,
                 stream=None, mem_cap=0, device=None, graph=False, nufft_tol=0.0,
                 fp32_products="bf16x3", fadi_1d=True):
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        pts = [_device_points(p, dev) for p in points_list]
        m_off = np.zeros(len(pts) + 1, dtype=np.int64)
        m_off[1:] = np.cumsum([p.shape[0] for p in pts])
        allp = torch.cat(pts, dim=0).contiguous()
        torch.cuda.current_stream(dev).synchronize()
        nx = np.ascontiguousarray(nx_list, dtype=np.int32)
        ny = np.ascontiguousarray(ny_list, dtype=np.int32)
        self.M = int(m_off[-1])
        self.m_off = m_off
        self.n_off = np.concatenate([[0], np.cumsum(nx.astype(np.int64) * ny)])
        self.N_shape = (int(self.n_off[-1]),)
        if stream is None:
            stream = _current_stream(dev)
        o = _opts(precision, eps, leaf, ir_tol, ir_maxit, refine, stream, mem_cap, graph,
                  nufft_tol, fp32_products, fadi_1d)
        self.ir_tol, self.ir_maxit, self.refine = float(ir_tol), int(ir_maxit), int(refine)
        h = C.c_void_p()
        with torch.cuda.device(dev):
            st = lib.nudft2_plan_batch(
                C.byref(h), len(pts), C.c_void_p(allp.data_ptr()),
                m_off.ctypes.data_as(C.POINTER(C.c_int64)),
                nx.ctypes.data_as(C.POINTER(C.c_int32)),
                ny.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(o))
        check(st, "nudft2_plan_batch")
        self._handle = h
        self.nx_list, self.ny_list = nx, ny


def lsq_solve(*args, **kwargs):
    """Differentiable least-squares solve (see .autograd)."""
    from .autograd import lsq_solve as _f
    return _f(*args, **kwargs)
