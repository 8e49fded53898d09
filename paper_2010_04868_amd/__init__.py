"""tvstencil: time-skewed temporal stencil sweeps on MI355X (gfx950).

Python binding over the C ABI declared in ``include/tvstencil.h``.  Each
function here marshals arguments and calls the native library; every step of
the computation runs in the HIP kernels.  PyTorch provides device memory
(tensors) and streams only.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

from . import _lib
from ._lib import StencilError, check
from .inputs import (BOX, DIRICHLET, F32, F64, GAUSS_SEIDEL, I32, JACOBI, PERIODIC, STAR,
                     Problem, npoints)

METHOD_PLAIN, METHOD_TSTP = 0, 1
RULE_WEIGHTED, RULE_LIFE = 0, 1

__all__ = ["Plan", "LifePlan", "LcsPlan", "run", "run_simple", "batch_run", "Server", "StencilError",
           "load", "STAR", "BOX", "JACOBI", "GAUSS_SEIDEL", "DIRICHLET", "PERIODIC", "F32", "F64",
           "I32", "METHOD_PLAIN", "METHOD_TSTP", "RULE_WEIGHTED", "RULE_LIFE", "version"]


def load():
    return _lib.load()


def version() -> str:
    return load().stencil_version().decode()


def _torch():
    import torch
    return torch


def _dtype_of(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.int32:
        return I32
    raise TypeError(f"unsupported tensor dtype {t.dtype}")


def _stream_handle(stream=None) -> Optional[int]:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _coeff_array(coeffs: Sequence[float]):
    arr = (ctypes.c_double * len(coeffs))(*[float(c) for c in coeffs])
    return arr


class Plan:
    """A validated stencil problem plus the schedule chosen to run it."""

    def __init__(self, dims: Sequence[int], dtype: int, shape: int, order: int,
                 dependence: int = JACOBI, boundary: int = DIRICHLET,
                 tuning: Optional[str] = None):
        lib = load()
        self._h = ctypes.c_void_p()
        d = (ctypes.c_int64 * len(dims))(*[int(x) for x in dims])
        check(lib.stencil_plan(ctypes.byref(self._h), len(dims), d, int(dtype), int(shape),
                               int(order), int(dependence), int(boundary),
                               tuning.encode() if tuning else None))
        self.dims = tuple(int(x) for x in dims)
        self.dtype, self.shape, self.order = dtype, shape, order
        self.dependence, self.boundary = dependence, boundary

    @classmethod
    def for_problem(cls, p: Problem, tuning: Optional[str] = None) -> "Plan":
        if p.dtype == I32:
            return LifePlan(p.dims, p.boundary, tuning)
        return cls(p.dims, p.dtype, p.shape, p.order, p.dependence, p.boundary, tuning)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def info(self) -> dict:
        inf = _lib.PlanInfo()
        check(load().stencil_plan_info(self._h, ctypes.byref(inf)))
        out = {f: getattr(inf, f) for f, _ in inf._fields_}
        out["dims"] = tuple(inf.dims[: inf.ndim])
        out["tuning"] = inf.tuning.decode()
        out["varcoef_tuning"] = inf.varcoef_tuning.decode()
        return out

    def tuning(self) -> str:
        """The plan's schedule as a tuning string (accepted by ``Plan(..., tuning=)``)."""
        return self.info()["tuning"]

    def run(self, grid, coeffs: Optional[Sequence[float]], T: int, stream=None) -> None:
        """Advance the device tensor ``grid`` by T steps, asynchronously on ``stream``."""
        if tuple(grid.shape) != self.dims or _dtype_of(grid) != self.dtype:
            raise ValueError("grid shape/dtype does not match the plan")
        if not grid.is_contiguous() or not grid.is_cuda:
            raise ValueError("grid must be a contiguous device tensor")
        c = None if coeffs is None else _coeff_array(coeffs)
        check(load().stencil_run(self._h, ctypes.c_void_p(grid.data_ptr()), c, int(T),
                                 ctypes.c_void_p(_stream_handle(stream))))

    def run_varcoef(self, grid, weights, T: int, stream=None) -> None:
        """T Jacobi steps with a weight per offset per point: ``weights`` is a
        device tensor of shape (order,) + dims in the grid's dtype."""
        if tuple(grid.shape) != self.dims or _dtype_of(grid) != self.dtype:
            raise ValueError("grid shape/dtype does not match the plan")
        if (tuple(weights.shape) != (self.order,) + self.dims or weights.dtype != grid.dtype
                or not weights.is_contiguous() or not weights.is_cuda):
            raise ValueError("weights must be a contiguous device tensor of shape "
                             "(order,) + dims in the grid's dtype")
        check(load().stencil_run_varcoef(self._h, ctypes.c_void_p(grid.data_ptr()),
                                         ctypes.c_void_p(weights.data_ptr()), int(T),
                                         ctypes.c_void_p(_stream_handle(stream))))

    def check(self) -> None:
        """Wait for the plan's last run and raise if a Gauss-Seidel launch of it
        (or of an earlier unreported run) aborted (``stencil_plan_check``)."""
        check(load().stencil_plan_check(self._h))

    def tune(self, grid, coeffs: Optional[Sequence[float]], T_probe: int, stream=None) -> str:
        buf = ctypes.create_string_buffer(256)
        c = None if coeffs is None else _coeff_array(coeffs)
        check(load().stencil_tune(self._h, ctypes.c_void_p(grid.data_ptr()), c, int(T_probe),
                                  ctypes.c_void_p(_stream_handle(stream)), buf, 256))
        return buf.value.decode()

    def close(self) -> None:
        if self._h:
            load().stencil_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LifePlan(Plan):
    """Game of Life B2S23 on an int32 board (``stencil_plan_life``): the 2D
    9-point box neighbourhood, Jacobi dependence, no weights."""

    def __init__(self, dims: Sequence[int], boundary: int = DIRICHLET,
                 tuning: Optional[str] = None):
        lib = load()
        self._h = ctypes.c_void_p()
        d = (ctypes.c_int64 * len(dims))(*[int(x) for x in dims])
        check(lib.stencil_plan_life(ctypes.byref(self._h), len(dims), d, int(boundary),
                                    tuning.encode() if tuning else None))
        self.dims = tuple(int(x) for x in dims)
        self.dtype, self.shape, self.order = I32, BOX, 9
        self.dependence, self.boundary = JACOBI, boundary

    def run(self, grid, coeffs=None, T: int = 0, stream=None) -> None:
        """Advance the int32 device tensor ``grid`` by T generations (``coeffs`` is ignored)."""
        super().run(grid, None, T, stream)

    def tune(self, grid, coeffs=None, T_probe: int = 1, stream=None) -> str:
        return super().tune(grid, None, T_probe, stream)


class LcsPlan:
    """Longest common subsequence of byte sequences of lengths m and n
    (``stencil_lcs_plan``): the 1D Gauss-Seidel-like dynamic program of
    Section 3.4 on device tensors."""

    def __init__(self, m: int, n: int, tuning: Optional[str] = None):
        self._h = ctypes.c_void_p()
        check(load().stencil_lcs_plan(ctypes.byref(self._h), int(m), int(n),
                                      tuning.encode() if tuning else None))
        self.m, self.n = int(m), int(n)

    @property
    def tile_width(self) -> int:
        return load().stencil_lcs_tile_width(self._h)

    @property
    def tile_rows(self) -> int:
        return load().stencil_lcs_tile_rows(self._h)

    def run(self, a, b, row, col, stream=None) -> None:
        """From the boundary row (int32, n+1) and column (int32, m+1; entry 0
        unused) to the last row and column, in place, asynchronously."""
        torch = _torch()
        for t, dt, size in ((a, torch.uint8, self.m), (b, torch.uint8, self.n),
                            (row, torch.int32, self.n + 1), (col, torch.int32, self.m + 1)):
            if t.dtype != dt or t.numel() != size or not t.is_cuda or not t.is_contiguous():
                raise ValueError("a, b: contiguous uint8 device tensors of m and n elements; "
                                 "row, col: contiguous int32 device tensors of n+1 and m+1")
        check(load().stencil_lcs_run(self._h, ctypes.c_void_p(a.data_ptr()),
                                     ctypes.c_void_p(b.data_ptr()),
                                     ctypes.c_void_p(row.data_ptr()),
                                     ctypes.c_void_p(col.data_ptr()),
                                     ctypes.c_void_p(_stream_handle(stream))))

    def close(self) -> None:
        if self._h:
            load().stencil_lcs_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run(problem: Problem, grid, T: Optional[int] = None, tuning: Optional[str] = None,
        stream=None) -> Plan:
    plan = Plan.for_problem(problem, tuning)
    plan.run(grid, problem.coeffs, problem.T if T is None else T, stream)
    return plan


def run_simple(grid, coeffs: Sequence[float], shape: int, order: int, dependence: int,
               boundary: int, T: int, stream=None) -> None:
    d = (ctypes.c_int64 * grid.dim())(*grid.shape)
    c = _coeff_array(coeffs)
    check(load().stencil_run_simple(ctypes.c_void_p(grid.data_ptr()), grid.dim(), d,
                                    _dtype_of(grid), c, shape, order, dependence, boundary,
                                    int(T), ctypes.c_void_p(_stream_handle(stream))))


def batch_run(plans: List[Plan], grids: list, coeffs: List[Sequence[float]], T: List[int],
              stream=None) -> None:
    n = len(plans)
    P = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    G = (ctypes.c_void_p * n)(*[g.data_ptr() for g in grids])
    arrs = [_coeff_array(c) for c in coeffs]
    C = (ctypes.POINTER(ctypes.c_double) * n)(*[ctypes.cast(a, ctypes.POINTER(ctypes.c_double))
                                                 for a in arrs])
    Tn = (ctypes.c_int64 * n)(*[int(t) for t in T])
    check(load().stencil_batch_run(n, P, G, C, Tn, ctypes.c_void_p(_stream_handle(stream))))


class Server:
    """Continuous-batching server for stencil solves (host buffers in, host buffers out)."""

    def __init__(self, hbm_budget: int = 0, max_slots: int = 0, chunk_steps: int = 0):
        self._h = ctypes.c_void_p()
        check(load().stencil_server_create(ctypes.byref(self._h), int(hbm_budget),
                                           int(max_slots), int(chunk_steps)))

    def submit(self, p: Problem, host_in) -> int:
        import numpy as np
        a = np.ascontiguousarray(host_in)
        req = _lib.Request()
        req.ndim = len(p.dims)
        for i, d in enumerate(p.dims):
            req.dims[i] = d
        req.dtype, req.shape, req.order = p.dtype, p.shape, p.order
        req.dependence, req.boundary = p.dependence, p.boundary
        c = _coeff_array(p.coeffs)
        req.coeffs = ctypes.cast(c, ctypes.POINTER(ctypes.c_double))
        req.T = p.T
        req.host_in = a.ctypes.data
        rid = ctypes.c_uint64()
        check(load().stencil_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        return rid.value

    def poll(self, rid: int, out) -> Optional[tuple]:
        st = ctypes.c_int()
        ts = (ctypes.c_double * 4)()
        check(load().stencil_server_poll(self._h, rid, ctypes.byref(st),
                                         ctypes.c_void_p(out.ctypes.data), ts))
        return tuple(ts) if st.value == 1 else None

    def wait(self, rid: int, out) -> tuple:
        ts = (ctypes.c_double * 4)()
        check(load().stencil_server_wait(self._h, rid, ctypes.c_void_p(out.ctypes.data), ts))
        return tuple(ts)

    def now(self) -> float:
        return load().stencil_server_now(self._h)

    def stats(self) -> dict:
        s = _lib.ServerStats()
        check(load().stencil_server_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def close(self) -> None:
        if self._h:
            load().stencil_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
