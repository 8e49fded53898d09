"""CPU oracle for the stencil sweeps -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps the plain C sweep in
``oracle.c`` (naive (d+1)-loop sweep of Section 1 / Algorithm 1, Gauss-Seidel
in place as in Section 3.4), which shares no code with the HIP library.

Every function here is pinned by ``tests/test_oracle_pins.py`` against exact
rational brute force, eigenmode closed forms and invariants.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

STAR, BOX = 0, 1
JACOBI, GAUSS_SEIDEL = 0, 1
DIRICHLET, PERIODIC = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
# TVS_ORACLE_LIBRARY: a sanitized build of the same source (oracle/build.py)
_LIB_PATH = os.environ.get("TVS_ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build  # compile on first use (gcc only)
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64p = ctypes.POINTER(ctypes.c_int64)
    for name, real in (("oracle_sweep_f64", ctypes.c_double), ("oracle_sweep_f32", ctypes.c_float)):
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                       ctypes.POINTER(real), ctypes.c_int64, ctypes.POINTER(real)]
        fn.restype = ctypes.c_int
    for name, real in (("oracle_sweep_f64_varcoef", ctypes.c_double),
                       ("oracle_sweep_f32_varcoef", ctypes.c_float)):
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                       ctypes.POINTER(real), ctypes.c_int64, ctypes.POINTER(real)]
        fn.restype = ctypes.c_int
    lib.oracle_offsets.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int)]
    lib.oracle_offsets.restype = ctypes.c_int
    lib.oracle_life.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_int32)]
    lib.oracle_life.restype = ctypes.c_int
    u8p, i32p = ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32)
    lib.oracle_lcs.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, i32p, i32p]
    lib.oracle_lcs.restype = ctypes.c_int
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def offsets(ndim: int, shape: int, npoints: int) -> np.ndarray:
    """Canonical offset list (lexicographic, axis 0 most significant)."""
    lib = _load()
    buf = (ctypes.c_int * (npoints * ndim))()
    P = lib.oracle_offsets(ndim, shape, npoints, buf)
    if P < 0:
        raise OracleError(f"oracle_offsets failed ({P})")
    return np.array(buf[:], dtype=np.int64).reshape(P, ndim)


def sweep(u: np.ndarray, coeffs: Sequence[float], shape: int, dependence: int, boundary: int,
          T: int, npoints: int | None = None, precision: str = "f64") -> np.ndarray:
    """Return u after T steps of the naive sweep (the input is not modified).

    ``precision="f64"`` (the reference) widens the input to float64 and uses
    the coefficients as given.  ``precision="f32"`` repeats the identical
    operation sequence in single precision with coefficients rounded to
    float32 (round to nearest even).
    """
    lib = _load()
    if npoints is None:
        npoints = len(coeffs)
    if len(coeffs) != npoints:
        raise OracleError("coefficient count differs from the point count")
    if precision == "f64":
        real, fn, np_real = ctypes.c_double, lib.oracle_sweep_f64, np.float64
    elif precision == "f32":
        real, fn, np_real = ctypes.c_float, lib.oracle_sweep_f32, np.float32
    else:
        raise OracleError(f"unknown precision {precision!r}")
    g = np.ascontiguousarray(u, dtype=np_real).copy()
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64).astype(np_real))
    dims = (ctypes.c_int64 * g.ndim)(*g.shape)
    rc = fn(g.ndim, dims, shape, npoints, dependence, boundary,
            c.ctypes.data_as(ctypes.POINTER(real)), int(T), g.ctypes.data_as(ctypes.POINTER(real)))
    if rc != 0:
        raise OracleError(f"oracle sweep failed ({rc})")
    return g


def life(u: np.ndarray, boundary: int, T: int) -> np.ndarray:
    """Return the int32 board u after T steps of Game of Life B2S23 (the input is not modified).

    The rule of the paper's Life stencil (Section 3.4): a dead cell becomes live
    with exactly 2 live neighbours of 8, a live cell stays live with 2 or 3.  A
    cell is live when non-zero; its neighbour count is the sum of the 8
    neighbour values.  Dirichlet keeps the outer layer; periodic wraps.
    """
    lib = _load()
    g = np.ascontiguousarray(u, dtype=np.int32).copy()
    if g.ndim != 2:
        raise OracleError("Life boards are 2D")
    rc = lib.oracle_life(g.shape[0], g.shape[1], boundary, int(T),
                         g.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc != 0:
        raise OracleError(f"oracle life failed ({rc})")
    return g


def lcs(a, b, row=None, col=None):
    """Longest-common-subsequence table of byte sequences a (m) and b (n), as
    the 1D Gauss-Seidel-like dynamic program of Section 3.4: from the boundary
    row lcs[0][0..n] (default zeros) and column lcs[1..m][0] (``col[1:]``,
    default zeros) to ``(last_row, last_col)`` = (lcs[m][0..n], lcs[0..m][n]).
    With zero boundaries ``last_row[-1]`` is the LCS length.  Inputs are not
    modified.
    """
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    m, n = a.size, b.size
    r = np.zeros(n + 1, np.int32) if row is None else np.array(row, dtype=np.int32, copy=True)
    c = np.zeros(m + 1, np.int32) if col is None else np.array(col, dtype=np.int32, copy=True)
    if r.shape != (n + 1,) or c.shape != (m + 1,):
        raise OracleError("row must hold n+1 values and col m+1")
    u8p, i32p = ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32)
    rc = lib.oracle_lcs(a.ctypes.data_as(u8p), m, b.ctypes.data_as(u8p), n,
                        r.ctypes.data_as(i32p), c.ctypes.data_as(i32p))
    if rc != 0:
        raise OracleError(f"oracle lcs failed ({rc})")
    return r, c


def sweep_varcoef(u: np.ndarray, weights: np.ndarray, shape: int, boundary: int, T: int,
                  npoints: int, precision: str = "f64") -> np.ndarray:
    """Jacobi sweep with a weight per offset per point (variable coefficients,
    fixed over time): ``weights`` has shape (npoints,) + u.shape, offsets in
    canonical order.  Same operation order as ``sweep``; the input is not
    modified."""
    lib = _load()
    real = np.float64 if precision == "f64" else np.float32
    ct = ctypes.c_double if precision == "f64" else ctypes.c_float
    g = np.ascontiguousarray(u, dtype=real).copy()
    w = np.ascontiguousarray(weights, dtype=real)
    if w.shape != (npoints,) + g.shape:
        raise OracleError("weights must have shape (npoints,) + grid shape")
    dims = (ctypes.c_int64 * g.ndim)(*g.shape)
    fn = lib.oracle_sweep_f64_varcoef if precision == "f64" else lib.oracle_sweep_f32_varcoef
    rc = fn(g.ndim, dims, shape, npoints, boundary, w.ctypes.data_as(ctypes.POINTER(ct)), int(T),
            g.ctypes.data_as(ctypes.POINTER(ct)))
    if rc != 0:
        raise OracleError(f"oracle varcoef sweep failed ({rc})")
    return g
