"""Seeded synthetic inputs for the stencil workloads.

This module only draws numbers and describes problem shapes; it performs no
stencil arithmetic.  Both the HIP path (through the tests and the benchmark)
and the CPU oracle are fed from here, so that they see identical bits.

Problem description (Section 1 of the paper): a time-iterated update of a
regular d-dimensional grid, classified by dimension, number of points (order),
shape (star/box), dependence (Jacobi/Gauss-Seidel) and boundary
(constant/periodic).  ``dims`` are full storage extents; with a constant
(Dirichlet) boundary the outer layer of width r is part of the array and is
never written.

Generator: numpy ``Generator(PCG64(seed))``.  FP64 problems draw float64
values, FP32 problems draw float32 values (the FP64 oracle then runs on those
same values widened, so that a comparison measures arithmetic error only).
Game of Life boards (int32 cells) draw each cell live (1) with probability
``density`` from the same generator.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

STAR, BOX = 0, 1
JACOBI, GAUSS_SEIDEL = 0, 1
DIRICHLET, PERIODIC = 0, 1
F32, F64, I32 = 0, 1, 2

_NP = {F32: np.float32, F64: np.float64, I32: np.int32}


def np_dtype(dtype: int):
    return _NP[dtype]


def npoints(ndim: int, shape: int, radius: int = 1) -> int:
    """Number of stencil points of a star or box stencil of the given radius."""
    if shape == STAR:
        return 2 * ndim * radius + 1
    return (2 * radius + 1) ** ndim


@dataclasses.dataclass
class Problem:
    """One stencil problem: everything a caller passes to ``stencil_plan``/``run``."""

    name: str
    dims: Tuple[int, ...]
    dtype: int
    shape: int
    order: int
    dependence: int
    boundary: int
    coeffs: Tuple[float, ...]
    T: int
    seed: int
    zero_border: bool = False

    @property
    def ndim(self) -> int:
        return len(self.dims)

    @property
    def radius(self) -> int:
        """r from the point count: star P = 2 d r + 1, box P = (2r + 1)^d."""
        if self.shape == STAR:
            return (self.order - 1) // (2 * self.ndim)
        side = int(round(self.order ** (1.0 / self.ndim)))
        return (side - 1) // 2

    def updated_points(self) -> int:
        """Points written per step (GStencil/s counts only these)."""
        if self.boundary == PERIODIC:
            return int(np.prod(self.dims))
        return int(np.prod([n - 2 * self.radius for n in self.dims]))

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def uniform_grid(dims: Sequence[int], dtype: int, seed, zero_border: bool = False,
                 radius: int = 1) -> np.ndarray:
    """uniform[0,1) values from PCG64(seed), in the storage dtype of the problem.

    ``seed`` may be an int or a tuple of ints (numpy SeedSequence entropy).
    With ``zero_border`` the outer ``radius`` layers are overwritten with 0.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.random(tuple(int(n) for n in dims), dtype=_NP[dtype])
    if zero_border:
        for ax in range(a.ndim):
            idx = [slice(None)] * a.ndim
            idx[ax] = slice(0, radius)
            a[tuple(idx)] = 0
            idx[ax] = slice(a.shape[ax] - radius, a.shape[ax])
            a[tuple(idx)] = 0
    return a


def life_board(dims: Sequence[int], seed, density: float = 0.5,
               zero_border: bool = False) -> np.ndarray:
    """int32 0/1 board: each cell live with probability ``density`` (PCG64(seed)).

    With ``zero_border`` the outer layer is dead.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    a = (rng.random(tuple(int(n) for n in dims)) < density).astype(np.int32)
    if zero_border:
        a[0, :] = a[-1, :] = 0
        a[:, 0] = a[:, -1] = 0
    return a


def make_grid(p: Problem) -> np.ndarray:
    if p.dtype == I32:
        return life_board(p.dims, p.seed, 0.5, p.zero_border)
    return uniform_grid(p.dims, p.dtype, p.seed, p.zero_border, p.radius)


def star_coeffs(ndim: int, centre: float, neighbour: float) -> Tuple[float, ...]:
    """Coefficients of a radius-1 star stencil in canonical offset order.

    Canonical order lists offsets lexicographically with axis 0 most
    significant, so the centre sits in the middle: ndim entries before it and
    ndim after it.
    """
    return tuple([neighbour] * ndim + [centre] + [neighbour] * ndim)


# ---------------------------------------------------------------------------
# The workloads.  Sizes, coefficients and step counts are the ones the
# throughput figures are quoted on; the generator recipe is described above.
# ---------------------------------------------------------------------------

def heat1d(periodic: bool = False, n: int = 100000, T: int = 1000) -> Problem:
    """1D 3-point Jacobi, coefficients (1/4, 1/2, 1/4), fixed ends (or periodic)."""
    return Problem("heat1d_3p" + ("_periodic" if periodic else ""), (n,), F64, STAR, 3,
                   JACOBI, PERIODIC if periodic else DIRICHLET, (0.25, 0.5, 0.25), T, 1)


def star1d5p(n: int = 100000, T: int = 1000) -> Problem:
    """1D 5-point (radius 2) Jacobi, weights (0.05, 0.2, 0.5, 0.2, 0.05), fixed ends."""
    return Problem("star1d5p", (n,), F64, STAR, 5, JACOBI, DIRICHLET,
                   (0.05, 0.2, 0.5, 0.2, 0.05), T, 11)


def vc1d3p(n: int = 100000, T: int = 1000) -> Problem:
    """1D 3-point Jacobi with variable coefficients (a heat equation with a
    diffusivity per point): weights (a(x), 1 - 2a(x), a(x)), a(x) uniform in
    [0.1, 0.4] from varcoef_weights; fixed ends.  ``coeffs`` is empty: the
    weights are an array."""
    return Problem("vc1d3p", (n,), F64, STAR, 3, JACOBI, DIRICHLET, (), T, 12)


def varcoef_weights(p: Problem) -> np.ndarray:
    """Weights of shape (P,) + dims for the variable-coefficient workloads,
    drawn after the grid from PCG64((seed, 1)): vc1d3p (a, 1 - 2a, a) with a
    uniform in [0.1, 0.4]; vc2d5p (a, a, 1 - 4a, a, a) with a uniform in
    [0.05, 0.2] (canonical order N, W, C, E, S)."""
    rng = np.random.Generator(np.random.PCG64((p.seed, 1)))
    if p.ndim == 1:
        a = rng.uniform(0.1, 0.4, size=p.dims[0])
        return np.stack([a, 1.0 - 2.0 * a, a]).astype(_NP[p.dtype])
    a = rng.uniform(0.05, 0.2, size=p.dims)
    return np.stack([a, a, 1.0 - 4.0 * a, a, a]).astype(_NP[p.dtype])


def vc2d5p(n: int = 4096, T: int = 1000) -> Problem:
    """2D 5-point Jacobi with variable coefficients (a heat equation with a
    diffusivity per point): weights (a, a, 1 - 4a, a, a), a uniform in
    [0.05, 0.2] from varcoef_weights; zero Dirichlet border."""
    return Problem("vc2d5p", (n, n), F64, STAR, 5, JACOBI, DIRICHLET, (), T, 14,
                   zero_border=True)


def star2d9p(n: int = 8192, T: int = 1000) -> Problem:
    """2D 9-point star of radius 2, weights 0.05 / 0.1 at distance 2 / 1 and
    0.4 at the centre (canonical order (-2,0), (-1,0), (0,-2), (0,-1), (0,0),
    (0,1), (0,2), (1,0), (2,0)), zero Dirichlet border two points deep."""
    return Problem("star2d9p", (n, n), F64, STAR, 9, JACOBI, DIRICHLET,
                   (0.05, 0.1, 0.05, 0.1, 0.4, 0.1, 0.05, 0.1, 0.05), T, 13, zero_border=True)


def gs1d3p(n: int = 100000, T: int = 1000) -> Problem:
    """1D 3-point Gauss-Seidel in place, coefficients (1/4, 1/2, 1/4), fixed ends."""
    return Problem("gs1d3p", (n,), F64, STAR, 3, GAUSS_SEIDEL, DIRICHLET, (0.25, 0.5, 0.25), T, 6)


def box2d9p(dtype: int = F64, n: int = 8192, T: int = 1000) -> Problem:
    """2D 9-point box Jacobi, all coefficients 1/9, zero Dirichlet border."""
    return Problem("box2d9p" + ("_f32" if dtype == F32 else ""), (n, n), dtype, BOX, 9,
                   JACOBI, DIRICHLET, tuple([1.0 / 9.0] * 9), T, 2, zero_border=True)


def star3d7p(dtype: int = F64, n: int = 512, T: int = 100) -> Problem:
    """3D 7-point star Jacobi, centre 0.4, six neighbours 0.1, periodic."""
    return Problem("star3d7p" + ("_f32" if dtype == F32 else ""), (n, n, n), dtype, STAR, 7,
                   JACOBI, PERIODIC, star_coeffs(3, 0.4, 0.1), T, 3)


def gs2d5p(n: int = 4096, T: int = 100) -> Problem:
    """2D 5-point Gauss-Seidel in place, all five coefficients 0.2, zero border."""
    return Problem("gs2d5p", (n, n), F64, STAR, 5, GAUSS_SEIDEL, DIRICHLET,
                   tuple([0.2] * 5), T, 4, zero_border=True)


def life2d(n: int = 8000, T: int = 2000) -> Problem:
    """Game of Life B2S23 on an n x n int32 board (the paper's Life workload,
    8000^2 cells over 2000 steps in Table 1): cells live with probability 1/2,
    dead fixed border.  The rule has no weights."""
    return Problem("life2d", (n, n), I32, BOX, 9, JACOBI, DIRICHLET, (), T, 8, zero_border=True)


@dataclasses.dataclass
class LcsProblem:
    """Longest common subsequence of two random byte sequences (Section 3.4)."""

    name: str
    m: int
    n: int
    alphabet: int
    seed: int

    def cells(self) -> int:
        return self.m * self.n


def lcs_sequences(m: int, n: int, seed, alphabet: int = 4) -> Tuple[np.ndarray, np.ndarray]:
    """Two uint8 sequences of lengths m and n, letters uniform over
    0..alphabet-1, drawn from PCG64(seed) (the first sequence first)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.integers(0, alphabet, size=int(m), dtype=np.uint8)
    b = rng.integers(0, alphabet, size=int(n), dtype=np.uint8)
    return a, b


def lcs200k(m: int = 200000, n: int = 200000) -> LcsProblem:
    """The paper's LCS size (Table 1: 200000 x 200000), a 4-letter alphabet."""
    return LcsProblem("lcs", m, n, 4, 9)


def gs3d7p(n: int = 800, T: int = 200) -> Problem:
    """3D 7-point Gauss-Seidel in place (Table 1's GS-3D size, 800^3 x 200):
    centre 0.4, six neighbours 0.1, zero border."""
    return Problem("gs3d7p", (n, n, n), F64, STAR, 7, GAUSS_SEIDEL, DIRICHLET,
                   star_coeffs(3, 0.4, 0.1), T, 10, zero_border=True)


WORKLOADS = {
    "heat1d_3p": heat1d,
    "box2d9p": box2d9p,
    "star3d7p": star3d7p,
    "gs2d5p": gs2d5p,
    "life2d": life2d,
    "gs3d7p": gs3d7p,
    "star1d5p": star1d5p,
}


# ---------------------------------------------------------------------------
# Serving mix: a Poisson stream of mixed solves.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    index: int
    arrival_s: float
    problem: Problem


def _log_uniform_int(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def serving_mix(n_requests: int = 2000, rate_per_s: float = 100.0, seed: int = 5,
                side2d: Tuple[int, int] = (64, 4096), side3d: Tuple[int, int] = (32, 256),
                n1d: Tuple[int, int] = (1000, 1000000), steps: Tuple[int, int] = (10, 1000)
                ) -> List[Request]:
    """Poisson arrivals of 1D/2D/3D Jacobi and 2D Gauss-Seidel solves.

    Kind is uniform over {1D 3-point Jacobi, 2D Jacobi (5-point star or
    9-point box, 50/50), 3D 7-point Jacobi, 2D 5-point Gauss-Seidel}; 2D
    sides are log-uniform in ``side2d``, 3D sides in ``side3d``, 1D lengths in
    ``n1d``; T is uniform in ``steps``; FP32/FP64 50/50; Jacobi boundaries are
    Dirichlet/periodic 50/50 and Gauss-Seidel is Dirichlet.  Request ``i``
    draws its grid from seed ``(seed, i)``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out: List[Request] = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        kind = int(rng.integers(0, 4))
        dtype = F32 if rng.random() < 0.5 else F64
        T = int(rng.integers(steps[0], steps[1] + 1))
        periodic = rng.random() < 0.5
        bnd = PERIODIC if periodic else DIRICHLET
        if kind == 0:
            n = _log_uniform_int(rng, *n1d)
            p = Problem(f"req{i}_1d3p", (n,), dtype, STAR, 3, JACOBI, bnd, (0.25, 0.5, 0.25), T,
                        (seed, i))
        elif kind == 1:
            ny, nx = _log_uniform_int(rng, *side2d), _log_uniform_int(rng, *side2d)
            if rng.random() < 0.5:
                p = Problem(f"req{i}_2d5p", (ny, nx), dtype, STAR, 5, JACOBI, bnd,
                            tuple([0.2] * 5), T, (seed, i))
            else:
                p = Problem(f"req{i}_2d9p", (ny, nx), dtype, BOX, 9, JACOBI, bnd,
                            tuple([1.0 / 9.0] * 9), T, (seed, i))
        elif kind == 2:
            s = [_log_uniform_int(rng, *side3d) for _ in range(3)]
            p = Problem(f"req{i}_3d7p", tuple(s), dtype, STAR, 7, JACOBI, bnd,
                        star_coeffs(3, 0.4, 0.1), T, (seed, i))
        else:
            ny, nx = _log_uniform_int(rng, *side2d), _log_uniform_int(rng, *side2d)
            p = Problem(f"req{i}_gs2d5p", (ny, nx), dtype, STAR, 5, GAUSS_SEIDEL, DIRICHLET,
                        tuple([0.2] * 5), T, (seed, i))
        out.append(Request(i, t, p))
    return out
