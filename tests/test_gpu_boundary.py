"""The C ABI's one-call form and abort reporting, and the equal-weight fast
path of the band kernels, against the oracle.

Interior tiles of the band kernels form each value's product once when all
weights have the same bit pattern; tiles that touch a fixed border multiply
every term by its own weight.  Both must give the canonical sum's bits, so
the grids here are large enough to hold interior tiles, and weights that
compare equal but differ in sign must not take the shared-product path.
"""
import threading

import numpy as np
import pytest

from helpers import assert_bitwise, gpu_sweep, oracle_sweep
from paper_2010_04868_amd.inputs import (BOX, DIRICHLET, F32, F64, GAUSS_SEIDEL, JACOBI,
                                         PERIODIC, STAR, np_dtype)

pytestmark = pytest.mark.gpu


def _grid(dims, dtype, seed):
    return np.random.default_rng(seed).random(dims).astype(np_dtype(dtype))


@pytest.mark.parametrize("dims,shape,order,dep", [
    ((5000,), STAR, 3, JACOBI), ((300, 410), BOX, 9, JACOBI), ((40, 50, 60), STAR, 7, JACOBI),
    ((200, 150), STAR, 5, GAUSS_SEIDEL)])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_run_simple_matches_oracle(dims, shape, order, dep, dtype):
    import torch

    import paper_2010_04868_amd as tvs
    c = [float(x) for x in np.random.default_rng(order).uniform(0.02, 0.2, order)]
    u0 = _grid(dims, dtype, 3)
    g = torch.from_numpy(u0).to("cuda")
    want = u0
    for T in (7, 1, 20):       # the cached plan serves every call
        tvs.run_simple(g, c, shape, order, dep, DIRICHLET, T)
        want = oracle_sweep(want, c, shape, order, dep, DIRICHLET, T)
    torch.cuda.synchronize()
    assert_bitwise(g.cpu().numpy(), want, f"run_simple {dims}")


@pytest.mark.parametrize("dep", [JACOBI, GAUSS_SEIDEL])
def test_run_simple_threads_and_streams(dep):
    """Four threads, each on its own stream, run the same problem through the
    one-call form at once: they share one cached plan (and its scratch), and
    every result must still be the oracle's."""
    import torch

    import paper_2010_04868_amd as tvs
    dims, order = (257, 300), 5
    c = [0.1, 0.15, 0.3, 0.25, 0.2]
    inputs = [_grid(dims, F64, 100 + i) for i in range(4)]
    T = 13
    outs, errors = [None] * 4, []

    def worker(i):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                g = torch.from_numpy(inputs[i]).to("cuda", non_blocking=False)
                s.synchronize()
                for _ in range(3):
                    tvs.run_simple(g, c, STAR, order, dep, DIRICHLET, T, stream=s)
                s.synchronize()
                outs[i] = g.cpu().numpy()
        except Exception as e:  # reported below
            errors.append(e)
    threads = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for i in range(4):
        ref = oracle_sweep(inputs[i], c, STAR, order, dep, DIRICHLET, 3 * T)
        assert_bitwise(outs[i], ref, f"thread {i}")


def test_plan_check_after_gauss_seidel_runs():
    import torch

    import paper_2010_04868_amd as tvs
    u0 = _grid((300, 333), F64, 5)
    c = [0.2] * 5
    plan = tvs.Plan(u0.shape, F64, STAR, 5, GAUSS_SEIDEL, DIRICHLET)
    g = torch.from_numpy(u0).to("cuda")
    for _ in range(3):
        plan.run(g, c, 9)
    plan.check()               # waits; no launch aborted
    assert_bitwise(g.cpu().numpy(), oracle_sweep(u0, c, STAR, 5, GAUSS_SEIDEL, DIRICHLET, 27),
                   "GS after check")


@pytest.mark.parametrize("ndim,shape,order", [(1, STAR, 3), (2, STAR, 5), (2, BOX, 9),
                                              (3, STAR, 7), (3, BOX, 27)])
@pytest.mark.parametrize("boundary", [DIRICHLET, PERIODIC])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_signed_zero_weights(ndim, shape, order, boundary, dtype):
    """Weights (-0.0, +0.0, ..., +0.0) compare equal but are not the same
    number: the canonical sum of positive values is (-0.0) + (+0.0) + ... =
    +0.0, where one shared product would give -0.0."""
    dims = {1: (3000,), 2: (700, 900), 3: (70, 80, 90)}[ndim]
    c = [-0.0] + [0.0] * (order - 1)
    u0 = _grid(dims, dtype, 9) + np.asarray(0.5, np_dtype(dtype))
    for T in (1, 3):
        ref = oracle_sweep(u0, c, shape, order, JACOBI, boundary, T)
        for tuning in (None, "method=plain"):
            got = gpu_sweep(u0, c, shape, order, JACOBI, boundary, T, tuning)
            assert_bitwise(got, ref, f"{dims} T={T} {tuning}")
    # the same weights in the other sign order, and exact equal weights
    c2 = [0.0] * (order - 1) + [-0.0]
    assert_bitwise(gpu_sweep(u0, c2, shape, order, JACOBI, boundary, 2),
                   oracle_sweep(u0, c2, shape, order, JACOBI, boundary, 2), "+0 ... -0")


@pytest.mark.parametrize("tuning", [None, "method=tstp,k=8,w=64,c=8,l=40",
                                    "method=tstp,k=8,w=128,c=8,l=100,lanemap=0",
                                    "method=tstp,k=6,w=128,c=4,l=64,lanemap=1"])
@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("boundary", [DIRICHLET, PERIODIC])
def test_uniform_weights_interior_tiles(tuning, dtype, boundary):
    """All weights 1/9 on a grid of many tiles: the interior tiles share
    products, the border tiles do not, and every seam between them must
    match the oracle."""
    u0 = _grid((1500, 1700), dtype, 21)
    if boundary == DIRICHLET:
        u0[0, :] = u0[-1, :] = u0[:, 0] = u0[:, -1] = 0
    c = [1.0 / 9] * 9
    T = 37
    ref = oracle_sweep(u0, c, BOX, 9, JACOBI, boundary, T)
    assert_bitwise(gpu_sweep(u0, c, BOX, 9, JACOBI, boundary, T, tuning), ref,
                   f"1/9 weights {tuning}")


@pytest.mark.parametrize("tuning", [None, "method=tstp,k=4,w=32,h=16,c=8,l=40",
                                    "method=tstp,k=3,w=64,h=16,c=8,l=64,lanemap=1"])
@pytest.mark.parametrize("boundary", [DIRICHLET, PERIODIC])
def test_uniform_weights_interior_tiles_3d(tuning, boundary):
    u0 = _grid((140, 150, 160), F64, 22)
    c = [1.0 / 7] * 7
    T = 9
    ref = oracle_sweep(u0, c, STAR, 7, JACOBI, boundary, T)
    assert_bitwise(gpu_sweep(u0, c, STAR, 7, JACOBI, boundary, T, tuning), ref,
                   f"1/7 weights {tuning}")
