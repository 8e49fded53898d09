"""Batched persistent launches: every grid of a mixed batch must come out
bit-identical to running it alone (and to the oracle), including when the
captured hipGraph of a repeated batch layout is replayed."""
import os

import numpy as np
import pytest

from helpers import assert_bitwise, gpu_sweep, oracle_sweep
from paper_2010_04868_amd.inputs import (BOX, DIRICHLET, F32, F64, GAUSS_SEIDEL, JACOBI,
                                         PERIODIC, STAR, np_dtype, npoints)

pytestmark = pytest.mark.gpu

MEMBERS = [
    # dims, shape, dependence, boundary, dtype, T, coeff kind
    ((1000,), STAR, JACOBI, DIRICHLET, F64, 70, "uni"),
    ((777,), STAR, JACOBI, PERIODIC, F32, 13, "rand"),
    ((130, 301), BOX, JACOBI, DIRICHLET, F64, 19, "uni"),
    ((64, 70), BOX, JACOBI, DIRICHLET, F64, 8, "uni"),      # one band
    ((97, 45), STAR, JACOBI, PERIODIC, F64, 23, "rand"),
    ((300, 77), STAR, JACOBI, DIRICHLET, F32, 9, "uni"),
    ((33, 40, 47), STAR, JACOBI, PERIODIC, F64, 7, "rand"),
    ((20, 21, 22), BOX, JACOBI, DIRICHLET, F32, 5, "uni"),
    ((66, 70), STAR, GAUSS_SEIDEL, DIRICHLET, F64, 6, "rand"),
    ((50, 60), BOX, JACOBI, DIRICHLET, F64, 0, "uni"),      # T = 0
    ((129, 130), BOX, JACOBI, DIRICHLET, F64, 17, "uni"),   # same variant as #2
    ((500,), STAR, GAUSS_SEIDEL, DIRICHLET, F64, 11, "rand"),  # 1D Gauss-Seidel
    ((131, 600), BOX, GAUSS_SEIDEL, DIRICHLET, F32, 5, "uni"),  # several on side streams
    ((17, 20, 23), BOX, GAUSS_SEIDEL, DIRICHLET, F64, 4, "rand"),  # 3D Gauss-Seidel
]


def _coeffs(P, kind, seed):
    if kind == "uni":
        return [1.0 / P] * P
    return [float(x) for x in np.random.default_rng(seed).uniform(0.02, 0.2, P)]


def _setup():
    import torch

    import paper_2010_04868_amd as tvs
    plans, grids, coeffs, Ts, inits = [], [], [], [], []
    for i, (dims, shape, dep, bnd, dt, T, kind) in enumerate(MEMBERS):
        P = npoints(len(dims), shape)
        u0 = np.random.default_rng(100 + i).random(dims).astype(np_dtype(dt))
        plans.append(tvs.Plan(dims, dt, shape, P, dep, bnd))
        grids.append(torch.from_numpy(u0).to("cuda"))
        coeffs.append(_coeffs(P, kind, 200 + i))
        Ts.append(T)
        inits.append(u0)
    return plans, grids, coeffs, Ts, inits


def _expected(i, u0, c, T):
    dims, shape, dep, bnd, dt, _, _ = MEMBERS[i]
    return oracle_sweep(u0, c, shape, npoints(len(dims), shape), dep, bnd, T)


@pytest.mark.parametrize("graph", ["0", "1"])
def test_batch_matches_alone_and_oracle(graph, monkeypatch):
    import torch

    import paper_2010_04868_amd as tvs
    monkeypatch.setenv("TVS_BATCH_GRAPH", graph)
    plans, grids, coeffs, Ts, inits = _setup()
    reps = 3 if graph == "1" else 1
    for rep in range(1, reps + 1):
        tvs.batch_run(plans, grids, coeffs, Ts)
        torch.cuda.synchronize()
        # some eager work between replays
        scratch = torch.ones(1000, device="cuda") * rep
        torch.cuda.synchronize()
        for i, g in enumerate(grids):
            got = g.cpu().numpy()
            want = _expected(i, inits[i], coeffs[i], Ts[i] * rep)
            assert_bitwise(got, want, f"member {i} {MEMBERS[i][:2]} replay {rep}")
            dims, shape, dep, bnd, dt, T, _ = MEMBERS[i]
            if rep == 1 and T > 0:
                alone = gpu_sweep(inits[i], coeffs[i], shape, npoints(len(dims), shape), dep,
                                  bnd, T)
                assert_bitwise(got, alone, f"member {i} alone")
        del scratch


def test_batch_rejects_bad_arguments():
    import torch

    import paper_2010_04868_amd as tvs
    p = tvs.Plan((10, 10), F64, STAR, 5)
    g = torch.zeros((10, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(tvs.StencilError):
        tvs.batch_run([p], [g], [[0.2] * 5], [-1])
