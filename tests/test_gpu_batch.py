"""Batched launches (band rounds, and one persistent launch): every grid of a
mixed batch must come out bit-identical to running it alone (and to the
oracle), including when the captured hipGraph of a repeated batch layout is
replayed.  Members keep their plans' schedules (explicit tunings below:
depths, tile widths, lane maps, 4 and 8 points per lane); a plan tuned to
plain steps, or to a 1D pipeline of 16 lanes, runs the batch's own
time-skewed schedule."""
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


# member index -> the tuning its plan is created with
TUNINGS = {
    0: "method=tstp,k=16,l=100,pl=16",
    2: "method=tstp,k=3,w=64,c=8,l=40,lanemap=0",
    4: "method=tstp,k=5,w=96,c=4,l=20,lanemap=1",
    5: "method=plain",
    6: "method=tstp,k=2,w=32,h=16,c=4,l=12,lanemap=0",
    10: "method=tstp,k=6,w=128,c=8,l=64,lanemap=1",
}


def _setup():
    import torch

    import paper_2010_04868_amd as tvs
    plans, grids, coeffs, Ts, inits = [], [], [], [], []
    for i, (dims, shape, dep, bnd, dt, T, kind) in enumerate(MEMBERS):
        P = npoints(len(dims), shape)
        u0 = np.random.default_rng(100 + i).random(dims).astype(np_dtype(dt))
        plans.append(tvs.Plan(dims, dt, shape, P, dep, bnd, TUNINGS.get(i)))
        grids.append(torch.from_numpy(u0).to("cuda"))
        coeffs.append(_coeffs(P, kind, 200 + i))
        Ts.append(T)
        inits.append(u0)
    return plans, grids, coeffs, Ts, inits


def _expected(i, u0, c, T):
    dims, shape, dep, bnd, dt, _, _ = MEMBERS[i]
    return oracle_sweep(u0, c, shape, npoints(len(dims), shape), dep, bnd, T)


@pytest.mark.parametrize("persistent", ["0", "1"])
@pytest.mark.parametrize("graph", ["0", "1"])
def test_batch_matches_alone_and_oracle(graph, persistent, monkeypatch):
    import torch

    import paper_2010_04868_amd as tvs
    monkeypatch.setenv("TVS_BATCH_GRAPH", graph)
    monkeypatch.setenv("TVS_BATCH_PERSISTENT", persistent)
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


@pytest.mark.parametrize("persistent", ["0", "1"])
def test_many_members_many_bands(persistent, monkeypatch):
    """Forty 2D and 3D grids with up to 40 bands each (in one persistent
    launch, bands of different grids interleave); each result must still be
    the oracle's."""
    import torch

    import paper_2010_04868_amd as tvs
    monkeypatch.setenv("TVS_BATCH_PERSISTENT", persistent)
    rng = np.random.default_rng(5)
    plans, grids, coeffs, Ts, inits, probs = [], [], [], [], [], []
    for i in range(40):
        if i % 4 == 3:
            dims = tuple(int(x) for x in rng.integers(10, 40, 3))
            shape, P = STAR, 7
        else:
            dims = tuple(int(x) for x in rng.integers(20, 300, 2))
            shape, P = (BOX, 9) if i % 2 else (STAR, 5)
        bnd = PERIODIC if i % 3 == 0 else DIRICHLET
        dt = F32 if i % 5 == 0 else F64
        k = int(rng.integers(1, 5))
        T = int(rng.integers(1, 41)) * k // 2 + 1
        u0 = rng.random(dims).astype(np_dtype(dt))
        tuning = (f"method=tstp,k={k},w=64,c=4,l=16" if len(dims) == 2 else
                  f"method=tstp,k={min(k, 3)},w=16,h=16,c=4,l=8")
        plans.append(tvs.Plan(dims, dt, shape, P, JACOBI, bnd, tuning))
        grids.append(torch.from_numpy(u0).to("cuda"))
        c = [float(x) for x in rng.uniform(0.02, 0.2, P)]
        coeffs.append(c)
        Ts.append(T)
        inits.append(u0)
        probs.append((dims, shape, P, bnd))
    tvs.batch_run(plans, grids, coeffs, Ts)
    torch.cuda.synchronize()
    for i, g in enumerate(grids):
        dims, shape, P, bnd = probs[i]
        want = oracle_sweep(inits[i], coeffs[i], shape, P, JACOBI, bnd, Ts[i])
        assert_bitwise(g.cpu().numpy(), want, f"member {i} {dims} T={Ts[i]}")


def test_batch_rejects_bad_arguments():
    import torch

    import paper_2010_04868_amd as tvs
    p = tvs.Plan((10, 10), F64, STAR, 5)
    g = torch.zeros((10, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(tvs.StencilError):
        tvs.batch_run([p], [g], [[0.2] * 5], [-1])
