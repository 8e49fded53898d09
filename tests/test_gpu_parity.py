"""GPU parity: the HIP library against the CPU oracle, element by element.

FP64 must be bit-identical to the oracle; FP32 must be bit-identical to the
oracle's FP32 mirror (same operation order in single precision).  Sizes are
small enough for the oracle, but span several tiles and ragged tails; every
method (plain one-step launches and the time-skewed pipeline with several
tile shapes, lane maps and depths) and step counts that leave a remainder
band are covered, as are the degenerate cases (T = 0, minimal extents,
tiles larger than the grid, periodic wrap across a whole tile).
"""
import numpy as np
import pytest

from helpers import assert_bitwise, gpu_sweep, oracle_sweep
from paper_2010_04868_amd.inputs import (BOX, DIRICHLET, F32, F64, GAUSS_SEIDEL, JACOBI,
                                         PERIODIC, STAR, np_dtype, npoints)

pytestmark = pytest.mark.gpu

SIZES = {
    1: [(3,), (4,), (97,), (1000,), (4099,)],
    2: [(3, 3), (5, 7), (37, 53), (70, 130), (131, 67)],
    3: [(3, 3, 3), (5, 6, 7), (17, 19, 23), (34, 20, 41)],
}
TUNINGS = {
    1: [None, "method=plain", "method=tstp,k=64,l=100,pl=64", "method=tstp,k=16,l=37,pl=16",
        "method=tstp,k=5,l=20,pl=16", "method=tstp,k=64,l=3,pl=64"],
    2: [None, "method=plain", "method=tstp,k=4,w=64,c=8,l=40,lanemap=0",
        "method=tstp,k=4,w=64,c=8,l=40,lanemap=1", "method=tstp,k=3,w=48,c=4,l=17,lanemap=0",
        "method=tstp,k=8,w=128,c=16,l=64,lanemap=1", "method=tstp,k=16,w=256,c=8,l=50"],
    3: [None, "method=plain", "method=tstp,k=2,w=16,h=8,c=4,l=10",
        "method=tstp,k=3,w=16,h=12,c=8,l=7,lanemap=0", "method=tstp,k=4,w=32,h=16,c=16,l=5",
        "method=tstp,k=2,w=64,h=32,c=8,l=9,lanemap=1"],
}
STEPS = [1, 2, 7, 19]


def _coeffs(P, seed):
    # distinct, asymmetric weights: any offset or orientation mix-up shows
    c = np.random.default_rng(seed).uniform(0.02, 0.2, size=P)
    return [float(x) for x in c]


@pytest.mark.parametrize("ndim,shape", [(1, STAR), (2, STAR), (2, BOX), (3, STAR), (3, BOX)])
@pytest.mark.parametrize("boundary", [DIRICHLET, PERIODIC])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_jacobi_matches_oracle(ndim, shape, boundary, dtype):
    P = npoints(ndim, shape)
    coeffs = _coeffs(P, seed=ndim * 10 + shape)
    failures = []
    for dims in SIZES[ndim]:
        u0 = np.random.default_rng(sum(dims)).random(dims).astype(np_dtype(dtype))
        for T in STEPS + ([130] if ndim == 1 else []):
            ref = oracle_sweep(u0, coeffs, shape, P, JACOBI, boundary, T)
            for tuning in TUNINGS[ndim]:
                got = gpu_sweep(u0, coeffs, shape, P, JACOBI, boundary, T, tuning)
                try:
                    assert_bitwise(got, ref, f"dims={dims} T={T} tuning={tuning}")
                except AssertionError as e:
                    failures.append(str(e))
    assert not failures, "\n".join(failures[:20])


@pytest.mark.parametrize("shape", [STAR, BOX])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_gauss_seidel_matches_oracle(shape, dtype):
    P = npoints(2, shape)
    coeffs = _coeffs(P, seed=40 + shape)
    failures = []
    for dims in [(3, 3), (5, 7), (66, 70), (67, 130), (131, 40), (200, 129)]:
        u0 = np.random.default_rng(sum(dims)).random(dims).astype(np_dtype(dtype))
        for T in (1, 2, 5, 9):
            ref = oracle_sweep(u0, coeffs, shape, P, GAUSS_SEIDEL, DIRICHLET, T)
            for tuning in ("method=plain", "method=tstp,k=1", "method=tstp,k=3,c=1",
                           "method=tstp,k=70", None):
                got = gpu_sweep(u0, coeffs, shape, P, GAUSS_SEIDEL, DIRICHLET, T, tuning)
                try:
                    assert_bitwise(got, ref, f"GS dims={dims} T={T} tuning={tuning}")
                except AssertionError as e:
                    failures.append(str(e))
    assert not failures, "\n".join(failures[:20])


@pytest.mark.parametrize("shape", [STAR, BOX])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_gauss_seidel_wide_rows(shape, dtype):
    # rows wide enough for interior intervals (no per-step tests) with each
    # sync interval: 600 columns take intervals of 64 steps, 2100 of 128
    P = npoints(2, shape)
    coeffs = _coeffs(P, seed=50 + shape)
    failures = []
    for dims in [(70, 600), (131, 2100)]:
        u0 = np.random.default_rng(sum(dims)).random(dims).astype(np_dtype(dtype))
        for T in (1, 3, 7):
            ref = oracle_sweep(u0, coeffs, shape, P, GAUSS_SEIDEL, DIRICHLET, T)
            for tuning in ("method=plain", "method=tstp,k=2", None):
                got = gpu_sweep(u0, coeffs, shape, P, GAUSS_SEIDEL, DIRICHLET, T, tuning)
                try:
                    assert_bitwise(got, ref, f"GS dims={dims} T={T} tuning={tuning}")
                except AssertionError as e:
                    failures.append(str(e))
    assert not failures, "\n".join(failures[:20])


@pytest.mark.parametrize("shape", [STAR, BOX])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_gauss_seidel_many_bands(shape, dtype):
    # 17 and 18 bands of 64 rows, the last of 1, 10 and 64 rows, rows narrow
    # and wide enough for 32-step intervals (inner intervals take a lane's
    # east value from its neighbour's south-east value of SIG steps before)
    P = npoints(2, shape)
    coeffs = _coeffs(P, seed=60 + shape)
    failures = []
    for dims in [(1027, 300), (1100, 700), (1090, 2100)]:
        u0 = np.random.default_rng(sum(dims)).random(dims).astype(np_dtype(dtype))
        for T in (1, 3, 8):
            ref = oracle_sweep(u0, coeffs, shape, P, GAUSS_SEIDEL, DIRICHLET, T)
            for tuning in ("method=tstp,k=2", "method=tstp,k=5", None):
                got = gpu_sweep(u0, coeffs, shape, P, GAUSS_SEIDEL, DIRICHLET, T, tuning)
                try:
                    assert_bitwise(got, ref, f"GS dims={dims} T={T} tuning={tuning}")
                except AssertionError as e:
                    failures.append(str(e))
    assert not failures, "\n".join(failures[:20])


@pytest.mark.parametrize("dtype", [F64, F32])
def test_gauss_seidel_1d_matches_oracle(dtype):
    # lanes are sweeps: 1, 3, 64 (one wave), 65 and 200 (chained waves) per launch
    coeffs = _coeffs(3, seed=60)
    failures = []
    for n in (3, 5, 70, 1000, 4099):
        u0 = np.random.default_rng(n).random(n).astype(np_dtype(dtype))
        for T in (1, 5, 65, 130):
            ref = oracle_sweep(u0, coeffs, STAR, 3, GAUSS_SEIDEL, DIRICHLET, T)
            for tuning in ("method=plain", "method=tstp,k=1", "method=tstp,k=3",
                           "method=tstp,k=64", "method=tstp,k=65", "method=tstp,k=200", None):
                got = gpu_sweep(u0, coeffs, STAR, 3, GAUSS_SEIDEL, DIRICHLET, T, tuning)
                try:
                    assert_bitwise(got, ref, f"GS-1D n={n} T={T} tuning={tuning}")
                except AssertionError as e:
                    failures.append(str(e))
    assert not failures, "\n".join(failures[:20])


def test_gauss_seidel_1d_sixteen_waves():
    """Up to 1024 sweeps per launch run as 16 one-wave workgroups chained
    through rings in device memory: long rows wrap every ring many times and
    make producers wait for their consumers; T = 2100 takes three launches."""
    coeffs = _coeffs(3, seed=61)
    n = 30011
    u0 = np.random.default_rng(n).random(n)
    for T in (1000, 1024, 2100):
        ref = oracle_sweep(u0, coeffs, STAR, 3, GAUSS_SEIDEL, DIRICHLET, T)
        got = gpu_sweep(u0, coeffs, STAR, 3, GAUSS_SEIDEL, DIRICHLET, T, "method=tstp,k=1024")
        assert_bitwise(got, ref, f"GS-1D n={n} T={T}")


@pytest.mark.parametrize("shape", [STAR, BOX])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_gauss_seidel_3d_matches_oracle(shape, dtype):
    # sweeps pipelined along the plane wavefront: 1, 3, 16 and the default
    # number of sweeps per group, against one sweep per group (plain)
    P = npoints(3, shape)
    coeffs = _coeffs(P, seed=70 + shape)
    failures = []
    for dims in [(3, 3, 3), (5, 6, 7), (17, 19, 23), (34, 20, 41), (20, 33, 9), (9, 4, 70)]:
        u0 = np.random.default_rng(sum(dims)).random(dims).astype(np_dtype(dtype))
        for T in (1, 2, 5, 9):
            ref = oracle_sweep(u0, coeffs, shape, P, GAUSS_SEIDEL, DIRICHLET, T)
            for tuning in ("method=plain", "method=tstp,k=1", "method=tstp,k=3",
                           "method=tstp,k=16", None):
                got = gpu_sweep(u0, coeffs, shape, P, GAUSS_SEIDEL, DIRICHLET, T, tuning)
                try:
                    assert_bitwise(got, ref, f"GS-3D dims={dims} T={T} tuning={tuning}")
                except AssertionError as e:
                    failures.append(str(e))
    assert not failures, "\n".join(failures[:20])


RADIUS_SIZES = {1: [(5,), (7,), (97,), (1000,), (4099,)],
                2: [(5, 5), (7, 9), (37, 53), (70, 130), (130, 301)],
                3: [(5, 5, 5), (7, 8, 9), (17, 19, 23), (30, 41, 50)]}
# 2D and 3D: the band kernel of radius r (skew 2r) at several depths, tile
# widths, points per lane and both lane maps, with ragged segments
RADIUS_TUNINGS = {1: [None, "method=plain", "method=tstp,k=1,l=16", "method=tstp,k=7,l=20",
                      "method=tstp,k=64,l=100", "method=tstp,k=20,l=37"],
                  2: [None, "method=plain", "method=tstp,k=1,w=32,c=4,l=16",
                      "method=tstp,k=3,w=64,c=4,l=20,lanemap=0",
                      "method=tstp,k=4,w=128,c=8,l=40", "method=tstp,k=2,w=64,c=8,l=9,lanemap=1"],
                  3: [None, "method=plain", "method=tstp,k=1,w=16,h=16,c=4,l=8",
                      "method=tstp,k=2,w=32,h=16,c=4,l=12,lanemap=0"]}


@pytest.mark.parametrize("ndim,shape,order", [(1, STAR, 5), (1, STAR, 7), (1, BOX, 5),
                                              (2, STAR, 9), (2, BOX, 25), (2, STAR, 13),
                                              (2, BOX, 49), (3, STAR, 13), (3, STAR, 19),
                                              (3, BOX, 125)])
@pytest.mark.parametrize("boundary", [DIRICHLET, PERIODIC])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_radius_matches_oracle(ndim, shape, order, boundary, dtype):
    # radius 2 and 3: the 1D pipeline with skew r + 1 (every depth, ragged
    # segments, remainder bands), the 2D/3D band kernel with skew 2r, and the
    # plain step in 1D, 2D and 3D (the only form of the boxes of more than 27
    # points: 2D radius 3, 3D radius 2)
    r = {(1, 5): 2, (1, 7): 3, (2, 9): 2, (2, 25): 2, (2, 13): 3, (2, 49): 3, (3, 13): 2,
         (3, 19): 3, (3, 125): 2}[(ndim, order)]
    coeffs = _coeffs(order, seed=80 + order)
    failures = []
    for dims in RADIUS_SIZES[ndim]:
        if min(dims) < 2 * r + 1:
            continue
        u0 = np.random.default_rng(sum(dims) + r).random(dims).astype(np_dtype(dtype))
        for T in STEPS + ([70] if ndim == 1 else []):
            ref = oracle_sweep(u0, coeffs, shape, order, JACOBI, boundary, T)
            for tuning in RADIUS_TUNINGS[ndim]:
                if (ndim == 3 and r == 3 or order > 27) and tuning and "tstp" in tuning:
                    continue  # 3D radius 3 and the large boxes run plain steps only
                got = gpu_sweep(u0, coeffs, shape, order, JACOBI, boundary, T, tuning)
                try:
                    assert_bitwise(got, ref, f"r={r} dims={dims} T={T} tuning={tuning}")
                except AssertionError as e:
                    failures.append(str(e))
    assert not failures, "\n".join(failures[:20])


def test_zero_steps_is_noop():
    u0 = np.random.default_rng(0).random((40, 50))
    got = gpu_sweep(u0, [1.0 / 9] * 9, BOX, 9, JACOBI, DIRICHLET, 0)
    assert_bitwise(got, u0, "T=0")


def test_operation_order_and_no_fma_on_gpu():
    # left-to-right sum: (1 + 1e16) - 1e16 = 0 at the centre point
    u = np.array([0.0, 1.0, 1e16, -1e16, 0.0])
    got = gpu_sweep(u, [1.0, 1.0, 1.0], STAR, 3, JACOBI, DIRICHLET, 1, "method=tstp,k=1,l=8,pl=16")
    assert got[2] == 0.0
    # no fused multiply-add: -1 + 3*(1/3) is exactly 0 with a rounded product
    u = np.array([0.0, -1.0, 1.0 / 3.0, 7.0])
    for tuning in ("method=plain", None):
        got = gpu_sweep(u, [1.0, 3.0, 0.0], STAR, 3, JACOBI, DIRICHLET, 1, tuning)
        assert got[2] == 0.0
    # the same in 2D and 3D kernels: weights put the pattern on one axis
    u2 = np.zeros((5, 6))
    u2[1, 2], u2[2, 2], u2[3, 2] = -1.0, 1.0 / 3.0, 7.0  # N, C, S of point (2, 2)
    c5 = [1.0, 0.0, 3.0, 0.0, 0.0]  # N, W, C, E, S
    for tuning in ("method=plain", "method=tstp,k=1,w=8,c=4,l=4", None):
        got = gpu_sweep(u2, c5, STAR, 5, JACOBI, DIRICHLET, 1, tuning)
        assert got[2, 2] == 0.0, tuning
    u3 = np.zeros((5, 5, 5))
    u3[1, 2, 2], u3[2, 2, 2] = -1.0, 1.0 / 3.0
    c7 = [1.0, 0.0, 0.0, 3.0, 0.0, 0.0, 0.0]
    for tuning in ("method=plain", "method=tstp,k=1,w=8,h=8,c=4,l=4", None):
        got = gpu_sweep(u3, c7, STAR, 7, JACOBI, DIRICHLET, 1, tuning)
        assert got[2, 2, 2] == 0.0, tuning


@pytest.mark.parametrize("dep", [JACOBI, GAUSS_SEIDEL])
def test_composition_bitwise(dep):
    u0 = np.random.default_rng(7).random((90, 77))
    c = _coeffs(5, 3)
    whole = gpu_sweep(u0, c, STAR, 5, dep, DIRICHLET, 23)
    part = gpu_sweep(gpu_sweep(u0, c, STAR, 5, dep, DIRICHLET, 10), c, STAR, 5, dep, DIRICHLET, 13)
    assert_bitwise(whole, part, "composition")
    ref = oracle_sweep(u0, c, STAR, 5, dep, DIRICHLET, 23)
    assert_bitwise(whole, ref, "vs oracle")


@pytest.mark.parametrize("dims,shape,order,tuning,T", [
    ((130, 301), BOX, 9, None, 70),                        # 9 launches: copy back
    ((5000,), STAR, 3, "method=tstp,k=16,l=64,pl=16", 200),  # 1D, 13 bands
    ((33, 40, 47), STAR, 7, None, 33),                     # 3D, 9 launches: copy back
    ((64, 70), STAR, 5, "method=plain", 12),               # plain steps, even count
])
@pytest.mark.parametrize("graph", ["0", "1"])
def test_repeated_runs_replay(dims, shape, order, tuning, T, graph, monkeypatch):
    """The same run requested again is replayed from a captured graph; every
    replay must equal the oracle at T * (replay count), with unrelated eager
    device work between the replays."""
    import torch

    import paper_2010_04868_amd as tvs
    monkeypatch.setenv("TVS_RUN_GRAPH", graph)
    u0 = np.random.default_rng(11).random(dims)
    c = _coeffs(order, 5)
    plan = tvs.Plan(dims, F64, shape, order, JACOBI, DIRICHLET, tuning)
    g = torch.from_numpy(u0).to("cuda")
    want = u0
    for rep in range(1, 5):
        plan.run(g, c, T)
        torch.cuda.synchronize()
        noise = torch.ones(4096, device="cuda", dtype=torch.float64).cumsum(0)
        torch.cuda.synchronize()
        want = oracle_sweep(want, c, shape, order, JACOBI, DIRICHLET, T)
        assert_bitwise(g.cpu().numpy(), want, f"{dims} replay {rep} graph={graph}")
        del noise
