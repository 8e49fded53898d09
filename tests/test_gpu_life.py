"""GPU parity for Game of Life B2S23: the HIP library against the CPU oracle,
cell by cell (integer work: bit-exact).

Boards span several tiles with ragged tails; every method (plain one-step
launches and the time-skewed pipeline with several tile shapes, lane maps
and depths) runs step counts that leave a remainder band, under both
boundaries.  Besides random 0/1 boards, boards with non-0/1 values (a live
cell is any non-zero value, the neighbour count is the sum of values) and
Dirichlet borders that hold live cells are covered.
"""
import numpy as np
import pytest

import oracle
from helpers import assert_bitwise
from paper_2010_04868_amd.inputs import DIRICHLET, PERIODIC, life_board

pytestmark = pytest.mark.gpu

SIZES = [(3, 3), (5, 7), (37, 53), (70, 130), (131, 67), (200, 301)]
TUNINGS = [None, "method=plain", "method=tstp,k=4,w=64,c=8,l=40,lanemap=0",
           "method=tstp,k=4,w=64,c=8,l=40,lanemap=1", "method=tstp,k=3,w=48,c=4,l=17,lanemap=0",
           "method=tstp,k=8,w=128,c=16,l=64,lanemap=1", "method=tstp,k=16,w=256,c=8,l=50"]
STEPS = [1, 2, 7, 19, 40]


def gpu_life(u0, boundary, T, tuning=None):
    import torch

    import paper_2010_04868_amd as tvs
    t = torch.from_numpy(np.ascontiguousarray(u0, dtype=np.int32)).to("cuda")
    tvs.LifePlan(u0.shape, boundary, tuning).run(t, None, T)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _check_all(boards, boundary, steps, tunings, tag):
    failures = []
    for u0 in boards:
        for T in steps:
            ref = oracle.life(u0, boundary, T)
            for tuning in tunings:
                got = gpu_life(u0, boundary, T, tuning)
                try:
                    assert_bitwise(got, ref, f"{tag} dims={u0.shape} T={T} tuning={tuning}")
                except AssertionError as e:
                    failures.append(str(e))
    assert not failures, "\n".join(failures[:20])


@pytest.mark.parametrize("boundary", [DIRICHLET, PERIODIC])
def test_life_matches_oracle(boundary):
    boards = [life_board(d, sum(d), 0.5) for d in SIZES]
    _check_all(boards, boundary, STEPS, TUNINGS, "Life")


@pytest.mark.parametrize("boundary", [DIRICHLET, PERIODIC])
def test_life_sparse_and_dense_boards(boundary):
    boards = [life_board((90, 77), 3, 0.1), life_board((90, 77), 4, 0.9),
              np.zeros((40, 50), np.int32), np.ones((40, 50), np.int32)]
    _check_all(boards, boundary, [1, 5, 23], TUNINGS[:3], "Life density")


def test_life_general_cell_values():
    # non-zero cells are live; the neighbour count is the sum of the values
    rng = np.random.default_rng(12)
    boards = [rng.integers(-3, 4, size=(61, 83)).astype(np.int32),
              rng.integers(0, 3, size=(40, 130)).astype(np.int32)]
    for boundary in (DIRICHLET, PERIODIC):
        _check_all(boards, boundary, [1, 3, 9], TUNINGS, "Life values")


def test_life_zero_steps_and_composition():
    u0 = life_board((150, 170), 9, 0.5)
    assert_bitwise(gpu_life(u0, DIRICHLET, 0), u0, "T=0")
    whole = gpu_life(u0, PERIODIC, 37)
    part = gpu_life(gpu_life(u0, PERIODIC, 20), PERIODIC, 17)
    assert_bitwise(whole, part, "composition")
    assert_bitwise(whole, oracle.life(u0, PERIODIC, 37), "vs oracle")


def test_life_repeated_runs_replay():
    """A repeated run is replayed from a captured graph; every replay must
    equal the oracle at T * (replay count), with eager work in between."""
    import torch

    import paper_2010_04868_amd as tvs
    u0 = life_board((130, 301), 10, 0.5)
    plan = tvs.LifePlan(u0.shape, DIRICHLET)
    g = torch.from_numpy(u0).to("cuda")
    want = u0
    for rep in range(1, 5):
        plan.run(g, None, 70)
        torch.cuda.synchronize()
        noise = torch.ones(4096, device="cuda", dtype=torch.float64).cumsum(0)
        torch.cuda.synchronize()
        want = oracle.life(want, DIRICHLET, 70)
        assert_bitwise(g.cpu().numpy(), want, f"Life replay {rep}")
        del noise


def test_life_tune_keeps_bits(tmp_path, monkeypatch):
    import torch

    import paper_2010_04868_amd as tvs
    monkeypatch.setenv("TVS_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    u0 = life_board((300, 520), 11, 0.5)
    plan = tvs.LifePlan(u0.shape, PERIODIC)
    g = torch.from_numpy(u0).to("cuda")
    best = plan.tune(g, None, 16)
    assert best.startswith("method=") and "kern=1" not in best
    torch.cuda.synchronize()
    assert_bitwise(g.cpu().numpy(), u0, "tune restores the board")
    plan.run(g, None, 33)
    torch.cuda.synchronize()
    assert_bitwise(g.cpu().numpy(), oracle.life(u0, PERIODIC, 33), f"tuned {best}")
