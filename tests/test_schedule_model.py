"""The time-skewed schedule, replayed on the CPU.

These tests check the scheduling ideas the kernels rely on, against the
counts and vector contents the paper prints (tests/golden), and replay the
GPU pipelines' step formulas to show that every (level, point) is computed
exactly once and only after everything it reads.
"""
import json
import os

import pytest

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "temporal_vectorization_counts.json")))


def skewed_vector(x, t, s, vl):
    """Lane i (0 = highest) of the vector that finishes a^{t+vl}_x: time t+vl-i at x+i*s."""
    return [(t + vl - i, x + i * s) for i in range(vl)]


def test_algorithm3_vector_contents():
    g = GOLDEN["algorithm3_vectors"]
    s, vl = g["s"], 4
    out = skewed_vector(0, 0, s, vl)
    assert [[tt, xx] for tt, xx in out] == [[a, b * s] for a, b in g["output_v3"]]
    # rotate: drop the finished top value, move the others up, blend in a
    # fresh time-0 value at x + vl*s
    rotated = out[1:] + [(0, vl * s)]
    assert [[tt, xx] for tt, xx in rotated] == [[a, b * s] for a, b in g["input_after_blend"]]


def fill_drain_points(s, vl):
    """Points of a vl-deep time tile that no full skewed vector covers.

    With lane i working i*s positions behind lane 0, the sweep starts with a
    triangle of i*s positions missing at level i and ends with the mirror
    triangle: sum over i of 2*i*s.
    """
    return sum(2 * i * s for i in range(vl))


def test_scalar_points_per_tile_match_paper():
    g = GOLDEN["scalar_points"]
    pts = fill_drain_points(g["s"], g["vl"])
    assert pts == g["points_per_tile"]
    for nx, pct in g["ratio_percent"].items():
        ratio = pts / (int(nx) * g["vl"])
        assert round(100 * ratio) == pct


def min_legal_stride(deps):
    """Smallest integer s with s > max dx/dt over dependences with dx > 0."""
    best = 0.0
    for dt, dx in deps:
        if dt > 0 and dx > 0:
            best = max(best, dx / dt)
    return int(best) + 1


def test_legality_rule():
    g = GOLDEN["legality"]
    assert min_legal_stride(g["deps_1d3p"]) == g["min_s"]


# ---------------------------------------------------------------------------
# replay of the GPU pipelines' step formulas
# ---------------------------------------------------------------------------

def replay_lds_pipeline(k, lin):
    """Lane group j (1..k) at step q consumes level j-1 row q-2j+1 and emits
    level j row q-2j; level 0 row q enters at step q."""
    produced = {}
    for q in range(lin + k + 1):
        if q < lin:
            produced[(0, q)] = q
        for j in range(1, k + 1):
            p = q - 2 * j + 1
            if p < 0 or p >= lin:
                continue
            # emitting row p-1 reads rows p-2, p-1, p of level j-1 (the running
            # sums carry p-2 and p-1 from earlier steps); when row p-1 lies in
            # level j's trapezoid [j, lin-j), those rows lie in level j-1's and
            # must have been produced by step q-1
            if j <= p - 1 < lin - j:
                for r in (p - 2, p - 1, p):
                    assert produced[(j - 1, r)] <= q - 1
            if p >= 1:
                key = (j, p - 1)
                assert key not in produced
                produced[key] = q
    return produced


@pytest.mark.parametrize("k,lin", [(1, 5), (3, 11), (8, 40), (16, 64)])
def test_lds_pipeline_schedule(k, lin):
    produced = replay_lds_pipeline(k, lin)
    # every valid row of the last level (the trapezoid's top) is produced
    for r in range(k, lin - k):
        assert (k, r) in produced


def replay_register_pipeline(k, lin):
    """Inside one lane: level j at step q emits row q-j from level j-1 row q-j+1."""
    produced = {}
    for q in range(lin):
        produced[(0, q)] = (q, 0)
        for j in range(1, k + 1):
            r = q - j
            if r < 0:
                continue
            for rr in (r - 1, r, r + 1):
                if 0 <= rr < lin:
                    assert produced[(j - 1, rr)] <= (q, j - 1)
            assert (j, r) not in produced
            produced[(j, r)] = (q, j)
    return produced


@pytest.mark.parametrize("k,lin", [(4, 20), (8, 37), (16, 70)])
def test_register_pipeline_schedule(k, lin):
    produced = replay_register_pipeline(k, lin)
    for r in range(k, lin - k):
        assert (k, r) in produced


def replay_gs_wavefront(rows, cols, sigma):
    """Gauss-Seidel band: lane i at step u updates column c = u - 1 - sigma*i.
    New neighbours (north row and west) must be updated earlier in this
    sweep; old ones (east, and the south row) later."""
    when = {}
    for u in range(cols + 2 + sigma * rows):
        for i in range(rows):
            c = u - 1 - sigma * i
            if 0 <= c < cols:
                when[(i, c)] = u
    for (i, c), u in when.items():
        north = [(i - 1, c + d) for d in ((-1, 0, 1) if sigma == 2 else (0,))]
        for n in north:
            if n in when:
                assert when[n] < u
        if (i, c - 1) in when:
            assert when[(i, c - 1)] < u
        south = [(i + 1, c + d) for d in ((-1, 0, 1) if sigma == 2 else (0,))]
        for s_ in south:
            if s_ in when:
                assert when[s_] > u
    return when


@pytest.mark.parametrize("sigma", [1, 2])
def test_gauss_seidel_wavefront_order(sigma):
    replay_gs_wavefront(64, 50, sigma)
