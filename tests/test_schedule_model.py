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


def replay_radius_pipeline(k, lin, r):
    """The 2D/3D band kernel of radius r (skew 2r): at step q, level j reads
    row p = q + r - 2rj of level j-1 from LDS slot (q - r) mod (r + 1) and
    emits row p - r into slot q mod (r + 1); level 0 row q enters slot
    q mod (r + 1) at step q.  Checks that every row a valid point reads is
    still in its slot when read (written at an earlier step, not yet
    overwritten), that a row emitted at step q is read no earlier than step
    q + 1, and that the running-sum ring slot (row mod 2r) a level uses for a
    row is the same at every level for a given step parity class."""
    slots = r + 1
    lds = {}          # (level, slot) -> (row, step written)
    produced = {}
    ring_slot = {}    # (q mod 2r, axis-0 offset) -> ring slot, must not depend on j
    for q in range(lin + r * k + 1):
        reads = []
        for j in range(1, k + 1):
            p = q + r - 2 * r * j
            if p < 0 or p >= lin:
                continue
            # the point p - dd receives its terms of axis-0 offset dd
            for dd in range(-r, r + 1):
                key = (q % (2 * r), dd)
                slot = (p - dd) % (2 * r)
                assert ring_slot.setdefault(key, slot) == slot
            reads.append((j, p))
        writes = []
        if q < lin:
            writes.append((0, q))
        for j in range(1, k + 1):
            p = q + r - 2 * r * j
            if 0 <= p < lin and p - r >= 0:
                writes.append((j, p - r))
        # reads of this step see the slots as left by earlier steps
        for j, p in reads:
            level_ok = j - 1 == 0 or (j - 1) * r <= p < lin - (j - 1) * r
            # row p feeds points p - r .. p + r of level j; it must be right
            # if any of them is a valid point of level j
            need = any(j * r <= z < lin - j * r for z in range(p - r, p + r + 1))
            if need:
                assert level_ok
                row, when = lds[(j - 1, (q - r) % slots)]
                assert row == p and when < q
        for lev, row in writes:
            lds[(lev, q % slots)] = (row, q)
            if lev > 0:
                assert (lev, row) not in produced
                produced[(lev, row)] = q
    return produced


@pytest.mark.parametrize("k,lin,r", [(1, 9, 2), (3, 30, 2), (4, 41, 2), (2, 25, 3), (3, 40, 3),
                                     (8, 40, 1)])
def test_radius_pipeline_schedule(k, lin, r):
    produced = replay_radius_pipeline(k, lin, r)
    # every valid row of the top level is emitted
    for row in range(k * r, lin - k * r):
        assert (k, row) in produced


def simulate_persistent_batch(tiles, workers, seed):
    """The persistent batch launch: items in round-major ticket order (band b
    of every grid before band b + 1 of any); a worker takes the next ticket,
    waits until its grid's completed-tile counter reaches the tiles of all
    earlier bands of that grid, runs the tile and bumps the counter.  Workers
    advance in a random order (any interleaving the hardware may produce).
    Returns the completion order; raises if no worker can advance (a
    deadlock) before every item is done."""
    import random
    rnd = random.Random(seed)
    items = []
    prefix = []
    for g, per_band in enumerate(tiles):
        acc = [0]
        for n in per_band:
            acc.append(acc[-1] + n)
        prefix.append(acc)
    nb = max(len(t) for t in tiles)
    for b in range(nb):
        for g, per_band in enumerate(tiles):
            if b < len(per_band):
                items += [(g, b, t) for t in range(per_band[b])]
    ticket = 0
    done = [0] * len(tiles)
    state = [None] * workers      # None: taking a ticket; else (item, phase)
    finished = []
    while len(finished) < len(items):
        movable = []
        for w in range(workers):
            st = state[w]
            if st is None:
                if ticket < len(items):
                    movable.append(w)
            else:
                (g, b, t), phase = st
                if phase == "wait" and done[g] >= prefix[g][b]:
                    movable.append(w)
                elif phase == "run":
                    movable.append(w)
        assert movable, f"deadlock after {len(finished)} of {len(items)} items"
        w = rnd.choice(movable)
        st = state[w]
        if st is None:
            state[w] = (items[ticket], "wait")
            ticket += 1
        elif st[1] == "wait":
            state[w] = (st[0], "run")
        else:
            g, b, t = st[0]
            # everything this tile reads or overwrites belongs to bands < b,
            # all complete
            assert done[g] >= prefix[g][b]
            done[g] += 1
            finished.append(st[0])
            state[w] = None
    return finished


@pytest.mark.parametrize("workers", [1, 2, 7, 64])
@pytest.mark.parametrize("seed", range(5))
def test_persistent_batch_drains(workers, seed):
    import random
    rnd = random.Random(100 + seed)
    tiles = [[rnd.randint(1, 9)] * rnd.randint(1, 6) for _ in range(rnd.randint(1, 12))]
    for per_band in tiles:      # a last band with fewer tiles, as a shallower band may have
        per_band[-1] = max(1, per_band[-1] - rnd.randint(0, 2))
    order = simulate_persistent_batch(tiles, workers, seed)
    assert len(order) == sum(sum(t) for t in tiles)
    # bands of one grid complete in order
    for g in range(len(tiles)):
        bands = [b for gg, b, _ in order if gg == g]
        assert bands == sorted(bands)


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


def simulate_gs_items(nb, rows, ncols, sweeps, ks, sig, seed, last_rows=None):
    """The 2D Gauss-Seidel item pipeline with its exact waits, at small size.

    Items (band b, sweep t), bands of `rows` rows (the last band may have
    fewer), run by independent workers in a random interleaving of single
    steps.  At step u lane i of item (b, t) updates row 1 + rows*b + i at
    column u - sig*i.  Before each interval of ks steps an item waits until
    (b, t-1) has completed us + ks + sig + 1 steps, (b+1, t-1) us + ks + 1 -
    sig*L steps (L its last lane) and (b-1, t) us + ks - 1 + sig*rows steps,
    the kernel's thresholds with `rows` for 64.  Every value carries the
    sweep that wrote it.  Checked: (1) when an interval starts, every value
    any of its steps reads already has the sweep it must have (loads may be
    issued anywhere in the interval); (2) no step overwrites a value some
    later step of another item still has to read in its old sweep."""
    import random
    rnd = random.Random(seed)
    nrow = 2 + rows * (nb - 1) + (last_rows if last_rows else rows)
    ver = {(x, y): 0 for x in range(nrow) for y in range(ncols + 2)}
    band_rows = [rows] * nb
    if last_rows:
        band_rows[-1] = last_rows
    box = sig == 2

    def reads(b, t, i, u):
        """(point, sweep it must hold) read from memory by lane i of (b, t) at
        step u.  The west value is the lane's own previous result and the
        north values of lanes i > 0 come from lane i - 1 of the same item (a
        lane shift): neither is read from memory."""
        x = 1 + rows * b + i
        y = u - sig * i
        if not 1 <= y <= ncols:
            return []
        out = [((x, y), t - 1), ((x, y + 1), t - 1)]
        cols = (y - 1, y, y + 1) if box else (y,)
        if i == 0:
            out += [((x - 1, c), t) for c in cols]
        out += [((x + 1, c), t - 1) for c in cols]
        return [((px, py), v) for (px, py), v in out
                if 1 <= px <= nrow - 2 and 1 <= py <= ncols]   # borders never change

    def steps_of(b):
        return ncols + 2 + sig * (band_rows[b] - 1)

    items = [(b, t) for t in range(1, sweeps + 1) for b in range(nb)]
    done = {it: 0 for it in items}
    FINISHED = 1 << 30
    pos = {it: 0 for it in items}          # next step
    pending = {}                           # (point, version) -> readers left
    for b, t in items:
        for u in range(steps_of(b)):
            for i in range(band_rows[b]):
                for pt, v in reads(b, t, i, u):
                    if v == t - 1:
                        pending[(pt, v)] = pending.get((pt, v), 0) + 1

    def ready(it):
        b, t = it
        us = pos[it]
        if us % ks:
            return True
        need = []
        if t > 1:
            need.append(((b, t - 1), us + ks + sig + 1))
            if b + 1 < nb and us + ks + 1 - sig * (band_rows[b] - 1) > 0:
                need.append(((b + 1, t - 1), us + ks + 1 - sig * (band_rows[b] - 1)))
        if b > 0:
            need.append(((b - 1, t), us + ks - 1 + sig * rows))
        return all(done[p] >= n for p, n in need)

    active = set(items)
    started = set()
    while active:
        cand = [it for it in active if ready(it)]
        assert cand, "deadlock"
        it = rnd.choice(cand)
        b, t = it
        u = pos[it]
        if u % ks == 0:
            # interval start: everything the interval reads is in place
            for uu in range(u, min(u + ks, steps_of(b))):
                for i in range(band_rows[b]):
                    for pt, v in reads(b, t, i, uu):
                        assert ver[pt] == v, (it, uu, i, pt, ver[pt], v)
        for i in range(band_rows[b]):
            for pt, v in reads(b, t, i, u):
                if v == t - 1:
                    pending[(pt, v)] -= 1
        for i in range(band_rows[b]):
            x, y = 1 + rows * b + i, u - sig * i
            if 1 <= y <= ncols:
                assert pending.get(((x, y), t - 1), 0) == 0, ("overwrite before read", it, u, i)
                ver[(x, y)] = t
        pos[it] = u + 1
        if pos[it] % ks == 0:
            done[it] = pos[it]
        if pos[it] >= steps_of(b):
            done[it] = FINISHED
            active.discard(it)
    assert all(v == sweeps for (x, y), v in ver.items() if 1 <= x <= nrow - 2 and 1 <= y <= ncols)


@pytest.mark.parametrize("sig", [1, 2])
@pytest.mark.parametrize("ks,last_rows", [(2, None), (4, 3), (8, 1), (4, None)])
@pytest.mark.parametrize("seed", range(3))
def test_gauss_seidel_item_waits(sig, ks, last_rows, seed):
    simulate_gs_items(nb=4, rows=5, ncols=13, sweeps=4, ks=ks, sig=sig, seed=seed,
                      last_rows=last_rows)


def simulate_gs1d_ring(waves, blocks, bs, ring_blocks, seed, slack=0):
    """Replay the block protocol of the multi-CU 1D Gauss-Seidel kernel with
    random interleavings of whole blocks.  Wave w > 0 reads, at block b, the
    inputs of steps bs*b - 2 .. bs*b + bs - 2 from its ring (slot q mod
    ring_blocks*bs), written by wave w-1 at the block of step q; it may start
    block b once wave w-1 has finished block b (count >= b + 1).  A wave that
    feeds another may start block b once that wave has finished block
    b - ring_blocks + 1 (count >= b - ring_blocks + 2; slack weakens that).  Checks that the
    launch never stalls and that every input read is the value of its own
    step (no slot overwritten before it was read)."""
    import random
    rng = random.Random(seed)
    rs = ring_blocks * bs
    slots = [[None] * rs for _ in range(waves)]  # ring of wave w: step whose value it holds
    done = [0] * waves                           # finished blocks per wave
    while min(done) < blocks:
        ready = []
        for w in range(waves):
            b = done[w]
            if b >= blocks:
                continue
            if w > 0 and done[w - 1] < b + 1:
                continue
            need = b - ring_blocks + 2 - slack
            if w + 1 < waves and need > 0 and done[w + 1] < need:
                continue
            ready.append(w)
        assert ready, f"stalled at {done}"
        w = rng.choice(ready)
        b = done[w]
        if w > 0:
            for q in range(bs * b - 2, bs * b + bs - 1):
                if q >= 0:
                    assert slots[w][q % rs] == q, (w, b, q, slots[w][q % rs])
        if w + 1 < waves:
            for q in range(bs * b, bs * b + bs):
                slots[w + 1][q % rs] = q
        done[w] += 1


@pytest.mark.parametrize("ring_blocks", [2, 3, 8])
@pytest.mark.parametrize("seed", range(4))
def test_gauss_seidel_1d_ring(ring_blocks, seed):
    simulate_gs1d_ring(waves=5, blocks=23, bs=4, ring_blocks=ring_blocks, seed=seed)


def test_gauss_seidel_1d_ring_needs_its_waits():
    # a producer allowed one block further ahead overwrites inputs not yet read
    with pytest.raises(AssertionError, match=r"^\("):
        for seed in range(50):
            simulate_gs1d_ring(waves=3, blocks=30, bs=4, ring_blocks=3, seed=seed, slack=1)
