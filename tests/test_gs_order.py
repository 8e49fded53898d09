"""Order of the 2D Gauss-Seidel items (band b, sweep t), CPU only: the
order of gs_order.hpp (built as a host-only program) is the mu = 2t + b
order of a brute-force enumeration, and the ticket drains: a replay with a
few waves, each taking the next item in that order and waiting exactly as
the kernel does before each interval, never stalls; the reversed order
does."""
import os
import random
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def listing():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out_dir = os.path.join(ROOT, "_build")
    os.makedirs(out_dir, exist_ok=True)
    exe = os.path.join(out_dir, "gs_order_check")
    src = os.path.join(ROOT, "tests", "gs_order_check.cpp")
    r = subprocess.run([hipcc, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", src,
                        "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    cases = {}
    cur = None
    for line in r.stdout.splitlines():
        if line.startswith("case "):
            nb, sweeps = map(int, line.split()[1:])
            cur = cases.setdefault((nb, sweeps), {})
        else:
            label, _, rest = line.partition(":")
            cur[label] = [tuple(map(int, p.split(","))) for p in rest.split()]
    return cases


def mu_order(nb, sweeps):
    items = [(b, t) for t in range(sweeps) for b in range(nb)]
    return sorted(items, key=lambda it: (2 * it[1] + it[0], it[1]))


def test_order_matches_brute_force(listing):
    assert len(listing) == 10
    for (nb, sweeps), lists in listing.items():
        assert lists["all"] == mu_order(nb, sweeps), (nb, sweeps)


def replay_tickets(order, nb, sweeps, waves_per_group, seed, rows=5, ncols=13, ks=4, sig=1):
    """Waves of group x take the items of order[x] in turn; an item runs
    ncols + 2 + sig*(rows-1) steps and, before each interval of ks steps,
    waits for (b, t-1), (b+1, t-1) and (b-1, t) with the kernel's thresholds.
    Returns the number of items finished before the replay stalled or ended."""
    rnd = random.Random(seed)
    S = ncols + 2 + sig * (rows - 1)
    L = rows - 1
    done = {}                      # item -> steps completed and published
    FIN = 1 << 30
    nxt = {x: 0 for x in order}    # ticket per group
    waves = [[x, None, 0] for x in order for _ in range(waves_per_group[x])]

    def prog(it):
        return done.get(it, 0)

    def ready(it, us):
        b, t = it
        need = []
        if t > 0:
            need.append(((b, t - 1), us + ks + sig + 1))
            if b + 1 < nb and us + ks + 1 - sig * L > 0:
                need.append(((b + 1, t - 1), us + ks + 1 - sig * L))
        if b > 0:
            need.append(((b - 1, t), us + ks - 1 + sig * rows))
        return all(prog(p) >= n for p, n in need)

    finished = 0
    while True:
        movable = []
        for w in waves:
            x, it, us = w
            if it is None:
                if nxt[x] < len(order[x]):
                    movable.append(w)
            elif ready(it, us):
                movable.append(w)
        if not movable:
            return finished
        w = rnd.choice(movable)
        x, it, us = w
        if it is None:
            w[1], w[2] = order[x][nxt[x]], 0
            nxt[x] += 1
            continue
        us = min(us + ks, S)
        w[2] = us
        done[it] = us if us < S else FIN
        if us >= S:
            finished += 1
            w[1] = None


@pytest.mark.parametrize("case", [(16, 7), (17, 2), (40, 9), (9, 3), (1, 5)])
@pytest.mark.parametrize("waves", [1, 2, 5])
@pytest.mark.parametrize("seed", range(3))
def test_ticket_order_drains(listing, case, waves, seed):
    nb, sweeps = case
    got = replay_tickets({0: listing[case]["all"]}, nb, sweeps, {0: waves}, seed)
    assert got == nb * sweeps


def test_reversed_order_stalls(listing):
    # the replay does catch an order in which an item waits for a later one
    order = {0: list(reversed(listing[(16, 7)]["all"]))}
    assert replay_tickets(order, 16, 7, {0: 1}, seed=0) < 16 * 7
