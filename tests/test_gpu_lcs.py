"""GPU parity for the longest-common-subsequence dynamic program (integer
work: bit-exact against the oracle).

Small cases span several tiles with ragged tails in both directions, empty
and one-letter sequences, binary, 4-letter and 256-letter alphabets, zero
and non-zero boundary arrays, and every tile width.  At the benchmark's size
(200000 x 200000) the oracle checks the first 1000 entries of the last row
and column (each a smaller LCS problem of its own), and the GPU result must
satisfy the table's properties: unit steps, transposition symmetry and the
chaining of rectangles through the wavefront arrays.
"""
import numpy as np
import pytest

import oracle
from helpers import assert_bitwise
from paper_2010_04868_amd.inputs import lcs200k, lcs_sequences

pytestmark = pytest.mark.gpu

TUNINGS = [None, "w=64,r=64", "w=1024,r=64", "w=64", "w=128,r=128", "w=256,r=512",
           "w=64,r=1024"]


def gpu_lcs(a, b, row=None, col=None, tuning=None, plan=None):
    import torch

    import paper_2010_04868_amd as tvs
    m, n = a.size, b.size
    da = torch.from_numpy(np.ascontiguousarray(a, np.uint8)).to("cuda")
    db = torch.from_numpy(np.ascontiguousarray(b, np.uint8)).to("cuda")
    r = torch.zeros(n + 1, dtype=torch.int32) if row is None else torch.from_numpy(
        np.array(row, np.int32))
    c = torch.zeros(m + 1, dtype=torch.int32) if col is None else torch.from_numpy(
        np.array(col, np.int32))
    r, c = r.to("cuda"), c.to("cuda")
    (plan or tvs.LcsPlan(m, n, tuning)).run(da, db, r, c)
    torch.cuda.synchronize()
    return r.cpu().numpy(), c.cpu().numpy()


def _check(a, b, row, col, tuning, tag):
    want_r, want_c = oracle.lcs(a, b, row, col)
    got_r, got_c = gpu_lcs(a, b, row, col, tuning)
    assert_bitwise(got_r, want_r, f"{tag} last row")
    assert_bitwise(got_c, want_c, f"{tag} last column")


@pytest.mark.parametrize("alphabet", [2, 4, 256])
def test_lcs_matches_oracle(alphabet):
    rng = np.random.default_rng(alphabet)
    failures = []
    for m, n in [(1, 1), (5, 3), (64, 64), (65, 130), (130, 64), (200, 300), (1, 500), (500, 1),
                 (1000, 1500), (3000, 2500)]:
        a = rng.integers(0, alphabet, m).astype(np.uint8)
        b = rng.integers(0, alphabet, n).astype(np.uint8)
        for boundary in ("zero", "random"):
            row = col = None
            if boundary == "random":
                row = rng.integers(0, 7, n + 1).astype(np.int32)
                col = rng.integers(0, 7, m + 1).astype(np.int32)
            for tuning in TUNINGS:
                try:
                    _check(a, b, row, col, tuning, f"m={m} n={n} A={alphabet} {boundary} {tuning}")
                except AssertionError as e:
                    failures.append(str(e))
    assert not failures, "\n".join(failures[:20])


def test_lcs_empty_sequences():
    s = np.arange(70, dtype=np.uint8)
    e = np.zeros(0, np.uint8)
    for a, b in ((e, s), (s, e), (e, e)):
        row = np.arange(b.size + 1, dtype=np.int32) + 3
        col = np.arange(a.size + 1, dtype=np.int32) * 2
        _check(a, b, row, col, None, f"empty m={a.size} n={b.size}")


def test_lcs_identical_and_disjoint():
    s = np.random.default_rng(4).integers(0, 4, 5000).astype(np.uint8)
    r, c = gpu_lcs(s, s)
    assert r[-1] == 5000 and np.array_equal(r, np.arange(5001)) and np.array_equal(c, r)
    r, _ = gpu_lcs(s, s + 4)
    assert not r.any()


def test_lcs_20000_exact():
    a, b = lcs_sequences(20000, 17000, seed=13)
    _check(a, b, None, None, None, "20000 x 17000")


def test_lcs_full_size_samples_and_properties():
    p = lcs200k()                             # 200000 x 200000, the benchmark's size
    a, b = lcs_sequences(p.m, p.n, p.seed, p.alphabet)
    r, c = gpu_lcs(a, b)
    # unit steps along the last row and the last column
    assert set(np.diff(r).tolist()) <= {0, 1} and set(np.diff(c).tolist()) <= {0, 1}
    assert r[0] == 0 and c[0] == 0 and r[-1] == c[-1]
    # the first 1000 entries of each are LCS problems the oracle can run
    want_r, _ = oracle.lcs(a, b[:1000])
    assert_bitwise(r[:1001], want_r, "last row, first 1000 columns")
    _, want_c = oracle.lcs(a[:1000], b)
    assert_bitwise(c[:1001], want_c, "last column, first 1000 rows")
    # transposition: swapping the sequences swaps the last row and column
    r_t, c_t = gpu_lcs(b, a)
    assert_bitwise(r_t, c, "transposed row")
    assert_bitwise(c_t, r, "transposed column")
    # two rectangles chained through the wavefront arrays equal the whole
    n1 = 123457
    r1, c1 = gpu_lcs(a, b[:n1])
    r2, c2 = gpu_lcs(a, b[n1:], np.zeros(p.n - n1 + 1, np.int32), c1, "w=512,r=256")
    assert_bitwise(np.concatenate([r1, r2[1:]]), r, "chained row")
    assert_bitwise(c2[1:], c[1:], "chained column")
