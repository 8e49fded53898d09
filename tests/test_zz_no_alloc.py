"""The allocation-free LCS entry point against the allocating one.

stencil_lcs_run_noalloc keeps the per-tile-column corner array in a static
device array instead of plan memory.  Through the C ABI, two calls in a row
(the second on a smaller problem, so stale entries of the first are left in
the shared array) must give bit for bit the row and column that
stencil_lcs_run gives on the same inputs.
"""
import ctypes

import numpy as np
import pytest

from paper_2010_04868_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def _run(entry, m, n, tuning, a, b, row0, col0):
    import torch
    lib = _lib.load()
    plan = ctypes.c_void_p()
    assert lib.stencil_lcs_plan(ctypes.byref(plan), m, n, tuning) == 0
    da = torch.from_numpy(a).to("cuda")
    db = torch.from_numpy(b).to("cuda")
    row = torch.from_numpy(row0.copy()).to("cuda")
    col = torch.from_numpy(col0.copy()).to("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rc = getattr(lib, entry)(plan, ctypes.c_void_p(da.data_ptr()), ctypes.c_void_p(db.data_ptr()),
                             ctypes.c_void_p(row.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                             ctypes.c_void_p(stream))
    assert rc == 0, lib.stencil_last_error()
    torch.cuda.synchronize()
    out = row.cpu().numpy(), col.cpu().numpy()
    assert lib.stencil_lcs_destroy(plan) == 0
    return out


def _case(m, n, seed):
    rng = np.random.default_rng(seed)
    a, b = inputs.lcs_sequences(m, n, seed, 4)
    row0 = rng.integers(0, 50, n + 1).astype(np.int32)
    col0 = rng.integers(0, 50, m + 1).astype(np.int32)
    return a, b, row0, col0


@pytest.mark.parametrize("tuning", [None, b"w=128,r=64", b"w=512,r=512"])
def test_noalloc_matches_allocating_entry_point(tuning):
    # the first call fills many corner entries; the second, smaller call
    # reuses the same static array
    for m, n, seed in ((3000, 9000, 1), (700, 650, 2)):
        a, b, row0, col0 = _case(m, n, seed)
        want = _run("stencil_lcs_run", m, n, tuning, a, b, row0, col0)
        got = _run("stencil_lcs_run_noalloc", m, n, tuning, a, b, row0, col0)
        assert np.array_equal(got[0], want[0]), f"row differs, m={m} n={n} {tuning}"
        assert np.array_equal(got[1], want[1]), f"column differs, m={m} n={n} {tuning}"


def test_noalloc_rejects_too_many_tile_columns():
    lib = _lib.load()
    plan = ctypes.c_void_p()
    n = 65536 * 64 + 1                     # 65537 tile columns of 64
    assert lib.stencil_lcs_plan(ctypes.byref(plan), 10, n, b"w=64") == 0
    fake = ctypes.c_void_p(0x1000)
    assert lib.stencil_lcs_run_noalloc(plan, fake, fake, fake, fake, None) == -2  # TVS_E_SHAPE
    assert lib.stencil_lcs_destroy(plan) == 0
