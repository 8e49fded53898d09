"""The C ABI without a GPU: the library loads, exports every function the
header declares, validates problems with the documented error codes, and
parses tunings.  The server's scheduling policy is checked with its
simulated executor (no device calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2010_04868_amd as tvs
from paper_2010_04868_amd import _lib, inputs
from paper_2010_04868_amd.inputs import (BOX, DIRICHLET, F32, F64, GAUSS_SEIDEL, JACOBI,
                                         PERIODIC, STAR)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tvstencil.h")

E = {v: k for k, v in _lib.ERRORS.items()}


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stencil_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == {n for n, _, _ in _lib.SIGNATURES}


def code_of(fn):
    with pytest.raises(tvs.StencilError) as ei:
        fn()
    return ei.value.code


@pytest.mark.parametrize("args,err", [
    (((8, 8), F64, STAR, 7, JACOBI, DIRICHLET), "TVS_E_ORDER"),
    (((8, 8), F64, BOX, 5, JACOBI, DIRICHLET), "TVS_E_ORDER"),
    (((8, 8, 8, 8), F64, STAR, 9, JACOBI, DIRICHLET), "TVS_E_SHAPE"),
    (((2, 8), F64, STAR, 5, JACOBI, DIRICHLET), "TVS_E_SHAPE"),
    (((8, 8), 7, STAR, 5, JACOBI, DIRICHLET), "TVS_E_INVALID"),
    (((8, 8), F64, 3, 5, JACOBI, DIRICHLET), "TVS_E_INVALID"),
    (((8, 8), F64, STAR, 5, 4, DIRICHLET), "TVS_E_INVALID"),
    (((8, 8), F64, STAR, 5, JACOBI, 5), "TVS_E_INVALID"),
    (((8, 8), F64, STAR, 5, GAUSS_SEIDEL, PERIODIC), "TVS_E_UNSUPPORTED"),
    (((9, 9, 9), F64, BOX, 343, JACOBI, DIRICHLET), "TVS_E_UNSUPPORTED"),  # 3D radius-3 box
    (((9, 9), F64, BOX, 49, GAUSS_SEIDEL, DIRICHLET), "TVS_E_UNSUPPORTED"),  # radius 3 GS
    (((20,), F64, STAR, 9, JACOBI, DIRICHLET), "TVS_E_UNSUPPORTED"),       # radius 4
    (((20,), F64, STAR, 5, GAUSS_SEIDEL, DIRICHLET), "TVS_E_UNSUPPORTED"),  # radius 2 GS
    (((70000, 3, 3), F64, STAR, 7, GAUSS_SEIDEL, DIRICHLET), "TVS_E_UNSUPPORTED"),
    (((8, 8, 8), F64, BOX, 27, GAUSS_SEIDEL, PERIODIC), "TVS_E_UNSUPPORTED"),
])
def test_plan_validation_codes(args, err):
    assert code_of(lambda: tvs.Plan(*args)) == E[err]
    msg = _lib.load().stencil_last_error().decode()
    assert msg


@pytest.mark.parametrize("tuning", ["k", "k=x", "method=fast", "bogus=1", "k=-1",
                                    "method=tstp,k=8,w=64,c=3",
                                    "method=tstp,k=8,s=3,w=256,c=4"])
def test_bad_tunings_rejected(tuning):
    assert code_of(lambda: tvs.Plan((64, 64), F64, BOX, 9, tuning=tuning)) == E["TVS_E_INVALID"]


def test_plan_info_reports_schedule():
    p = tvs.Plan((8192, 8192), F64, BOX, 9)
    inf = p.info()
    assert inf["dims"] == (8192, 8192) and inf["radius"] == 1 and inf["method"] == 1
    assert inf["k"] >= 1 and inf["s"] == 2 and inf["tile_w"] > 2 * inf["k"]
    q = tvs.Plan((100, 100), F32, STAR, 5, tuning="method=plain")
    assert q.info()["method"] == 0 and q.info()["k"] == 1
    r = tvs.Plan((64, 64), F64, STAR, 5, tuning="method=tstp,k=8,w=128,c=4")
    assert r.info()["k"] == 8 and r.info()["lane_c"] == 4 and r.info()["kern"] == 0
    # only the LDS level-plane kernel exists
    assert code_of(lambda: tvs.Plan((64, 64), F64, STAR, 5, tuning="method=tstp,kern=1,k=8,c=4")) \
        == E["TVS_E_INVALID"]


def test_varcoef_schedule():
    """Variable-coefficient runs take at most 4 points per lane; a 2D
    radius-1 plan without a tuning string takes the weight-ring geometry (8
    levels on 128-wide tiles), a tuning string keeps its tile and depth, and
    the reported schedule re-creates itself."""
    def vc(plan):
        return dict(kv.split("=") for kv in plan.info()["varcoef_tuning"].split(","))
    d = vc(tvs.Plan((4096, 4096), F64, STAR, 5))
    assert (d["method"], d["k"], d["w"], d["c"]) == ("tstp", "8", "128", "4")
    e = vc(tvs.Plan((4096, 4096), F64, STAR, 5, tuning="method=tstp,k=3,w=64,c=8"))
    assert (e["k"], e["w"], e["c"]) == ("3", "64", "4")
    assert vc(tvs.Plan((4096, 4096), F64, STAR, 5, tuning="method=plain"))["method"] == "plain"
    # narrow grids shrink the tile; 1D keeps the plan's pipeline
    n = vc(tvs.Plan((4096, 40), F64, BOX, 9))
    assert int(n["w"]) <= 64 and int(n["w"]) > 2 * int(n["k"])
    assert vc(tvs.Plan((100000,), F64, STAR, 3))["k"] == str(tvs.Plan((100000,), F64, STAR, 3).info()["k"])
    t = tvs.Plan((4096, 4096), F64, STAR, 5).info()["varcoef_tuning"]
    assert tvs.Plan((4096, 4096), F64, STAR, 5, tuning=t).info()["varcoef_tuning"] == t


@pytest.mark.parametrize("dims,shape,order,dep", [
    ((8192, 8192), BOX, 9, 0), ((512, 512, 512), STAR, 7, 0), ((100000,), STAR, 3, 0),
    ((4096, 4096), STAR, 5, 1), ((100, 100), STAR, 5, 0)])
def test_tuning_string_roundtrips(dims, shape, order, dep):
    """The schedule a plan reports re-creates exactly that schedule."""
    a = tvs.Plan(dims, F64, shape, order, dep)
    t = a.tuning()
    assert t.startswith("method=")
    b = tvs.Plan(dims, F64, shape, order, dep, tuning=t)
    ia, ib = a.info(), b.info()
    for f in ("method", "k", "s", "tile_w", "tile_h", "tile_l", "lane_c", "lanemap", "pl", "kern",
              "tuning"):
        assert ia[f] == ib[f], f


def test_huge_plane_runs_plain():
    """A 3D grid whose stream-axis plane is 2 GiB or more cannot use the band
    kernels (31-bit plane offsets); the default schedule is then the plain sweep,
    and an explicit band schedule is rejected."""
    p = tvs.Plan((3, 16384, 16384), F64, STAR, 7)
    assert p.info()["method"] == 0
    assert code_of(lambda: tvs.Plan((3, 16384, 16384), F64, STAR, 7,
                                    tuning="method=tstp,k=2,w=64,h=32,c=8")) == E["TVS_E_INVALID"]


def test_varcoef_argument_errors_without_device():
    lib = _lib.load()
    fake = ctypes.c_void_p(0x1000)
    p = tvs.Plan((16, 16), F64, STAR, 5)
    assert lib.stencil_run_varcoef(p.handle, fake, None, 3, None) == E["TVS_E_INVALID"]
    assert lib.stencil_run_varcoef(p.handle, fake, fake, -1, None) == E["TVS_E_INVALID"]
    assert lib.stencil_run_varcoef(p.handle, fake, fake, 0, None) == 0
    gs = tvs.Plan((16, 16), F64, STAR, 5, GAUSS_SEIDEL)
    assert lib.stencil_run_varcoef(gs.handle, fake, fake, 3, None) == E["TVS_E_UNSUPPORTED"]
    life = tvs.LifePlan((16, 16))
    assert lib.stencil_run_varcoef(life.handle, fake, fake, 3, None) == E["TVS_E_INVALID"]


def test_radius_plans_without_device():
    p = tvs.Plan((1000,), F64, STAR, 5)              # radius 2: the 1D pipeline, skew 3
    inf = p.info()
    assert inf["radius"] == 2 and inf["method"] == 1 and inf["s"] == 3 and inf["pl"] == 64
    # 2D and 3D radius 2: the band kernel with skew 2r
    b = tvs.Plan((500, 600), F64, BOX, 25).info()
    assert b["method"] == 1 and b["s"] == 4 and b["radius"] == 2
    assert tvs.Plan((50, 60, 70), F64, STAR, 13).info()["s"] == 4
    t = tvs.Plan((500, 600), F32, STAR, 13, tuning="method=tstp,k=3,w=64,c=4,l=20").info()
    assert (t["k"], t["s"], t["tile_w"], t["lane_c"], t["tile_l"]) == (3, 6, 64, 4, 20)
    r3 = tvs.Plan((9, 9, 9), F32, STAR, 19).info()                  # 3D radius 3: plain steps
    assert r3["radius"] == 3 and r3["method"] == 0
    # boxes of more than 27 points (2D radius 3, 3D radius 2): plain steps,
    # and no band schedule is accepted for them
    for dims, P, r in (((500, 600), 49, 3), ((50, 60, 70), 125, 2)):
        big = tvs.Plan(dims, F64, BOX, P).info()
        assert big["radius"] == r and big["method"] == 0 and big["order"] == P
    assert code_of(lambda: tvs.Plan((500, 600), F64, BOX, 49, tuning="method=tstp,k=2,w=64,c=4")) \
        == E["TVS_E_INVALID"]
    for bad in ("method=tstp,k=4,w=64,c=4,s=3",                      # the skew is 2r
                "method=tstp,k=8,w=32,c=4",                          # 2kr halo columns >= w
                "method=tstp,k=2,w=64,c=16"):                        # 4 or 8 points per lane
        assert code_of(lambda: tvs.Plan((50, 60), F64, STAR, 9, tuning=bad)) == E["TVS_E_INVALID"]
    assert code_of(lambda: tvs.Plan((9, 9, 9), F64, STAR, 19, tuning="method=tstp,k=1,w=16,h=16,c=4")) \
        == E["TVS_E_INVALID"]
    q = tvs.Plan((1000,), F64, STAR, 7, tuning="method=tstp,k=16,l=100")
    assert q.info()["k"] == 16 and q.info()["s"] == 4
    for bad in ("method=tstp,k=8,l=64,pl=16", "method=tstp,k=8,s=2", "method=tstp,k=8,l=4000"):
        assert code_of(lambda: tvs.Plan((1000,), F64, STAR, 5, tuning=bad)) == E["TVS_E_INVALID"]
    lib = _lib.load()
    P = (ctypes.c_void_p * 1)(p.handle.value)
    G = (ctypes.c_void_p * 1)(0x1000)
    c = (ctypes.c_double * 5)(*([0.2] * 5))
    C = (ctypes.POINTER(ctypes.c_double) * 1)(ctypes.cast(c, ctypes.POINTER(ctypes.c_double)))
    Tn = (ctypes.c_int64 * 1)(3)
    assert lib.stencil_batch_run(1, P, G, C, Tn, None) == E["TVS_E_UNSUPPORTED"]


def test_life_plans_without_device():
    lib = _lib.load()
    p = tvs.LifePlan((64, 80), DIRICHLET)
    inf = p.info()
    assert inf["rule"] == tvs.RULE_LIFE and inf["dtype"] == tvs.I32
    assert (inf["shape"], inf["order"], inf["dependence"]) == (BOX, 9, JACOBI)
    assert inf["kern"] == 0 and inf["method"] == 1
    assert tvs.Plan((64, 64), F64, BOX, 9).info()["rule"] == tvs.RULE_WEIGHTED
    q = tvs.LifePlan((64, 80), PERIODIC, "method=plain")
    assert q.info()["method"] == 0 and q.info()["boundary"] == PERIODIC
    r = tvs.LifePlan((64, 80), DIRICHLET, inf["tuning"])
    assert r.info()["tuning"] == inf["tuning"]
    # 2D only; kern=1 and weighted int32 grids do not exist
    assert code_of(lambda: tvs.LifePlan((8, 8, 8))) == E["TVS_E_SHAPE"]
    assert code_of(lambda: tvs.LifePlan((2, 8))) == E["TVS_E_SHAPE"]
    assert code_of(lambda: tvs.LifePlan((8, 8), 3)) == E["TVS_E_INVALID"]
    assert code_of(lambda: tvs.LifePlan((64, 64), DIRICHLET, "method=tstp,kern=1,k=8,c=4")) \
        == E["TVS_E_INVALID"]
    assert code_of(lambda: tvs.Plan((8, 8), tvs.I32, BOX, 9)) == E["TVS_E_INVALID"]
    fake = ctypes.c_void_p(0x1000)
    # Life: coeffs NULL is accepted (T = 0 enqueues nothing); weighted plans need them
    assert lib.stencil_run(p.handle, fake, None, 0, None) == 0
    w = tvs.Plan((16, 16), F64, STAR, 5)
    assert lib.stencil_run(w.handle, fake, None, 3, None) == E["TVS_E_INVALID"]
    P = (ctypes.c_void_p * 1)(p.handle.value)
    G = (ctypes.c_void_p * 1)(0x1000)
    C = (ctypes.POINTER(ctypes.c_double) * 1)()
    Tn = (ctypes.c_int64 * 1)(3)
    assert lib.stencil_batch_run(1, P, G, C, Tn, None) == E["TVS_E_UNSUPPORTED"]


def test_lcs_plans_without_device():
    lib = _lib.load()
    p = tvs.LcsPlan(200000, 1000)
    assert p.tile_width == 1024 and p.tile_rows == 256
    assert tvs.LcsPlan(10, 10, "w=1024").tile_width == 1024
    assert tvs.LcsPlan(0, 0).tile_width == 1024
    assert tvs.LcsPlan(10, 10, "w=512,r=1024").tile_rows == 1024
    assert tvs.LcsPlan(10, 10, "w=64").tile_rows == 256
    for bad in ("w=100", "w=32", "w=8192", "k=4", "w=", "r=32", "r=2048", "w=4096,r=1024"):
        assert code_of(lambda: tvs.LcsPlan(10, 10, bad)) == E["TVS_E_INVALID"]
    assert code_of(lambda: tvs.LcsPlan(-1, 10)) == E["TVS_E_SHAPE"]
    assert code_of(lambda: tvs.LcsPlan(10, 1 << 31)) == E["TVS_E_SHAPE"]
    # rows and columns are indexed in 32 bits: lengths up to 2^30, so the last
    # tile plus its pipeline lag stays below 2^31 for every tiling
    assert tvs.LcsPlan(1 << 30, 1 << 30, "w=4096,r=512").tile_width == 4096
    assert code_of(lambda: tvs.LcsPlan((1 << 30) + 1, 10, "r=1024")) == E["TVS_E_SHAPE"]
    assert code_of(lambda: tvs.LcsPlan(10, (1 << 30) + 1)) == E["TVS_E_SHAPE"]
    assert code_of(lambda: tvs.LcsPlan((1 << 31) - 256, 10)) == E["TVS_E_SHAPE"]
    fake = ctypes.c_void_p(0x1000)
    assert lib.stencil_lcs_run(p.handle if hasattr(p, "handle") else p._h, None, fake, fake,
                               fake, None) == E["TVS_E_INVALID"]
    assert lib.stencil_lcs_run(None, fake, fake, fake, fake, None) == E["TVS_E_INVALID"]
    assert lib.stencil_lcs_tile_width(None) == E["TVS_E_INVALID"]
    assert lib.stencil_lcs_destroy(None) == 0


def test_run_argument_errors_without_device():
    lib = _lib.load()
    p = tvs.Plan((16, 16), F64, STAR, 5)
    c = (ctypes.c_double * 5)(*([0.2] * 5))
    fake = ctypes.c_void_p(0x1000)
    assert lib.stencil_run(p.handle, fake, c, -1, None) == E["TVS_E_INVALID"]
    assert lib.stencil_run(p.handle, None, c, 3, None) == E["TVS_E_INVALID"]
    assert lib.stencil_run(None, fake, c, 3, None) == E["TVS_E_INVALID"]
    assert lib.stencil_run(p.handle, fake, c, 0, None) == 0   # T = 0 enqueues nothing
    assert lib.stencil_batch_run(0, None, None, None, None, None) == 0
    assert lib.stencil_batch_run(-1, None, None, None, None, None) == E["TVS_E_INVALID"]
    assert lib.stencil_plan_destroy(None) == 0
    # a plan that never ran has no abort to report
    assert lib.stencil_plan_check(p.handle) == 0
    assert lib.stencil_plan_check(None) == E["TVS_E_INVALID"]
    g = tvs.Plan((16, 16), F64, STAR, 5, GAUSS_SEIDEL)
    assert lib.stencil_plan_check(g.handle) == 0


def test_batch_rejects_repeated_plans_and_grids():
    """Members run at the same time: one plan (its scratch) or one grid given
    twice would be shared by two of them.  Rejected before any device work."""
    lib = _lib.load()
    a = tvs.Plan((16, 16), F64, STAR, 5)
    b = tvs.Plan((16, 16), F64, STAR, 5)
    gs = tvs.Plan((16, 16), F64, STAR, 5, GAUSS_SEIDEL)
    w = (ctypes.c_double * 5)(*([0.2] * 5))
    C = (ctypes.POINTER(ctypes.c_double) * 2)(w, w)

    def batch(p0, p1, g0, g1, t0=3, t1=3):
        P = (ctypes.c_void_p * 2)(p0.handle.value, p1.handle.value)
        G = (ctypes.c_void_p * 2)(g0, g1)
        Tn = (ctypes.c_int64 * 2)(t0, t1)
        return lib.stencil_batch_run(2, P, G, C, Tn, None)
    assert batch(a, a, 0x1000, 0x2000) == E["TVS_E_INVALID"]
    assert batch(gs, gs, 0x1000, 0x2000) == E["TVS_E_INVALID"]
    assert batch(a, b, 0x1000, 0x1000) == E["TVS_E_INVALID"]
    assert batch(a, gs, 0x3000, 0x3000) == E["TVS_E_INVALID"]
    assert "twice" in lib.stencil_last_error().decode()


def test_tuning_cache_roundtrip(tmp_path, monkeypatch):
    path = tmp_path / "tune.jsonl"
    key = "nd2:300x200:f64:box9:jacobi:dirichlet"
    path.write_text('{"key": "%s", "tuning": "method=tstp,k=6,w=256,h=1,l=40,c=4,lanemap=1,kern=0"}\n' % key)
    monkeypatch.setenv("TVS_TUNE_CACHE", str(path))
    inf = tvs.Plan((300, 200), F64, BOX, 9).info()
    assert (inf["k"], inf["tile_w"], inf["tile_l"], inf["lane_c"], inf["lanemap"]) == (6, 256, 40, 4, 1)
    # another problem keeps the model-based default
    assert tvs.Plan((301, 200), F64, BOX, 9).info()["k"] == 8


# ---------------------------------------------------------------------------
# server policy with the simulated executor
# ---------------------------------------------------------------------------

@pytest.fixture
def sim_server(monkeypatch):
    monkeypatch.setenv("TVS_SERVER_SIMULATE", "1")
    made = []

    def make(**kw):
        s = tvs.Server(**kw)
        made.append(s)
        return s
    yield make
    for s in made:
        s.close()


def test_server_completes_everything_fifo(sim_server):
    srv = sim_server(hbm_budget=8 << 20, max_slots=3, chunk_steps=8)
    reqs = inputs.serving_mix(40, seed=11, side2d=(16, 300), side3d=(8, 40), n1d=(50, 5000),
                              steps=(1, 60))
    ids = []
    for r in reqs:
        u = inputs.make_grid(r.problem)
        ids.append((srv.submit(r.problem, u), u))
    stamps = []
    for rid, u in ids:
        out = np.empty_like(u)
        ts = srv.wait(rid, out)
        assert np.array_equal(out, u)           # simulated executor returns the input
        arrival, admit, start, finish = ts
        assert arrival <= admit <= start <= finish
        stamps.append(ts)
    admits = [t[1] for t in stamps]
    assert admits == sorted(admits)              # admission in arrival order
    st = srv.stats()
    assert st["submitted"] == st["admitted"] == st["completed"] == 40
    assert st["resident"] == 0 and st["bytes_in_use"] == 0


def test_server_budget_and_rejection(sim_server):
    srv = sim_server(hbm_budget=1 << 20, max_slots=64, chunk_steps=4)
    big = inputs.box2d9p(n=400, T=10)           # 2 x 1.28 MB > 1 MiB
    with pytest.raises(tvs.StencilError) as ei:
        srv.submit(big, inputs.make_grid(big))
    assert ei.value.code == E["TVS_E_BUSY"]
    small = inputs.box2d9p(n=100, T=10)         # 2 x 80 KB each: 6 fit at once
    ids = [srv.submit(small, inputs.make_grid(small)) for _ in range(20)]
    for rid in ids:
        srv.wait(rid, np.empty((100, 100)))
    st = srv.stats()
    assert st["rejected"] == 1 and st["completed"] == 20


def test_server_poll_and_unknown_ids(sim_server):
    srv = sim_server()
    p = inputs.heat1d(n=1000, T=5)
    rid = srv.submit(p, inputs.make_grid(p))
    out = np.empty(1000)
    while srv.poll(rid, out) is None:
        pass
    with pytest.raises(tvs.StencilError) as ei:
        srv.poll(rid, out)
    assert ei.value.code == E["TVS_E_NOTFOUND"]
