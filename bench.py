#!/usr/bin/env python3
"""Benchmark: GStencil/s of the time-skewed pipeline on one MI355X.

One "step" of this benchmark is one full solve of the headline workload --
2D 9-point box Jacobi on an 8192 x 8192 FP64 grid (zero border, all weights
1/9), T = 1000 time steps -- on a grid already resident in HBM, with the
schedule the autotuner picks.  The JSON line also carries:
  * the plain one-step-per-launch sweep on the same grid (the baseline the
    time-skewed forms must beat);
  * the roofline position of the dominant kernel (one band of k steps),
    timed live with HIP events;
  * a serving run: a Poisson stream of mixed 1D/2D/3D Jacobi and 2D
    Gauss-Seidel solves through the continuous-batching server, p50/p99
    latency and throughput, next to the same requests run one at a time;
  * the CPU oracle timed on a bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# Vector ALU rates, from 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane
# instructions per second.  FP64 (and unpacked FP32) counts a fused
# multiply-add as two operations: 78.6 TFLOP/s, MI355X's published FP64 vector
# peak and the FP32 rate without packed math, which the library is built
# without.  The bit-exact update issues every multiply and add on its own, so
# 39.3 T ops/s is the ceiling it can actually reach; the roofline reports the
# fraction of both.  Integer kernels have no fused form: 39.3 T ops/s.
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
FMA_PEAK_TFLOPS = 2 * ALU_PEAK_TOPS
PUBLISHED_VECTOR_TFLOPS = {"f64": 78.6, "f32": 157.3}


def alu_peak(achieved, dt_name):
    """The "alu" roofline's peak fields for a kernel of this dtype."""
    if dt_name == "i32":
        return {"peak": round(ALU_PEAK_TOPS, 2), "unit": "TOP/s (int32)",
                "frac": round(achieved / ALU_PEAK_TOPS, 4),
                "peak_note": "int32 vector issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz"}
    return {"peak": round(FMA_PEAK_TFLOPS, 2), "unit": "TFLOP/s",
            "frac": round(achieved / FMA_PEAK_TFLOPS, 4),
            "issue_ceiling": round(ALU_PEAK_TOPS, 2),
            "frac_of_issue_ceiling": round(achieved / ALU_PEAK_TOPS, 4),
            "peak_note": ("peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz = MI355X's "
                          "published FP64 vector rate; the unpacked FP32 rate (published "
                          f"{PUBLISHED_VECTOR_TFLOPS[dt_name]} counts packed FP32, which this "
                          "library is built without)" if dt_name == "f32" else
                          "peak: MI355X's published FP64 vector rate, 256 CUs x 4 SIMDs x 16 "
                          "lanes x 2 (FMA) x 2.4 GHz") +
                         "; issue_ceiling: the same lanes issuing the separate multiplies and "
                         "adds of the unfused, bit-exact update"}


# The paper's own measurements, for context (Section 4.1: two 12-core Xeon
# E5-2670 at 2.7 GHz, AVX2 256-bit vectors, ICC -O3 -xHost; Section 4.2).  It
# prints almost no absolute rates; its figures are relative.
PAPER_CONTEXT = ("paper (2x 12-core Xeon E5-2670, 2.7 GHz, AVX2): scalar Gauss-Seidel about "
                 "0.4 Gstencil/s for every GS stencil; temporal vectorization 3x scalar and "
                 "1.6x compiler auto-vectorization on Heat-1D at every core count; GS-2D 2.2x "
                 "scalar on 24 cores; LCS 5.3x scalar on 24 cores (Section 4.2)")
METRIC = "GStencil/s + % HBM roofline vs plain sweep; p50/p99 latency mixed load"
# workload -> (rocprof summary of its band kernel, that kernel's source and instantiation unit)
PROFILES = {
    "box2d9p": ("tstp_nd_box2d9p_8192_f64.md", ["tstp_nd.hpp", "tstp_nd_f64_2d.hip"]),
    "box2d9p_f32": ("tstp_nd_box2d9p_8192_f32.md", ["tstp_nd.hpp", "tstp_nd_f32_2d.hip"]),
    "star3d7p": ("tstp_nd_star3d7p_512_f64.md", ["tstp_nd.hpp", "tstp_nd_f64_3d.hip"]),
    "heat1d": ("tstp1d_heat1d_100000_f64.md", ["tstp1d.hpp", "tstp1d.hip"]),
    "star2d9p": ("tstp_ndr_star2d9p_8192_f64.md", ["tstp_ndr.hpp", "tstp_ndr_w_f64.hip"]),
    "life2d": ("tstp_nd_life2d_8000_i32.md", ["tstp_nd.hpp", "tstp_nd_life_2d.hip"]),
    "vc2d5p": ("tstp_ndr_vc2d5p_4096_f64.md", ["tstp_ndr.hpp", "tstp_ndr_vc2d_f64.hip"]),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash(workload: str = "box2d9p") -> str:
    h = hashlib.sha256()
    for f in PROFILES[workload][1]:
        with open(os.path.join(ROOT, "paper_2010_04868_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(workload: str, schedule: str):
    """HBM bytes per band launch from the committed rocprof summary, if it was
    taken on the current kernel sources and on this schedule (else None)."""
    if workload not in PROFILES:
        return None
    try:
        text = open(os.path.join(ROOT, "profiles", PROFILES[workload][0])).read()
    except OSError:
        return None
    m = re.search(r"kernel sources hash: `([0-9a-f]+)`", text)
    t = re.search(r"HBM traffic per band launch \(bytes\): `([0-9.eE+]+)`", text)
    s = re.search(r"profiled schedule: `([^`]+)`", text)
    if not m or not t or not s or m.group(1) != kernel_hash(workload) or s.group(1) != schedule:
        return None
    return float(t.group(1))


def _tile_ranges(n, valid, ext, k, periodic):
    """Tiles along one axis and the interior range [lo, hi) of tiles that
    touch no fixed border (the band kernel's own test)."""
    nt = -(-n // valid)
    if periodic:
        return nt, 0, nt
    inner = [t for t in range(nt) if t * valid - k > 0 and t * valid - k + ext - 1 < n - 1]
    return (nt, inner[0], inner[-1] + 1) if inner else (nt, 0, 0)


def band_work(p, info, inputs, uniform):
    """(computed point updates, executed arithmetic ops) of one band launch of
    the 2D/3D band kernel.  A workgroup computes every point of its tile
    (halo columns included) at every level; an interior tile runs whole
    groups of 4 steps, Lin + k + 1 rounded up (its lanes compute outside the
    trapezoid too, with no test), a border tile computes only the Lin stream
    rows of each level.  Per computed point: P - 1 sums, and P products --
    or, in interior tiles with equal weights, each value's product once:
    (C + 2) / C per point in 2D; in 3D (C + 2) / C per stencil row of the
    box and (C + 2 + 2C) / C in all for the star."""
    k, W, H, Lv, C = info["k"], info["tile_w"], info["tile_h"], info["tile_l"], info["lane_c"]
    per = p.boundary == inputs.PERIODIC
    D, P = p.ndim, p.order
    Lin = Lv + 2 * k
    Q = -(-(Lin + k + 1) // 4) * 4
    nz, nx = p.dims[0], p.dims[-1]
    ntx, x0, x1 = _tile_ranges(nx, W - 2 * k, W, k, per)
    nts, s0, s1 = _tile_ranges(nz, Lv, Lin, k, per)
    if D == 3:
        nty, y0, y1 = _tile_ranges(p.dims[1], H - 2 * k, H, k, per)
    else:
        nty, y0, y1 = 1, 0, 1
    n_int = (x1 - x0) * (y1 - y0) * (s1 - s0)
    n_all = ntx * nty * nts
    if not per and (x1 <= x0 or y1 <= y0 or s1 <= s0):
        n_int = 0
    pts = W * (H if D == 3 else 1)
    upd_int = n_int * k * pts * Q
    upd_bdr = (n_all - n_int) * k * pts * Lin
    full = (P - 1) + P
    if uniform and p.dtype != inputs.I32:
        if D == 2:
            prods = (C + 2) / C
        elif p.shape == inputs.BOX:
            prods = 3 * (C + 2) / C
        else:
            prods = (C + 2 + 2 * C) / C
        shared = (P - 1) + prods
    elif p.dtype == inputs.I32:
        full = shared = LIFE_EXEC_OPS
    else:
        shared = full
    return upd_int + upd_bdr, upd_int * shared + upd_bdr * full


# name -> (builder, description); builders take (n, T) overrides or None
WORKLOADS = {
    "box2d9p": (lambda inp, n, T: inp.box2d9p(**_kw(n, T)), "2D 9-point box Jacobi FP64"),
    "box2d9p_f32": (lambda inp, n, T: inp.box2d9p(inp.F32, **_kw(n, T)),
                    "2D 9-point box Jacobi FP32"),
    "star3d7p": (lambda inp, n, T: inp.star3d7p(**_kw(n, T)), "3D 7-point star Jacobi FP64"),
    "star3d7p_f32": (lambda inp, n, T: inp.star3d7p(inp.F32, **_kw(n, T)),
                     "3D 7-point star Jacobi FP32"),
    "heat1d": (lambda inp, n, T: inp.heat1d(**_kw(n, T)), "1D 3-point Jacobi FP64"),
    "gs2d5p": (lambda inp, n, T: inp.gs2d5p(**_kw(n, T)), "2D 5-point Gauss-Seidel FP64"),
    "gs1d3p": (lambda inp, n, T: inp.gs1d3p(**_kw(n, T)), "1D 3-point Gauss-Seidel FP64"),
    "life2d": (lambda inp, n, T: inp.life2d(**_kw(n, T)), "Game of Life B2S23, int32 cells"),
    "gs3d7p": (lambda inp, n, T: inp.gs3d7p(**_kw(n, T)), "3D 7-point Gauss-Seidel FP64"),
    "star1d5p": (lambda inp, n, T: inp.star1d5p(**_kw(n, T)), "1D 5-point (radius 2) Jacobi FP64"),
    "star2d9p": (lambda inp, n, T: inp.star2d9p(**_kw(n, T)),
                 "2D 9-point star (radius 2) Jacobi FP64"),
    "vc2d5p": (None, "2D 5-point Jacobi with variable coefficients FP64"),
    "lcs": (None, "longest common subsequence, 200000 x 200000"),
    "vc1d3p": (None, "1D 3-point Jacobi with variable coefficients FP64"),
}

# Integer operations of one LCS cell in the branch-free form of the
# recurrence: the letter comparison, the diagonal +1, the max of north and
# west, and the select between the two.
LCS_OPS = 4

# Integer operations of one Life update as the band kernel executes it: 8
# additions (the running sums of 9 values), the centre's subtraction, 3
# compares and a select.
LIFE_EXEC_OPS = 13


def _kw(n, T):
    kw = {}
    if n is not None:
        kw["n"] = n
    if T is not None:
        kw["T"] = T
    return kw


def describe(p, inputs) -> str:
    if p.dtype == inputs.I32:
        dims = "x".join(str(d) for d in p.dims)
        bnd = "periodic" if p.boundary == inputs.PERIODIC else "dead fixed border"
        return f"2D Game of Life B2S23 {dims} int32 cells, T={p.T}, {bnd}, cells live w.p. 1/2"
    kind = {(inputs.STAR, 3): "3-point", (inputs.STAR, 5): "5-point", (inputs.STAR, 7): "7-point",
            (inputs.BOX, 9): "9-point box"}.get((p.shape, p.order), f"{p.order}-point")
    if p.radius > 1:
        kind += f" {'box' if p.shape == inputs.BOX else 'star'} (radius {p.radius})"
    dep = "Gauss-Seidel (in place, lexicographic)" if p.dependence == inputs.GAUSS_SEIDEL else \
        "Jacobi"
    dims = "x".join(str(d) for d in p.dims)
    dt = "FP64" if p.dtype == inputs.F64 else "FP32"
    bnd = "periodic" if p.boundary == inputs.PERIODIC else \
        ("zero Dirichlet border" if p.zero_border else "fixed Dirichlet ends")
    w = sorted(set(p.coeffs))
    wt = "weights " + ("1/9" if w == [1.0 / 9.0] else "/".join(f"{x:g}" for x in p.coeffs))
    if p.radius > 1 and p.zero_border:
        bnd = f"zero Dirichlet border {p.radius} points deep"
    return f"{p.ndim}D {kind} {dep} {dims} {dt}, T={p.T}, {bnd}, {wt}"


def time_runs(torch, fn, reps):
    """Average device time (ms) of fn() over reps, with events on the current stream."""
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def kernel_name(p, info, inputs) -> str:
    if info["method"] == 0:
        return "plain step"
    if p.dependence == inputs.GAUSS_SEIDEL:
        return {1: "gs1d sweep pipeline", 2: "gs2d wavefront", 3: "gs3d_planes"}[p.ndim]
    if p.ndim == 1:
        return "tstp1d_r" if info.get("radius", 1) > 1 else "tstp1d"
    return "tstp_ndr" if info.get("radius", 1) > 1 else "tstp_nd"


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, budget_s=15.0):
    """The oracle as it stands, on a bounded number of steps of the same grid."""
    import oracle
    from paper_2010_04868_amd import inputs
    u0 = inputs.make_grid(p)
    if p.dtype == inputs.I32:
        def sweep(u, steps):
            return oracle.life(u, p.boundary, steps)
    else:
        def sweep(u, steps):
            return oracle.sweep(u, p.coeffs, p.shape, p.dependence, p.boundary, steps)
    t0 = time.perf_counter()
    u = sweep(u0, 1)
    one = time.perf_counter() - t0
    steps = max(1, min(p.T, int(budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    sweep(u, steps)
    dt = time.perf_counter() - t0
    return {"value": round(p.updated_points() * steps / dt / 1e9, 4), "unit": "GStencil/s",
            "cores": 1, "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{describe(p, inputs)}: {steps} of {p.T} steps, single thread, "
                      f"{dt:.1f} s"}


def serving_run(torch, tvs, inputs, n_req, rhos, seed=5, budget=4 << 30):
    """A Poisson stream through the server at offered loads rho of its
    capacity, next to the same requests run one at a time (tuned schedules,
    then the plain one-step-per-launch sweep).  The requests follow the
    serving mix's full distribution (2D sides 64..4096, 3D 32..256, 1D
    1e3..1e6, T 10..1000); n_req of them.  Every form starts from the host
    input and ends with the result on the host, as a served request does."""
    import numpy as np
    side2d, side3d, n1d, steps = (64, 4096), (32, 256), (1000, 1000000), (10, 1000)
    mix = inputs.serving_mix(n_req, seed=seed, side2d=side2d, side3d=side3d, n1d=n1d,
                             steps=steps)
    t_gen = time.perf_counter()
    grids = [inputs.make_grid(r.problem) for r in mix]
    log(f"serving: {len(mix)} request grids generated ({sum(g.nbytes for g in grids) / 2**30:.2f} "
        f"GiB, {time.perf_counter() - t_gen:.1f} s)")
    outs = [np.empty_like(g) for g in grids]
    total_updates = sum(r.problem.updated_points() * r.problem.T for r in mix)

    def serve(arrivals):
        srv = tvs.Server(hbm_budget=budget, max_slots=64, chunk_steps=0)
        try:
            t_base = time.perf_counter()
            ids = []
            for r, g, a in zip(mix, grids, arrivals):
                delay = a - (time.perf_counter() - t_base)
                if delay > 0:
                    time.sleep(delay)
                ids.append(srv.submit(r.problem, g))
            stamps = [srv.wait(i, o) for i, o in zip(ids, outs)]
            st = srv.stats()
        finally:
            srv.close()
        return stamps, st

    def one_at_a_time(tuning):
        t0 = time.perf_counter()
        for r, g in zip(mix, grids):
            d = torch.from_numpy(g).to("cuda")
            tvs.Plan.for_problem(r.problem, tuning).run(d, r.problem.coeffs, r.problem.T)
            d.cpu()
        return time.perf_counter() - t0

    serve([0.0] * min(8, len(mix)))  # warm-up: kernels loaded, arena touched
    # capacity: everything submitted at once
    t0 = time.perf_counter()
    stamps, st_cap = serve([0.0] * len(mix))
    makespan = max(s[3] for s in stamps) - min(s[0] for s in stamps)
    capacity_rps = len(mix) / makespan
    capacity = total_updates / makespan / 1e9
    log(f"serving: capacity {capacity:.1f} GStencil/s, {capacity_rps:.1f} requests/s "
        f"({time.perf_counter() - t0:.1f} s)")
    loads = []
    for rho in rhos:
        # Poisson arrivals at rho * capacity
        t0 = time.perf_counter()
        rng = np.random.default_rng((seed, int(rho * 1000)))
        gaps = rng.exponential(1.0 / (rho * capacity_rps), size=len(mix))
        arrivals = np.cumsum(gaps) - gaps[0]
        stamps, st = serve(list(arrivals))
        lat = np.array([s[3] - s[0] for s in stamps])
        span = max(s[3] for s in stamps) - min(s[0] for s in stamps)
        loads.append({"offered_load": rho,
                      "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                      "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
                      "throughput_GStencil_s": round(total_updates / span / 1e9, 2),
                      "chunks": int(st["chunks"])})
        log(f"serving: load {rho}: {loads[-1]} ({time.perf_counter() - t0:.1f} s)")
    alone_s = one_at_a_time(None)
    plain_s = one_at_a_time("method=plain")
    return {
        "requests": len(mix),
        "loads": loads,
        "capacity_GStencil_s": round(capacity, 2),
        "sequential_alone_GStencil_s": round(total_updates / alone_s / 1e9, 2),
        "sequential_plain_GStencil_s": round(total_updates / plain_s / 1e9, 2),
        "capacity_vs_plain": round(capacity / (total_updates / plain_s / 1e9), 3),
        "capacity_vs_alone": round(capacity / (total_updates / alone_s / 1e9), 3),
        "device_busy_frac": round(st_cap["busy_seconds"] / makespan, 3),
        "hbm_budget_GiB": budget / 2**30,
        "mix": f"Poisson stream, seed {seed}, the first {len(mix)} requests of the serving "
               f"mix: 1D 3-point / 2D 5- or 9-point / 3D 7-point Jacobi and 2D 5-point "
               f"Gauss-Seidel; 2D sides log-uniform {side2d[0]}..{side2d[1]}, 3D "
               f"{side3d[0]}..{side3d[1]}, 1D {n1d[0]:g}..{n1d[1]:g}, T uniform "
               f"{steps[0]}..{steps[1]}, FP32/FP64 50/50; host input and output included "
               f"in every form",
    }


def batch_measure(torch, tvs, inputs, n_grids=48, seed=7, reps=3):
    """Many uneven device-resident grids in one stencil_batch_run call, next to
    the same grids run one at a time (tuned schedules, then the plain
    one-step-per-launch sweep).  Inputs stay in HBM; no host transfer is timed."""
    side2d, side3d, n1d, steps = (64, 2048), (32, 160), (1000, 1000000), (10, 200)
    mix = inputs.serving_mix(n_grids, seed=seed, side2d=side2d, side3d=side3d, n1d=n1d,
                             steps=steps)
    probs = [r.problem for r in mix]
    dev = [torch.from_numpy(inputs.make_grid(p)).to("cuda") for p in probs]
    total = sum(p.updated_points() * p.T for p in probs)
    plans = [tvs.Plan.for_problem(p) for p in probs]
    plain = [tvs.Plan.for_problem(p, "method=plain") for p in probs]
    coeffs = [p.coeffs for p in probs]
    Ts = [p.T for p in probs]

    def timed(fn):
        fn()  # warm-up (a repeated batch layout is captured and then replayed)
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    t_batch = timed(lambda: tvs.batch_run(plans, dev, coeffs, Ts))
    # the same batch as one persistent launch per kernel variant
    os.environ["TVS_BATCH_PERSISTENT"] = "1"
    try:
        t_pers = timed(lambda: tvs.batch_run(plans, dev, coeffs, Ts))
    finally:
        del os.environ["TVS_BATCH_PERSISTENT"]
    t_alone = timed(lambda: [pl.run(g, c, T) for pl, g, c, T in zip(plans, dev, coeffs, Ts)])
    t_plain = timed(lambda: [pl.run(g, c, T) for pl, g, c, T in zip(plain, dev, coeffs, Ts)])
    for pl in plans + plain:
        pl.close()
    n_gs = sum(1 for p in probs if p.dependence == inputs.GAUSS_SEIDEL)
    return {
        "grids": len(probs), "gauss_seidel_grids": n_gs,
        "batch_GStencil_s": round(total / t_batch / 1e9, 2),
        "persistent_launch_GStencil_s": round(total / t_pers / 1e9, 2),
        "sequential_alone_GStencil_s": round(total / t_alone / 1e9, 2),
        "sequential_plain_GStencil_s": round(total / t_plain / 1e9, 2),
        "batch_vs_plain": round(t_plain / t_batch, 3),
        "batch_vs_alone": round(t_alone / t_batch, 3),
        "mix": f"seed {seed}, the serving mix's kinds and sizes (2D sides {side2d[0]}..{side2d[1]}, "
               f"3D {side3d[0]}..{side3d[1]}, 1D {n1d[0]:g}..{n1d[1]:g}, T {steps[0]}..{steps[1]}); "
               f"grids resident in HBM, each plan's default schedule, band-round launches "
               f"(and one persistent launch per kernel variant), best of {reps}",
    }


def lcs_bench(torch, tvs, inputs, args, copy_gbs):
    """LCS of two random 4-letter sequences, Table 1's size unless --n is given
    (then n x n).  A step is one whole table from zero boundaries."""
    p = inputs.lcs200k() if args.n is None else inputs.lcs200k(args.n, args.n)
    a, b = inputs.lcs_sequences(p.m, p.n, p.seed, p.alphabet)
    da, db = torch.from_numpy(a).to("cuda"), torch.from_numpy(b).to("cuda")
    row = torch.zeros(p.n + 1, dtype=torch.int32, device="cuda")
    col = torch.zeros(p.m + 1, dtype=torch.int32, device="cuda")
    plan = tvs.LcsPlan(p.m, p.n, args.tuning)
    tw, tr = plan.tile_width, plan.tile_rows

    def solve():
        row.zero_()
        col.zero_()
        plan.run(da, db, row, col)

    for _ in range(1 + args.warmup):
        solve()
    torch.cuda.synchronize()
    ms = time_runs(torch, solve, args.steps)
    cells = p.m * p.n
    value = cells / (ms / 1e3) / 1e9
    launches = (p.m + tr - 1) // tr + (p.n + tw - 1) // tw - 1
    kernel_ms = ms / launches                  # average tile launch (init and zeroing included)
    ops = cells * LCS_OPS / launches
    achieved = ops / (kernel_ms / 1e3) / 1e12
    log(f"lcs: w={tw} r={tr} {ms:.2f} ms/solve, {value:.1f} GCells/s, {launches} launches, "
        f"{kernel_ms * 1e3:.2f} us per launch, LCS length {int(row[-1].item())}")
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GCells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": f"synthetic: two uniform 4-letter sequences, PCG64(seed {p.seed})",
        "config": {"workload": f"longest common subsequence {p.m} x {p.n}, 4-letter alphabet, "
                               "zero boundaries", "schedule": f"w={tw},r={tr}", "cells": cells,
                   "lcs_length": int(row[-1].item())},
        "copy_GBs": round(copy_gbs, 1),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     **alu_peak(achieved, "i32"), "traffic": None,
                     "kernel": f"lcs_diag (one launch per anti-diagonal of {tr} x {tw} tiles)",
                     "kernel_ms": round(kernel_ms, 5),
                     "algorithmic_bytes": p.m + p.n + 8 * (p.m + p.n)},
    }
    if not args.no_cpu:
        import oracle
        rows = 64
        t0 = time.perf_counter()
        oracle.lcs(a[:rows], b)
        one = time.perf_counter() - t0
        rows = max(64, min(p.m, int(64 * 15.0 / max(one, 1e-6))))
        t0 = time.perf_counter()
        oracle.lcs(a[:rows], b)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(rows * p.n / dt / 1e9, 4), "unit": "GCells/s",
                               "cores": 1, "kind": "oracle", "cpu": cpu_model(),
                               "sample": f"the first {rows} rows of the table ({rows} x {p.n}), "
                                         f"single thread, {dt:.1f} s"}
    return out


def varcoef_bench(torch, tvs, inputs, args, copy_gbs):
    """Variable-coefficient Jacobi (a weight per point and offset): 1D 1e5
    points x 1000 steps (the time-skewed pipeline with the weights staged in
    LDS) or 2D 4096^2 x 1000 steps (the band kernel reading each weight per
    term), against plain steps reading them from memory."""
    import oracle
    p = (inputs.vc1d3p if args.workload == "vc1d3p" else inputs.vc2d5p)(**_kw(args.n, args.T))
    u0 = inputs.make_grid(p)
    W = inputs.varcoef_weights(p)
    grid = torch.from_numpy(u0).to("cuda")
    w = torch.from_numpy(W).to("cuda")
    plan = tvs.Plan.for_problem(p, args.tuning)
    info = plan.info()
    for _ in range(1 + args.warmup):
        plan.run_varcoef(grid, w, p.T)
    torch.cuda.synchronize()
    ms = time_runs(torch, lambda: plan.run_varcoef(grid, w, p.T), args.steps)
    nu = p.updated_points()
    value = nu * p.T / (ms / 1e3) / 1e9
    # the schedule variable-coefficient runs take (2D: the band kernel's own
    # tile and depth, with the weights staged in its LDS ring)
    vtune = info["varcoef_tuning"]
    k = int(dict(kv.split("=") for kv in vtune.split(","))["k"])
    band_ms = time_runs(torch, lambda: plan.run_varcoef(grid, w, 2 * k), 10) / 2
    ops = nu * k * (2 * p.order - 1)
    achieved = ops / (band_ms / 1e3) / 1e12
    # a band reads the grid and the P weights of a point once and writes the
    # point once: (2 + P) x 8 bytes per point per launch of k steps
    alg_bytes = (2 + p.order) * 8 * nu
    achieved_gbs = alg_bytes / (band_ms / 1e3) / 1e9
    # k (2P - 1) operations per (2 + P) x 8 bytes: below the FP64 ridge
    # (78.6 TFLOP/s over 8 TB/s) the band is bound by HBM
    hbm_bound = ops / alg_bytes < 78.64e12 / (HBM_PEAK_GBS * 1e9)
    plain = tvs.Plan.for_problem(p, "method=plain")
    plain.run_varcoef(grid, w, p.T)
    plain_ms = time_runs(torch, lambda: plain.run_varcoef(grid, w, p.T), args.plain_steps)
    plain_value = nu * p.T / (plain_ms / 1e3) / 1e9
    log(f"varcoef: {vtune} {ms:.3f} ms/solve, {value:.1f} GStencil/s; band {band_ms:.4f} ms; "
        f"plain {plain_value:.1f} GStencil/s")
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GStencil/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": (f"synthetic: uniform[0,1) grid, diffusivity uniform[0.1,0.4], PCG64(seed {p.seed})"
                 if p.ndim == 1 else f"synthetic: uniform[0,1) grid, diffusivity uniform"
                                     f"[0.05,0.2], PCG64(seed {p.seed})"),
        "config": {"workload": (f"1D 3-point Jacobi with variable coefficients {p.dims[0]} FP64, "
                                f"T={p.T}, fixed ends, weights (a, 1-2a, a) per point"
                                if p.ndim == 1 else
                                f"2D 5-point Jacobi with variable coefficients "
                                f"{p.dims[0]}x{p.dims[1]} FP64, T={p.T}, zero Dirichlet border, "
                                f"weights (a, a, 1-4a, a, a) per point"),
                   "schedule": vtune, "updated_points": nu},
        "copy_GBs": round(copy_gbs, 1),
        "plain_sweep": {"value": round(plain_value, 2), "unit": "GStencil/s",
                        "speedup": round(value / plain_value, 3)},
    }
    alu = {"achieved": round(achieved, 3), **alu_peak(achieved, "f64")}
    hbm = {"achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": alg_bytes}
    kernel = ("tstp1d_r with LDS-staged weights" if p.ndim == 1 else
              "tstp_ndr with the weights staged in its LDS ring") + " (one launch of k steps)"
    traffic = (profiled_traffic(args.workload, vtune)
               if args.n is None and args.T is None else None)
    if hbm_bound:
        out["roofline"] = {"bound": "hbm", **hbm, "traffic": traffic, "alu": alu,
                           "kernel": kernel, "kernel_ms": round(band_ms, 4)}
    else:
        out["roofline"] = {"bound": "alu", **alu, "traffic": traffic, "hbm": hbm,
                           "kernel": kernel, "kernel_ms": round(band_ms, 4)}
    if not args.no_cpu:
        t0 = time.perf_counter()
        oracle.sweep_varcoef(u0, W, p.shape, p.boundary, 50, p.order)
        one = (time.perf_counter() - t0) / 50
        steps = max(1, min(p.T, int(15.0 / max(one, 1e-9))))
        t0 = time.perf_counter()
        oracle.sweep_varcoef(u0, W, p.shape, p.boundary, steps, p.order)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(nu * steps / dt / 1e9, 4), "unit": "GStencil/s",
                               "cores": 1, "kind": "oracle", "cpu": cpu_model(),
                               "sample": f"{steps} of {p.T} steps of the same grid, single thread, "
                                         f"{dt:.1f} s"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tuning", default=None, help="fixed schedule instead of the autotuner")
    ap.add_argument("--plain-steps", type=int, default=2, help="timed solves of the plain sweep")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=300,
                    help="requests of the serving mix per load level (the full stream is 2000)")
    ap.add_argument("--serve-loads", default="0.5,0.8,1.0",
                    help="offered loads, as fractions of the measured capacity")
    ap.add_argument("--workload", default="box2d9p", choices=sorted(WORKLOADS),
                    help="problem to time (default: the headline 2D 9-point box FP64)")
    ap.add_argument("--n", type=int, default=None, help="grid side (default: the workload's)")
    ap.add_argument("--T", type=int, default=None, help="time steps (default: the workload's)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: --gpus N with N > 1 is not supported (the sweep runs "
              "on a single device; a larger grid would be split into slabs along axis 0, one "
              "per GPU, exchanging k-deep halos per band)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2010_04868_amd as tvs
    from paper_2010_04868_amd import inputs

    tvs.load()
    props = torch.cuda.get_device_properties(0)
    log(f"device: {props.name} CUs={props.multi_processor_count} "
        f"mem={props.total_memory / 2**30:.1f} GiB")
    # HBM calibration: a device-to-device copy of 1 GiB
    src = torch.empty(2**27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    copy_ms = time_runs(torch, lambda: dst.copy_(src), 10)
    copy_gbs = 2 * src.numel() * 8 / (copy_ms / 1e3) / 1e9
    log(f"copy 1 GiB: {copy_ms:.3f} ms = {copy_gbs:.0f} GB/s (read + write)")
    del src, dst

    if args.workload == "lcs":
        print(json.dumps(lcs_bench(torch, tvs, inputs, args, copy_gbs)), flush=True)
        return
    if args.workload in ("vc1d3p", "vc2d5p"):
        print(json.dumps(varcoef_bench(torch, tvs, inputs, args, copy_gbs)), flush=True)
        return
    p = WORKLOADS[args.workload][0](inputs, args.n, args.T)
    u0 = inputs.make_grid(p)
    grid = torch.from_numpy(u0).to("cuda")
    plan = tvs.Plan.for_problem(p, args.tuning)
    if args.tuning is None:
        t0 = time.perf_counter()
        chosen = plan.tune(grid, p.coeffs, 16)
        log(f"autotuner: {chosen} ({time.perf_counter() - t0:.1f} s)")
    info = plan.info()
    log("plan:", info)
    nu = p.updated_points()
    eb = 8 if p.dtype == inputs.F64 else 4
    life = p.dtype == inputs.I32

    # time-skewed solves; one setup run first (a repeated run is replayed from
    # a graph recorded on its second request, so that recording stays out of
    # the timed region whatever --warmup is)
    plan.run(grid, p.coeffs, p.T)
    for _ in range(args.warmup):
        plan.run(grid, p.coeffs, p.T)
    torch.cuda.synchronize()
    ms = time_runs(torch, lambda: plan.run(grid, p.coeffs, p.T), args.steps)
    value = nu * p.T / (ms / 1e3) / 1e9
    log(f"tstp: {ms:.3f} ms/solve, {value:.1f} GStencil/s")

    # dominant kernel: one band of k steps per launch (two per run, so that
    # the result lands in the caller's buffer with no copy)
    k = info["k"]
    if p.dependence == inputs.GAUSS_SEIDEL and p.ndim == 3:
        # one launch updates one plane of every sweep in flight: the average
        # launch of the timed solves (groups of k sweeps, planes + G (k - 1)
        # launches each)
        n0, n1, n2 = p.dims
        wts, G = ((4, 2, 1), 8) if p.shape == inputs.BOX else ((1, 1, 1), 2)
        planes = sum(w * (e - 3) for w, e in zip(wts, p.dims)) + 1
        launches, left = 0, p.T
        while left > 0:
            g = min(k, left)
            launches += planes + G * (g - 1)
            left -= g
        band_ms = ms / launches
        band_updates = nu * p.T / launches
    else:
        band_ms = time_runs(torch, lambda: plan.run(grid, p.coeffs, 2 * k), 10) / 2
        band_updates = nu * k
    # the arithmetic the band kernel executes: the 2D/3D band kernel counts
    # its redundant halo and pipeline-fill work and its shared products
    # (band_work); the other kernels count P products + (P - 1) sums per
    # update (Life: its integer operations)
    nd_band = (info["method"] == 1 and p.ndim >= 2 and p.dependence == inputs.JACOBI and
               info["radius"] == 1)
    if nd_band:
        uniform = len({np.float64(c).tobytes() for c in p.coeffs}) == 1
        computed, exec_ops = band_work(p, info, inputs, uniform)
        ops_note = (f"executed: {computed / band_updates:.3f} computed points per update "
                    f"(trapezoid halo and pipeline fill) x "
                    f"{exec_ops / computed:.3f} ops per computed point "
                    f"({'shared products, ' if uniform and not life else ''}no FMA)")
    else:
        exec_ops = band_updates * (LIFE_EXEC_OPS if life else 2 * p.order - 1)
        ops_note = ("executed: " + ("13 integer ops" if life else f"{2 * p.order - 1} ops "
                    f"({p.order} products + {p.order - 1} sums)") + " per update")
    achieved_tops = exec_ops / (band_ms / 1e3) / 1e12
    alg_bytes = 2 * eb * band_updates / k            # each point read and written once per band
    achieved_gbs = alg_bytes / (band_ms / 1e3) / 1e9
    log(f"band kernel: {band_ms:.4f} ms, {achieved_tops:.2f} T ops/s executed "
        f"({ops_note}), {achieved_gbs:.0f} GB/s algorithmic")

    # plain one-step-per-launch sweep on the same grid
    plain = tvs.Plan.for_problem(p, "method=plain")
    plain.run(grid, p.coeffs, p.T)
    plain_ms = time_runs(torch, lambda: plain.run(grid, p.coeffs, p.T), args.plain_steps)
    plain_value = nu * p.T / (plain_ms / 1e3) / 1e9
    step_ms = time_runs(torch, lambda: plain.run(grid, p.coeffs, 2), 25) / 2
    plain_gbs = 2 * eb * nu / (step_ms / 1e3) / 1e9
    log(f"plain: {plain_ms:.3f} ms/solve, {plain_value:.1f} GStencil/s, step {step_ms:.4f} ms "
        f"= {plain_gbs:.0f} GB/s")
    del grid
    torch.cuda.empty_cache()

    dt_name = "i32" if life else ("f64" if eb == 8 else "f32")
    traffic = (profiled_traffic(args.workload, plan.tuning())
               if args.n is None and args.T is None else None)
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GStencil/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt_name,
        "data": (f"synthetic: 0/1 board, cells live w.p. 1/2, PCG64(seed {p.seed})" if life
                 else f"synthetic: uniform[0,1) PCG64(seed {p.seed})"),
        "config": {"workload": describe(p, inputs),
                   "schedule": plan.tuning(),
                   "updated_points": nu},
        "hbm_effective_frac": round(value * 2 * eb / HBM_PEAK_GBS, 4),
        "copy_GBs": round(copy_gbs, 1),
        "plain_sweep": {"value": round(plain_value, 2), "unit": "GStencil/s",
                        "hbm_GBs": round(plain_gbs, 1),
                        "hbm_frac": round(plain_gbs / HBM_PEAK_GBS, 4),
                        "speedup": round(value / plain_value, 3)},
        "roofline": {"bound": "alu", "achieved": round(achieved_tops, 3),
                     **alu_peak(achieved_tops, dt_name),
                     "traffic": traffic,
                     "ops_counted": ops_note,
                     "hbm": {"achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                             "algorithmic_bytes": alg_bytes},
                     "kernel": f"{kernel_name(p, info, inputs)} (one launch of k steps)",
                     "kernel_ms": round(band_ms, 4)},
        "paper_context": PAPER_CONTEXT,
    }
    if not args.no_serve and args.workload == "box2d9p":
        t0 = time.perf_counter()
        out["serving"] = serving_run(torch, tvs, inputs, args.serve_requests,
                                     [float(x) for x in args.serve_loads.split(",")])
        log(f"serving: {out['serving']} ({time.perf_counter() - t0:.1f} s)")
        t0 = time.perf_counter()
        out["batch"] = batch_measure(torch, tvs, inputs)
        log(f"batch: {out['batch']} ({time.perf_counter() - t0:.1f} s)")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
