"""GPU parity for variable-coefficient Jacobi stencils (a weight per offset
per point, fixed over time): bit-exact against the oracle's variable-
coefficient sweep (FP64, and FP32 against its FP32 mirror).  1D runs the
time-skewed pipeline at several depths and segment lengths; 2D and 3D run
the band kernel (radius 1 and 2; 3D radius 3 runs plain steps), in 2D both
with the weights read per term and staged in the LDS ring.  Weights are
distinct per point and offset, so an offset or point mix-up shows."""
import numpy as np
import pytest

import oracle
from helpers import assert_bitwise
from paper_2010_04868_amd.inputs import BOX, DIRICHLET, F32, F64, PERIODIC, STAR, np_dtype

pytestmark = pytest.mark.gpu

CASES = [((97,), STAR, 3), ((1000,), STAR, 3), ((4099,), STAR, 3), ((300,), STAR, 5),
         ((301,), STAR, 7), ((5,), STAR, 3), ((37, 53), STAR, 5), ((37, 53), BOX, 9),
         ((40, 41), STAR, 9), ((17, 19, 23), STAR, 7), ((9, 10, 11), BOX, 27),
         ((11, 12, 13), STAR, 13), ((70, 130), STAR, 5), ((66, 140), BOX, 9),
         ((80, 150), STAR, 9), ((70, 140), BOX, 25), ((60, 130), STAR, 13),
         ((20, 40, 44), STAR, 7), ((18, 36, 40), BOX, 27), ((24, 40, 44), STAR, 13),
         ((12, 14, 16), STAR, 19), ((30, 37), BOX, 49), ((12, 13, 14), BOX, 125)]
# 2D: k = 2 and 3 read each weight per term; k = 5 and 6 (one staged element
# per thread) stage the weights of radius-1 stencils in the LDS ring, with
# ragged row shares (P x W not a multiple of the thread count: 9 x 40 over
# 50 threads, 5 x 64 over 96)
BAND_TUNINGS = {2: ["method=tstp,k=2,w=32,c=4,l=16", "method=tstp,k=3,w=64,c=4,l=20,lanemap=0",
                    "method=tstp,k=5,w=40,c=4,l=16", "method=tstp,k=6,w=64,c=4,l=24,lanemap=1"],
                3: ["method=tstp,k=1,w=16,h=16,c=4,l=8",
                    "method=tstp,k=2,w=32,h=16,c=4,l=12,lanemap=1"]}


def gpu_varcoef(u0, W, shape, order, boundary, T, tuning=None):
    import torch

    import paper_2010_04868_amd as tvs
    dt = F64 if u0.dtype == np.float64 else F32
    g = torch.from_numpy(np.ascontiguousarray(u0)).to("cuda")
    w = torch.from_numpy(np.ascontiguousarray(W)).to("cuda")
    tvs.Plan(u0.shape, dt, shape, order, 0, boundary, tuning).run_varcoef(g, w, T)
    torch.cuda.synchronize()
    return g.cpu().numpy()


@pytest.mark.parametrize("boundary", [DIRICHLET, PERIODIC])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_varcoef_matches_oracle(boundary, dtype):
    failures = []
    for dims, shape, P in CASES:
        rng = np.random.default_rng(sum(dims) + P)
        u0 = rng.random(dims).astype(np_dtype(dtype))
        W = rng.uniform(0.02, 0.2, (P,) + dims).astype(np_dtype(dtype))
        prec = "f64" if dtype == F64 else "f32"
        tunings = [None, "method=plain"]
        if len(dims) == 1:
            tunings += ["method=tstp,k=1,l=16", "method=tstp,k=5,l=20", "method=tstp,k=64,l=100"]
        elif not (len(dims) == 3 and P == 19) and P <= 27:
            tunings += BAND_TUNINGS[len(dims)]
        for T in (1, 2, 7, 70):
            ref = oracle.sweep_varcoef(u0, W, shape, boundary, T, P, precision=prec)
            for tuning in tunings:
                got = gpu_varcoef(u0, W, shape, P, boundary, T, tuning)
                try:
                    assert_bitwise(got, ref, f"dims={dims} P={P} T={T} tuning={tuning}")
                except AssertionError as e:
                    failures.append(str(e))
    assert not failures, "\n".join(failures[:20])


def test_varcoef_constant_weights_equal_plain_run():
    import torch

    import paper_2010_04868_amd as tvs
    u0 = np.random.default_rng(1).random((3000,))
    c = [0.25, 0.5, 0.25]
    W = np.broadcast_to(np.array(c).reshape(3, 1), (3, 3000)).copy()
    a = gpu_varcoef(u0, W, STAR, 3, DIRICHLET, 100)
    g = torch.from_numpy(u0).to("cuda")
    tvs.Plan((3000,), F64, STAR, 3).run(g, c, 100)
    torch.cuda.synchronize()
    assert_bitwise(a, g.cpu().numpy(), "constant weights vs the weighted sweep")
