"""Shared helpers for the tests: device round trips through the C ABI and
the oracle reference for the same seeded inputs."""
import numpy as np

import oracle
from paper_2010_04868_amd.inputs import F32, F64, np_dtype


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def gpu_sweep(u0: np.ndarray, coeffs, shape, order, dependence, boundary, T, tuning=None,
              plan=None):
    """Run T steps of the HIP library on a copy of u0; returns a host array."""
    import torch

    import paper_2010_04868_amd as tvs
    dtype = F64 if u0.dtype == np.float64 else F32
    t = torch.from_numpy(np.ascontiguousarray(u0)).to("cuda")
    p = plan or tvs.Plan(u0.shape, dtype, shape, order, dependence, boundary, tuning)
    p.run(t, coeffs, T)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def oracle_sweep(u0, coeffs, shape, order, dependence, boundary, T):
    """Reference in the grid's own precision (FP64 oracle, or its FP32 mirror)."""
    prec = "f64" if u0.dtype == np.float64 else "f32"
    return oracle.sweep(u0, coeffs, shape, dependence, boundary, T, npoints=order, precision=prec)


def max_rel_err(got, ref, mask=None):
    g = got.astype(np.float64)
    r = ref.astype(np.float64)
    if mask is not None:
        g, r = g[mask], r[mask]
    denom = np.maximum(np.abs(r), np.finfo(np.float64).tiny)
    return float(np.max(np.abs(g - r) / denom)) if g.size else 0.0


def assert_bitwise(got, ref, what=""):
    if not np.array_equal(got.view(np.uint8), ref.view(np.uint8)):
        diff = got != ref
        idx = np.argwhere(diff)
        first = tuple(idx[0]) if len(idx) else None
        raise AssertionError(f"{what}: {int(diff.sum())} of {got.size} elements differ; "
                             f"first at {first}: got {got[first] if first else None!r} "
                             f"want {ref[first] if first else None!r}")
