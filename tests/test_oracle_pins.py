"""Pins for the CPU oracle, from mathematics that does not use its arithmetic.

The oracle implements the naive (d+1)-loop sweep (Section 1, Algorithm 1;
Gauss-Seidel "newest values" in place, Section 3.4).  Each test below checks
it against something fixed independently of that code:

* exact integer brute force: the Jacobi iteration matrix applied T times and
  the Gauss-Seidel matrix splitting (I - L) u' = (D + U) u solved by a library
  triangular solver -- with integer coefficients every intermediate value is
  an integer below 2**53, so the comparison is exact and independent of the
  summation order, and asymmetric coefficients catch any offset/sign mix-up;
* the operation order itself (left-to-right sum, no fused multiply-add) on
  inputs where another order or a fused operation gives a different double;
* closed forms: Fourier eigenmodes under periodic boundaries, sine modes
  under zero Dirichlet borders, the binomial kernel of the (1/4, 1/2, 1/4)
  smoother, checkerboards;
* invariants: constant fields, fixed borders, translation invariance,
  composition, the maximum principle;
* textbook Gauss-Seidel facts: convergence factor cos^2(pi/(m+1)) against
  Jacobi's cos(pi/(m+1)) for the discrete Laplacian, and the fixed point
  equal to a direct solve of the Laplace system.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import BOX, DIRICHLET, GAUSS_SEIDEL, JACOBI, PERIODIC, STAR


# ---------------------------------------------------------------------------
# helpers that know the stencil only through its definition
# ---------------------------------------------------------------------------

def offset_list(ndim, shape, r):
    """All offsets in {-r..r}^ndim (star: at most one non-zero component),
    in lexicographic order with axis 0 most significant."""
    out = []
    for d in itertools.product(range(-r, r + 1), repeat=ndim):
        if shape == STAR and sum(1 for x in d if x) > 1:
            continue
        out.append(d)
    return out


def is_updated(idx, dims, r, boundary):
    if boundary == PERIODIC:
        return True
    return all(r <= i < n - r for i, n in zip(idx, dims))


def neighbour(idx, d, dims):
    return tuple((i + di) % n for i, di, n in zip(idx, d, dims))


def stencil_matrices(dims, shape, r, coeffs, boundary):
    """(A, L, M) as exact integer object arrays.

    A   : Jacobi iteration matrix (identity rows on fixed border points).
    L   : coefficients of neighbours that precede the point in C order.
    M   : coefficients of the centre and the neighbours after it, with
          identity rows on fixed border points.  Gauss-Seidel in place is
          (I - L) u' = M u.
    """
    n = int(np.prod(dims))
    offs = offset_list(len(dims), shape, r)
    assert len(offs) == len(coeffs)
    A = np.zeros((n, n), dtype=object)
    L = np.zeros((n, n), dtype=object)
    M = np.zeros((n, n), dtype=object)
    A[:] = 0
    L[:] = 0
    M[:] = 0
    for idx in itertools.product(*[range(k) for k in dims]):
        i = int(np.ravel_multi_index(idx, dims))
        if not is_updated(idx, dims, r, boundary):
            A[i, i] = 1
            M[i, i] = 1
            continue
        for d, c in zip(offs, coeffs):
            j = int(np.ravel_multi_index(neighbour(idx, d, dims), dims))
            A[i, j] += c
            if j < i:
                L[i, j] += c
            else:
                M[i, j] += c
    return A, L, M


def jacobi_bruteforce(u0, shape, r, coeffs, boundary, T):
    A, _, _ = stencil_matrices(u0.shape, shape, r, coeffs, boundary)
    v = np.array([int(x) for x in u0.ravel()], dtype=object)
    for _ in range(T):
        v = A.dot(v)
    return v.reshape(u0.shape)


def gs_bruteforce(u0, shape, r, coeffs, T):
    _, L, M = stencil_matrices(u0.shape, shape, r, coeffs, DIRICHLET)
    n = L.shape[0]
    ImL = np.eye(n) - L.astype(np.float64)
    Mf = M.astype(np.float64)
    v = u0.ravel().astype(np.float64)
    for _ in range(T):
        v = scipy.linalg.solve_triangular(ImL, Mf @ v, lower=True, unit_diagonal=True)
    return v.reshape(u0.shape)


def int_inputs(dims, seed, lo=-3, hi=4):
    return np.random.default_rng(seed).integers(lo, hi, size=dims).astype(np.float64)


def int_coeffs(P, seed, lo=-2, hi=3):
    c = np.random.default_rng(seed).integers(lo, hi, size=P)
    c[c == 0] = 1  # every neighbour participates
    return [int(x) for x in c]


# ---------------------------------------------------------------------------
# canonical offsets
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ndim,shape,r", [(1, STAR, 1), (1, STAR, 2), (2, STAR, 1), (2, BOX, 1),
                                          (3, STAR, 1), (3, BOX, 1), (2, STAR, 2), (3, BOX, 2)])
def test_offsets_match_definition(ndim, shape, r):
    P = len(offset_list(ndim, shape, r))
    got = oracle.offsets(ndim, shape, P)
    assert [tuple(x) for x in got] == offset_list(ndim, shape, r)


def test_offsets_written_out():
    assert [tuple(x) for x in oracle.offsets(2, STAR, 5)] == [(-1, 0), (0, -1), (0, 0), (0, 1), (1, 0)]
    assert [tuple(x) for x in oracle.offsets(3, STAR, 7)] == [
        (-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)]
    assert [tuple(x) for x in oracle.offsets(1, STAR, 3)] == [(-1,), (0,), (1,)]


def test_inconsistent_point_count_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.sweep(np.zeros(8), [1.0] * 4, STAR, JACOBI, DIRICHLET, 1)
    with pytest.raises(oracle.OracleError):
        oracle.sweep(np.zeros((5, 5)), [1.0] * 7, BOX, JACOBI, DIRICHLET, 1)


# ---------------------------------------------------------------------------
# exact brute force
# ---------------------------------------------------------------------------

BRUTE_CASES = [
    ((11,), STAR, 1, 6),
    ((13,), STAR, 2, 4),
    ((5, 6), STAR, 1, 5),
    ((5, 6), BOX, 1, 4),
    ((7, 6), STAR, 2, 3),
    ((4, 4, 5), STAR, 1, 3),
    ((4, 4, 5), BOX, 1, 2),
    ((6, 7), BOX, 2, 2),
    ((5, 5, 6), STAR, 2, 2),
    ((17,), STAR, 3, 3),
    ((8, 9), BOX, 3, 2),
    ((6, 6, 7), BOX, 2, 1),
]


@pytest.mark.parametrize("dims,shape,r,T", BRUTE_CASES)
@pytest.mark.parametrize("boundary", [DIRICHLET, PERIODIC])
def test_jacobi_exact_bruteforce(dims, shape, r, T, boundary):
    P = len(offset_list(len(dims), shape, r))
    c = int_coeffs(P, seed=P * 7 + T)
    u0 = int_inputs(dims, seed=sum(dims))
    exact = jacobi_bruteforce(u0, shape, r, c, boundary, T)
    assert max(abs(int(x)) for x in exact.ravel()) < 2 ** 53
    got = oracle.sweep(u0, c, shape, JACOBI, boundary, T, npoints=P)
    assert np.array_equal(got, exact.astype(np.float64))
    got32 = oracle.sweep(u0, c, shape, JACOBI, boundary, T, npoints=P, precision="f32")
    if max(abs(int(x)) for x in exact.ravel()) < 2 ** 24:
        assert np.array_equal(got32.astype(np.float64), exact.astype(np.float64))


@pytest.mark.parametrize("dims,shape,r,T", [((12,), STAR, 1, 4), ((5, 6), STAR, 1, 3),
                                            ((5, 6), BOX, 1, 2), ((4, 4, 5), STAR, 1, 2),
                                            ((4, 5, 4), BOX, 1, 1), ((9,), STAR, 2, 3)])
def test_gauss_seidel_matrix_splitting(dims, shape, r, T):
    P = len(offset_list(len(dims), shape, r))
    c = int_coeffs(P, seed=P + 3, lo=-1, hi=2)
    u0 = int_inputs(dims, seed=len(dims) + T, lo=-2, hi=3)
    exact = gs_bruteforce(u0, shape, r, c, T)
    assert np.all(np.abs(exact) < 2 ** 50) and np.array_equal(exact, np.round(exact))
    got = oracle.sweep(u0, c, shape, GAUSS_SEIDEL, DIRICHLET, T, npoints=P)
    assert np.array_equal(got, exact)


def test_gauss_seidel_differs_from_jacobi():
    u0 = int_inputs((6, 7), seed=1)
    c = [1, 1, 1, 1, 1]
    gs = oracle.sweep(u0, c, STAR, GAUSS_SEIDEL, DIRICHLET, 1)
    ja = oracle.sweep(u0, c, STAR, JACOBI, DIRICHLET, 1)
    # the first interior point has no updated predecessor: identical there
    assert gs[1, 1] == ja[1, 1]
    assert not np.array_equal(gs, ja)


def test_gauss_seidel_periodic_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.sweep(np.zeros((5, 5)), [0.2] * 5, STAR, GAUSS_SEIDEL, PERIODIC, 1)


# ---------------------------------------------------------------------------
# operation order and rounding
# ---------------------------------------------------------------------------

def test_left_to_right_summation():
    # centre point: 1*1 + 1*1e16 + 1*(-1e16).  Left to right: (1 + 1e16)
    # rounds to 1e16, minus 1e16 gives 0.  Any other association gives 1.
    u = np.array([0.0, 1.0, 1e16, -1e16, 0.0])
    got = oracle.sweep(u, [1.0, 1.0, 1.0], STAR, JACOBI, DIRICHLET, 1)
    assert got[2] == 0.0
    # the first term enters as a product, not as (+0) + product: every term
    # of point 1 is -0.0, and only a sum that starts from the first product
    # keeps the sign (+0 + -0 is +0).
    u = np.array([-0.0, -1.0, -5.0, 0.0])
    got = oracle.sweep(u, [1.0, 0.0, 0.0], STAR, JACOBI, DIRICHLET, 1)
    assert got[1] == 0.0 and math.copysign(1.0, got[1]) == -1.0


def test_no_fused_multiply_add():
    # point 2 reads (u1, u2, u3) = (-1, 1/3, 7) with weights (1, 3, 0):
    # acc = 1*(-1); the separately rounded product 3*(1/3) is exactly 1.0
    # (a tie that rounds to even), so acc becomes 0, and 0*7 keeps it 0.  A
    # fused multiply-add keeps the exact product and gives -2**-54 instead.
    third = 1.0 / 3.0
    u = np.array([0.0, -1.0, third, 7.0])
    got = oracle.sweep(u, [1.0, 3.0, 0.0], STAR, JACOBI, DIRICHLET, 1)
    assert got[2] == 0.0
    exact_product = Fraction(3) * Fraction(third)
    assert exact_product != 1 and float(exact_product) == 1.0


# The FP32 mirror must follow the same order and rounding in single
# precision: every product and sum rounded to float32 on its own.  These
# inputs give a different float32 result if the mirror accumulated in double
# (or any wider type), reassociated, or fused a multiply and an add.

def test_left_to_right_summation_f32():
    # 1 + 1e8 rounds to 1e8 in float32 (the spacing there is 8), and 1e8 - 1e8
    # is 0.  Accumulating in double keeps 100000001 and ends at 1; summing in
    # another order also gives 1.
    assert np.float32(1.0) + np.float32(1e8) == np.float32(1e8)
    u = np.array([0.0, 1.0, 1e8, -1e8, 0.0], np.float32)
    got = oracle.sweep(u, [1.0, 1.0, 1.0], STAR, JACOBI, DIRICHLET, 1, precision="f32")
    assert got.dtype == np.float32 and got[2] == 0.0
    # the first term enters as a product: -0.0 survives only without a +0 start
    u = np.array([-0.0, -1.0, -5.0, 0.0], np.float32)
    got = oracle.sweep(u, [1.0, 0.0, 0.0], STAR, JACOBI, DIRICHLET, 1, precision="f32")
    assert got[1] == 0.0 and math.copysign(1.0, float(got[1])) == -1.0


def test_no_fused_multiply_add_f32():
    # float32(1/3) = 11184811 * 2**-25, so 3 * float32(1/3) = 1 + 2**-25
    # exactly; rounded to float32 (spacing 2**-23 at 1) it is 1.0, and
    # -1 + 1.0 = 0.  A fused multiply-add, or a product kept in double, leaves
    # 2**-25 instead.
    third = np.float32(1.0) / np.float32(3.0)
    exact = Fraction(3) * Fraction(float(third))
    assert exact == 1 + Fraction(1, 2**25) and np.float32(3.0) * third == np.float32(1.0)
    u = np.array([0.0, -1.0, third, 7.0], np.float32)
    got = oracle.sweep(u, [1.0, 3.0, 0.0], STAR, JACOBI, DIRICHLET, 1, precision="f32")
    assert got[2] == 0.0
    # the weights themselves are rounded to float32 first (nearest even):
    # 0.1 becomes 13421773 * 2**-27, and 0.1f * 10 rounds to exactly 1.0f
    u = np.array([0.0, 10.0, 0.0], np.float32)
    got = oracle.sweep(u, [0.0, 0.1, 0.0], STAR, JACOBI, DIRICHLET, 1, precision="f32")
    w = Fraction(13421773, 2**27)
    assert float(np.float32(0.1)) == float(w)
    assert got[1] == np.float32(float(w * 10))


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

def test_binomial_kernel_1d3p_periodic():
    # (1/4,1/2,1/4) is ((1/2)(shift^-1 + 1))((1/2)(1 + shift)); T steps are the
    # binomial filter C(2T,k)/4^T.  Integer inputs and T <= 20 keep every
    # value exactly representable, so equality is exact.
    n, T = 37, 12
    u0 = np.random.default_rng(0).integers(0, 16, size=n)
    exact = [sum(Fraction(math.comb(2 * T, k) * int(u0[(x + k - T) % n]), 4 ** T)
                 for k in range(2 * T + 1)) for x in range(n)]
    got = oracle.sweep(u0.astype(np.float64), [0.25, 0.5, 0.25], STAR, JACOBI, PERIODIC, T)
    assert [Fraction(float(g)) for g in got] == exact


def _fourier_eigenvalue(offs, coeffs, theta):
    return sum(c * np.exp(1j * np.dot(theta, d)) for d, c in zip(offs, coeffs))


@pytest.mark.parametrize("dims,shape,coeffs,modes,T", [
    ((1000,), STAR, (0.25, 0.5, 0.25), (7,), 200),
    ((1000,), STAR, (0.3, 0.5, 0.2), (13,), 150),           # asymmetric: a phase drift
    ((48, 40), BOX, tuple([1.0 / 9.0] * 9), (3, 5), 60),
    ((48, 40), STAR, (0.1, 0.25, 0.3, 0.2, 0.15), (2, 7), 40),
    ((16, 20, 24), STAR, (0.1, 0.1, 0.1, 0.4, 0.1, 0.1, 0.1), (1, 3, 2), 30),
    ((12, 10, 8), BOX, tuple(np.linspace(0.01, 0.06, 27)), (2, 1, 3), 12),
])
def test_fourier_modes_periodic(dims, shape, coeffs, modes, T):
    offs = offset_list(len(dims), shape, 1)
    theta = np.array([2 * np.pi * m / n for m, n in zip(modes, dims)])
    grid = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    phase = sum(t * g for t, g in zip(theta, grid))
    u0 = np.cos(phase)
    lam = _fourier_eigenvalue(offs, coeffs, theta)
    expect = np.real(lam ** T * np.exp(1j * phase))
    got = oracle.sweep(u0, coeffs, shape, JACOBI, PERIODIC, T)
    assert np.max(np.abs(got - expect)) < 1e-13 * T


def test_fourier_config_1d_modes():
    # the 100000-point 1D problem, periodic: lambda_m = cos^2(pi m / N)
    n, T = 100000, 1000
    x = np.arange(n)
    for m in (1, 1007, 3000):
        u0 = np.cos(2 * np.pi * m * x / n)
        got = oracle.sweep(u0, [0.25, 0.5, 0.25], STAR, JACOBI, PERIODIC, T)
        lam = np.cos(np.pi * m / n) ** 2
        assert np.max(np.abs(got - lam ** T * u0)) < 1e-12


@pytest.mark.parametrize("dims,shape,coeffs,modes,T", [
    ((66,), STAR, (0.25, 0.5, 0.25), (3,), 100),
    ((34, 50), BOX, tuple([1.0 / 9.0] * 9), (2, 3), 50),
    ((34, 50), STAR, (0.2,) * 5, (1, 4), 50),
    ((18, 20, 22), STAR, (0.1, 0.1, 0.1, 0.4, 0.1, 0.1, 0.1), (1, 2, 3), 20),
])
def test_sine_modes_dirichlet(dims, shape, coeffs, modes, T):
    # storage extent n holds the two zero border layers; interior sine
    # sin(pi m i/(n-1)) vanishes on both of them.
    offs = offset_list(len(dims), shape, 1)
    grid = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    ang = [np.pi * m / (n - 1) for m, n in zip(modes, dims)]
    u0 = np.prod([np.sin(a * g) for a, g in zip(ang, grid)], axis=0)
    for ax in range(len(dims)):  # exact zeros on the border
        sl = [slice(None)] * len(dims)
        sl[ax] = 0
        u0[tuple(sl)] = 0
        sl[ax] = -1
        u0[tuple(sl)] = 0
    lam = sum(c * np.prod([np.cos(a * di) for a, di in zip(ang, d)]) for d, c in zip(offs, coeffs))
    got = oracle.sweep(u0, coeffs, shape, JACOBI, DIRICHLET, T)
    assert np.max(np.abs(got - lam ** T * u0)) < 1e-13 * T


def test_checkerboards():
    x = np.arange(64)
    u0 = (-1.0) ** x
    got = oracle.sweep(u0, [0.25, 0.5, 0.25], STAR, JACOBI, PERIODIC, 1)
    assert np.all(got == 0.0)
    g = np.indices((8, 8, 8)).sum(axis=0)
    u0 = (-1.0) ** g
    c = (0.125, 0.125, 0.125, 0.25, 0.125, 0.125, 0.125)
    for T in (1, 5, 9):
        got = oracle.sweep(u0, c, STAR, JACOBI, PERIODIC, T)
        assert np.array_equal(got, (-0.5) ** T * u0)


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims,shape,coeffs,dep,bnd", [
    ((40,), STAR, (0.25, 0.5, 0.25), JACOBI, PERIODIC),
    ((17, 23), BOX, (1 / 16,) * 4 + (0.5,) + (1 / 16,) * 4, JACOBI, DIRICHLET),
    ((9, 10, 11), STAR, (0.125,) * 3 + (0.25,) + (0.125,) * 3, JACOBI, PERIODIC),
    ((17, 23), STAR, (0.125, 0.125, 0.5, 0.125, 0.125), GAUSS_SEIDEL, DIRICHLET),
])
def test_constant_field_dyadic(dims, shape, coeffs, dep, bnd):
    c = 0.375
    got = oracle.sweep(np.full(dims, c), coeffs, shape, dep, bnd, 25)
    assert np.all(got == c)


@pytest.mark.parametrize("dims,shape,P,dep", [((50,), STAR, 3, JACOBI), ((20, 30), BOX, 9, JACOBI),
                                              ((20, 30), STAR, 5, GAUSS_SEIDEL),
                                              ((8, 9, 10), STAR, 7, JACOBI),
                                              ((8, 9, 10), BOX, 27, GAUSS_SEIDEL)])
def test_dirichlet_border_fixed(dims, shape, P, dep):
    u0 = np.random.default_rng(1).random(dims)
    got = oracle.sweep(u0, [1.0 / P] * P, shape, dep, DIRICHLET, 17)
    inner = tuple(slice(1, n - 1) for n in dims)
    mask = np.ones(dims, bool)
    mask[inner] = False
    assert np.array_equal(got[mask], u0[mask])
    assert not np.array_equal(got[inner], u0[inner])


def test_translation_invariance_periodic():
    u0 = np.random.default_rng(2).random((13, 17))
    c = (0.05, 0.1, 0.15, 0.2, 0.1, 0.1, 0.1, 0.1, 0.1)
    a = oracle.sweep(np.roll(u0, (3, -5), axis=(0, 1)), c, BOX, JACOBI, PERIODIC, 9)
    b = np.roll(oracle.sweep(u0, c, BOX, JACOBI, PERIODIC, 9), (3, -5), axis=(0, 1))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dep,bnd", [(JACOBI, PERIODIC), (JACOBI, DIRICHLET), (GAUSS_SEIDEL, DIRICHLET)])
def test_composition(dep, bnd):
    u0 = np.random.default_rng(3).random((19, 21))
    c = (0.1, 0.2, 0.3, 0.25, 0.15)
    whole = oracle.sweep(u0, c, STAR, dep, bnd, 13)
    parts = oracle.sweep(oracle.sweep(u0, c, STAR, dep, bnd, 6), c, STAR, dep, bnd, 7)
    assert np.array_equal(whole, parts)
    assert np.array_equal(oracle.sweep(u0, c, STAR, dep, bnd, 0), u0)


def test_maximum_principle():
    u0 = np.random.default_rng(4).random((30, 30))
    got = oracle.sweep(u0, [1.0 / 9.0] * 9, BOX, JACOBI, DIRICHLET, 50)
    assert got.min() >= u0.min() - 1e-12 and got.max() <= u0.max() + 1e-12
    got = oracle.sweep(u0, [0.2] * 5, STAR, GAUSS_SEIDEL, DIRICHLET, 50)
    assert got.min() >= u0.min() - 1e-12 and got.max() <= u0.max() + 1e-12


def test_f32_mirror_close_to_f64():
    u0 = np.random.default_rng(5).random((64, 64)).astype(np.float32)
    c = [1.0 / 9.0] * 9
    ref = oracle.sweep(u0, c, BOX, JACOBI, DIRICHLET, 100)
    f32 = oracle.sweep(u0, c, BOX, JACOBI, DIRICHLET, 100, precision="f32")
    assert f32.dtype == np.float32
    inner = (slice(1, -1), slice(1, -1))
    rel = np.max(np.abs(f32[inner] - ref[inner]) / np.abs(ref[inner]))
    assert 0 < rel < 1e-5


# ---------------------------------------------------------------------------
# Gauss-Seidel against textbook facts for the discrete Laplacian
# ---------------------------------------------------------------------------

def test_gauss_seidel_convergence_factor():
    m = 14  # interior points per side
    n = m + 2
    u = np.zeros((n, n))
    u[1:-1, 1:-1] = np.random.default_rng(6).random((m, m)) + 0.5
    c = (0.25, 0.25, 0.0, 0.25, 0.25)  # N, W, C, E, S
    gs_norms, ja_norms = [], []
    g, j = u.copy(), u.copy()
    for _ in range(400):
        g = oracle.sweep(g, c, STAR, GAUSS_SEIDEL, DIRICHLET, 1)
        j = oracle.sweep(j, c, STAR, JACOBI, DIRICHLET, 1)
        gs_norms.append(np.linalg.norm(g))
        ja_norms.append(np.linalg.norm(j))
    rho_gs = gs_norms[-1] / gs_norms[-2]
    rho_ja = (ja_norms[-1] / ja_norms[-3]) ** 0.5  # Jacobi's extreme modes alternate sign
    assert abs(rho_gs - math.cos(math.pi / (m + 1)) ** 2) < 1e-5
    assert abs(rho_ja - math.cos(math.pi / (m + 1))) < 1e-5


def test_gauss_seidel_fixed_point_is_laplace_solution():
    m = 10
    n = m + 2
    u = np.zeros((n, n))
    u[0, :] = 1.0           # hot top border, the rest cold
    u[:, -1] = np.linspace(1.0, 0.0, n)
    c = (0.25, 0.25, 0.0, 0.25, 0.25)
    got = oracle.sweep(u, c, STAR, GAUSS_SEIDEL, DIRICHLET, 1500)
    # direct solve of 4 u_ij - (N + S + W + E) = 0 on the interior
    N = m * m
    A = np.zeros((N, N))
    b = np.zeros(N)
    for i in range(m):
        for j in range(m):
            k = i * m + j
            A[k, k] = 4.0
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < m and 0 <= jj < m:
                    A[k, ii * m + jj] = -1.0
                else:
                    b[k] += u[ii + 1, jj + 1]
    x = np.linalg.solve(A, b).reshape(m, m)
    assert np.max(np.abs(got[1:-1, 1:-1] - x)) < 1e-12


# ---------------------------------------------------------------------------
# Game of Life B2S23 (Section 3.4, "Game of life"): born with 2 live
# neighbours of 8, survives with 2 or 3.  Expected boards below are derived by
# counting neighbours by hand; none re-implements the rule.
# ---------------------------------------------------------------------------
def _board(shape, live):
    b = np.zeros(shape, np.int32)
    for r, c in live:
        b[r, c] = 1
    return b


@pytest.mark.parametrize("boundary", [DIRICHLET, PERIODIC])
def test_life_dead_board_stays_dead(boundary):
    assert not oracle.life(np.zeros((9, 11), np.int32), boundary, 5).any()


def test_life_lone_cell_dies_and_begets_nothing():
    # the cell has no live neighbour; each of its 8 neighbours has exactly 1
    got = oracle.life(_board((9, 9), [(4, 4)]), DIRICHLET, 1)
    assert not got.any()


def test_life_domino_moves_to_both_sides():
    # live cells each see 1 neighbour and die; the 4 cells directly above and
    # below the pair see both (2, born); every other cell sees at most 1
    got = oracle.life(_board((8, 9), [(3, 4), (3, 5)]), DIRICHLET, 1)
    want = _board((8, 9), [(2, 4), (2, 5), (4, 4), (4, 5)])
    assert np.array_equal(got, want)


def test_life_block_survives_and_grows_its_edges():
    # each block cell sees the other 3 (survives); each of the 8 cells that
    # share an edge with the block sees 2 (born); the 4 diagonal corners see 1
    block = [(4, 4), (4, 5), (5, 4), (5, 5)]
    edges = [(3, 4), (3, 5), (6, 4), (6, 5), (4, 3), (5, 3), (4, 6), (5, 6)]
    got = oracle.life(_board((10, 10), block), DIRICHLET, 1)
    assert np.array_equal(got, _board((10, 10), block + edges))


def test_life_l_tromino_corner_stays_dead_and_cells_survive_with_two():
    # live A(4,4), B(4,5), C(5,4).  Each live cell sees the other two (2:
    # survives).  The empty corner (5,5) of their 2x2 box sees all three (3:
    # a dead cell with 3 stays dead under B2).  (3,4), (3,5) see A and B, and
    # (4,3), (5,3) see A and C (2: born).  Every other cell sees at most 1.
    got = oracle.life(_board((10, 10), [(4, 4), (4, 5), (5, 4)]), DIRICHLET, 1)
    want = _board((10, 10), [(4, 4), (4, 5), (5, 4), (3, 4), (3, 5), (4, 3), (5, 3)])
    assert np.array_equal(got, want)


def test_life_blinker_middle_survives_with_two():
    # row (4,3), (4,4), (4,5).  The middle sees 2 (survives); the ends see 1
    # (die).  (3,4) and (5,4) see all three (3: stay dead).  The four diagonal
    # cells (3,3), (3,5), (5,3), (5,5) see 2 each (born); the rest see <= 1.
    got = oracle.life(_board((9, 9), [(4, 3), (4, 4), (4, 5)]), DIRICHLET, 1)
    want = _board((9, 9), [(4, 4), (3, 3), (3, 5), (5, 3), (5, 5)])
    assert np.array_equal(got, want)


def test_life_plus_centre_dies_with_four():
    # centre (4,4) and its four edge neighbours.  The centre sees 4 (dies); each
    # arm sees the centre and the two arms beside it (3: survives); the four
    # diagonal corners see 3 (stay dead); every other cell sees at most 1.
    arms = [(3, 4), (5, 4), (4, 3), (4, 5)]
    got = oracle.life(_board((9, 9), arms + [(4, 4)]), DIRICHLET, 1)
    assert np.array_equal(got, _board((9, 9), arms))


def test_life_full_square_and_square_less_a_corner():
    # full 3x3 square, rows and columns 3..5.  Centre sees 8 and the edge
    # middles 5 (die); corners see 3 (survive).  Outside, the cells beside an
    # edge middle, e.g. (2,4), see 3 (stay dead); (2,3), (2,5), (3,2), (5,2),
    # (6,3), (6,5), (3,6), (5,6) see 2 (born); (2,2)-type corners see 1.
    sq = [(i, j) for i in range(3, 6) for j in range(3, 6)]
    got = oracle.life(_board((9, 9), sq), DIRICHLET, 1)
    corners = [(3, 3), (3, 5), (5, 3), (5, 5)]
    born = [(2, 3), (2, 5), (3, 2), (5, 2), (6, 3), (6, 5), (3, 6), (5, 6)]
    assert np.array_equal(got, _board((9, 9), corners + born))
    # the same square without (5,5): the centre sees 7, (4,5) and (5,4) see 4,
    # (3,4) and (4,3) see 5 (all die); corners (3,3), (3,5), (5,3) see 3
    # (survive); (5,5) sees 3 (stays dead); outside, (2,3), (2,5), (3,2),
    # (5,2), (3,6), (6,3), (4,6) and (6,4) see 2 (born), (2,4) and (4,2) see
    # 3 (stay dead), (5,6) and (6,5) see 1.
    sq7 = [c for c in sq if c != (5, 5)]
    got = oracle.life(_board((9, 9), sq7), DIRICHLET, 1)
    want = [(3, 3), (3, 5), (5, 3), (2, 3), (2, 5), (3, 2), (5, 2), (3, 6), (6, 3), (4, 6),
            (6, 4)]
    assert np.array_equal(got, _board((9, 9), want))


def test_life_full_torus_dies():
    # on a full periodic board every cell sees 8 live neighbours
    assert not oracle.life(np.ones((6, 7), np.int32), PERIODIC, 1).any()


def test_life_fixed_border_and_isotropy():
    rng = np.random.default_rng(11)
    u = (rng.random((23, 23)) < 0.4).astype(np.int32)
    got = oracle.life(u, DIRICHLET, 6)
    # the outer layer never changes
    for edge in (np.s_[0, :], np.s_[-1, :], np.s_[:, 0], np.s_[:, -1]):
        assert np.array_equal(got[edge], u[edge])
    # the rule has the square's symmetries: transposes and mirror images commute with it
    assert np.array_equal(oracle.life(u.T.copy(), DIRICHLET, 6), got.T)
    assert np.array_equal(oracle.life(u[:, ::-1].copy(), DIRICHLET, 6), got[:, ::-1])


def test_life_periodic_translation_and_composition():
    rng = np.random.default_rng(12)
    u = (rng.random((17, 19)) < 0.5).astype(np.int32)
    got = oracle.life(u, PERIODIC, 7)
    shifted = np.roll(np.roll(u, 5, axis=0), -3, axis=1)
    assert np.array_equal(oracle.life(shifted, PERIODIC, 7),
                          np.roll(np.roll(got, 5, axis=0), -3, axis=1))
    assert np.array_equal(oracle.life(oracle.life(u, PERIODIC, 3), PERIODIC, 4), got)


# Longest common subsequence (Section 3.4, "Longest common subsequence"): the
# dynamic program's table is pinned by the definition of a longest common
# subsequence itself (brute force over subsequences), a textbook example,
# symmetry, and the chaining of rectangles through the wavefront arrays.
def _is_subsequence(s, t):
    it = iter(t)
    return all(any(c == d for d in it) for c in s)


def _lcs_brute(a, b):
    best = 0
    for mask in range(1 << len(a)):
        sub = [a[i] for i in range(len(a)) if mask >> i & 1]
        if len(sub) > best and _is_subsequence(sub, b):
            best = len(sub)
    return best


def test_lcs_brute_force_all_prefixes():
    rng = np.random.default_rng(21)
    for trial in range(40):
        m, n = int(rng.integers(0, 8)), int(rng.integers(0, 8))
        k = int(rng.integers(1, 4))
        a = rng.integers(0, k, m).astype(np.uint8)
        b = rng.integers(0, k, n).astype(np.uint8)
        row, col = oracle.lcs(a, b)
        # last row: prefixes of b; last column: prefixes of a
        assert [int(v) for v in row] == [_lcs_brute(list(a), list(b[:y])) for y in range(n + 1)]
        assert [int(v) for v in col] == [_lcs_brute(list(a[:x]), list(b)) for x in range(m + 1)]


def test_lcs_textbook_and_special_cases():
    a = np.frombuffer(b"ABCBDAB", np.uint8)
    b = np.frombuffer(b"BDCABA", np.uint8)
    assert oracle.lcs(a, b)[0][-1] == 4      # e.g. "BCBA"
    s = np.random.default_rng(3).integers(0, 4, 500).astype(np.uint8)
    assert oracle.lcs(s, s)[0][-1] == 500    # identical strings
    assert oracle.lcs(s, s + 4)[0][-1] == 0  # disjoint alphabets
    r, c = oracle.lcs(s, np.zeros(0, np.uint8))
    assert r.tolist() == [0] and c.tolist() == [0] * 501
    r, c = oracle.lcs(np.zeros(0, np.uint8), s)
    assert r.tolist() == [0] * 501 and c.tolist() == [0]


def test_lcs_symmetry_and_unit_steps():
    rng = np.random.default_rng(5)
    a = rng.integers(0, 4, 300).astype(np.uint8)
    b = rng.integers(0, 4, 410).astype(np.uint8)
    r_ab, c_ab = oracle.lcs(a, b)
    r_ba, c_ba = oracle.lcs(b, a)
    assert r_ab[-1] == r_ba[-1]
    # transposing the table swaps the last row and the last column
    assert np.array_equal(r_ab, c_ba) and np.array_equal(c_ab, r_ba)
    for v in (r_ab, c_ab):
        assert set(np.diff(v).tolist()) <= {0, 1}


def test_lcs_rectangles_chain_through_wavefront_arrays():
    rng = np.random.default_rng(8)
    a = rng.integers(0, 3, 257).astype(np.uint8)
    b = rng.integers(0, 3, 333).astype(np.uint8)
    row, col = oracle.lcs(a, b)
    # split b: the right rectangle starts from the left one's last column
    n1 = 150
    r1, c1 = oracle.lcs(a, b[:n1])
    r2, c2 = oracle.lcs(a, b[n1:], row=np.zeros(b.size - n1 + 1, np.int32), col=c1)
    assert np.array_equal(np.concatenate([r1, r2[1:]]), row)
    assert np.array_equal(c2[1:], col[1:])
    # split a: the lower rectangle starts from the upper one's last row
    m1 = 100
    r1, c1 = oracle.lcs(a[:m1], b)
    r2, c2 = oracle.lcs(a[m1:], b, row=r1, col=np.zeros(a.size - m1 + 1, np.int32))
    assert np.array_equal(r2, row)
    assert np.array_equal(np.concatenate([c1, c2[1:]]), col)
    # a 3 x 4 grid of rectangles, in anti-diagonal order, equals the whole
    xs, ys = [0, 90, 200, 257], [0, 60, 61, 250, 333]
    rows = {j: np.zeros(ys[j + 1] - ys[j] + 1, np.int32) for j in range(4)}
    cols = {i: np.zeros(xs[i + 1] - xs[i] + 1, np.int32) for i in range(3)}
    for d in range(6):
        for i in range(3):
            j = d - i
            if not 0 <= j < 4:
                continue
            # a rectangle's last row starts with its corner (the boundary
            # column's last value): it is the next rectangle's whole top row
            r, c = oracle.lcs(a[xs[i]:xs[i + 1]], b[ys[j]:ys[j + 1]], row=rows[j], col=cols[i])
            rows[j], cols[i] = r, c
    assert np.array_equal(np.concatenate([rows[0]] + [rows[j][1:] for j in range(1, 4)]), row)
    assert np.array_equal(np.concatenate([cols[0]] + [cols[i][1:] for i in range(1, 3)])[1:],
                          col[1:])


# Variable coefficients (a weight per offset per point, fixed over time; the
# paper's LCS treats one sequence as such a coefficient, Section 3.4): exact
# integer brute force through the dense iteration matrix, and the reduction
# to the constant-coefficient sweep when every point carries the same weights.
def varcoef_bruteforce(u0, shape, r, W, boundary, T):
    dims = u0.shape
    n = int(np.prod(dims))
    offs = offset_list(len(dims), shape, r)
    A = np.zeros((n, n), dtype=object)
    A[:] = 0
    for idx in itertools.product(*[range(k) for k in dims]):
        i = int(np.ravel_multi_index(idx, dims))
        if not is_updated(idx, dims, r, boundary):
            A[i, i] = 1
            continue
        for q, d in enumerate(offs):
            j = int(np.ravel_multi_index(neighbour(idx, d, dims), dims))
            A[i, j] += int(W[q][idx])
    v = np.array([int(x) for x in u0.ravel()], dtype=object)
    for _ in range(T):
        v = A.dot(v)
    return v.reshape(dims)


@pytest.mark.parametrize("dims,shape,r,T", [((12,), STAR, 1, 4), ((13,), STAR, 2, 3),
                                            ((5, 6), STAR, 1, 3), ((5, 6), BOX, 1, 2),
                                            ((4, 4, 5), STAR, 1, 2), ((8, 9), BOX, 3, 1),
                                            ((6, 6, 7), BOX, 2, 1)])
@pytest.mark.parametrize("boundary", [DIRICHLET, PERIODIC])
def test_varcoef_exact_bruteforce(dims, shape, r, T, boundary):
    P = len(offset_list(len(dims), shape, r))
    W = np.random.default_rng(P + T).integers(-2, 3, size=(P,) + dims).astype(np.float64)
    u0 = int_inputs(dims, seed=sum(dims) + 1)
    exact = varcoef_bruteforce(u0, shape, r, W, boundary, T)
    assert max(abs(int(x)) for x in exact.ravel()) < 2 ** 53
    got = oracle.sweep_varcoef(u0, W, shape, boundary, T, P)
    assert np.array_equal(got, exact.astype(np.float64))


@pytest.mark.parametrize("dims,shape,P", [((40,), STAR, 5), ((9, 11), BOX, 9), ((6, 7, 8), STAR, 7)])
@pytest.mark.parametrize("boundary", [DIRICHLET, PERIODIC])
def test_varcoef_constant_weights_reduce_to_sweep(dims, shape, P, boundary):
    rng = np.random.default_rng(P)
    c = rng.uniform(0.02, 0.2, P)
    u0 = rng.random(dims)
    W = np.broadcast_to(c.reshape((P,) + (1,) * len(dims)), (P,) + dims)
    for prec in ("f64", "f32"):
        a = oracle.sweep_varcoef(u0, W, shape, boundary, 7, P, precision=prec)
        b = oracle.sweep(u0, list(c), shape, JACOBI, boundary, 7, npoints=P, precision=prec)
        assert np.array_equal(a, b)
