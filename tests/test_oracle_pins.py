"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests compares the oracle with itself: each checks it against a
closed form (eigenvalues/eigenvectors of the 5-point Laplacian), a library
routine (dense Cholesky, dense eigensolver, scipy sparse products), an exact
integer computation, an invariant of CG, or the stencil the paper prints.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from oracle import MODE_CANONICAL, MODE_SEQUENTIAL, VARIANT_CLASSIC, VARIANT_PIPELINED

HERE = os.path.dirname(os.path.abspath(__file__))
VARIANTS = (VARIANT_CLASSIC, VARIANT_PIPELINED)
GPU_LIKE = oracle.Order(2, 64, 4, 16, 256)


def dense_A(nx, ny, order=0):
    rp, col, val = oracle.csr(nx, ny, order)
    return sp.csr_matrix((val, col, rp), shape=(nx * ny, nx * ny)).toarray()


def sparse_A(nx, ny):
    rp, col, val = oracle.csr(nx, ny, 0)
    return sp.csr_matrix((val, col, rp), shape=(nx * ny, nx * ny))


def closed_form_eigs(nx, ny):
    a = np.arange(1, nx + 1)[None, :]
    b = np.arange(1, ny + 1)[:, None]
    return 4 - 2 * np.cos(a * np.pi / (nx + 1)) - 2 * np.cos(b * np.pi / (ny + 1))


def mode(nx, ny, a, b):
    """Eigenvector phi_ab on the (ny, nx) grid, unknown (i, j) at [j, i]."""
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    return np.sin(a * np.pi * (i + 1) / (nx + 1)) * np.sin(b * np.pi * (j + 1) / (ny + 1))


def mode_eig(nx, ny, a, b):
    return 4 - 2 * math.cos(a * math.pi / (nx + 1)) - 2 * math.cos(b * math.pi / (ny + 1))


# ------------------------------------------------------------ the operator --

def test_golden_stencil_from_paper():
    """Interior row of A equals the 3x3 stencil printed in Section II-B."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "stencil_3x3.txt"))
            if l.strip() and not l.startswith("#")]
    st = np.array(rows, dtype=float)
    assert st.shape == (3, 3)
    nx, ny = 7, 6
    for order in (0, 1):
        A = dense_A(nx, ny, order)
        i, j = 3, 2
        row = A[j * nx + i].reshape(ny, nx)
        # window centred on (i, j): rows j+1, j, j-1 (north first), columns i-1..i+1
        win = row[[j + 1, j, j - 1]][:, i - 1:i + 2]
        np.testing.assert_array_equal(win, st)
        assert np.count_nonzero(row) == 5


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 5), (5, 7), (16, 16), (9, 4), (13, 11)])
def test_eigenvalues_closed_form(nx, ny):
    """Dense eigvalsh of the assembled A equals 4-2cos(a pi/(nx+1))-2cos(b pi/(ny+1))."""
    A = dense_A(nx, ny)
    got = np.sort(np.linalg.eigvalsh(A))
    want = np.sort(closed_form_eigs(nx, ny).ravel())
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("nx,ny", [(5, 7), (12, 12), (3, 1)])
def test_matrix_structure(nx, ny):
    for order in (0, 1):
        A = dense_A(nx, ny, order)
        np.testing.assert_array_equal(A, A.T)
        np.testing.assert_array_equal(A, dense_A(nx, ny, 1 - order))
        # a row sums to the number of that node's neighbours on the Dirichlet ring
        g = np.zeros((ny, nx))
        g[0, :] += 1; g[-1, :] += 1; g[:, 0] += 1; g[:, -1] += 1
        np.testing.assert_array_equal(A.sum(axis=1), g.ravel())


@pytest.mark.parametrize("nx,ny", [(37, 23), (64, 1), (100, 100)])
def test_eigenvector_identity(nx, ny):
    for (a, b) in [(1, 1), (2, 1), (nx, ny), (max(1, nx // 3), max(1, ny // 2))]:
        phi = mode(nx, ny, a, b)
        lam = mode_eig(nx, ny, a, b)
        for order in (0, 1):
            y = oracle.spmv(phi, nx, ny, order)
            np.testing.assert_allclose(y, lam * phi, rtol=0, atol=1e-14 * 8)


def test_spmv_matches_scipy():
    nx, ny = 31, 17
    u = np.random.default_rng(0).standard_normal((ny, nx))
    want = sparse_A(nx, ny) @ u.ravel()
    for order in (0, 1):
        np.testing.assert_allclose(oracle.spmv(u, nx, ny, order).ravel(), want, rtol=0,
                                   atol=1e-14)


# ------------------------------------------------------------------- dots --

@pytest.mark.parametrize("nx,ny", [(1, 1), (127, 1), (129, 65), (300, 77), (1000, 3)])
@pytest.mark.parametrize("order", [GPU_LIKE, oracle.Order(4, 64, 4, 8, 256),
                                   oracle.Order(1, 4, 3, 5, 8), oracle.Order(2, 64, 1, 37, 256),
                                   oracle.Order(2, 64, 4, 16, 256, alt=1),
                                   oracle.Order(1, 4, 3, 5, 8, alt=1)])
def test_canonical_dot_exact_on_integers(nx, ny, order):
    """Integer data: every partial sum is exact, so any correct order returns the
    exact sum; a dropped, repeated or misplaced term would not."""
    rng = np.random.default_rng(nx * 1000 + ny)
    a = rng.integers(-8, 9, size=(ny, nx)).astype(float)
    b = rng.integers(-8, 9, size=(ny, nx)).astype(float)
    exact = float(np.sum(a.astype(np.int64) * b.astype(np.int64)))
    assert oracle.dot(a, b, nx, ny, MODE_CANONICAL, order) == exact
    assert oracle.dot(a, b, nx, ny, MODE_SEQUENTIAL) == exact
    # weights that identify every position: term k gets weight k+1
    w = np.arange(1, nx * ny + 1, dtype=float).reshape(ny, nx)
    one = np.ones((ny, nx))
    assert oracle.dot(w, one, nx, ny, MODE_CANONICAL, order) == (nx * ny) * (nx * ny + 1) / 2


def test_alt_order_sums_odd_wavefronts_upward():
    """alt = 1: the odd wavefronts of a tile add their strip's rows from the
    last up, the even ones top down.  One column, two wavefronts of three
    rows: 1, 1e16, -1e16 top down gives 0 (1 + 1e16 rounds to 1e16), bottom up
    gives 1."""
    o0 = oracle.Order(1, 1, 2, 3, 1)
    o1 = oracle.Order(1, 1, 2, 3, 1, alt=1)
    one = np.ones((6, 1))
    odd = np.array([0.0, 0.0, 0.0, 1.0, 1e16, -1e16]).reshape(6, 1)
    even = np.array([1.0, 1e16, -1e16, 0.0, 0.0, 0.0]).reshape(6, 1)
    assert oracle.dot(odd, one, 1, 6, MODE_CANONICAL, o0) == 0.0
    assert oracle.dot(odd, one, 1, 6, MODE_CANONICAL, o1) == 1.0
    assert oracle.dot(even, one, 1, 6, MODE_CANONICAL, o0) == 0.0
    assert oracle.dot(even, one, 1, 6, MODE_CANONICAL, o1) == 0.0
    # a ragged strip (four-row strips, seven rows: the second wavefront holds
    # three): bottom up from the last row of the grid
    o4 = oracle.Order(1, 1, 2, 4, 1, alt=1)
    rag = np.array([0.0, 0.0, 0.0, 0.0, 1.0, 1e16, -1e16]).reshape(7, 1)
    assert oracle.dot(rag, np.ones((7, 1)), 1, 7, MODE_CANONICAL, o4) == 1.0
    assert oracle.dot(rag, np.ones((7, 1)), 1, 7, MODE_CANONICAL,
                      oracle.Order(1, 1, 2, 4, 1)) == 0.0


def seg_order(nx, ny, rows, lanes, spare_waves=1, ghosts=1):
    """Column-segment order covering the grid, with `ghosts` idle threads per
    row of segments and idle threads in spare waves."""
    cols = nx + ghosts
    need = cols * -(-ny // rows)
    return oracle.Order.segments(rows, lanes, -(-need // lanes) + spare_waves, cols)


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 37), (37, 1), (100, 100), (129, 65), (1000, 3)])
@pytest.mark.parametrize("rows,lanes,ghosts", [(10, 64, 1), (1, 64, 0), (3, 4, 2), (7, 16, 1)])
def test_segment_dot_exact_on_integers(nx, ny, rows, lanes, ghosts):
    """The column-segment order counts every term exactly once: exact on
    integer data, and the position-weighted sum identifies every term."""
    order = seg_order(nx, ny, rows, lanes, ghosts=ghosts)
    rng = np.random.default_rng(nx * 7 + ny)
    a = rng.integers(-8, 9, size=(ny, nx)).astype(float)
    b = rng.integers(-8, 9, size=(ny, nx)).astype(float)
    exact = float(np.sum(a.astype(np.int64) * b.astype(np.int64)))
    assert oracle.dot(a, b, nx, ny, MODE_CANONICAL, order) == exact
    w = np.arange(1, nx * ny + 1, dtype=float).reshape(ny, nx)
    assert oracle.dot(w, np.ones((ny, nx)), nx, ny, MODE_CANONICAL, order) == \
        (nx * ny) * (nx * ny + 1) / 2
    # squares of the position weights: a term counted twice or dropped changes it
    assert oracle.dot(w, w, nx, ny, MODE_CANONICAL, order) == \
        sum(k * k for k in range(1, nx * ny + 1))


def test_segment_order_must_cover_the_grid():
    one = np.ones((100, 100))
    short = oracle.Order.segments(10, 64, 15, 100)  # 960 threads < 100 * 10 segments
    narrow = oracle.Order.segments(10, 64, 20, 99)  # fewer threads per row than columns
    for o in (short, narrow):
        assert math.isnan(oracle.dot(one, one, 100, 100, MODE_CANONICAL, o))
        with pytest.raises(ValueError):
            oracle.cg(one, 100, 100, mode=MODE_CANONICAL, order=o)
    for o in (oracle.Order.segments(10, 64, 16, 100), oracle.Order.segments(20, 64, 8, 101)):
        assert oracle.dot(one, one, 100, 100, MODE_CANONICAL, o) == 1e4


def test_segment_dot_error_bound():
    nx, ny, rows = 100, 100, 10
    o = seg_order(nx, ny, rows, 64)
    rng = np.random.default_rng(8)
    a = rng.standard_normal((ny, nx))
    b = rng.standard_normal((ny, nx))
    exact = math.fsum((a * b).ravel())
    mag = float(np.sum(np.abs(a * b)))
    u = 2.0 ** -53
    depth = rows + 6 + o.waves + 2
    got = oracle.dot(a, b, nx, ny, MODE_CANONICAL, o)
    assert abs(got - exact) <= 2 * depth * u * mag + 1e-300


@pytest.mark.parametrize("nx,ny", [(300, 77), (513, 129)])
def test_canonical_dot_error_bound(nx, ny):
    rng = np.random.default_rng(7)
    a = rng.standard_normal((ny, nx))
    b = rng.standard_normal((ny, nx))
    exact = math.fsum((a * b).ravel())  # products rounded, then summed exactly
    mag = float(np.sum(np.abs(a * b)))
    u = 2.0 ** -53
    o = GPU_LIKE
    T = math.ceil(nx / (o.cols_per_lane * o.lanes)) * math.ceil(ny / (o.waves * o.rows))
    depth = o.rows + o.cols_per_lane + 6 + o.waves + math.ceil(T / o.threads2) + 6 + 4 + 2
    got = oracle.dot(a, b, nx, ny, MODE_CANONICAL, o)
    # fma rounds once per term, so the product rounding of fsum adds n*u*mag at most
    assert abs(got - exact) <= 2 * depth * u * mag + 1e-300
    assert abs(oracle.dot(a, b, nx, ny, MODE_SEQUENTIAL) - exact) <= nx * ny * u * mag


# -------------------------------------------------------------- CG solves --

def kappa(nx, ny):
    e = closed_form_eigs(nx, ny)
    return e.max() / e.min()


@pytest.mark.parametrize("nx,ny", [(6, 5), (16, 16), (11, 3)])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("mode_", [MODE_SEQUENTIAL, MODE_CANONICAL, "segments"])
def test_solve_vs_dense_cholesky(nx, ny, variant, mode_):
    b = np.random.default_rng(nx + 31 * ny).uniform(-1, 1, (ny, nx))
    c = sla.cho_factor(dense_A(nx, ny))
    xc = sla.cho_solve(c, b.ravel())
    tol = 1e-12
    order = GPU_LIKE
    if mode_ == "segments":
        mode_, order = MODE_CANONICAL, seg_order(nx, ny, 3, 4)
    x, r = oracle.cg(b, nx, ny, variant=variant, tol=tol, maxit=1000, mode=mode_,
                     order=order)
    assert r.status == oracle.OR_OK
    assert r.rel_res_recursive <= tol
    err = np.linalg.norm(x.ravel() - xc) / np.linalg.norm(xc)
    assert err <= 2 * tol * kappa(nx, ny)
    # the reported true residual matches a scipy recomputation
    rt = np.linalg.norm(b.ravel() - sparse_A(nx, ny) @ x.ravel()) / np.linalg.norm(b)
    assert abs(rt - r.rel_res_true) <= 1e-3 * rt + 1e-16


@pytest.mark.parametrize("variant", VARIANTS)
def test_single_eigenvector_one_iteration(variant):
    nx, ny = 13, 9
    phi = mode(nx, ny, 3, 2)
    lam = mode_eig(nx, ny, 3, 2)
    x, r = oracle.cg(phi, nx, ny, variant=variant, tol=1e-12, maxit=50)
    assert r.status == oracle.OR_OK and r.iterations == 1
    np.testing.assert_allclose(x, phi / lam, rtol=0, atol=1e-14)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("K", [2, 3, 5])
def test_finite_termination(variant, K):
    """b spanning K eigenvectors with distinct eigenvalues: CG ends after K
    iterations in exact arithmetic (K or K+1 in FP64)."""
    nx, ny = 13, 7
    modes = [(1, 1), (4, 2), (7, 5), (2, 6), (12, 3)][:K]
    lams = [mode_eig(nx, ny, a, b) for a, b in modes]
    assert min(abs(x - y) for i, x in enumerate(lams) for y in lams[i + 1:]) > 1e-2
    coef = [1.0, -0.7, 0.45, 0.9, -0.3][:K]
    b = sum(c * mode(nx, ny, a, bb) for c, (a, bb) in zip(coef, modes))
    x, r = oracle.cg(b, nx, ny, variant=variant, tol=1e-10, maxit=100)
    assert r.status == oracle.OR_OK
    assert r.iterations in (K, K + 1)
    want = sum(c / l * mode(nx, ny, a, bb) for c, l, (a, bb) in zip(coef, lams, modes))
    np.testing.assert_allclose(x, want, rtol=0, atol=1e-9)


def test_one_by_one_and_two_by_one_brute_force():
    x, r = oracle.cg(np.array([[3.0]]), 1, 1, tol=1e-14)
    assert r.iterations == 1 and x[0, 0] == 0.75
    b = np.array([[1.0, 2.0]])
    want = np.linalg.solve(np.array([[4.0, -1.0], [-1.0, 4.0]]), b.ravel())
    for v in VARIANTS:
        x, r = oracle.cg(b, 2, 1, variant=v, tol=1e-14)
        assert r.status == oracle.OR_OK and r.iterations <= 2
        np.testing.assert_allclose(x.ravel(), want, rtol=1e-15, atol=1e-15)


def test_classic_invariants():
    """Residuals mutually orthogonal, directions A-conjugate, A-norm error
    non-increasing (first 20 iterations)."""
    nx, ny = 12, 12
    b = np.random.default_rng(3).uniform(-1, 1, (ny, nx))
    m = 21
    x, r, h = oracle.cg(b, nx, ny, tol=0.0, maxit=m - 1, history=m)
    assert h["r"].shape[0] == m
    R, P, X = h["r"], h["p"], h["x"]
    A = sparse_A(nx, ny)
    G = R @ R.T
    d = np.sqrt(np.diag(G))
    off = np.abs(G / np.outer(d, d) - np.eye(m))
    assert off.max() <= 1e-10
    AP = (A @ P.T).T
    H = P @ AP.T
    dh = np.sqrt(np.diag(H))
    assert np.abs(H / np.outer(dh, dh) - np.eye(m)).max() <= 1e-10
    xs = sla.cho_solve(sla.cho_factor(dense_A(nx, ny)), b.ravel())
    E = X - xs
    anorm = np.sqrt(np.einsum("ij,ij->i", E, (A @ E.T).T))
    assert np.all(np.diff(anorm) <= 1e-12 * anorm[0])
    # recorded gamma is (r, r)
    np.testing.assert_allclose(h["gamma"], np.einsum("ij,ij->i", R, R), rtol=1e-14)


@pytest.mark.parametrize("nx,ny", [(6, 5), (16, 16), (9, 14)])
def test_variant_agreement(nx, ny):
    """Classic and modified CG produce the same iterates in exact arithmetic;
    a wrong sign or a misplaced parenthesis in the modified recurrences breaks this."""
    b = np.random.default_rng(nx * ny).uniform(-1, 1, (ny, nx))
    for m in (1, 2, 5, 10, 20):
        xc, rc = oracle.cg(b, nx, ny, variant=VARIANT_CLASSIC, tol=0.0, maxit=m)
        xp, rp = oracle.cg(b, nx, ny, variant=VARIANT_PIPELINED, tol=0.0, maxit=m)
        assert rc.iterations == rp.iterations == m
        assert np.linalg.norm(xc - xp) / np.linalg.norm(xc) <= 1e-12
    xc, rc = oracle.cg(b, nx, ny, variant=VARIANT_CLASSIC, tol=1e-8)
    xp, rp = oracle.cg(b, nx, ny, variant=VARIANT_PIPELINED, tol=1e-8)
    assert abs(rc.iterations - rp.iterations) <= 1


def test_modes_agree_on_workload_shape():
    """Sequential and canonical orders are two valid FP64 runs of the same method."""
    nx, ny = 100, 100
    b = np.random.default_rng(11).uniform(-1, 1, (ny, nx))
    for v, lim in ((VARIANT_CLASSIC, 1e-13), (VARIANT_PIPELINED, 1e-9)):
        xs, rs = oracle.cg(b, nx, ny, variant=v, tol=1e-8)
        xk, rk = oracle.cg(b, nx, ny, variant=v, tol=1e-8, mode=MODE_CANONICAL, order=GPU_LIKE)
        assert abs(rs.iterations - rk.iterations) <= 1
        assert np.linalg.norm(xs - xk) / np.linalg.norm(xs) <= lim


# ------------------------------------------------------------- edge cases --

@pytest.mark.parametrize("variant", VARIANTS)
def test_zero_rhs(variant):
    x, r = oracle.cg(np.zeros((4, 5)), 5, 4, variant=variant, x0=np.ones((4, 5)))
    assert r.status == oracle.OR_OK and r.iterations == 0
    assert not x.any()


@pytest.mark.parametrize("variant", VARIANTS)
def test_fixed_iterations_and_maxit(variant):
    b = np.random.default_rng(5).uniform(-1, 1, (20, 30))
    x, r = oracle.cg(b, 30, 20, variant=variant, tol=0.0, maxit=7)
    assert r.status == oracle.OR_OK and r.iterations == 7
    x, r = oracle.cg(b, 30, 20, variant=variant, tol=1e-12, maxit=7)
    assert r.status == oracle.OR_NOT_CONVERGED and r.iterations == 7


@pytest.mark.parametrize("variant", VARIANTS)
def test_exact_start_takes_no_iteration(variant):
    nx, ny = 8, 6
    b = np.random.default_rng(2).uniform(-1, 1, (ny, nx))
    xs = sla.cho_solve(sla.cho_factor(dense_A(nx, ny)), b.ravel()).reshape(ny, nx)
    x, r = oracle.cg(b, nx, ny, variant=variant, tol=1e-8, x0=xs)
    assert r.iterations == 0 and r.status == oracle.OR_OK
    np.testing.assert_array_equal(x, xs)


@pytest.mark.parametrize("variant", VARIANTS)
def test_nonfinite_rhs_is_breakdown(variant):
    b = np.ones((3, 3)); b[1, 1] = np.nan
    x, r = oracle.cg(b, 3, 3, variant=variant)
    assert r.status == oracle.OR_BREAKDOWN and r.iterations == 0


def test_rejects_invalid():
    with pytest.raises(ValueError):
        oracle.cg(np.ones((2, 2)), 2, 2, tol=1.5)
    with pytest.raises(ValueError):
        oracle.cg(np.ones((2, 2)), 2, 2, maxit=0)


# ------------------------------------------------------------- refinement --

@pytest.mark.parametrize("nx,ny", [(16, 16), (40, 25)])
def test_refinement_reaches_fp64_accuracy(nx, ny):
    b = np.random.default_rng(9).standard_normal((ny, nx))
    tol = 1e-10
    x, r = oracle.refine(b, nx, ny, tol=tol, inner_tol=1e-4)
    assert r.status == oracle.OR_OK and r.outer_iterations >= 2
    rt = np.linalg.norm(b.ravel() - sparse_A(nx, ny) @ x.ravel()) / np.linalg.norm(b)
    assert rt <= tol
    xc = sla.cho_solve(sla.cho_factor(dense_A(nx, ny)), b.ravel())
    assert np.linalg.norm(x.ravel() - xc) / np.linalg.norm(xc) <= 2 * tol * kappa(nx, ny)


def test_refinement_inner_cap_and_zero():
    b = np.random.default_rng(4).standard_normal((30, 30))
    x, r = oracle.refine(b, 30, 30, tol=1e-12, inner_tol=1e-4, maxit=10)
    assert r.status == oracle.OR_NOT_CONVERGED and r.iterations == 10
    x, r = oracle.refine(np.zeros((3, 3)), 3, 3)
    assert r.status == oracle.OR_OK and r.iterations == 0 and not x.any()


# ------------------------------------------- refinement: the FP32 inner solve --
#
# The refinement oracle's inner solve keeps its vectors, its stencil and its
# axpys in binary32 and forms its dot products and scalar ratios in binary64,
# rounding alpha and beta to binary32 once.  On a right-hand side built so that
# every quantity of the first inner iteration is exact (integers of at most 21
# bits scaled by a power of two, ||b|| a power of two), that iteration has one
# correct outcome, fixed by the definitions alone: alpha = (rho, rho) /
# (rho, A rho) evaluated exactly, rounded to binary64 and then to binary32,
# and d = fl32(alpha * rho).

def _rhs_with_power_of_two_norm(nx, ny, seed):
    """Integers in [-4095, 4095] whose squares sum to 4^m: the last few
    entries (greedy squares) complete the sum.  Returns (b, m)."""
    n = nx * ny
    rng = np.random.default_rng(seed)
    while True:
        v = rng.integers(-4095, 4096, n).astype(np.int64)
        head = n - 16
        S = int(np.sum(v[:head] * v[:head]))
        m = (S.bit_length() + 1) // 2 + 1          # 4^m > S
        R = 4 ** m - S
        tail = []
        while R > 0 and len(tail) < 16:
            a = math.isqrt(R)
            tail.append(a)
            R -= a * a
        if R == 0:
            v[head:] = 0
            v[head:head + len(tail)] = np.asarray(tail) * rng.choice([-1, 1], len(tail))
            assert int(np.sum(v * v)) == 4 ** m
            return v.reshape(ny, nx), m


def _stencil_int(v):
    """A v in exact integer arithmetic (the 5-point Laplacian, zero ring)."""
    out = 4 * v
    out[:, 1:] -= v[:, :-1]
    out[:, :-1] -= v[:, 1:]
    out[1:, :] -= v[:-1, :]
    out[:-1, :] -= v[1:, :]
    return out


def _first_inner_step_pin(refine, nx=64, ny=64, seed=77):
    """True when one outer step with one inner iteration of `refine` gives
    x = ||b|| * fl32(alpha32 * rho) exactly."""
    from fractions import Fraction
    bi, m = _rhs_with_power_of_two_norm(nx, ny, seed)
    b = bi.astype(np.float64)
    x, r = refine(b, nx, ny, tol=1e-12, inner_tol=1e-4, maxit=1)
    assert r.status == oracle.OR_NOT_CONVERGED and r.iterations == 1
    assert r.outer_iterations == 1
    scale = 2.0 ** m                                  # ||b||, exactly
    rho = (b / scale).astype(np.float32)              # exact: 21-bit integers / 2^m
    assert np.array_equal(rho.astype(np.float64) * scale, b)
    Ab = _stencil_int(bi)
    gamma = Fraction(int(np.sum(bi * bi)), 4 ** m)    # = 1
    pi = Fraction(int(np.sum(bi * Ab)), 4 ** m)
    alpha32 = np.float32(float(gamma / pi))           # binary64, then binary32
    d_want = np.float32(alpha32) * rho                # one binary32 rounding each
    return bool(np.array_equal(x / scale, d_want.astype(np.float64)))


def test_refinement_first_inner_step_is_binary32_with_binary64_dots():
    assert _first_inner_step_pin(oracle.refine)


def test_refinement_inner_accuracy_is_binary32_limited():
    """Whatever the inner tolerance, one outer step cannot take the true
    residual below what binary32 vectors hold (about kappa * 2^-24 of ||b||):
    even with inner tol 1e-12 a tolerance of 1e-11 needs a second outer step;
    after each outer step x / ||r|| increment is binary32 (d is stored so)."""
    nx, ny = 40, 30
    b = np.random.default_rng(12).standard_normal((ny, nx))
    x, r = oracle.refine(b, nx, ny, tol=1e-11, inner_tol=1e-12)
    assert r.status == oracle.OR_OK and r.outer_iterations >= 2
    rt = np.linalg.norm(b.ravel() - sparse_A(nx, ny) @ x.ravel()) / np.linalg.norm(b)
    assert rt <= 1e-11
    # one outer step only (maxit = the first inner solve's length is not
    # known, so cap the inner iterations well inside it): x = ||b|| * d
    x1, r1 = oracle.refine(b, nx, ny, tol=1e-11, inner_tol=1e-12, maxit=20)
    assert r1.outer_iterations == 1 and r1.iterations == 20
    d = x1 / math.sqrt(math.fsum((b * b).ravel()))
    nz = d != 0
    assert nz.sum() > 0.9 * d.size
    rel32 = np.abs(d[nz] - d[nz].astype(np.float32)) / np.abs(d[nz])
    assert rel32.max() <= 1e-15


@pytest.mark.parametrize("mutant", [1, 2, 3])
def test_refinement_pins_catch_planted_mistakes(tmp_path, mutant):
    """Copies of the oracle built with a planted mistake (1: binary64 inner
    vectors, 2: binary32 inner dots, 3: alpha and beta left in binary64) fail
    the first-inner-step pin that the real oracle passes."""
    import ctypes as C
    import subprocess
    from oracle import oracle as _oracle_mod
    src = os.path.join(os.path.dirname(oracle.lib_path()), "cg_oracle.c")
    lib_path = str(tmp_path / ("mutant%d.so" % mutant))
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-DORACLE_MUTANT=%d" % mutant, "-o", lib_path, src, "-lm"],
                   check=True)
    lib = C.CDLL(lib_path)
    P = C.c_void_p
    lib.oracle_refine.restype = C.c_int
    lib.oracle_refine.argtypes = [C.c_int32, C.c_int32, P, P, P, C.c_double, C.c_double,
                                  C.c_int32, C.POINTER(_oracle_mod._Result)]

    def refine(b, nx, ny, tol, inner_tol, maxit):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        res = _oracle_mod._Result()
        rc = lib.oracle_refine(nx, ny, b.ctypes.data, None, x.ctypes.data, tol, inner_tol, maxit,
                               C.byref(res))
        assert rc >= 0
        return x, _oracle_mod.Result(status=res.status, iterations=res.iterations,
                                outer_iterations=res.outer_iterations)

    assert not _first_inner_step_pin(refine)


def test_refinement_last_inner_solve_stops_at_what_tol_needs():
    """tol 1e-6, inner tol 1e-4 from x0 = 0: the first inner solve takes the
    residual to about 1e-4, the second only needs a further factor of about
    tol / 1e-4 / 2 = 5e-3 (not 1e-4): two outer steps end with a true
    residual below tol but far above what a second 1e-4 step gives (1e-8)."""
    nx, ny = 40, 30
    b = np.random.default_rng(15).standard_normal((ny, nx))
    x, r = oracle.refine(b, nx, ny, tol=1e-6, inner_tol=1e-4)
    rt = np.linalg.norm(b.ravel() - sparse_A(nx, ny) @ x.ravel()) / np.linalg.norm(b)
    assert r.status == oracle.OR_OK and r.outer_iterations == 2
    assert 1e-8 < rt <= 1e-6


def test_openmp_build_canonical_mode_gives_the_same_bits():
    """The OpenMP build's canonical mode (tile partials formed in parallel,
    then summed in tile order) returns the single-thread build's bits for both
    variants, in the tile order with and without the alternating walk."""
    nx, ny = 300, 190
    b = np.random.default_rng(8).uniform(-1, 1, (ny, nx))
    for o in (GPU_LIKE, oracle.Order(2, 64, 4, 32, 256, alt=1)):
        for v in (0, 1):
            x1, r1 = oracle.cg(b, nx, ny, variant=v, tol=1e-10, maxit=3000,
                               mode=MODE_CANONICAL, order=o)
            x2, r2 = oracle.cg(b, nx, ny, variant=v, tol=1e-10, maxit=3000,
                               mode=MODE_CANONICAL, order=o, all_cores=True)
            assert r1.iterations == r2.iterations
            np.testing.assert_array_equal(x1, x2)
            assert r1.rel_res_true == r2.rel_res_true
