"""Pins of the Chebyshev-preconditioned CG oracle (oracle_cheb_*, oracle_pcg in
cg_oracle.c) against closed forms, a dense textbook implementation and the
already pinned CG oracle.

The preconditioner is the s-step Chebyshev semi-iteration on A y = r from
y = 0 over [lambda_max / (2 s^2), lambda_max]; its residual polynomial is the
scaled Chebyshev polynomial T_s((theta - lambda)/delta) / T_s(theta/delta), so
on an eigenvector of A it multiplies by p_s(lambda) = (1 - that) / lambda.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from oracle import MODE_CANONICAL, MODE_SEQUENTIAL

GPU_LIKE = oracle.Order(2, 64, 4, 16, 256)
# (r, z) of the library's Chebyshev pass: tiles of one wavefront, 20 rows
CHEB_LIKE = oracle.Order(2, 64, 1, 20, 256)
MODES = (MODE_SEQUENTIAL, MODE_CANONICAL)


def mode_vec(nx, ny, a, b):
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    return np.sin(a * np.pi * (i + 1) / (nx + 1)) * np.sin(b * np.pi * (j + 1) / (ny + 1))


def spectrum(nx, ny):
    c = 2 * math.cos(math.pi / (nx + 1)) + 2 * math.cos(math.pi / (ny + 1))
    return 4 - c, 4 + c


def interval(nx, ny, s):
    """The Chebyshev interval: the top of the spectrum and 1/(2 s^2) of it."""
    hi = spectrum(nx, ny)[1]
    return hi / (2 * s * s), hi


def cheb_T(s, x):
    """T_s(x) for any real x."""
    if abs(x) <= 1:
        return math.cos(s * math.acos(x))
    return math.copysign(1, x) ** s * math.cosh(s * math.acosh(abs(x)))


def p_closed(s, lam, nx, ny):
    lo, hi = interval(nx, ny, s)
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    return (1 - cheb_T(s, (theta - lam) / delta) / cheb_T(s, theta / delta)) / lam


def dense_A(nx, ny):
    rp, col, val = oracle.csr(nx, ny, 0)
    return sp.csr_matrix((val, col, rp), shape=(nx * ny, nx * ny)).toarray()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("s", [1, 2, 3, 5, 8])
def test_eigenvectors_scale_by_the_polynomial(mode, s):
    for nx, ny in ((37, 23), (64, 1), (100, 100)):
        for a, b in ((1, 1), (2, 1), (nx, ny), (nx // 2 + 1, 1)):
            if b > ny:
                continue
            phi = mode_vec(nx, ny, a, b)
            lam = 4 - 2 * math.cos(a * math.pi / (nx + 1)) - 2 * math.cos(b * math.pi / (ny + 1))
            z = oracle.cheb_apply(phi, nx, ny, s, mode)
            want = p_closed(s, lam, nx, ny) * phi
            # p_s(lambda) is small where the residual polynomial nears 1 (the
            # lowest modes): the cancellation there is measured against ||phi||
            err = np.linalg.norm(z - want)
            assert err <= 1e-10 * np.linalg.norm(want) + 1e-12 * np.linalg.norm(phi), \
                (nx, ny, a, b)


def test_coefficients():
    for nx, ny in ((1, 1), (10, 3), (4096, 4096)):
        c0, c1, c2 = oracle.cheb_coeffs(nx, ny, 6)
        lo, hi = interval(nx, ny, 6)
        assert abs(c0 - 1 / ((lo + hi) / 2)) <= 1e-15
        assert len(c1) == len(c2) == 5
        # rho_k of the three-term recurrence: rho_k = 1/(2 sigma - rho_(k-1))
        sigma = ((hi + lo) / 2) / ((hi - lo) / 2)
        rho = 1 / sigma
        for k in range(5):
            rn = 1 / (2 * sigma - rho)
            assert c1[k] == pytest.approx(rn * rho, rel=1e-14)
            assert c2[k] == pytest.approx(2 * rn / ((hi - lo) / 2), rel=1e-14)
            rho = rn


def test_residual_polynomial_bounds():
    """On [lo, hi] the residual polynomial is at most 1/T_s(sigma) in size; below
    lo it lies in [1/T_s(sigma), 1), so p_s > 0 over the whole spectrum, at
    the top (where an interval ending below lambda_max would fail for even s)
    and at the bottom."""
    nx, ny = 300, 200
    lmin, lmax = spectrum(nx, ny)
    for s in (1, 2, 3, 4, 6, 8):
        lo, hi = interval(nx, ny, s)
        theta, delta = (hi + lo) / 2, (hi - lo) / 2
        bound = 1 / cheb_T(s, theta / delta)
        for lam in np.linspace(lmin, lmax, 2001):
            p = p_closed(s, lam, nx, ny)
            R = 1 - lam * p
            assert p > 0
            if lam >= lo:
                assert abs(R) <= bound * (1 + 1e-12)
            else:
                assert bound * (1 - 1e-12) <= R < 1
        # the operator's largest mode keeps a gain of at least 1 - 1/T_s(sigma)
        phi = mode_vec(nx, ny, nx, ny)
        lam = 4 + 2 * math.cos(math.pi / (nx + 1)) + 2 * math.cos(math.pi / (ny + 1))
        gain = (oracle.cheb_apply(phi, nx, ny, s) * phi).sum() / (phi * phi).sum() * lam
        assert gain >= 1 - bound - 1e-12, s


@pytest.mark.parametrize("s", [1, 2, 4, 7])
def test_preconditioner_is_symmetric_positive_definite(s):
    nx, ny = 13, 9
    n = nx * ny
    M = np.column_stack([oracle.cheb_apply(np.eye(n)[:, k].reshape(ny, nx), nx, ny, s).ravel()
                         for k in range(n)])
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    ev = np.linalg.eigvalsh((M + M.T) / 2)
    assert ev.min() > 0
    # M = p_s(A): the eigenvalues are p_s at A's eigenvalues
    lams = np.linalg.eigvalsh(dense_A(nx, ny))
    want = np.sort([p_closed(s, l, nx, ny) for l in lams])
    np.testing.assert_allclose(np.sort(ev), want, rtol=1e-10)


def _textbook_pcg(A, M, b, iters):
    """Dense preconditioned CG, the textbook recurrence, iters steps."""
    x = np.zeros_like(b)
    r = b - A @ x
    z = M @ r
    p = z.copy()
    rho = r @ z
    for _ in range(iters):
        s = A @ p
        alpha = rho / (p @ s)
        x = x + alpha * p
        r = r - alpha * s
        z = M @ r
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x


@pytest.mark.parametrize("s", [2, 3, 5])
def test_iterates_match_a_dense_textbook_pcg(s):
    nx, ny = 12, 9
    n = nx * ny
    A = dense_A(nx, ny)
    M = np.column_stack([oracle.cheb_apply(np.eye(n)[:, k].reshape(ny, nx), nx, ny, s).ravel()
                         for k in range(n)])
    b = np.random.default_rng(s).uniform(-1, 1, n)
    for k in (1, 2, 5, 12):
        xt = _textbook_pcg(A, M, b, k)
        for mode in MODES:
            o = GPU_LIKE if mode == MODE_CANONICAL else None
            x, r = oracle.pcg(b.reshape(ny, nx), nx, ny, s, tol=0.0, maxit=k, mode=mode, order=o)
            assert r.iterations == k
            assert np.linalg.norm(x.ravel() - xt) <= 1e-11 * np.linalg.norm(xt), (s, k, mode)
        # rho in the Chebyshev pass's own tile order
        x, r = oracle.pcg(b.reshape(ny, nx), nx, ny, s, tol=0.0, maxit=k, mode=MODE_CANONICAL,
                          order=GPU_LIKE, order_rho=CHEB_LIKE)
        assert r.iterations == k
        assert np.linalg.norm(x.ravel() - xt) <= 1e-11 * np.linalg.norm(xt), (s, k)


def test_rho_order_is_the_one_given():
    """order_rho changes only how rho = (r,z) is summed: with tiles of one
    wavefront the iterates differ in the last bits from the default order
    (so the argument is used) and agree to rounding; the default is order."""
    nx, ny = 300, 70
    b = np.random.default_rng(8).uniform(-1, 1, (ny, nx))
    xa, ra = oracle.pcg(b, nx, ny, 4, tol=0.0, maxit=30, mode=MODE_CANONICAL, order=GPU_LIKE)
    xd, rd = oracle.pcg(b, nx, ny, 4, tol=0.0, maxit=30, mode=MODE_CANONICAL, order=GPU_LIKE,
                        order_rho=GPU_LIKE)
    xb, rb = oracle.pcg(b, nx, ny, 4, tol=0.0, maxit=30, mode=MODE_CANONICAL, order=GPU_LIKE,
                        order_rho=CHEB_LIKE)
    np.testing.assert_array_equal(xa, xd)
    assert not np.array_equal(xa, xb)
    assert np.linalg.norm(xa - xb) <= 1e-12 * np.linalg.norm(xa)


@pytest.mark.parametrize("mode", MODES)
def test_one_step_is_plain_cg(mode):
    """s = 1: M = c0 I with c0 = 1/theta = 4/(3 lambda_max); CG is invariant
    under a scalar preconditioner (z = c0 r scales rho and p by c0 and alpha
    by 1/c0), so the iterates are CG's up to rounding."""
    nx, ny = 50, 37
    b = np.random.default_rng(3).uniform(-1, 1, (ny, nx))
    o = GPU_LIKE if mode == MODE_CANONICAL else None
    hi = spectrum(nx, ny)[1]
    assert oracle.cheb_coeffs(nx, ny, 1)[0] == pytest.approx(4 / (3 * hi), rel=1e-15)
    for tol, maxit in ((0.0, 17), (1e-9, 5000)):
        xp, rp = oracle.pcg(b, nx, ny, 1, tol=tol, maxit=maxit, mode=mode, order=o)
        xc, rc = oracle.cg(b, nx, ny, tol=tol, maxit=maxit, mode=mode, order=o)
        assert abs(rp.iterations - rc.iterations) <= 1 and rp.status == rc.status
        assert np.linalg.norm(xp - xc) <= 1e-10 * np.linalg.norm(xc)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("s", [3, 8])
def test_solution_against_cholesky(mode, s):
    nx, ny = 40, 31
    A = dense_A(nx, ny)
    b = np.random.default_rng(7).uniform(-1, 1, (ny, nx))
    xs = sla.cho_solve(sla.cho_factor(A), b.ravel()).reshape(ny, nx)
    o = GPU_LIKE if mode == MODE_CANONICAL else None
    x, r = oracle.pcg(b, nx, ny, s, tol=1e-12, maxit=5000, mode=mode, order=o)
    lo, hi = spectrum(nx, ny)
    assert r.status == 0 and r.rel_res_true <= 1.5e-12
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 2 * 1e-12 * hi / lo


def test_fewer_iterations_than_cg():
    """The bulk of the spectrum of p_s(A) A is squeezed to 1 -+ 1/T_s(sigma),
    and p_s(0) grows like s^2: at 128^2 the iterations fall roughly as 1/s
    (0.53, 0.28 and 0.16 of CG's measured for s = 2, 4, 8)."""
    n = 128
    b = np.random.default_rng(5).uniform(-1, 1, (n, n))
    _, rc = oracle.cg(b, n, n, tol=1e-8, maxit=20000)
    its = {}
    for s in (2, 4, 8):
        x, r = oracle.pcg(b, n, n, s, tol=1e-8, maxit=20000)
        assert r.status == 0 and r.rel_res_true <= 1.2e-8
        its[s] = r.iterations
    assert its[2] <= 0.6 * rc.iterations
    assert its[4] <= 0.35 * rc.iterations
    assert its[8] <= 0.2 * rc.iterations


def test_edge_cases_and_rejections():
    nx, ny = 9, 7
    b = np.random.default_rng(1).uniform(-1, 1, (ny, nx))
    x, r = oracle.pcg(np.zeros_like(b), nx, ny, 4, x0=np.ones_like(b))
    assert r.status == 0 and r.iterations == 0 and not x.any()
    x, r = oracle.pcg(b, nx, ny, 4, tol=1e-14, maxit=2)
    assert r.status == 2 and r.iterations == 2
    b2 = b.copy()
    b2[3, 3] = np.nan
    x, r = oracle.pcg(b2, nx, ny, 4)
    assert r.status == 3 and r.iterations == 0
    for bad in (0, 65):
        with pytest.raises(ValueError):
            oracle.pcg(b, nx, ny, bad)
    with pytest.raises(ValueError):
        oracle.cheb_apply(b, nx, ny, 0)


# --------------------------------------------- preconditioned pipelined CG --
PIPE = oracle.VARIANT_PIPELINED


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("nx,ny,s", [(6, 5, 2), (16, 16, 5), (13, 9, 8), (1, 7, 3)])
def test_pipelined_iterates_match_classic(mode, nx, ny, s):
    """In exact arithmetic the preconditioned pipelined recurrences (r, u, w,
    s, q, z) give the iterates of preconditioned classic CG; in FP64 they
    agree to rounding over the first 20 iterations (a sign or beta slip in
    any of the eight updates breaks this)."""
    b = np.random.default_rng(nx * ny + s).uniform(-1, 1, (ny, nx))
    o = GPU_LIKE if mode == MODE_CANONICAL else None
    for k in range(1, min(21, nx * ny + 1)):
        xc, rc = oracle.pcg(b, nx, ny, s, tol=0.0, maxit=k, mode=mode, order=o)
        xp, rp = oracle.pcg(b, nx, ny, s, tol=0.0, maxit=k, mode=mode, order=o, variant=PIPE)
        assert rp.iterations == rc.iterations == k
        assert np.linalg.norm(xp - xc) <= 1e-12 * np.linalg.norm(xc), (k, mode)


@pytest.mark.parametrize("mode", MODES)
def test_pipelined_iterates_match_a_dense_textbook_pcg(mode):
    nx, ny, s = 12, 9, 3
    n = nx * ny
    A = dense_A(nx, ny)
    M = np.column_stack([oracle.cheb_apply(np.eye(n)[:, k].reshape(ny, nx), nx, ny, s).ravel()
                         for k in range(n)])
    b = np.random.default_rng(17).uniform(-1, 1, n)
    o = GPU_LIKE if mode == MODE_CANONICAL else None
    for k in (1, 2, 5, 12):
        xt = _textbook_pcg(A, M, b, k)
        x, r = oracle.pcg(b.reshape(ny, nx), nx, ny, s, tol=0.0, maxit=k, mode=mode, order=o,
                          variant=PIPE)
        assert np.linalg.norm(x.ravel() - xt) <= 1e-11 * np.linalg.norm(xt), k


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("s", [2, 8])
def test_pipelined_solution_against_cholesky(mode, s):
    nx, ny = 40, 31
    A = dense_A(nx, ny)
    b = np.random.default_rng(9).uniform(-1, 1, (ny, nx))
    xs = sla.cho_solve(sla.cho_factor(A), b.ravel()).reshape(ny, nx)
    o = GPU_LIKE if mode == MODE_CANONICAL else None
    x, r = oracle.pcg(b, nx, ny, s, tol=1e-12, maxit=5000, mode=mode, order=o, variant=PIPE)
    lo, hi = spectrum(nx, ny)
    # the pipelined recurrences let the true residual drift a little above
    # the recursive one (reading 11 of the unpreconditioned variant)
    assert r.status == 0 and r.rel_res_recursive <= 1e-12 and r.rel_res_true <= 1e-11
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 20 * 1e-12 * hi / lo


def test_pipelined_single_mode_and_edge_cases():
    nx, ny = 20, 11
    phi = mode_vec(nx, ny, 3, 2)
    lam = 4 - 2 * math.cos(3 * math.pi / (nx + 1)) - 2 * math.cos(2 * math.pi / (ny + 1))
    x, r = oracle.pcg(phi, nx, ny, 4, tol=1e-10, maxit=50, variant=PIPE)
    assert r.status == 0 and r.iterations == 1
    assert np.linalg.norm(x - phi / lam) <= 1e-12 * np.linalg.norm(phi / lam)
    b = np.random.default_rng(2).uniform(-1, 1, (ny, nx))
    x, r = oracle.pcg(np.zeros_like(b), nx, ny, 4, x0=np.ones_like(b), variant=PIPE)
    assert r.status == 0 and r.iterations == 0 and not x.any()
    x, r = oracle.pcg(b, nx, ny, 4, tol=1e-14, maxit=3, variant=PIPE)
    assert r.status == 2 and r.iterations == 3
    b2 = b.copy()
    b2[4, 4] = np.inf
    x, r = oracle.pcg(b2, nx, ny, 4, variant=PIPE)
    assert r.status == 3 and r.iterations == 0
    x0 = np.random.default_rng(3).uniform(-1, 1, (ny, nx))
    xp, rp = oracle.pcg(b, nx, ny, 4, tol=1e-10, maxit=500, x0=x0, variant=PIPE)
    xc, rc = oracle.pcg(b, nx, ny, 4, tol=1e-10, maxit=500, x0=x0)
    assert rp.status == 0 and abs(rp.iterations - rc.iterations) <= 1
    assert np.linalg.norm(xp - xc) <= 1e-9 * np.linalg.norm(xc)
    with pytest.raises(ValueError):
        oracle.pcg(b, nx, ny, 4, variant=2)


# ------------------------ refinement with a preconditioned binary32 inner solve --

@pytest.mark.parametrize("s", [2, 3, 5, 8])
def test_binary32_chebyshev_on_eigenvectors(s):
    """z = M^-1 phi in binary32 equals p_s(lambda) phi to binary32 accuracy
    (the recurrence's cancellation on the highest modes costs up to about 1e-5
    relative at s = 8; a wrong coefficient, sign or step costs O(1))."""
    nx, ny = 24, 17
    for a, b in ((1, 1), (5, 9), (24, 17), (12, 3)):
        i = np.arange(nx)[None, :]
        j = np.arange(ny)[:, None]
        phi = np.sin(a * np.pi * (i + 1) / (nx + 1)) * np.sin(b * np.pi * (j + 1) / (ny + 1))
        lam = 4 - 2 * math.cos(a * math.pi / (nx + 1)) - 2 * math.cos(b * math.pi / (ny + 1))
        phi32 = phi.astype(np.float32)
        z = oracle.cheb_apply_f32(phi32, nx, ny, s).astype(np.float64)
        want = p_closed(s, lam, nx, ny) * phi32.astype(np.float64)
        assert np.abs(z - want).max() <= 1e-5 * np.abs(want).max()


def test_binary32_chebyshev_one_step_is_one_rounding():
    """s = 1: z = fl32(fl32(c0) r), bitwise."""
    nx, ny = 19, 11
    r = np.random.default_rng(2).standard_normal((ny, nx)).astype(np.float32)
    c0, _, _ = oracle.cheb_coeffs(nx, ny, 1)
    z = oracle.cheb_apply_f32(r, nx, ny, 1)
    np.testing.assert_array_equal(z, np.float32(c0) * r)


@pytest.mark.parametrize("nx,ny", [(16, 16), (40, 25)])
@pytest.mark.parametrize("s", [2, 4, 8])
def test_preconditioned_refinement_accuracy(nx, ny, s):
    b = np.random.default_rng(nx * s).standard_normal((ny, nx))
    tol = 1e-10
    x, r = oracle.refine(b, nx, ny, tol=tol, inner_tol=1e-4, precond=s)
    A = dense_A(nx, ny)
    rt = np.linalg.norm(b.ravel() - A @ x.ravel()) / np.linalg.norm(b)
    assert r.status == oracle.OR_OK and rt <= tol and r.outer_iterations >= 2
    xc = sla.cho_solve(sla.cho_factor(A), b.ravel())
    w = np.linalg.eigvalsh(A)
    assert np.linalg.norm(x.ravel() - xc) / np.linalg.norm(xc) <= 2 * tol * w[-1] / w[0]


def test_preconditioned_refinement_takes_fewer_inner_iterations():
    """128^2, tol 1e-10: the preconditioned inner solves take 0.55 / 0.3 / 0.16
    of the plain ones' iterations at s = 2 / 4 / 8 (the FP64 preconditioned CG
    ratios), with the same number of outer steps."""
    n = 128
    b = np.random.default_rng(3).standard_normal((n, n))
    x0, r0 = oracle.refine(b, n, n, tol=1e-10, inner_tol=1e-4)
    for s, ratio in ((2, 0.55), (4, 0.3), (8, 0.16)):
        x, r = oracle.refine(b, n, n, tol=1e-10, inner_tol=1e-4, precond=s)
        assert r.status == oracle.OR_OK and r.outer_iterations <= r0.outer_iterations + 1
        assert r.iterations <= ratio * r0.iterations
        assert np.linalg.norm(x - x0) <= 1e-8 * np.linalg.norm(x0)


def test_preconditioned_refinement_rejects():
    with pytest.raises(ValueError):
        oracle.refine(np.ones((4, 4)), 4, 4, precond=65)
