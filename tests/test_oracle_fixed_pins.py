"""Pins of the fixed-point oracle (cg_oracle_fixed.c) against facts fixed by
the definition of the paper's number format (Section II-B: 50 bits, 20 above
the binary point, round to nearest, saturate), by exact rational arithmetic,
by the FP64 oracle (itself pinned in test_oracle_pins.py) and by the paper's
fixed versus floating comparison (Section III).

The brute-force test runs a second implementation written here with Python
integers and the dense matrix of the operator on tiny grids, saturating and
tie-breaking inputs included.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import VARIANT_CLASSIC, VARIANT_PIPELINED
from oracle.oracle import (FX_MAX, FX_MIN, FX_ONE, cg_fixed, fx_axmy, fx_axpy, fx_div, fx_dot,
                           fx_mul, fx_quantize, fx_spmv, fx_value)

HERE = os.path.dirname(os.path.abspath(__file__))
VARIANTS = (VARIANT_CLASSIC, VARIANT_PIPELINED)
Q = 2.0 ** -30


def paper_rows():
    rows = []
    for line in open(os.path.join(HERE, "golden", "fixed_point_tables.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append(tuple(int(v) for v in line.split()))
    return rows


# ----------------------------------------------------------- the format --

def test_format_matches_the_paper():
    for n, t, i, _ in paper_rows():
        assert (t, i) == (50, 20)
    # 50 bits: 2^49 - 1 and -2^49 counts of 2^-(50-20)
    assert FX_ONE == 2 ** (50 - 20)
    assert FX_MAX == 2 ** 49 - 1 and FX_MIN == -(2 ** 49)
    assert fx_value(FX_MAX) == 2.0 ** 19 - Q and fx_value(FX_MIN) == -(2.0 ** 19)


def test_quantize_round_to_nearest_ties_up():
    assert fx_quantize(0.0) == 0 and fx_quantize(-0.0) == 0
    assert fx_quantize(1.0) == FX_ONE
    assert fx_quantize(-2.5) == -5 * FX_ONE // 2
    assert fx_quantize(0.25 * Q) == 0
    assert fx_quantize(0.75 * Q) == 1
    assert fx_quantize(0.5 * Q) == 1            # tie: towards +infinity
    assert fx_quantize(-0.5 * Q) == 0           # tie: towards +infinity
    assert fx_quantize(-1.5 * Q) == -1
    assert fx_quantize(-0.75 * Q) == -1
    assert fx_quantize(1.0 + 0.5 * Q) == FX_ONE + 1
    rng = np.random.default_rng(1)
    for k in rng.integers(FX_MIN, FX_MAX, size=200, endpoint=True):
        assert fx_quantize(fx_value(int(k))) == k   # representable values are fixed points


def test_quantize_saturates():
    assert fx_quantize(2.0 ** 19) == FX_MAX
    assert fx_quantize(2.0 ** 19 - Q) == FX_MAX
    assert fx_quantize(2.0 ** 19 - 0.25 * Q) == FX_MAX   # rounds to 2^19: saturates
    assert fx_quantize(1e30) == FX_MAX and fx_quantize(float("inf")) == FX_MAX
    assert fx_quantize(-(2.0 ** 19)) == FX_MIN
    assert fx_quantize(-(2.0 ** 19) - Q) == FX_MIN
    assert fx_quantize(-1e30) == FX_MIN and fx_quantize(float("-inf")) == FX_MIN
    assert fx_quantize(float("nan")) == 0


def rnd_exact(num, den=1 << 30):
    """floor(num/den + 1/2) of exact integers (den > 0), saturated."""
    v = (2 * num + den) // (2 * den)
    return max(FX_MIN, min(FX_MAX, v))


EDGE = [0, 1, -1, 2, -2, FX_ONE // 2, -FX_ONE // 2, FX_ONE, -FX_ONE, 3 * FX_ONE + 7, FX_MAX,
        FX_MIN, FX_MAX - 1, FX_MIN + 1, 1 << 40, -(1 << 40), (1 << 30) - 1, -(1 << 30) + 1]


def test_multiply_against_exact_rationals():
    rng = np.random.default_rng(2)
    vals = EDGE + [int(v) for v in rng.integers(FX_MIN, FX_MAX, size=60, endpoint=True)] + \
        [int(v) for v in rng.integers(-(1 << 32), 1 << 32, size=60)]
    for a in vals:
        for b in vals[::3]:
            exact = Fraction(a * b, 1 << 60)
            assert fx_mul(a, b) == rnd_exact(a * b), (a, b)
            assert abs(Fraction(fx_mul(a, b), 1 << 30) - exact) <= Fraction(1, 1 << 31) or \
                fx_mul(a, b) in (FX_MAX, FX_MIN)


def test_multiply_special_cases():
    assert fx_mul(FX_ONE, 12345) == 12345 and fx_mul(-FX_ONE, 12345) == -12345
    assert fx_mul(FX_ONE // 2, FX_ONE // 2) == FX_ONE // 4
    assert fx_mul(1, FX_ONE // 2) == 1       # 2^-31: half a quantum rounds up
    assert fx_mul(-1, FX_ONE // 2) == 0
    assert fx_mul(FX_MAX, FX_MAX) == FX_MAX and fx_mul(FX_MIN, FX_MAX) == FX_MIN
    assert fx_mul(FX_MIN, FX_MIN) == FX_MAX
    rng = np.random.default_rng(3)
    for a, b in rng.integers(FX_MIN, FX_MAX, size=(100, 2), endpoint=True):
        assert fx_mul(int(a), int(b)) == fx_mul(int(b), int(a))


def test_update_statements_round_once():
    """y + a x and y - a x are formed exactly and quantized once: the
    subtraction rounds its own tie upwards (it is not the negated sum)."""
    h = FX_ONE // 2
    assert fx_axpy(1, h, 0) == 1 and fx_axmy(1, h, 0) == 0
    assert fx_axpy(3, h, 10) == 12 and fx_axmy(3, h, 10) == 9      # y -+ 1.5 quanta
    assert fx_axmy(FX_ONE, 5, 7) == 2 and fx_axpy(-FX_ONE, 5, 7) == 2
    assert fx_axpy(FX_ONE, -FX_MAX, FX_MAX) == 0                   # exact cancellation
    assert fx_axpy(FX_MAX, FX_MAX, FX_MIN) == FX_MAX                # huge product wins
    assert fx_axmy(FX_MAX, FX_MAX, FX_MAX) == FX_MIN
    assert fx_axpy(FX_ONE, FX_MAX, 1) == FX_MAX and fx_axmy(FX_ONE, FX_MAX, -2) == FX_MIN
    rng = np.random.default_rng(7)
    for a, x, y in rng.integers(FX_MIN, FX_MAX, size=(300, 3), endpoint=True):
        a, x, y = int(a), int(x), int(y)
        assert fx_axpy(a, x, y) == max(FX_MIN, min(FX_MAX, y + (2 * a * x + (1 << 30)) // (1 << 31)))
        assert fx_axmy(a, x, y) == max(FX_MIN, min(FX_MAX, y + (-2 * a * x + (1 << 30)) // (1 << 31)))
    for a, x, y in rng.integers(-(1 << 31), 1 << 31, size=(300, 3)):
        a, x, y = int(a), int(x), int(y)
        assert fx_axmy(a, x, y) == max(FX_MIN, min(FX_MAX, y + (-2 * a * x + (1 << 30)) // (1 << 31)))


def test_divide():
    assert fx_div(FX_ONE, FX_ONE) == FX_ONE
    assert fx_div(3 * FX_ONE, 4 * FX_ONE) == 3 * FX_ONE // 4
    assert fx_div(FX_ONE, 1) == FX_MAX            # 2^30 does not fit
    assert fx_div(1, 2 * FX_ONE) == 1             # half a quantum: up
    assert fx_div(-1, 2 * FX_ONE) == 0
    assert fx_div(-3, 2 * FX_ONE) == -1           # -1.5 quanta: up to -1
    rng = np.random.default_rng(4)
    for n, d in zip(rng.integers(FX_MIN, FX_MAX, size=300, endpoint=True),
                    rng.integers(1, FX_MAX, size=300, endpoint=True)):
        n, d = int(n), int(d)
        assert fx_div(n, d) == rnd_exact(n << 30, d)
        if fx_div(n, d) not in (FX_MAX, FX_MIN):
            assert abs(Fraction(fx_div(n, d), 1 << 30) - Fraction(n, d)) <= Fraction(1, 1 << 31)
    for d in (1, 7, FX_ONE, FX_MAX):            # a * d / d == a when a * d is exact
        for a in (0, 1, -5, FX_ONE, 1234567):
            if abs(a * d) >> 30 <= FX_MAX and (a * d) % (1 << 30) == 0:
                assert fx_div((a * d) >> 30, d) == a


def test_dot_is_exact_and_order_free():
    rng = np.random.default_rng(5)
    for n in (1, 7, 1000):
        a = rng.integers(-(1 << 40), 1 << 40, size=n)
        b = rng.integers(-(1 << 40), 1 << 40, size=n)
        want = max(FX_MIN, min(FX_MAX, sum((2 * int(x) * int(y) + (1 << 30)) // (1 << 31)
                                           for x, y in zip(a, b))))
        assert fx_dot(a, b) == want
        for _ in range(3):
            p = rng.permutation(n)
            assert fx_dot(a[p], b[p]) == want
    # huge terms that cancel: the sum is exact, saturation comes only at the end
    a = np.array([FX_MAX, FX_MAX, FX_MAX, 3], np.int64)
    b = np.array([FX_MAX, -FX_MAX, FX_MAX, FX_ONE], np.int64)
    assert fx_dot(a, b[[0, 1, 2, 3]]) == FX_MAX
    b2 = np.array([FX_MAX, -FX_MAX, 0, FX_ONE], np.int64)
    assert fx_dot(a, b2) == 3
    assert fx_dot(np.full(4, FX_MIN), np.full(4, FX_MAX)) == FX_MIN


def test_stencil_matches_the_fp64_operator_on_small_integers():
    rng = np.random.default_rng(6)
    for nx, ny in ((1, 1), (1, 9), (9, 1), (7, 5), (33, 17)):
        u = rng.integers(-(1 << 44), 1 << 44, size=(ny, nx))
        y = fx_spmv(u, nx, ny)
        # counts below 2^47 keep the FP64 stencil exact
        yd = oracle.spmv(u.astype(np.float64), nx, ny)
        np.testing.assert_array_equal(y, yd.astype(np.int64))


def test_stencil_saturates():
    nx, ny = 4, 3
    u = np.full((ny, nx), FX_MAX, np.int64)
    y = fx_spmv(u, nx, ny)
    # corners 2 neighbours, edges 3, interior 4: 4u - (neighbours) u
    assert y[0, 0] == FX_MAX and y[0, 1] == FX_MAX and y[1, 1] == 0
    y = fx_spmv(-u, nx, ny)
    assert y[0, 0] == FX_MIN and y[1, 2] == 0


# ------------------------------------------------------------ CG itself --

@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("bval,xval", [(1.0, 0.25), (3.0, 0.75), (-2.0, -0.5)])
def test_one_unknown(variant, bval, xval):
    """A = [4]: one step gives b/4 exactly for dyadic b."""
    x, xq, r = cg_fixed(np.full((1, 1), bval), 1, 1, variant=variant, tol=1e-6, maxit=10)
    assert r.status == 0 and r.iterations == 1
    assert x[0, 0] == xval and xq[0, 0] == fx_quantize(xval)
    assert r.rel_res_recursive == 0.0 and r.rel_res_true == 0.0


@pytest.mark.parametrize("variant", VARIANTS)
def test_zero_and_vanishing_rhs(variant):
    for scale in (0.0, 0.25 * Q):     # quantizes to zero: x = 0 after no iteration
        x, xq, r = cg_fixed(np.full((5, 4), scale), 4, 5, variant=variant,
                            x0=np.ones((5, 4)))
        assert r.status == 0 and r.iterations == 0 and not xq.any() and not x.any()


@pytest.mark.parametrize("variant", VARIANTS)
def test_breakdown_when_rounding_zeroes_the_curvature(variant):
    """A smooth right-hand side of a few quanta per product: (r, r) keeps 16
    quanta while every product of (p, A p) = (w, r) rounds to zero, so the
    first step divides by zero and must stop as a breakdown with x = x0."""
    n = 10
    s = np.sin(np.pi * np.arange(1, n + 1) / (n + 1))
    b = 0.9 * 2.0 ** -15 * np.outer(s, s)
    bq = np.vectorize(fx_quantize)(b).astype(np.int64)
    assert fx_dot(bq, bq) == 16 and fx_dot(bq, fx_spmv(bq, n, n)) == 0
    x, xq, r = cg_fixed(b, n, n, variant=variant, tol=0.0, maxit=5)
    assert r.status == 3 and r.iterations == 0 and not xq.any()
    assert r.rel_res_recursive == 1.0 and r.rel_res_true == 1.0


def test_rejects_bad_arguments():
    b = np.ones((2, 2))
    for kw in (dict(maxit=0), dict(tol=1.0), dict(tol=-1.0), dict(tol=float("nan"))):
        with pytest.raises(ValueError):
            cg_fixed(b, 2, 2, **kw)
    with pytest.raises(ValueError):
        cg_fixed(b, 0, 2)


# A second implementation: Python integers, the dense matrix, the algorithm's
# statements in order.  Only for tiny grids.

def _dense(nx, ny):
    n = nx * ny
    A = [[0] * n for _ in range(n)]
    for j in range(ny):
        for i in range(nx):
            k = j * nx + i
            A[k][k] = 4
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                if 0 <= i + di < nx and 0 <= j + dj < ny:
                    A[k][(j + dj) * nx + i + di] = -1
    return A


def _sat(v):
    return max(FX_MIN, min(FX_MAX, v))


def _q(v):
    if v != v:
        return 0
    f = Fraction(v) * (1 << 30) + Fraction(1, 2)
    return _sat(int(f // 1))


def _brute(b, nx, ny, variant, tol, maxit, x0=None):
    A = _dense(nx, ny)
    n = nx * ny
    mv = lambda u: [_sat(sum(A[k][m] * u[m] for m in range(n))) for k in range(n)]
    dot = lambda u, v: _sat(sum((2 * s * t + (1 << 30)) // (1 << 31) for s, t in zip(u, v)))
    ax = lambda a, u, v: [_sat(t + (2 * a * s + (1 << 30)) // (1 << 31)) for s, t in zip(u, v)]
    axm = lambda a, u, v: [_sat(t + (-2 * a * s + (1 << 30)) // (1 << 31)) for s, t in zip(u, v)]
    div = lambda p, d: _sat(((p << 31) + d) // (2 * d))
    bq = [_q(v) for v in b.ravel()]
    x = [_q(v) for v in x0.ravel()] if x0 is not None else [0] * n
    bb = dot(bq, bq)
    if bb == 0:
        return [0] * n, 0, 0
    thr = _q(tol * tol * (bb * 2.0 ** -30))
    r = [_sat(s - t) for s, t in zip(bq, mv(x))]
    g = dot(r, r)
    it = 0

    def stop(g, it):
        if g <= thr:
            return 0
        if it >= maxit:
            return 0 if tol == 0.0 else 2
        return None

    if variant == VARIANT_CLASSIC:
        p, beta = None, 0
        while True:
            st = stop(g, it)
            if st is not None:
                return x, it, st
            p = list(r) if it == 0 else ax(beta, p, r)
            s = mv(p)
            pi = dot(p, s)
            if pi <= 0:
                return x, it, 3
            al = div(g, pi)
            x = ax(al, p, x)
            r = axm(al, s, r)
            g2 = dot(r, r)
            beta = div(g2, g)
            g = g2
            it += 1
    w = mv(r)
    de = dot(w, r)
    st = stop(g, 0)
    if st is not None:
        return x, 0, st
    if de <= 0:
        return x, 0, 3
    nn = mv(w)
    al = div(g, de)
    z, q, p = nn, list(w), list(r)
    x = ax(al, p, x)
    r = axm(al, q, r)
    w = axm(al, z, w)
    it = 1
    while True:
        g_old = g
        g = dot(r, r)
        de = dot(w, r)
        st = stop(g, it)
        if st is not None:
            return x, it, st
        nn = mv(w)
        beta = div(g, g_old)
        if al <= 0:
            return x, it, 3
        den = _sat(div(de, g) - div(beta, al))
        if den <= 0:
            return x, it, 3
        al = div(FX_ONE, den)
        z = ax(beta, z, nn)
        q = ax(beta, q, w)
        p = ax(beta, p, r)
        x = ax(al, p, x)
        r = axm(al, q, r)
        w = axm(al, z, w)
        it += 1


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 1), (1, 3), (2, 2), (3, 2), (2, 3)])
def test_brute_force_tiny_grids(variant, nx, ny):
    rng = np.random.default_rng(10 * nx + ny + 100 * variant)
    cases = [
        (rng.uniform(-1, 1, (ny, nx)), None, 1e-6, 50),
        (rng.uniform(-1, 1, (ny, nx)), rng.uniform(-1, 1, (ny, nx)), 0.0, 7),
        # dyadic inputs with ties in the first products
        (rng.integers(-8, 8, (ny, nx)) * 0.125 + 0.5 * Q, None, 1e-9, 30),
        # saturating magnitudes
        (rng.uniform(-1, 1, (ny, nx)) * 6e5, None, 1e-6, 20),
        (np.full((ny, nx), 4e5), rng.uniform(-3e5, 3e5, (ny, nx)), 1e-3, 20),
    ]
    for b, x0, tol, maxit in cases:
        xb, itb, stb = _brute(b, nx, ny, variant, tol, maxit, x0)
        x, xq, r = cg_fixed(b, nx, ny, variant=variant, tol=tol, maxit=maxit, x0=x0)
        assert (r.status, r.iterations) == (stb, itb)
        assert xq.ravel().tolist() == xb


@pytest.mark.parametrize("variant", VARIANTS)
def test_tracks_floating_point_at_the_paper_sizes(variant):
    """Section III: with the paper's grids and iteration counts, the fixed and
    floating residual histories nearly coincide.  Here: the relative residual
    after the synthesized iteration count within 15% (0.06 decades) of FP64's,
    and the iterates within 1e-4 relative."""
    for n, _, _, iters in paper_rows():
        b = np.random.default_rng(n).uniform(-1, 1, (n, n))
        x, _, r = cg_fixed(b, n, n, variant=variant, tol=0.0, maxit=iters)
        xf, rf = oracle.cg(b, n, n, variant=variant, tol=0.0, maxit=iters)
        assert r.status == 0 and r.iterations == iters
        assert abs(np.log10(r.rel_res_true / rf.rel_res_true)) <= 0.06, n
        assert np.linalg.norm(x - xf) / np.linalg.norm(xf) <= 1e-4, n


def test_classic_converges_like_fp64():
    """Stopping on the residual: the classic variant reaches tol = 1e-6 on the
    100 x 100 grid within 10% of the FP64 iteration count, to the threshold's
    own quantization (the threshold is a whole number of quanta)."""
    b = np.random.default_rng(0).uniform(-1, 1, (100, 100))
    x, _, r = cg_fixed(b, 100, 100, variant=VARIANT_CLASSIC, tol=1e-6, maxit=5000)
    xf, rf = oracle.cg(b, 100, 100, variant=VARIANT_CLASSIC, tol=1e-6, maxit=5000)
    assert r.status == 0
    assert abs(r.iterations - rf.iterations) <= 0.1 * rf.iterations
    assert r.rel_res_true <= 1.1e-6 and r.rel_res_true == r.rel_res_recursive
    assert np.linalg.norm(x - xf) / np.linalg.norm(xf) <= 1e-3
