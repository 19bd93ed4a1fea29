"""GPU parity of both CG variants on the 3D 7-point Laplacian (cg_problem.nz > 1):
the tile passes marching along z (each wavefront walks one in-plane row through
its planes), against the 3D oracle in the library's z-march tile order
(bitwise) and in the textbook order (FP64 tolerance); at 256^3 (16.8M unknowns)
single-mode and finite-termination properties."""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import MODE_CANONICAL, MODE_SEQUENTIAL
from paper_1803_03797_amd import cg

pytestmark = pytest.mark.gpu

# single cells and rows, one-row planes, tiles ragged in y (rows % 4) and in z
# (planes % the planes per strip), several tile columns
SHAPES = [(1, 1, 2), (2, 3, 4), (64, 1, 3), (130, 7, 5), (37, 40, 23), (100, 64, 64),
          (257, 30, 9)]
VARIANTS = (cg.CG_VARIANT_CLASSIC, cg.CG_VARIANT_PIPELINED)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    c = cg.Context(device=0, arena_bytes=4 << 30)
    yield c
    c.close()


def tile_order(ctx, nx, ny, nz, variant):
    """The z-march order of the plan: tiles of `waves` in-plane rows by `rows`
    planes, each wavefront summing its row over the planes."""
    info = ctx.cg_plan(nx, ny, variant=variant, nz=nz)
    assert info.path == 0 and info.cols_per_lane == 2 and info.walk_z == 1
    assert info.walk_alt == 0
    return oracle.Order.zmarch(info.cols_per_lane, info.lanes, info.waves, info.rows,
                               info.threads2, ny)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb else 1.0)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("nx,ny,nz", SHAPES)
def test_lockstep_bitwise(ctx, nx, ny, nz, variant):
    b = np.random.default_rng(nx + 7 * ny + 13 * nz).uniform(-1, 1, (ny * nz, nx))
    o = tile_order(ctx, nx, ny, nz, variant)
    for m in (1, 2, 7):
        say("3d lockstep", nx, ny, nz, "variant", variant, "maxit", m)
        x = np.zeros_like(b)
        rc, res = ctx.solve(b, x, nx, ny, tol=0.0, maxit=m, variant=variant, nz=nz)
        xo, ro = oracle.cg3(b, nx, ny, nz, variant=variant, tol=0.0, maxit=m,
                            mode=MODE_CANONICAL, order=o)
        assert rc == ro.status and res.iterations == ro.iterations
        np.testing.assert_array_equal(x, xo)
        assert res.rel_res_recursive == ro.rel_res_recursive
        assert res.rel_res_true == ro.rel_res_true


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("nx,ny,nz", [(37, 40, 23), (100, 64, 64)])
def test_natural_stop(ctx, nx, ny, nz, variant):
    b = np.random.default_rng(3 * nx + nz).uniform(-1, 1, (ny * nz, nx))
    o = tile_order(ctx, nx, ny, nz, variant)
    say("3d natural stop", nx, ny, nz, "variant", variant)
    x = np.zeros_like(b)
    rc, res = ctx.solve(b, x, nx, ny, tol=1e-8, maxit=20000, variant=variant, nz=nz)
    xk, rk = oracle.cg3(b, nx, ny, nz, variant=variant, tol=1e-8, maxit=20000,
                        mode=MODE_CANONICAL, order=o)
    xs, rs = oracle.cg3(b, nx, ny, nz, variant=variant, tol=1e-8, maxit=20000,
                        mode=MODE_SEQUENTIAL)
    assert rc == cg.CG_OK and res.iterations == rk.iterations
    np.testing.assert_array_equal(x, xk)
    assert abs(res.iterations - rs.iterations) <= 2
    say("  iterations %d, textbook-order spread %.2e, true residual %.3g" %
        (res.iterations, rel(x, xs), res.rel_res_true))
    assert rel(x, xs) <= (1e-10 if variant == cg.CG_VARIANT_CLASSIC else 1e-9)
    assert res.rel_res_true <= (1.2e-8 if variant == cg.CG_VARIANT_CLASSIC else 1e-7)


def lam3(n, a, b, c):
    s = lambda k: 4 * math.sin(k * math.pi / (2 * (n + 1))) ** 2
    return s(a) + s(b) + s(c)


def mode3(torch, n, a, b, c):
    dev = torch.device("cuda:0")
    i = torch.arange(1, n + 1, dtype=torch.float64, device=dev)
    fx = torch.sin(a * math.pi * i / (n + 1))
    fy = torch.sin(b * math.pi * i / (n + 1))
    fz = torch.sin(c * math.pi * i / (n + 1))
    return (fz[:, None, None] * fy[None, :, None] * fx[None, None, :]).reshape(n * n, n)


@pytest.mark.parametrize("variant", VARIANTS)
def test_full_size_modes(ctx, torch, variant):
    """256^3: a single grid mode takes one iteration to x = b / lambda; four
    modes with distinct eigenvalues take four (or five) iterations to the
    closed-form solution.  (b's rounding returns amplified by up to
    lambda / lambda_min ~ 2e4 through A^-1: 1e-11 covers it.  The four modes
    have eigenvalues 1.9 .. 7.5: with a wide spread the residual polynomial
    amplifies the rounding of the other modes by up to the spread, and a few
    more iterations reach the tolerance.)"""
    n = 256
    for a, b_, c in ((1, 1, 1), (30, 200, 7)):
        say("3d full size mode", variant, a, b_, c)
        phi = mode3(torch, n, a, b_, c)
        x = torch.zeros_like(phi)
        rc, res = ctx.cg_solve(cg.make_problem(phi, x, n, n, tol=1e-8, maxit=10,
                                               variant=variant, nz=n))
        assert rc == cg.CG_OK and res.iterations == 1
        lam = lam3(n, a, b_, c)
        err = float(torch.linalg.norm(x - phi / lam) / torch.linalg.norm(phi / lam))
        say("  rel err %.2e" % err)
        assert err <= 1e-11
    modes = [(100, 60, 40), (128, 128, 128), (200, 200, 50), (70, 90, 20)]
    coef = [1.0, -0.5, 0.25, 0.125]
    assert len({round(lam3(n, *m), 6) for m in modes}) == 4
    b = sum(mode3(torch, n, *m) * c for c, m in zip(coef, modes))
    xw = sum(mode3(torch, n, *m) * (c / lam3(n, *m)) for c, m in zip(coef, modes))
    x = torch.zeros_like(b)
    rc, res = ctx.cg_solve(cg.make_problem(b, x, n, n, tol=1e-10, maxit=50, variant=variant,
                                           nz=n))
    err = float(torch.linalg.norm(x - xw) / torch.linalg.norm(xw))
    say("3d finite termination", variant, res.iterations, "err %.2e" % err)
    assert rc == cg.CG_OK and res.iterations in (4, 5) and err <= 1e-10


@pytest.mark.parametrize("variant", VARIANTS)
def test_edge_cases(ctx, variant):
    nx, ny, nz = 50, 20, 12
    b = np.random.default_rng(4).uniform(-1, 1, (ny * nz, nx))
    o = tile_order(ctx, nx, ny, nz, variant)
    kw = dict(variant=variant, nz=nz)
    x = np.full_like(b, 2.0)
    rc, res = ctx.solve(np.zeros_like(b), x, nx, ny, x0=np.ones_like(b), **kw)
    assert rc == cg.CG_OK and res.iterations == 0 and not x.any()
    x = np.zeros_like(b)
    rc, res = ctx.solve(b, x, nx, ny, tol=1e-14, maxit=3, **kw)
    assert rc == cg.CG_NOT_CONVERGED and res.iterations == 3
    b2 = b.copy()
    b2[5, 5] = np.nan
    rc, res = ctx.solve(b2, x, nx, ny, **kw)
    assert rc == cg.CG_BREAKDOWN and res.iterations == 0
    x0 = np.random.default_rng(6).uniform(-1, 1, (ny * nz, nx))
    x = x0.copy()
    rc, res = ctx.solve(b, x, nx, ny, x0=x, tol=1e-9, maxit=5000, **kw)
    xo, ro = oracle.cg3(b, nx, ny, nz, variant=variant, tol=1e-9, maxit=5000, x0=x0,
                        mode=MODE_CANONICAL, order=o)
    assert rc == cg.CG_OK and res.iterations == ro.iterations
    np.testing.assert_array_equal(x, xo)


def _served(ctx, probs):
    import time
    tickets = []
    for k, p in enumerate(probs):
        tickets.append(ctx.cg_submit(p))
        if k % 3 == 2:
            time.sleep(0.002)
    out = {}
    deadline = time.time() + 120
    while len(out) < len(tickets) and time.time() < deadline:
        for t in tickets:
            if t not in out:
                rc, r = ctx.cg_poll(t)
                if rc != cg.CG_PENDING:
                    out[t] = (rc, cg.cg_result.from_buffer_copy(r))
        time.sleep(0.001)
    assert len(out) == len(tickets)
    return [out[t] for t in tickets]


def test_batch_and_served_3d_solves_match_alone(ctx):
    """3D requests of both variants beside 2D ones, batched and served: each
    result bitwise the solve alone (the 3D ones on their own step kernel,
    in the same z-march tiles and order), and the 3D ones bitwise the oracle
    in that order."""
    rng = np.random.default_rng(41)
    mix = [(37, 40, 23, 0), (100, 64, 64, 1), (64, 64, 0, 0), (130, 7, 5, 1), (300, 190, 0, 1),
           (2, 3, 4, 0), (257, 30, 9, 0)]
    bs = [rng.uniform(-1, 1, (ny * max(nz, 1), nx)) for nx, ny, nz, _ in mix]

    def prob(k, x):
        nx, ny, nz, v = mix[k]
        return cg.make_problem(bs[k], x, nx, ny, tol=1e-9, maxit=20000, variant=v, nz=nz)
    xb = [np.zeros_like(b) for b in bs]
    say("batch with 3D solves:", len(mix))
    rc, res = ctx.cg_solve_batch([prob(k, x) for k, x in enumerate(xb)])
    assert rc == cg.CG_OK
    xv = [np.zeros_like(b) for b in bs]
    served = _served(ctx, [prob(k, x) for k, x in enumerate(xv)])
    for k, (nx, ny, nz, v) in enumerate(mix):
        xa = np.zeros_like(bs[k])
        rca, ra = ctx.cg_solve(prob(k, xa))
        say("  %dx%dx%d v%d: batch %d served %d alone %d iterations" %
            (nx, ny, nz, v, res[k].iterations, served[k][1].iterations, ra.iterations))
        assert res[k].status == rca == served[k][0] == cg.CG_OK
        assert res[k].iterations == served[k][1].iterations == ra.iterations
        np.testing.assert_array_equal(xb[k], xa)
        np.testing.assert_array_equal(xv[k], xa)
        assert res[k].rel_res_true == ra.rel_res_true
        if nz > 1 and nx * ny * nz <= 40000:
            o = tile_order(ctx, nx, ny, nz, v)
            xo, ro = oracle.cg3(bs[k], nx, ny, nz, variant=v, tol=1e-9, maxit=20000,
                                mode=MODE_CANONICAL, order=o)
            assert ro.iterations == ra.iterations
            np.testing.assert_array_equal(xa, xo)


def test_rejections(ctx):
    nx, ny, nz = 8, 8, 8
    b = np.ones((ny * nz, nx))
    x = np.zeros_like(b)
    for kw in (dict(precond=4), dict(precision=cg.CG_PREC_FP32_REFINED),
               dict(precision=cg.CG_PREC_FIXED)):
        args = dict(nz=nz)
        args.update(kw)
        with pytest.raises(cg.CGError):
            ctx.solve(b, x, nx, ny, **args)
    # nz = 1 is the 2D problem
    x1 = np.zeros((ny, nx))
    x2 = np.zeros((ny, nx))
    b1 = np.random.default_rng(2).uniform(-1, 1, (ny, nx))
    ctx.solve(b1, x1, nx, ny, nz=1, tol=0.0, maxit=5)
    ctx.solve(b1, x2, nx, ny, tol=0.0, maxit=5)
    np.testing.assert_array_equal(x1, x2)
