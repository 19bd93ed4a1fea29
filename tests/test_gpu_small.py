"""GPU parity of the on-chip small-grid solver (cg_plan_info.path 2): the whole
solve in one work-group, every vector in registers or LDS, dot products in the
column-segment order.  Compared through the C ABI with the CPU oracle in that
order: iterates bitwise equal, iteration counts equal, and within the FP64
tolerance (rel. error <= 1e-10, iterations +-2) of the sequential oracle.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import MODE_CANONICAL, MODE_SEQUENTIAL
from paper_1803_03797_amd import cg, workloads

pytestmark = pytest.mark.gpu

VARIANTS = (cg.CG_VARIANT_CLASSIC, cg.CG_VARIANT_PIPELINED)

# shapes the solver takes: (nx + 1) * ceil(ny / rows) <= threads; single rows
# and columns, one segment, ragged last segments, exactly full, a column of
# 256 segments, the 100 x 100 workload
SHAPES = [(1, 1), (1, 20), (1, 21), (20, 1), (3, 5), (63, 20), (64, 21), (90, 70), (100, 100),
          (511, 20), (7, 1260), (1, 5120), (33, 300), (127, 80)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    c = cg.Context(device=0, arena_bytes=1 << 30)
    yield c
    c.close()


def seg_order(ctx, nx, ny, variant):
    info = ctx.cg_plan(nx, ny, variant)
    assert info.path == 2, (nx, ny, info.path)
    assert info.seg_cols == nx + 1
    assert info.seg_waves * info.lanes >= info.seg_cols * -(-ny // info.seg_rows)
    return oracle.Order.segments(info.seg_rows, info.lanes, info.seg_waves, info.seg_cols)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb else 1.0)


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("variant", VARIANTS)
def test_lockstep_bitwise(ctx, nx, ny, variant):
    rng = np.random.default_rng(nx * 31 + ny + variant)
    b = rng.uniform(-1, 1, (ny, nx))
    o = seg_order(ctx, nx, ny, variant)
    for m in (1, 2, 7, 40):
        say("on-chip lockstep", nx, ny, "variant", variant, "m", m)
        x = np.zeros_like(b)
        rc, res = ctx.solve(b, x, nx, ny, tol=0.0, maxit=m, variant=variant)
        xo, ro = oracle.cg(b, nx, ny, variant=variant, tol=0.0, maxit=m, mode=MODE_CANONICAL,
                           order=o)
        assert rc == ro.status
        assert res.iterations == ro.iterations
        np.testing.assert_array_equal(x, xo)
        assert res.rel_res_recursive == ro.rel_res_recursive
        assert res.rel_res_true == ro.rel_res_true


@pytest.mark.parametrize("nx,ny", [(100, 100), (90, 70), (7, 1260), (511, 20), (33, 300)])
@pytest.mark.parametrize("variant", VARIANTS)
def test_natural_stop(ctx, nx, ny, variant):
    rng = np.random.default_rng(500 + nx + ny)
    b = rng.uniform(-1, 1, (ny, nx))
    o = seg_order(ctx, nx, ny, variant)
    say("on-chip natural stop", nx, ny, "variant", variant)
    x = np.zeros_like(b)
    rc, res = ctx.solve(b, x, nx, ny, tol=1e-8, maxit=20000, variant=variant)
    xk, rk = oracle.cg(b, nx, ny, variant=variant, tol=1e-8, maxit=20000, mode=MODE_CANONICAL,
                       order=o)
    xs, rs = oracle.cg(b, nx, ny, variant=variant, tol=1e-8, maxit=20000, mode=MODE_SEQUENTIAL)
    assert rc == cg.CG_OK and res.iterations == rk.iterations
    np.testing.assert_array_equal(x, xk)
    assert abs(res.iterations - rs.iterations) <= 2
    assert rel(x, xs) <= 1e-10


@pytest.mark.parametrize("variant", VARIANTS)
def test_small_workload_against_tile_path(variant, torch):
    """The 100 x 100 workload on the on-chip solver and, with it switched off,
    on the tile path: each bitwise equal to the oracle in its own order, and
    both within the FP64 tolerance of each other."""
    nx, ny = workloads.SMALL["nx"], workloads.SMALL["ny"]
    b = workloads.small_problem()
    out = {}
    for rr in ("1", "0"):
        os.environ["CG_RR"] = rr
        try:
            with cg.Context(device=0, arena_bytes=256 << 20) as c:
                info = c.cg_plan(nx, ny, variant)
                assert info.path == (2 if rr == "1" else 1)
                o = (oracle.Order.segments(info.seg_rows, info.lanes, info.seg_waves, info.seg_cols)
                     if info.path == 2 else
                     oracle.Order(info.cols_per_lane, info.lanes, info.waves, info.rows,
                                  info.threads2, alt=info.walk_alt))
                x = np.zeros_like(b)
                rc, res = c.solve(b, x, nx, ny, tol=1e-8, maxit=2000, variant=variant)
                xo, ro = oracle.cg(b, nx, ny, variant=variant, tol=1e-8, maxit=2000,
                                   mode=MODE_CANONICAL, order=o)
                assert rc == cg.CG_OK and res.iterations == ro.iterations
                np.testing.assert_array_equal(x, xo)
                out[rr] = (x, res.iterations)
        finally:
            os.environ.pop("CG_RR", None)
    assert rel(out["1"][0], out["0"][0]) <= 1e-10
    assert abs(out["1"][1] - out["0"][1]) <= 2


@pytest.mark.parametrize("variant", VARIANTS)
def test_edge_cases(ctx, variant):
    nx, ny = 45, 38
    say("on-chip edge cases", variant)
    b = np.random.default_rng(4).uniform(-1, 1, (ny, nx))
    o = seg_order(ctx, nx, ny, variant)
    # zero right-hand side: x = 0 after no iteration, whatever x0 is
    x = np.full((ny, nx), 3.0)
    rc, res = ctx.solve(np.zeros_like(b), x, nx, ny, x0=np.ones_like(b), variant=variant)
    assert rc == cg.CG_OK and res.iterations == 0 and not x.any()
    # maxit reached
    x = np.zeros_like(b)
    rc, res = ctx.solve(b, x, nx, ny, tol=1e-14, maxit=5, variant=variant)
    assert rc == cg.CG_NOT_CONVERGED and res.iterations == 5
    # non-finite input: breakdown before the first update
    b2 = b.copy()
    b2[7, 11] = np.inf
    rc, res = ctx.solve(b2, x, nx, ny, variant=variant)
    assert rc == cg.CG_BREAKDOWN and res.iterations == 0
    # warm start aliasing x, against the oracle from the same x0
    x0 = np.random.default_rng(5).uniform(-1, 1, (ny, nx))
    x = x0.copy()
    rc, res = ctx.solve(b, x, nx, ny, x0=x, tol=1e-9, maxit=5000, variant=variant)
    xo, ro = oracle.cg(b, nx, ny, variant=variant, tol=1e-9, maxit=5000, x0=x0,
                       mode=MODE_CANONICAL, order=o)
    assert rc == cg.CG_OK and res.iterations == ro.iterations
    np.testing.assert_array_equal(x, xo)
    # an exact start takes no iteration
    xs, _ = oracle.cg(b, nx, ny, variant=variant, tol=1e-13, maxit=5000)
    x = xs.copy()
    rc, res = ctx.solve(b, x, nx, ny, x0=x, tol=1e-6, maxit=50, variant=variant)
    assert rc == cg.CG_OK and res.iterations == 0


def test_shapes_outside_the_solver_take_tiles(ctx):
    for nx, ny in ((512, 20), (100, 103), (1, 5121), (127, 81)):
        info = ctx.cg_plan(nx, ny)
        assert info.path != 2 and info.seg_rows == 0 and info.seg_waves == 0
    assert ctx.cg_plan(100, 100, precision=cg.CG_PREC_FP32_REFINED).path == 0


def test_batch_of_small_solves_bitwise_alone(ctx):
    """Small solves in a batch run one work-group each beside the step
    engine's solves; every result equals the solve alone bitwise."""
    rng = np.random.default_rng(77)
    shapes = [(100, 100), (32, 32), (300, 200), (90, 70), (7, 1260), (200, 150), (1, 1),
              (63, 20)]
    probs, xs, bs = [], [], []
    for k, (nx, ny) in enumerate(shapes):
        b = rng.uniform(-1, 1, (ny, nx))
        x = np.zeros_like(b)
        bs.append(b)
        xs.append(x)
        probs.append(cg.make_problem(b, x, nx, ny, tol=1e-8, maxit=20000, variant=k % 2))
    say("batch of small solves", len(shapes))
    rc, res = ctx.cg_solve_batch(probs)
    assert rc == cg.CG_OK
    for k, ((nx, ny), b, x, r) in enumerate(zip(shapes, bs, xs, res)):
        xa = np.zeros_like(b)
        rca, ra = ctx.solve(b, xa, nx, ny, tol=1e-8, maxit=20000, variant=k % 2)
        assert r.status == rca == cg.CG_OK
        assert r.iterations == ra.iterations
        np.testing.assert_array_equal(x, xa)
