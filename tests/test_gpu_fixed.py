"""GPU parity of the fixed-point path (cg_plan_info.path 3): Algorithms 1 and 2
in the paper's 50-bit format, one work-group per solve.  Integer arithmetic,
so the bar is bitwise: status, iteration count, every bit of x and both
relative residuals equal to the fixed-point oracle's, alone, in a batch and
through the serving queue."""
import sys

import numpy as np
import pytest

import oracle
from oracle.oracle import cg_fixed
from paper_1803_03797_amd import cg, workloads

pytestmark = pytest.mark.gpu

VARIANTS = (cg.CG_VARIANT_CLASSIC, cg.CG_VARIANT_PIPELINED)
FX = cg.CG_PREC_FIXED

# one unknown per thread (<= 1024), ragged waves, every compiled count of
# unknowns per thread (2, 3, 4, 6, 8, 10), the largest grids the solver takes
# ((nx + 1)(ny + 2) + nx ny <= 20352: 100 x 100, 98 x 102, a single column of
# 6782, a single row of 5087), single rows and columns
SHAPES = [(1, 1), (1, 7), (7, 1), (16, 16), (33, 17), (32, 32), (40, 40), (50, 50), (60, 60),
          (64, 65), (75, 75), (90, 90), (100, 100), (98, 102), (1, 6782), (5087, 1),
          (127, 78)]


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


def check_same(rc, res, x, ro, xo):
    assert rc == ro.status, (rc, ro.status)
    assert res.iterations == ro.iterations, (res.iterations, ro.iterations)
    np.testing.assert_array_equal(x, xo)
    assert res.rel_res_recursive == ro.rel_res_recursive
    assert res.rel_res_true == ro.rel_res_true


def test_plan_reports_the_fixed_path(ctx):
    for nx, ny in SHAPES:
        info = ctx.cg_plan(nx, ny, precision=FX)
        assert info.path == 3
    for nx, ny in ((101, 101), (100, 101), (1, 6783), (5088, 1), (96, 106), (200, 60)):
        with pytest.raises(cg.CGError):
            ctx.cg_plan(nx, ny, precision=FX)
        b = np.zeros((ny, nx))
        assert cg.cg_validate(cg.make_problem(b, b.copy(), nx, ny, precision=FX)) == cg.CG_E_INVALID


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("variant", VARIANTS)
def test_lockstep_bitwise(ctx, nx, ny, variant):
    rng = np.random.default_rng(nx * 7 + ny + 100 * variant)
    b = rng.uniform(-1, 1, (ny, nx))
    for m in (1, 2, 7, 40):
        say("fixed lockstep", nx, ny, "variant", variant, "maxit", m)
        x = np.zeros_like(b)
        rc, res = ctx.solve(b, x, nx, ny, tol=0.0, maxit=m, variant=variant, precision=FX)
        xo, _, ro = cg_fixed(b, nx, ny, variant=variant, tol=0.0, maxit=m)
        check_same(rc, res, x, ro, xo)


@pytest.mark.parametrize("variant", VARIANTS)
def test_paper_grids_and_iteration_counts(ctx, variant):
    """The paper's synthesized configurations (N, iterations) of Section III."""
    for n, iters in zip(workloads.FIXED["sides"], workloads.FIXED["iterations"]):
        b = workloads.fixed_rhs(n)
        say("fixed paper grid", n, "iterations", iters, "variant", variant)
        x = np.zeros_like(b)
        rc, res = ctx.solve(b, x, n, n, tol=0.0, maxit=iters, variant=variant, precision=FX)
        xo, _, ro = cg_fixed(b, n, n, variant=variant, tol=0.0, maxit=iters)
        check_same(rc, res, x, ro, xo)
        assert rc == cg.CG_OK and res.iterations == iters


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("nx,ny", [(16, 16), (40, 40), (100, 100), (1, 6782), (127, 78)])
def test_natural_stop(ctx, variant, nx, ny):
    """Stopping on the residual, breakdowns included (Algorithm 2 in this
    format can lose (r, r) to rounding before tol 1e-6 on 100 x 100)."""
    b = np.random.default_rng(nx + 3 * ny).uniform(-1, 1, (ny, nx))
    say("fixed natural stop", nx, ny, "variant", variant)
    x = np.zeros_like(b)
    rc, res = ctx.solve(b, x, nx, ny, tol=1e-6, maxit=20000, variant=variant, precision=FX)
    xo, _, ro = cg_fixed(b, nx, ny, variant=variant, tol=1e-6, maxit=20000)
    check_same(rc, res, x, ro, xo)


@pytest.mark.parametrize("variant", VARIANTS)
def test_edge_cases(ctx, variant):
    nx, ny = 45, 38
    rng = np.random.default_rng(9)
    b = rng.uniform(-1, 1, (ny, nx))
    cases = {
        "zero rhs": (np.zeros_like(b), np.ones_like(b), 1e-6, 50),
        "rhs below half a quantum": (np.full_like(b, 2.0 ** -32), None, 1e-6, 50),
        "saturating rhs": (rng.uniform(-6e5, 6e5, (ny, nx)), None, 1e-6, 30),
        "saturating start": (b, rng.uniform(-1e6, 1e6, (ny, nx)), 1e-3, 30),
        "non-finite entries": (np.where(rng.random((ny, nx)) < 0.1, np.nan, b), None, 1e-6, 500),
        "infinite entries": (np.where(rng.random((ny, nx)) < 0.05, -np.inf, b), None, 1e-6, 30),
        "ties in the input": (np.round(b * 8) / 8 + 2.0 ** -31, None, 1e-6, 500),
        "maxit reached": (b, None, 1e-9, 5),
        "warm start": (b, rng.uniform(-1, 1, (ny, nx)), 1e-6, 500),
    }
    for name, (bb, x0, tol, maxit) in cases.items():
        say("fixed edge case:", name, "variant", variant)
        x = np.zeros_like(bb)
        rc, res = ctx.solve(bb, x, nx, ny, x0=x0, tol=tol, maxit=maxit, variant=variant,
                            precision=FX)
        xo, _, ro = cg_fixed(bb, nx, ny, variant=variant, tol=tol, maxit=maxit, x0=x0)
        check_same(rc, res, x, ro, xo)
    # warm start aliasing x
    x0 = rng.uniform(-1, 1, (ny, nx))
    x = x0.copy()
    rc, res = ctx.solve(b, x, nx, ny, x0=x, tol=1e-6, maxit=500, variant=variant, precision=FX)
    xo, _, ro = cg_fixed(b, nx, ny, variant=variant, tol=1e-6, maxit=500, x0=x0)
    check_same(rc, res, x, ro, xo)


@pytest.mark.parametrize("variant", VARIANTS)
def test_breakdown_when_rounding_zeroes_the_curvature(ctx, variant):
    n = 10
    s = np.sin(np.pi * np.arange(1, n + 1) / (n + 1))
    b = 0.9 * 2.0 ** -15 * np.outer(s, s)
    x = np.full_like(b, 5.0)
    rc, res = ctx.solve(b, x, n, n, tol=0.0, maxit=5, variant=variant, precision=FX)
    xo, _, ro = cg_fixed(b, n, n, variant=variant, tol=0.0, maxit=5)
    check_same(rc, res, x, ro, xo)
    assert rc == cg.CG_BREAKDOWN and res.iterations == 0 and not x.any()


def test_device_memory_and_torch_tensors(ctx, torch):
    n = 40
    b = workloads.fixed_rhs(n, 3)
    bd = torch.from_numpy(b).to("cuda:0")
    for variant in VARIANTS:
        x = torch.zeros_like(bd)
        rc, res = ctx.solve(bd, x, n, n, tol=1e-6, maxit=1000, variant=variant, precision=FX)
        xo, _, ro = cg_fixed(b, n, n, variant=variant, tol=1e-6, maxit=1000)
        check_same(rc, res, x.cpu().numpy(), ro, xo)


def test_batch_mixed_with_fp64(ctx):
    """Fixed-point solves run one work-group each beside the step engine's
    FP64 solves; every fixed result equals the oracle's bitwise, every FP64
    result equals its solve alone."""
    rng = np.random.default_rng(31)
    specs = []
    for k, n in enumerate((16, 100, 32, 40, 100, 7)):
        specs.append(("fixed", n, n, k % 2))
    for k, (nx, ny) in enumerate(((300, 200), (100, 100), (64, 1024))):
        specs.append(("fp64", nx, ny, k % 2))
    probs, xs, bs = [], [], []
    for kind, nx, ny, variant in specs:
        b = rng.uniform(-1, 1, (ny, nx))
        x = np.zeros_like(b)
        prec = FX if kind == "fixed" else cg.CG_PREC_FP64
        tol = 1e-6 if kind == "fixed" else 1e-8
        probs.append(cg.make_problem(b, x, nx, ny, tol=tol, maxit=20000, variant=variant,
                                     precision=prec))
        bs.append(b)
        xs.append(x)
    say("fixed batch mixed with FP64", len(specs))
    rc, results = ctx.cg_solve_batch(probs)
    for (kind, nx, ny, variant), b, x, r in zip(specs, bs, xs, results):
        if kind == "fixed":
            xo, _, ro = cg_fixed(b, nx, ny, variant=variant, tol=1e-6, maxit=20000)
            check_same(r.status, r, x, ro, xo)
        else:
            xa = np.zeros_like(b)
            rca, ra = ctx.solve(b, xa, nx, ny, tol=1e-8, maxit=20000, variant=variant)
            assert r.status == rca and r.iterations == ra.iterations
            np.testing.assert_array_equal(x, xa)


def test_batch_every_compiled_size(ctx):
    """One launch per (variant, unknowns per thread) group inside a batch:
    every group size, both variants, each result the oracle's."""
    rng = np.random.default_rng(77)
    specs = [(n, v) for n in (7, 40, 50, 60, 75, 90, 100) for v in VARIANTS]
    rng.shuffle(specs)
    bs = [rng.uniform(-1, 1, (n, n)) for n, _ in specs]
    xs = [np.zeros_like(b) for b in bs]
    probs = [cg.make_problem(b, x, n, n, tol=1e-6, maxit=3000, variant=v, precision=FX)
             for (n, v), b, x in zip(specs, bs, xs)]
    say("fixed batch, every size", len(specs))
    rc, results = ctx.cg_solve_batch(probs)
    for (n, v), b, x, r in zip(specs, bs, xs, results):
        xo, _, ro = cg_fixed(b, n, n, variant=v, tol=1e-6, maxit=3000)
        check_same(r.status, r, x, ro, xo)


def test_batch_of_the_paper_grid(ctx):
    """Many copies of the largest paper grid at its synthesized iteration
    count, all in one launch: each bitwise the oracle's."""
    n, iters = 100, 120
    count = 24
    bs = [workloads.fixed_rhs(n, m) for m in range(count)]
    xs = [np.zeros_like(b) for b in bs]
    probs = [cg.make_problem(b, x, n, n, tol=0.0, maxit=iters, variant=m % 2, precision=FX)
             for m, (b, x) in enumerate(zip(bs, xs))]
    say("fixed batch of", count, "paper grids")
    rc, results = ctx.cg_solve_batch(probs)
    assert rc == cg.CG_OK
    for m, (b, x, r) in enumerate(zip(bs, xs, results)):
        xo, _, ro = cg_fixed(b, n, n, variant=m % 2, tol=0.0, maxit=iters)
        check_same(r.status, r, x, ro, xo)


def test_serving_queue(torch):
    with cg.Context(device=0, arena_bytes=256 << 20) as c:
        reqs = []
        for m, n in enumerate((16, 32, 40, 100, 100, 16)):
            b = workloads.fixed_rhs(n, 50 + m)
            x = np.zeros_like(b)
            t = c.cg_submit(cg.make_problem(b, x, n, n, tol=1e-6, maxit=5000, variant=m % 2,
                                            precision=FX))
            reqs.append((t, b, x, n, m % 2))
        say("fixed serving", len(reqs))
        for t, b, x, n, variant in reqs:
            rc, res = _poll(c, t)
            xo, _, ro = cg_fixed(b, n, n, variant=variant, tol=1e-6, maxit=5000)
            check_same(rc, res, x, ro, xo)


def _poll(c, t):
    import time
    t0 = time.time()
    while True:
        rc, res = c.cg_poll(t)
        if rc != cg.CG_PENDING:
            return rc, res
        assert time.time() - t0 < 60, "request not finished within a minute"
        time.sleep(0.002)


@pytest.mark.parametrize("variant", VARIANTS)
def test_huge_step_takes_the_general_update_form(ctx, variant):
    """A smooth right-hand side whose curvature (p, A p) rounds to a few
    quanta: the first alpha exceeds 2^13 (updates by the general 128-bit-free
    form with saturation checks), and the iterates saturate.  Bitwise against
    the oracle, a few iterations and a natural stop."""
    from oracle.oracle import fx_div, fx_dot, fx_quantize, fx_spmv
    nx, ny = 127, 78
    i, j = np.arange(1, nx + 1), np.arange(1, ny + 1)
    b = 4.635057289939733e-4 * np.outer(np.sin(np.pi * j / (ny + 1)), np.sin(np.pi * i / (nx + 1)))
    bq = np.vectorize(fx_quantize)(b).astype(np.int64)
    alpha = fx_div(fx_dot(bq, bq), fx_dot(bq, fx_spmv(bq, nx, ny)))
    assert alpha >= 2 ** 43, alpha
    for tol, maxit in ((0.0, 1), (0.0, 3), (1e-6, 200)):
        say("fixed general form", variant, tol, maxit)
        x = np.zeros_like(b)
        rc, res = ctx.solve(b, x, nx, ny, tol=tol, maxit=maxit, variant=variant, precision=FX)
        xo, _, ro = cg_fixed(b, nx, ny, variant=variant, tol=tol, maxit=maxit)
        check_same(rc, res, x, ro, xo)
