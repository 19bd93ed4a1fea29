"""GPU parity of residual replacement in the pipelined CG (cg_problem.rr_period):
every rr_period iterations the library recomputes q = A p, z = A q (stencil
passes), r = b - A x and w = A r (the initial-residual passes, with their
sums), bitwise the oracle's pipelined CG with the same replacement in the
library's order, on the 5-point and the variable-coefficient operators,
alone, in batches and served."""
import sys

import numpy as np
import pytest

import oracle
from oracle import MODE_CANONICAL
from paper_1803_03797_amd import cg, workloads

pytestmark = pytest.mark.gpu
PIPE = cg.CG_VARIANT_PIPELINED


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


def order(ctx, nx, ny, vc=False):
    info = ctx.cg_plan(nx, ny, PIPE, vc=vc, rr_period=2)
    assert info.path == 0
    return oracle.Order(info.cols_per_lane, info.lanes, info.waves, info.rows, info.threads2,
                        alt=info.walk_alt)


@pytest.mark.parametrize("nx,ny", [(300, 200), (129, 67), (513, 257), (40, 30), (1, 77)])
@pytest.mark.parametrize("period", [2, 4, 10])
def test_lockstep_bitwise(ctx, nx, ny, period):
    """Small grids too (they take the multi-work-group passes when replacing)."""
    b = np.random.default_rng(nx + ny + period).uniform(-1, 1, (ny, nx))
    o = order(ctx, nx, ny)
    for m in (1, 6, 40, 71):
        say("rr lockstep", nx, ny, "period", period, "m", m)
        x = np.zeros_like(b)
        rc, res = ctx.solve(b, x, nx, ny, tol=0.0, maxit=m, variant=PIPE, rr_period=period)
        xo, ro = oracle.cg(b, nx, ny, variant=PIPE, tol=0.0, maxit=m, mode=MODE_CANONICAL,
                           order=o, rr_period=period)
        # past convergence (the 77-unknown column converges in fewer than 40
        # iterations) a run with tol = 0 ends in a breakdown on both sides
        assert rc == ro.status and res.iterations == ro.iterations
        assert ro.status == cg.CG_BREAKDOWN or ro.iterations == m
        np.testing.assert_array_equal(x, xo)
        assert res.rel_res_recursive == ro.rel_res_recursive
        assert res.rel_res_true == ro.rel_res_true


def test_variable_coefficient_attainable_accuracy(ctx, torch):
    """256 x 256 variable coefficients, tol 1e-12: plain pipelined CG breaks
    down; with replacement every 50 iterations the solve converges to a true
    residual of tol, bitwise the oracle's replaced run in the library's order."""
    n, tol = 256, 1e-12
    kx, ky = workloads.vc_faces(n, n)
    b = workloads.vc_rhs(n, n)
    o = order(ctx, n, n, vc=True)
    say("vc 256^2 tol 1e-12: plain and replaced")
    x = np.zeros_like(b)
    rc0, r0 = ctx.solve(b, x, n, n, tol=tol, maxit=60000, variant=PIPE,
                        kx=kx, ky=ky)
    assert rc0 != cg.CG_OK or r0.rel_res_true > 100 * tol
    x = np.zeros_like(b)
    rc, r = ctx.solve(b, x, n, n, tol=tol, maxit=60000, variant=PIPE, kx=kx, ky=ky, rr_period=50)
    xo, ro = oracle.cg_vc(b, n, n, kx, ky, variant=PIPE, tol=tol, maxit=60000,
                          mode=MODE_CANONICAL, order=o, rr_period=50)
    say("  replaced: %d iterations, true residual %.2e (oracle %d)" %
        (r.iterations, r.rel_res_true, ro.iterations))
    assert rc == cg.CG_OK and r.iterations == ro.iterations
    assert r.rel_res_true <= 1.5 * tol
    np.testing.assert_array_equal(x, xo)


def test_full_size_lockstep(ctx, torch):
    """The 4096 x 4096 workload, 40 iterations with a replacement every 8
    (five replacements, two graph chunks), bitwise against the oracle."""
    n, m, period = 4096, 40, 8
    xs = workloads.large_solution(n, n)
    b = oracle.spmv(xs, n, n, order=0)
    o = order(ctx, n, n)
    say("4096^2 rr lockstep")
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    rc, res = ctx.solve(bd, xd, n, n, tol=0.0, maxit=m, variant=PIPE, rr_period=period)
    xo, ro = oracle.cg(b, n, n, variant=PIPE, tol=0.0, maxit=m, mode=MODE_CANONICAL, order=o,
                       rr_period=period)
    assert rc == cg.CG_OK and res.iterations == m
    np.testing.assert_array_equal(xd.cpu().numpy(), xo)


def test_batch_and_served_with_replacement_match_alone(ctx):
    """Pipelined solves with residual replacement (both operators, periods 2 to
    50, a single column among them) beside plain ones, batched and served on
    the step engine: each result bitwise the solve alone, and the replaced
    ones bitwise the oracle's replaced run in the library's order."""
    import time
    rng = np.random.default_rng(61)
    # (nx, ny, rr_period, variable coefficients)
    mix = [(300, 200, 4, False), (129, 67, 0, False), (513, 257, 10, False),
           (256, 256, 50, True), (100, 100, 2, False), (40, 30, 6, True), (1, 77, 4, False),
           (64, 64, 0, True)]
    bs = [rng.uniform(-1, 1, (ny, nx)) for nx, ny, _, _ in mix]
    ks = [workloads.vc_faces(nx, ny) if vc else (None, None) for nx, ny, _, vc in mix]

    def prob(k, x):
        nx, ny, per, vc = mix[k]
        return cg.make_problem(bs[k], x, nx, ny, tol=1e-10, maxit=20000, variant=PIPE,
                               rr_period=per, kx=ks[k][0], ky=ks[k][1])
    xb = [np.zeros_like(b) for b in bs]
    say("batch with residual replacement:", len(mix))
    rc, res = ctx.cg_solve_batch([prob(k, x) for k, x in enumerate(xb)])
    xv = [np.zeros_like(b) for b in bs]
    tickets = [ctx.cg_submit(prob(k, x)) for k, x in enumerate(xv)]
    served = {}
    deadline = time.time() + 120
    while len(served) < len(tickets) and time.time() < deadline:
        for t in tickets:
            if t not in served:
                rc2, r2 = ctx.cg_poll(t)
                if rc2 != cg.CG_PENDING:
                    served[t] = (rc2, cg.cg_result.from_buffer_copy(r2))
        time.sleep(0.001)
    assert len(served) == len(tickets)
    for k, (nx, ny, per, vc) in enumerate(mix):
        xa = np.zeros_like(bs[k])
        rca, ra = ctx.cg_solve(prob(k, xa))
        rcs, rs = served[tickets[k]]
        say("  %dx%d rr %d vc %d: batch %d served %d alone %d iterations (status %d)" %
            (nx, ny, per, vc, res[k].iterations, rs.iterations, ra.iterations, rca))
        assert res[k].status == rca == rcs
        assert res[k].iterations == rs.iterations == ra.iterations
        np.testing.assert_array_equal(xb[k], xa)
        np.testing.assert_array_equal(xv[k], xa)
        assert res[k].rel_res_true == rs.rel_res_true == ra.rel_res_true
        if per:
            o = order(ctx, nx, ny, vc=vc)
            if vc:
                xo, ro = oracle.cg_vc(bs[k], nx, ny, ks[k][0], ks[k][1], variant=PIPE, tol=1e-10,
                                      maxit=20000, mode=MODE_CANONICAL, order=o, rr_period=per)
            else:
                xo, ro = oracle.cg(bs[k], nx, ny, variant=PIPE, tol=1e-10, maxit=20000,
                                   mode=MODE_CANONICAL, order=o, rr_period=per)
            assert ro.status == rca and ro.iterations == ra.iterations
            np.testing.assert_array_equal(xa, xo)


def test_batch_fixed_iterations_ending_on_a_replacement(ctx):
    """tol = 0 runs whose last iteration is a replacement point (maxit a
    multiple of the period) or not: batched, each equals its solve alone in x,
    status, iterations and both residuals (the recursive one comes from the
    replaced r when the replacement follows the last iteration)."""
    rng = np.random.default_rng(67)
    # (nx, ny, rr_period, maxit)
    mix = [(300, 200, 4, 40), (129, 67, 10, 71), (40, 30, 2, 6), (513, 257, 10, 40),
           (1, 77, 4, 8)]
    bs = [rng.uniform(-1, 1, (ny, nx)) for nx, ny, _, _ in mix]

    def prob(k, x):
        nx, ny, per, m = mix[k]
        return cg.make_problem(bs[k], x, nx, ny, tol=0.0, maxit=m, variant=PIPE, rr_period=per)
    xb = [np.zeros_like(b) for b in bs]
    say("batch of fixed-iteration replaced solves:", len(mix))
    rc, res = ctx.cg_solve_batch([prob(k, x) for k, x in enumerate(xb)])
    for k, (nx, ny, per, m) in enumerate(mix):
        xa = np.zeros_like(bs[k])
        rca, ra = ctx.cg_solve(prob(k, xa))
        say("  %dx%d rr %d maxit %d: batch %d alone %d (status %d)" %
            (nx, ny, per, m, res[k].iterations, ra.iterations, rca))
        assert res[k].status == rca and res[k].iterations == ra.iterations
        np.testing.assert_array_equal(xb[k], xa)
        assert res[k].rel_res_recursive == ra.rel_res_recursive
        assert res[k].rel_res_true == ra.rel_res_true


def test_rejections(ctx):
    b = np.ones((20, 30))
    x = np.zeros_like(b)
    for kw in (dict(rr_period=3), dict(rr_period=-2), dict(rr_period=4, variant=0),
               dict(rr_period=4, variant=PIPE, precision=cg.CG_PREC_FP32_REFINED),
               dict(rr_period=4, variant=PIPE, precond=2)):
        with pytest.raises(cg.CGError):
            ctx.solve(b, x, 30, 20, **kw)
        with pytest.raises(cg.CGError):
            ctx.cg_solve_batch([cg.make_problem(b, x, 30, 20, **kw)])
        with pytest.raises(cg.CGError):
            ctx.cg_submit(cg.make_problem(b, x, 30, 20, **kw))
