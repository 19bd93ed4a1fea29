"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Parity bar (FP64): relative solution error <= 1e-10 and iteration counts
within +-2 against the oracle; against the oracle's canonical order (the
library's documented arithmetic contract) the iterates are expected to be
bitwise identical, which is asserted too.  Stencil and dot products are
compared element by element.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import MODE_CANONICAL, MODE_SEQUENTIAL
from paper_1803_03797_amd import cg, workloads

pytestmark = pytest.mark.gpu

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
    c = cg.Context(device=0, arena_bytes=6 << 30)
    yield c
    c.close()


def order_of(ctx, nx, ny, variant=0):
    """The reduction order a solve of this shape uses, and the plan."""
    info = ctx.cg_plan(nx, ny, variant)
    if info.path == 2:
        return oracle.Order.segments(info.seg_rows, info.lanes, info.seg_waves, info.seg_cols), info
    return tile_order(info), info


def tile_order(info):
    """The tile order of the shape (cg_dot and cg_apply use it on every path)."""
    return oracle.Order(info.cols_per_lane, info.lanes, info.waves, info.rows, info.threads2,
                        alt=info.walk_alt)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb else 1.0)


def mode(nx, ny, a, b):
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    return np.sin(a * np.pi * (i + 1) / (nx + 1)) * np.sin(b * np.pi * (j + 1) / (ny + 1))


def mode_eig(nx, ny, a, b):
    return 4 - 2 * math.cos(a * math.pi / (nx + 1)) - 2 * math.cos(b * math.pi / (ny + 1))


GRIDS = [(1, 1), (1, 9), (9, 1), (3, 5), (127, 3), (129, 67), (300, 200), (513, 257)]


@pytest.mark.parametrize("nx,ny", GRIDS)
def test_stencil_matches_oracle_bitwise(ctx, torch, nx, ny):
    say("stencil", nx, ny)
    u = np.random.default_rng(nx * 7 + ny).standard_normal((ny, nx))
    y = np.zeros_like(u)
    ctx.cg_apply(u, y, nx, ny)
    want = oracle.spmv(u, nx, ny, order=1)  # centre, west, east, south, north
    np.testing.assert_array_equal(y, want)
    # device memory path
    ud = torch.from_numpy(u).cuda()
    yd = torch.zeros_like(ud)
    ctx.cg_apply(ud, yd, nx, ny)
    np.testing.assert_array_equal(yd.cpu().numpy(), want)


@pytest.mark.parametrize("nx,ny", GRIDS + [(1000, 1000)])
def test_dot_matches_canonical_order(ctx, nx, ny):
    say("dot", nx, ny)
    rng = np.random.default_rng(nx + 13 * ny)
    a = rng.standard_normal((ny, nx))
    b = rng.standard_normal((ny, nx))
    o = tile_order(ctx.cg_plan(nx, ny))
    got = ctx.cg_dot(a, b, nx, ny)
    assert got == oracle.dot(a, b, nx, ny, MODE_CANONICAL, o)
    exact = math.fsum((a * b).ravel())
    assert abs(got - exact) <= 1e-13 * float(np.sum(np.abs(a * b)))
    # integer data: exact
    ai = rng.integers(-9, 10, (ny, nx)).astype(float)
    bi = rng.integers(-9, 10, (ny, nx)).astype(float)
    assert ctx.cg_dot(ai, bi, nx, ny) == float(np.sum(ai.astype(np.int64) * bi.astype(np.int64)))


def test_dot_deterministic(ctx):
    nx, ny = 2048, 1536
    say("dot determinism", nx, ny)
    rng = np.random.default_rng(5)
    a = rng.standard_normal((ny, nx))
    b = rng.standard_normal((ny, nx))
    vals = {ctx.cg_dot(a, b, nx, ny) for _ in range(5)}
    assert len(vals) == 1


@pytest.mark.parametrize("nx,ny", [(300, 200), (129, 67), (513, 130), (200, 300)])
@pytest.mark.parametrize("variant", VARIANTS)
def test_lockstep_bitwise_vs_canonical(ctx, nx, ny, variant):
    """tol = 0: exactly m iterations; the library must reproduce the oracle's
    canonical-order iterates."""
    rng = np.random.default_rng(nx * ny + variant)
    b = rng.uniform(-1, 1, (ny, nx))
    o, info = order_of(ctx, nx, ny, variant)
    for m in (1, 2, 7, 40):
        say("lockstep", nx, ny, "variant", variant, "m", m, "path", info.path)
        x = np.zeros_like(b)
        rc, res = ctx.solve(b, x, nx, ny, tol=0.0, maxit=m, variant=variant)
        xo, ro = oracle.cg(b, nx, ny, variant=variant, tol=0.0, maxit=m, mode=MODE_CANONICAL,
                           order=o)
        assert rc == cg.CG_OK and res.iterations == ro.iterations == m
        assert rel(x, xo) <= 1e-10
        np.testing.assert_array_equal(x, xo)
        assert res.rel_res_recursive == pytest.approx(ro.rel_res_recursive, rel=0, abs=0)
        assert res.rel_res_true == ro.rel_res_true


@pytest.mark.parametrize("nx,ny", [(100, 100), (300, 200), (77, 250), (640, 128)])
@pytest.mark.parametrize("variant", VARIANTS)
def test_natural_stop(ctx, nx, ny, variant):
    rng = np.random.default_rng(1000 + nx + ny)
    b = rng.uniform(-1, 1, (ny, nx))
    o, info = order_of(ctx, nx, ny, variant)
    say("natural stop", nx, ny, "variant", variant, "path", info.path)
    x = np.zeros_like(b)
    rc, res = ctx.solve(b, x, nx, ny, tol=1e-8, maxit=5000, variant=variant)
    xk, rk = oracle.cg(b, nx, ny, variant=variant, tol=1e-8, maxit=5000, mode=MODE_CANONICAL,
                       order=o)
    xs, rs = oracle.cg(b, nx, ny, variant=variant, tol=1e-8, maxit=5000, mode=MODE_SEQUENTIAL)
    assert rc == cg.CG_OK and res.rel_res_recursive <= 1e-8
    assert res.iterations == rk.iterations
    assert abs(res.iterations - rs.iterations) <= 2
    assert rel(x, xk) <= 1e-10
    np.testing.assert_array_equal(x, xk)
    # the sequential-order spread is a property of FP64 CG itself; report it
    say("  iters", res.iterations, "seq", rs.iterations, "spread vs sequential %.2e" % rel(x, xs))
    assert rel(x, xs) <= (1e-12 if variant == 0 else 1e-8)


@pytest.mark.parametrize("variant", VARIANTS)
def test_small_workload_device_memory(ctx, torch, variant):
    """The 100x100 workload through device pointers (on-chip solver)."""
    nx, ny = workloads.SMALL["nx"], workloads.SMALL["ny"]
    b = workloads.small_problem()
    say("small workload device", variant)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    rc, res = ctx.solve(bd, xd, nx, ny, tol=1e-8, maxit=2000, variant=variant)
    o, info = order_of(ctx, nx, ny, variant)
    assert info.path == 2 and info.seg_rows * info.seg_waves * info.lanes >= nx * ny
    xk, rk = oracle.cg(b, nx, ny, variant=variant, tol=1e-8, maxit=2000, mode=MODE_CANONICAL,
                       order=o)
    xs, rs = oracle.cg(b, nx, ny, variant=variant, tol=1e-8, maxit=2000)
    x = xd.cpu().numpy()
    assert rc == cg.CG_OK and res.iterations == rk.iterations
    assert abs(res.iterations - rs.iterations) <= 2
    np.testing.assert_array_equal(x, xk)
    assert rel(x, xs) <= 1e-10


# ----------------------------------------------------------- edge cases --

@pytest.mark.parametrize("nx,ny", [(5, 4), (300, 200)])
@pytest.mark.parametrize("variant", VARIANTS)
def test_zero_rhs(ctx, nx, ny, variant):
    say("zero rhs", nx, ny, variant)
    b = np.zeros((ny, nx))
    x = np.full((ny, nx), 7.0)
    x0 = np.ones((ny, nx))
    rc, res = ctx.solve(b, x, nx, ny, x0=x0, variant=variant)
    assert rc == cg.CG_OK and res.iterations == 0 and not x.any()


@pytest.mark.parametrize("nx,ny", [(30, 20), (300, 200)])
@pytest.mark.parametrize("variant", VARIANTS)
def test_maxit_and_nonfinite(ctx, nx, ny, variant):
    say("maxit/nonfinite", nx, ny, variant)
    b = np.random.default_rng(3).uniform(-1, 1, (ny, nx))
    x = np.zeros_like(b)
    rc, res = ctx.solve(b, x, nx, ny, tol=1e-12, maxit=7, variant=variant)
    assert rc == cg.CG_NOT_CONVERGED and res.iterations == 7
    b2 = b.copy()
    b2[ny // 2, nx // 3] = np.nan
    rc, res = ctx.solve(b2, x, nx, ny, variant=variant)
    assert rc == cg.CG_BREAKDOWN and res.iterations == 0


@pytest.mark.parametrize("nx,ny", [(40, 30), (300, 200)])
@pytest.mark.parametrize("variant", VARIANTS)
def test_warm_start_and_alias(ctx, nx, ny, variant):
    """x0 given (and aliasing x): continuing from a partial solve."""
    say("warm start", nx, ny, variant)
    b = np.random.default_rng(8).uniform(-1, 1, (ny, nx))
    o, _ = order_of(ctx, nx, ny, variant)
    x0 = np.random.default_rng(9).uniform(-1, 1, (ny, nx))
    x = x0.copy()
    rc, res = ctx.solve(b, x, nx, ny, x0=x, tol=1e-9, maxit=5000, variant=variant)
    xo, ro = oracle.cg(b, nx, ny, variant=variant, tol=1e-9, maxit=5000, x0=x0,
                       mode=MODE_CANONICAL, order=o)
    assert rc == cg.CG_OK and res.iterations == ro.iterations
    np.testing.assert_array_equal(x, xo)


@pytest.mark.parametrize("variant", VARIANTS)
def test_single_eigenvector_full_size(ctx, torch, variant):
    """4096 x 4096: b = one grid mode -> one iteration, x = b / lambda."""
    nx = ny = 4096
    say("eigenvector 4096^2", variant)
    # a mode with an O(1) eigenvalue: low modes (lambda ~ 1e-5) lose ~1e-11 of
    # relative accuracy to the stencil's cancellation, more than tol allows
    phi = mode(nx, ny, 2048, 1365)
    lam = mode_eig(nx, ny, 2048, 1365)
    bd = torch.from_numpy(phi).cuda()
    xd = torch.zeros_like(bd)
    rc, res = ctx.solve(bd, xd, nx, ny, tol=1e-12, maxit=50, variant=variant)
    assert rc == cg.CG_OK and res.iterations == 1
    err = (xd - bd / lam).abs().max().item()
    assert err <= 1e-13


@pytest.mark.parametrize("variant", VARIANTS)
def test_finite_termination_full_size(ctx, torch, variant):
    """4096 x 4096: b spanning 4 modes with distinct eigenvalues -> 4 (or 5)
    iterations and the closed-form solution."""
    nx = ny = 4096
    say("finite termination 4096^2", variant)
    modes = [(1000, 1000), (2048, 100), (3000, 3500), (500, 2500)]  # lambda 1.1 .. 7.1
    coef = [1.0, -0.5, 0.25, 0.125]
    b = sum(c * mode(nx, ny, a, bb) for c, (a, bb) in zip(coef, modes))
    want = sum(c / mode_eig(nx, ny, a, bb) * mode(nx, ny, a, bb) for c, (a, bb) in zip(coef, modes))
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    rc, res = ctx.solve(bd, xd, nx, ny, tol=1e-10, maxit=100, variant=variant)
    assert rc == cg.CG_OK and res.iterations in (4, 5)
    assert (xd.cpu() - torch.from_numpy(want)).abs().max().item() <= 1e-9


@pytest.mark.parametrize("variant", VARIANTS)
def test_full_size_lockstep_sampled(ctx, torch, variant):
    """The 4096 x 4096 workload (b = A x*), 3 iterations in the launch
    configuration the benchmark uses, against the canonical oracle."""
    nx = ny = 4096
    say("4096^2 lockstep 3 iterations", variant)
    xs = workloads.large_solution(nx, ny)
    b = oracle.spmv(xs, nx, ny, order=0)
    o, info = order_of(ctx, nx, ny, variant)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    rc, res = ctx.solve(bd, xd, nx, ny, tol=0.0, maxit=3, variant=variant)
    xo, ro = oracle.cg(b, nx, ny, variant=variant, tol=0.0, maxit=3, mode=MODE_CANONICAL, order=o)
    assert rc == cg.CG_OK and res.iterations == 3
    x = xd.cpu().numpy()
    assert rel(x, xo) <= 1e-10
    np.testing.assert_array_equal(x, xo)


@pytest.mark.parametrize("variant", VARIANTS)
def test_full_size_lockstep_across_graph_chunks(ctx, torch, variant):
    """The 4096 x 4096 workload for 70 iterations: more than two captured
    chunks of iterations (the benchmark replays chunks of 32), a ragged last
    chunk and an even stop (deferred x applied by the stopping pass), bitwise
    against the canonical oracle."""
    nx = ny = 4096
    m = 70
    say("4096^2 lockstep %d iterations" % m, variant)
    xs = workloads.large_solution(nx, ny)
    b = oracle.spmv(xs, nx, ny, order=0)
    o, info = order_of(ctx, nx, ny, variant)
    assert info.path == 0
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    rc, res = ctx.solve(bd, xd, nx, ny, tol=0.0, maxit=m, variant=variant)
    xo, ro = oracle.cg(b, nx, ny, variant=variant, tol=0.0, maxit=m, mode=MODE_CANONICAL, order=o)
    assert rc == cg.CG_OK and res.iterations == ro.iterations == m
    np.testing.assert_array_equal(xd.cpu().numpy(), xo)
    assert res.rel_res_recursive == ro.rel_res_recursive
    assert res.rel_res_true == ro.rel_res_true


@pytest.mark.parametrize("variant", VARIANTS)
def test_huge_grid_lockstep_bitwise(torch, variant):
    """8192 x 8192 (the refinement workload's grid and right-hand side), 4
    iterations in the plan solves of that size take (pipelined: two work-groups
    per CU, interleaved rows), in both tile-walk directions and with the
    deferred x of an even stop: bitwise against the canonical oracle."""
    n = workloads.HUGE["nx"]
    m = 4
    b = workloads.huge_rhs(n, n)
    with cg.Context(device=0, arena_bytes=(72 * n * n) + (1 << 30)) as c:
        o, info = order_of(c, n, n, variant)
        say("8192^2 lockstep %d iterations variant %d: rows %d grid %d tiles %d" %
            (m, variant, info.rows, info.grid, info.tiles))
        assert info.path == 0
        bd = torch.from_numpy(b).cuda()
        xd = torch.zeros_like(bd)
        rc, res = c.solve(bd, xd, n, n, tol=0.0, maxit=m, variant=variant)
        x = xd.cpu().numpy()
        del bd, xd
    xo, ro = oracle.cg(b, n, n, variant=variant, tol=0.0, maxit=m, mode=MODE_CANONICAL, order=o)
    assert rc == cg.CG_OK and res.iterations == ro.iterations == m
    np.testing.assert_array_equal(x, xo)
    assert res.rel_res_recursive == ro.rel_res_recursive
    assert res.rel_res_true == ro.rel_res_true


# ----------------------------------------------------------- refinement --

@pytest.mark.parametrize("nx,ny", [(256, 256), (300, 190)])
def test_refinement_parity(ctx, nx, ny):
    say("refinement", nx, ny)
    b = np.random.default_rng(31).standard_normal((ny, nx))
    x = np.zeros_like(b)
    rc, res = ctx.solve(b, x, nx, ny, tol=1e-10, maxit=200000,
                        precision=cg.CG_PREC_FP32_REFINED, inner_tol=1e-4)
    xo, ro = oracle.cg(b, nx, ny, tol=1e-10, maxit=200000)
    xr, rr = oracle.refine(b, nx, ny, tol=1e-10, inner_tol=1e-4)
    say("  refined outer %d inner %d (oracle refine %d/%d, fp64 %d); err vs fp64 %.2e"
        % (res.outer_iterations, res.iterations, rr.outer_iterations, rr.iterations,
           ro.iterations, rel(x, xo)))
    assert rc == cg.CG_OK
    assert res.rel_res_true <= 1e-10
    assert rel(x, xo) <= 1e-9
    assert abs(res.outer_iterations - rr.outer_iterations) <= 1


def test_refinement_parity_1024(ctx):
    """FP32-refined to a true relative residual of 1e-10 on 1024 x 1024 (b ~
    N(0,1), inner tol 1e-4): within 1e-9 of the FP64 oracle's solution at the
    same tolerance."""
    n = 1024
    say("refinement 1024^2")
    b = np.random.default_rng(1024).standard_normal((n, n))
    x = np.zeros_like(b)
    rc, res = ctx.solve(b, x, n, n, tol=1e-10, maxit=200000, precision=cg.CG_PREC_FP32_REFINED,
                        inner_tol=1e-4)
    xo, ro = oracle.cg(b, n, n, tol=1e-10, maxit=200000)
    err = rel(x, xo)
    say("  refined outer %d inner %d, fp64 oracle %d iterations; err vs fp64 oracle %.2e"
        % (res.outer_iterations, res.iterations, ro.iterations, err))
    assert rc == cg.CG_OK and ro.status == 0
    assert res.rel_res_true <= 1e-10
    assert err <= 1e-9
