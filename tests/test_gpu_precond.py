"""GPU parity of Chebyshev-preconditioned CG (cg_problem.precond = s), against
the oracle's preconditioned CG in the library's tile order (bitwise) and in
the textbook order (FP64 tolerance):
- classic: the Chebyshev pass (stop test, z = p_s(A) r, partials of (r,z))
  plus the two classic passes;
- pipelined: the Chebyshev pass m = p_s(A) w after the scalar step, plus the
  fused pass n = A m with the eight updates and the sums (r,u), (w,u), (r,r)."""
import sys

import numpy as np
import pytest

import oracle
from oracle import MODE_CANONICAL, MODE_SEQUENTIAL
from paper_1803_03797_amd import cg

pytestmark = pytest.mark.gpu

# one tile, ragged tiles, single rows / columns, grids that would otherwise
# take the on-chip or single-work-group solvers, several tile rows
SHAPES = [(1, 1), (2, 2), (64, 1), (1, 300), (100, 100), (130, 70), (300, 190), (513, 257),
          (1024, 1024)]
STEPS = (1, 2, 4, 8)
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
    c = cg.Context(device=0, arena_bytes=2 << 30)
    yield c
    c.close()


def tile_order(ctx, nx, ny, s, variant=cg.CG_VARIANT_CLASSIC):
    """The pass tiles' order, and the order of rho = (r,z): tiles of the
    Chebyshev pass, 128 columns by cheb_rows rows with one wavefront each."""
    info = ctx.cg_plan(nx, ny, variant=variant, precond=s)
    assert info.path == 0 and info.cols_per_lane == 2
    assert info.cheb_rows >= 1 and info.cheb_grid >= 8 and info.cheb_grid % 8 == 0
    assert info.cheb_tiles == (info.pitch // 128) * -(-ny // info.cheb_rows)
    return (oracle.Order(info.cols_per_lane, info.lanes, info.waves, info.rows, info.threads2,
                         alt=info.walk_alt),
            oracle.Order(2, info.lanes, 1, info.cheb_rows, info.threads2))


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb else 1.0)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("s", STEPS)
def test_lockstep_bitwise(ctx, nx, ny, s, variant):
    b = np.random.default_rng(nx * 13 + ny + s).uniform(-1, 1, (ny, nx))
    o, orho = tile_order(ctx, nx, ny, s, variant)
    for m in (1, 2, 7):
        say("precond lockstep", nx, ny, "s", s, "variant", variant, "maxit", m)
        x = np.zeros_like(b)
        rc, res = ctx.solve(b, x, nx, ny, tol=0.0, maxit=m, precond=s, variant=variant)
        xo, ro = oracle.pcg(b, nx, ny, s, tol=0.0, maxit=m, mode=MODE_CANONICAL, order=o,
                            order_rho=orho, variant=variant)
        assert rc == ro.status and res.iterations == ro.iterations
        np.testing.assert_array_equal(x, xo)
        assert res.rel_res_recursive == ro.rel_res_recursive
        assert res.rel_res_true == ro.rel_res_true


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("nx,ny", [(100, 100), (300, 190), (513, 257)])
@pytest.mark.parametrize("s", [2, 4, 8])
def test_natural_stop(ctx, nx, ny, s, variant):
    b = np.random.default_rng(3 * nx + ny).uniform(-1, 1, (ny, nx))
    o, orho = tile_order(ctx, nx, ny, s, variant)
    say("precond natural stop", nx, ny, "s", s, "variant", variant)
    x = np.zeros_like(b)
    rc, res = ctx.solve(b, x, nx, ny, tol=1e-8, maxit=20000, precond=s, variant=variant)
    xk, rk = oracle.pcg(b, nx, ny, s, tol=1e-8, maxit=20000, mode=MODE_CANONICAL, order=o,
                        order_rho=orho, variant=variant)
    xs, rs = oracle.pcg(b, nx, ny, s, tol=1e-8, maxit=20000, mode=MODE_SEQUENTIAL,
                        variant=variant)
    assert rc == cg.CG_OK and res.iterations == rk.iterations
    np.testing.assert_array_equal(x, xk)
    assert abs(res.iterations - rs.iterations) <= 2
    say("  iterations %d, textbook-order spread %.2e, true residual %.3g" %
        (res.iterations, rel(x, xs), res.rel_res_true))
    if variant == cg.CG_VARIANT_CLASSIC:
        assert rel(x, xs) <= 1e-10
        assert res.rel_res_true <= 1.2e-8
    else:
        # the pipelined recurrences: the order spread grows with the
        # iterations and the true residual drifts above the recursive one
        # (both reported; the gate is the bitwise canonical parity above)
        assert rel(x, xs) <= 1e-8
        assert res.rel_res_true <= 1e-7


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("s", [2, 8])
def test_full_size_eigenvector(ctx, torch, s, variant):
    """At 4096 x 4096, in the configuration the time-to-solution bench runs: a
    single eigenvector b = phi_ab of A is one of p_s(A) too, so preconditioned
    CG stops after one iteration with x = b / lambda_ab.  (The rounding of
    phi in the other modes comes back amplified by up to kappa(p_s(A) A),
    about 1e6 for the lowest mode at s = 2: the residual after the step is
    about 1e-10, so the stop is tested at the bench's tolerance 1e-8.  The
    error bound: b carries ~4e-16 relative rounding, which A^-1 amplifies by
    up to lambda_ab / lambda_min (1.7e6 for mode (37, 2000)), spread over
    the lowest modes; (p, A p) loses ~8 u / lambda_min / sqrt(n) ~ 1e-13 to
    the stencil's cancellation: 1e-11 covers both.)"""
    n = 4096
    dev = torch.device("cuda:0")
    i = torch.arange(1, n + 1, dtype=torch.float64, device=dev)
    for a_, b_ in ((1, 1), (37, 2000)):
        say("precond full size eigenvector s", s, "variant", variant, "mode", a_, b_)
        # 2 - 2 cos(t) = 4 sin^2(t/2): no cancellation for the lowest modes
        lam = 4 * np.sin(a_ * np.pi / (2 * (n + 1))) ** 2 + 4 * np.sin(b_ * np.pi / (2 * (n + 1))) ** 2
        phi = torch.outer(torch.sin(b_ * np.pi * i / (n + 1)), torch.sin(a_ * np.pi * i / (n + 1)))
        x = torch.zeros_like(phi)
        rc, res = ctx.cg_solve(cg.make_problem(phi, x, n, n, tol=1e-8, maxit=10, precond=s,
                                               variant=variant))
        assert rc == cg.CG_OK and res.iterations == 1, (rc, res.iterations)
        assert res.rel_res_true <= 1e-8
        err = float(torch.linalg.norm(x - phi / lam) / torch.linalg.norm(phi / lam))
        say("  rel err vs b/lambda %.2e" % err)
        assert err <= 1e-11


def test_one_step_is_plain_cg_on_the_gpu(ctx):
    """s = 1 scales r by the scalar 1/theta, under which CG is invariant: the
    preconditioned solve tracks the unpreconditioned one up to rounding (both
    on the tile passes here; bitwise parity with the oracle is checked
    above)."""
    nx, ny = 513, 257
    b = np.random.default_rng(11).uniform(-1, 1, (ny, nx))
    assert ctx.cg_plan(nx, ny).path == 0
    for tol, maxit in ((0.0, 9), (1e-9, 5000)):
        xp = np.zeros_like(b)
        xc = np.zeros_like(b)
        rcp, rp = ctx.solve(b, xp, nx, ny, tol=tol, maxit=maxit, precond=1)
        rcc, rc_ = ctx.solve(b, xc, nx, ny, tol=tol, maxit=maxit)
        assert rcp == rcc and abs(rp.iterations - rc_.iterations) <= 1
        assert np.linalg.norm(xp - xc) <= 1e-10 * np.linalg.norm(xc)


def test_fewer_iterations(ctx):
    n = 512
    b = np.random.default_rng(2).uniform(-1, 1, (n, n))
    x = np.zeros_like(b)
    _, r0 = ctx.solve(b, x, n, n, tol=1e-8, maxit=20000)
    its = {}
    for s in (4, 8):
        x = np.zeros_like(b)
        rc, r = ctx.solve(b, x, n, n, tol=1e-8, maxit=20000, precond=s)
        assert rc == cg.CG_OK and r.rel_res_true <= 1.2e-8
        its[s] = r.iterations
    say("iterations: CG", r0.iterations, "PCG", its)
    assert its[8] <= 0.2 * r0.iterations and its[4] <= 0.35 * r0.iterations


@pytest.mark.parametrize("variant", VARIANTS)
def test_edge_cases(ctx, variant):
    nx, ny, s = 200, 150, 4
    b = np.random.default_rng(4).uniform(-1, 1, (ny, nx))
    o, orho = tile_order(ctx, nx, ny, s, variant)
    kw = dict(precond=s, variant=variant)
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
    x0 = np.random.default_rng(6).uniform(-1, 1, (ny, nx))
    x = x0.copy()
    rc, res = ctx.solve(b, x, nx, ny, x0=x, tol=1e-9, maxit=5000, **kw)
    xo, ro = oracle.pcg(b, nx, ny, s, tol=1e-9, maxit=5000, x0=x0, mode=MODE_CANONICAL,
                        order=o, order_rho=orho, variant=variant)
    assert rc == cg.CG_OK and res.iterations == ro.iterations
    np.testing.assert_array_equal(x, xo)


def test_rejections(ctx):
    b = np.ones((8, 8))
    x = np.zeros_like(b)
    for bad in (9, -1):
        with pytest.raises(cg.CGError):
            ctx.solve(b, x, 8, 8, precond=bad)
    # the fixed-point solve takes no preconditioner (the refinement's FP32
    # inner solve does: tests/test_gpu_refine_pc.py)
    with pytest.raises(cg.CGError):
        ctx.solve(b, x, 8, 8, precond=4, precision=cg.CG_PREC_FIXED)


def test_profiled_passes(ctx):
    n, s, m = 512, 4, 5
    b = np.random.default_rng(1).uniform(-1, 1, (n, n))
    x = np.zeros_like(b)
    ctx.cg_set_profiling(True)
    ctx.cg_kernel_stats(reset=True)
    ctx.solve(b, x, n, n, tol=0.0, maxit=m, precond=s)
    st = ctx.cg_kernel_stats(reset=True)
    ctx.cg_set_profiling(False)
    # one Chebyshev pass per iteration; the iteration after maxit only
    # classifies the final state (its three passes count as final_check)
    assert st["cheb_precond"]["launches"] == m
    assert st["cheb_precond"]["bytes"] == m * 16 * n * n
    assert st["stencil_dot"]["launches"] == m
    assert st["final_check"]["launches"] == 3


def test_profiled_passes_pipelined(ctx):
    n, s, m = 512, 4, 5
    b = np.random.default_rng(1).uniform(-1, 1, (n, n))
    x = np.zeros_like(b)
    ctx.cg_set_profiling(True)
    ctx.cg_kernel_stats(reset=True)
    ctx.solve(b, x, n, n, tol=0.0, maxit=m, precond=s, variant=cg.CG_VARIANT_PIPELINED)
    st = ctx.cg_kernel_stats(reset=True)
    ctx.cg_set_profiling(False)
    # u = M^-1 r once, then per iteration m = M^-1 w and the fused pass; the
    # scalar step after maxit only classifies the final state
    assert st["cheb_precond"]["launches"] == 1 and st["init_wu"]["launches"] == 1
    assert st["cheb_precond_w"]["launches"] == m
    assert st["ppcg_pass"]["launches"] == m
    assert st["ppcg_pass"]["bytes"] == m * 136 * n * n


# ------------------------------------------------ batches and serving --

MIX = [(300, 190, 4, 0), (513, 257, 8, 1), (1, 1, 2, 0), (64, 1, 1, 1), (100, 100, 0, 1),
       (130, 70, 2, 1), (1024, 1024, 8, 0), (257, 129, 0, 0), (200, 150, 4, 1),
       (1, 300, 3, 0), (640, 128, 8, 1), (77, 250, 5, 0)]


def mix_problems(seed):
    rng = np.random.default_rng(seed)
    return [dict(nx=nx, ny=ny, s=sd, variant=v, b=rng.uniform(-1, 1, (ny, nx)),
                 tol=1e-8 if k % 2 else 1e-6) for k, (nx, ny, sd, v) in enumerate(MIX)]


def make(d, x):
    return cg.make_problem(d["b"], x, d["nx"], d["ny"], tol=d["tol"], maxit=20000,
                           variant=d["variant"], precond=d["s"])


def test_batch_with_preconditioned_solves_matches_alone(ctx):
    """Preconditioned solves of both variants and several s side by side with
    unpreconditioned ones in one batch: each result is bitwise its standalone
    solve, and the preconditioned ones bitwise the oracle's preconditioned CG
    in the library's order."""
    probs = mix_problems(31)
    xs = [np.zeros_like(d["b"]) for d in probs]
    say("batch with preconditioned solves:", len(probs))
    rc, res = ctx.cg_solve_batch([make(d, x) for d, x in zip(probs, xs)])
    assert rc == cg.CG_OK
    for d, x, r in zip(probs, xs, res):
        xa = np.zeros_like(d["b"])
        rca, ra = ctx.cg_solve(make(d, xa))
        say("  %dx%d s=%d v%d: batch %d alone %d iterations" % (d["nx"], d["ny"], d["s"],
                                                                d["variant"], r.iterations,
                                                                ra.iterations))
        assert r.status == rca == cg.CG_OK and r.iterations == ra.iterations
        np.testing.assert_array_equal(x, xa)
        assert r.rel_res_true == ra.rel_res_true
        if d["s"] and d["nx"] * d["ny"] <= 300 * 300:
            o, orho = tile_order(ctx, d["nx"], d["ny"], d["s"], d["variant"])
            xo, ro = oracle.pcg(d["b"], d["nx"], d["ny"], d["s"], tol=d["tol"], maxit=20000,
                                mode=MODE_CANONICAL, order=o, order_rho=orho,
                                variant=d["variant"])
            assert ro.iterations == r.iterations
            np.testing.assert_array_equal(x, xo)


def test_served_preconditioned_solves_match_alone(ctx):
    """The same mix served (requests arriving while others run): each result
    is bitwise its standalone solve; maxit and a zero right-hand side keep
    their outcomes."""
    import time
    probs = mix_problems(32)
    probs.append(dict(nx=90, ny=70, s=4, variant=1, b=np.zeros((70, 90)), tol=1e-8))
    xs = [np.zeros_like(d["b"]) for d in probs]
    tickets = []
    say("serving preconditioned requests:", len(probs))
    for k, (d, x) in enumerate(zip(probs, xs)):
        tickets.append(ctx.cg_submit(make(d, x)))
        if k % 4 == 3:
            time.sleep(0.002)
    xm = np.zeros_like(probs[0]["b"])
    tm = ctx.cg_submit(cg.make_problem(probs[0]["b"], xm, probs[0]["nx"], probs[0]["ny"],
                                       tol=1e-14, maxit=5, precond=4, variant=1))
    out = {}
    deadline = time.time() + 120
    while len(out) < len(tickets) + 1 and time.time() < deadline:
        for t in tickets + [tm]:
            if t not in out:
                rc, r = ctx.cg_poll(t)
                if rc != cg.CG_PENDING:
                    out[t] = (rc, cg.cg_result.from_buffer_copy(r))
        time.sleep(0.001)
    assert len(out) == len(tickets) + 1
    for d, x, t in zip(probs, xs, tickets):
        rc, r = out[t]
        xa = np.zeros_like(d["b"])
        rca, ra = ctx.cg_solve(make(d, xa))
        assert rc == rca == cg.CG_OK and r.iterations == ra.iterations
        np.testing.assert_array_equal(x, xa)
    assert out[tickets[-1]][1].iterations == 0 and not xs[-1].any()
    rc, r = out[tm]
    assert rc == cg.CG_NOT_CONVERGED and r.iterations == 5
