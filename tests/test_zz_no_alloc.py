"""The entry point for callers that cannot allocate (cg_solve_batch_small_noalloc):
through the C ABI, each result equals cg_solve_batch's for the same problem,
bitwise, over two calls in a row (the second with fewer and smaller problems,
so stale contents of the library's fixed device array would show)."""
import sys

import numpy as np
import pytest

from paper_1803_03797_amd import cg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def problems(torch, shapes, seed, x0_every=0):
    rng = np.random.default_rng(seed)
    out = []
    for m, (nx, ny) in enumerate(shapes):
        b = torch.from_numpy(rng.uniform(-1, 1, (ny, nx))).cuda()
        x0 = torch.from_numpy(rng.uniform(-1, 1, (ny, nx))).cuda() if x0_every and \
            m % x0_every == 0 else None
        out.append(dict(nx=nx, ny=ny, b=b, x0=x0, variant=m % 2,
                        tol=1e-8 if m % 3 else 1e-6, maxit=2000))
    return out


def run(torch, probs, noalloc, ctx=None):
    xs = [torch.full_like(d["b"], 5.0) for d in probs]
    ps = [cg.make_problem(d["b"], x, d["nx"], d["ny"], x0=d["x0"], tol=d["tol"],
                          maxit=d["maxit"], variant=d["variant"]) for d, x in zip(probs, xs)]
    if noalloc:
        rc, res = cg.cg_solve_batch_small_noalloc(ps)
    else:
        rc, res = ctx.cg_solve_batch(ps)
    return rc, res, xs


def same_float(u, v):
    return u == v or (u != u and v != v)  # equal, or both NaN


def same(torch, ra, xa, rb, xb):
    for a, xa_, b, xb_ in zip(ra, xa, rb, xb):
        assert a.status == b.status and a.iterations == b.iterations
        assert same_float(a.rel_res_recursive, b.rel_res_recursive)
        assert same_float(a.rel_res_true, b.rel_res_true)
        assert torch.equal(xa_, xb_) or (a.status == cg.CG_BREAKDOWN and
                                         torch.equal(xa_.isnan(), xb_.isnan()))


def test_noalloc_matches_batch_two_calls(torch):
    first = [(100, 100), (511, 20), (3, 5), (64, 64), (100, 99), (1, 1), (47, 80), (255, 40),
             (100, 100), (20, 100), (9, 1), (1, 9)]
    second = [(30, 20), (5, 4), (60, 7)]
    p1 = problems(torch, first, 1, x0_every=4)
    p2 = problems(torch, second, 2, x0_every=2)
    with cg.Context(device=0, arena_bytes=1 << 30) as ctx:
        for k in (p1[0], p1[2]):
            assert ctx.cg_plan(k["nx"], k["ny"], k["variant"]).path == 2
        say("no-alloc call 1:", len(p1), "solves")
        rc1, r1, x1 = run(torch, p1, True)
        say("no-alloc call 2:", len(p2), "solves")
        rc2, r2, x2 = run(torch, p2, True)
        rb1, q1, y1 = run(torch, p1, False, ctx)
        rb2, q2, y2 = run(torch, p2, False, ctx)
    assert rc1 == rb1 and rc2 == rb2 == cg.CG_OK
    same(torch, r1, x1, q1, y1)
    same(torch, r2, x2, q2, y2)
    assert all(r.status == cg.CG_OK and r.iterations > 0 for r in r1 + r2)


def test_noalloc_edge_cases(torch):
    """Zero right-hand side (x = 0), a non-finite one (breakdown), x0 aliasing
    x, maxit reached: the same outcomes as cg_solve_batch."""
    nx, ny = 40, 30
    rng = np.random.default_rng(5)
    b = torch.from_numpy(rng.uniform(-1, 1, (ny, nx))).cuda()
    bad = b.clone()
    bad[3, 4] = float("nan")
    zero = torch.zeros_like(b)
    x2_start = torch.from_numpy(rng.uniform(-1, 1, (ny, nx))).cuda()
    with cg.Context(device=0, arena_bytes=1 << 30) as ctx:
        outs = []
        for noalloc in (True, False):
            xs = [torch.full_like(b, 3.0) for _ in range(4)]
            xs[2] = x2_start.clone()
            ps = [cg.make_problem(zero, xs[0], nx, ny),
                  cg.make_problem(bad, xs[1], nx, ny, variant=1),
                  cg.make_problem(b, xs[2], nx, ny, x0=xs[2], tol=1e-9),
                  cg.make_problem(b, xs[3], nx, ny, tol=1e-12, maxit=6, variant=1)]
            if noalloc:
                rc, res = cg.cg_solve_batch_small_noalloc(ps)
            else:
                rc, res = ctx.cg_solve_batch(ps)
            outs.append((rc, res, xs))
    (rca, ra, xa), (rcb, rb, xb) = outs
    assert rca == rcb == cg.CG_BREAKDOWN
    assert [r.status for r in ra] == [cg.CG_OK, cg.CG_BREAKDOWN, cg.CG_OK, cg.CG_NOT_CONVERGED]
    assert ra[0].iterations == 0 and not xa[0].any()
    assert ra[3].iterations == 6
    same(torch, ra, xa, rb, xb)


def test_noalloc_rejects():
    """Problems outside the on-chip solver, host memory, more than 64 solves."""
    import torch as t
    b = t.ones((30, 20), dtype=t.float64, device="cuda")
    x = t.zeros_like(b)
    ok = cg.make_problem(b, x, 20, 30)
    big_b = t.ones((200, 200), dtype=t.float64, device="cuda")
    big = cg.make_problem(big_b, t.zeros_like(big_b), 200, 200)
    hb = np.ones((30, 20))
    host = cg.make_problem(hb, np.zeros_like(hb), 20, 30)
    refined = cg.make_problem(b, x, 20, 30, precision=cg.CG_PREC_FP32_REFINED)
    for bad in ([big], [host], [refined], [ok] * 65):
        with pytest.raises(cg.CGError) as e:
            cg.cg_solve_batch_small_noalloc(bad)
        assert e.value.code == cg.CG_E_INVALID
    xs = [t.zeros_like(b) for _ in range(64)]
    rc, res = cg.cg_solve_batch_small_noalloc([cg.make_problem(b, xk, 20, 30) for xk in xs])
    assert rc == cg.CG_OK and all(r.iterations == res[0].iterations for r in res)
    assert all(t.equal(xk, xs[0]) for xk in xs)
