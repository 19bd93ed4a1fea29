"""GPU tests of the multi-solve batch engine (cg_solve_batch) and the
continuous-batching server (cg_submit / cg_poll): every solve gives the same
bits in a batch or in a served mix as when solved alone (same tile geometry,
same reduction order), and the first few also match the CPU oracle."""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1803_03797_amd import cg, workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def mixed_problems(count, seed, refined_every=0, big=False):
    rng = np.random.default_rng(seed)
    sides = [3, 17, 64, 100, 128, 200, 257, 512] + ([1024] if big else [])
    out = []
    for m in range(count):
        nx, ny = int(rng.choice(sides)), int(rng.choice(sides))
        b = rng.uniform(-1, 1, (ny, nx))
        variant = int(rng.integers(0, 2))
        prec = cg.CG_PREC_FP32_REFINED if refined_every and m % refined_every == 0 else 0
        tol = 1e-10 if prec else float(rng.choice([1e-6, 1e-8]))
        out.append(dict(nx=nx, ny=ny, b=b, variant=variant, precision=prec, tol=tol))
    return out


def order_of(ctx, nx, ny, variant):
    """The reduction order of the plan a solve of this shape takes."""
    info = ctx.cg_plan(nx, ny, variant)
    if info.path == 2:
        return oracle.Order.segments(info.seg_rows, info.lanes, info.seg_waves, info.seg_cols)
    return oracle.Order(info.cols_per_lane, info.lanes, info.waves, info.rows, info.threads2,
                        alt=info.walk_alt)


def make(d, x, maxit=20000):
    return cg.make_problem(d["b"], x, d["nx"], d["ny"], tol=d["tol"], maxit=maxit,
                           variant=d["variant"], precision=d["precision"], inner_tol=1e-4)


def alone(ctx, d, maxit=20000):
    x = np.zeros_like(d["b"])
    rc, r = ctx.cg_solve(make(d, x, maxit))
    return rc, r, x


def test_batch_matches_alone_bitwise():
    with cg.Context(device=0, arena_bytes=4 << 30) as ctx:
        probs = mixed_problems(40, 7, refined_every=5)
        xs = [np.zeros_like(d["b"]) for d in probs]
        say("batch of", len(probs))
        rc, res = ctx.cg_solve_batch([make(d, x) for d, x in zip(probs, xs)])
        assert rc in (cg.CG_OK, cg.CG_NOT_CONVERGED)
        for m, (d, x, r) in enumerate(zip(probs, xs, res)):
            rca, ra, xa = alone(ctx, d)
            say("  #%d %dx%d v%d p%d: batch %s/%d alone %s/%d" % (
                m, d["nx"], d["ny"], d["variant"], d["precision"], cg.cg_status_str(r.status),
                r.iterations, cg.cg_status_str(rca), ra.iterations))
            assert r.status == rca
            assert r.iterations == ra.iterations and r.outer_iterations == ra.outer_iterations
            np.testing.assert_array_equal(x, xa)
            assert r.rel_res_true == ra.rel_res_true
        # a few against the oracle (FP64 ones)
        checked = 0
        for d, x, r in zip(probs, xs, res):
            if d["precision"] or checked >= 6:
                continue
            xo, ro = oracle.cg(d["b"], d["nx"], d["ny"], variant=d["variant"], tol=d["tol"],
                               maxit=20000)
            assert abs(r.iterations - ro.iterations) <= 2
            assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo) * (
                1 if d["variant"] == 0 else 1e2)
            checked += 1


def test_batch_failure_isolated_and_edge_cases():
    with cg.Context(device=0, arena_bytes=1 << 30) as ctx:
        rng = np.random.default_rng(3)
        good = [rng.uniform(-1, 1, (70, 90)) for _ in range(3)]
        bad = good[0].copy()
        bad[5, 5] = np.inf
        zero = np.zeros((40, 33))
        bs = [good[0], bad, zero, good[1], good[2]]
        shapes = [(90, 70), (90, 70), (33, 40), (90, 70), (90, 70)]
        xs = [np.full_like(b, 3.0) for b in bs]
        maxits = [20000, 20000, 20000, 5, 20000]
        probs = [cg.make_problem(b, x, nx, ny, tol=1e-8, maxit=mi, variant=k % 2)
                 for k, (b, x, (nx, ny), mi) in enumerate(zip(bs, xs, shapes, maxits))]
        say("batch edge cases")
        rc, res = ctx.cg_solve_batch(probs)
        assert rc == cg.CG_BREAKDOWN
        assert [r.status for r in res] == [cg.CG_OK, cg.CG_BREAKDOWN, cg.CG_OK,
                                           cg.CG_NOT_CONVERGED, cg.CG_OK]
        assert res[2].iterations == 0 and not xs[2].any()
        assert res[3].iterations == 5
        for k in (0, 4):
            rca, ra, xa = alone(ctx, dict(nx=90, ny=70, b=bs[k], variant=k % 2, precision=0,
                                          tol=1e-8))
            np.testing.assert_array_equal(xs[k], xa)


def test_batch_refined_slow_inner_solves_stay_isolated():
    """A refined request whose inner solves stop after about one iteration
    (inner tol 0.99) reaches maxit as CG_NOT_CONVERGED, with about six passes
    per inner iteration, in a batch and served, and leaves the others intact."""
    rng = np.random.default_rng(21)
    shapes = [(300, 200), (257, 129), (300, 200)]
    bs = [rng.uniform(-1, 1, (ny, nx)) for nx, ny in shapes]
    with cg.Context(device=0, arena_bytes=1 << 30) as ctx:
        for maxit in (15, 40):
            xs = [np.zeros_like(b) for b in bs]
            probs = [cg.make_problem(bs[0], xs[0], 300, 200, tol=1e-8, maxit=20000, variant=1),
                     cg.make_problem(bs[1], xs[1], 257, 129, tol=1e-10, maxit=maxit,
                                     precision=cg.CG_PREC_FP32_REFINED, inner_tol=0.99),
                     cg.make_problem(bs[2], xs[2], 300, 200, tol=1e-8, maxit=20000, variant=0)]
            say("refined inner tol 0.99, maxit", maxit)
            rc, res = ctx.cg_solve_batch(probs)
            assert [r.status for r in res] == [cg.CG_OK, cg.CG_NOT_CONVERGED, cg.CG_OK]
            assert res[1].iterations == maxit
            for k in (0, 2):
                rca, ra, xa = alone(ctx, dict(nx=300, ny=200, b=bs[k], variant=1 - k // 2,
                                              precision=0, tol=1e-8))
                np.testing.assert_array_equal(xs[k], xa)
            xa = np.zeros_like(bs[1])
            rca, ra = ctx.cg_solve(cg.make_problem(bs[1], xa, 257, 129, tol=1e-10, maxit=maxit,
                                                   precision=cg.CG_PREC_FP32_REFINED,
                                                   inner_tol=0.99))
            assert rca == cg.CG_NOT_CONVERGED and ra.iterations == maxit
            np.testing.assert_array_equal(xs[1], xa)
            # served
            xsv = np.zeros_like(bs[1])
            t = ctx.cg_submit(cg.make_problem(bs[1], xsv, 257, 129, tol=1e-10, maxit=maxit,
                                              precision=cg.CG_PREC_FP32_REFINED, inner_tol=0.99))
            deadline = time.time() + 60
            while time.time() < deadline:
                rc, r = ctx.cg_poll(t)
                if rc != cg.CG_PENDING:
                    break
                time.sleep(0.001)
            assert rc == cg.CG_NOT_CONVERGED and r.iterations == maxit
            np.testing.assert_array_equal(xsv, xa)


def test_batch_more_solves_than_slots_and_small_arena():
    """8 slots and an arena that holds only a few solves at once: admission
    waits for memory and slots, results are unchanged."""
    probs = mixed_problems(20, 11)
    need = max(cg.cg_footprint(make(d, np.zeros_like(d["b"]))) for d in probs)
    with cg.Context(device=0, arena_bytes=3 * need + (8 << 20), max_slots=8) as ctx:
        xs = [np.zeros_like(d["b"]) for d in probs]
        say("batch with 8 slots, small arena")
        rc, res = ctx.cg_solve_batch([make(d, x) for d, x in zip(probs, xs)])
        assert rc == cg.CG_OK
    with cg.Context(device=0, arena_bytes=1 << 30) as ctx2:
        for d, x, r in zip(probs, xs, res):
            rca, ra, xa = alone(ctx2, d)
            assert r.iterations == ra.iterations
            np.testing.assert_array_equal(x, xa)


def test_batch_rejects_oversized():
    with cg.Context(device=0, arena_bytes=64 << 20) as ctx:
        b = np.ones((2048, 2048))
        x = np.zeros_like(b)
        rc = ctx.lib.cg_solve_batch(ctx.h, (cg.cg_problem * 1)(cg.make_problem(b, x, 2048, 2048)),
                                    1, (cg.cg_result * 1)())
        assert rc == cg.CG_E_NOMEM


def test_batch_workload_sample_device_memory(torch):
    """A 32-solve sample of the batch workload (sides from {64..1024}, p-CG,
    tol 1e-8), device pointers; each equals its standalone solve."""
    shapes = workloads.batch_shapes(256)[:32]
    with cg.Context(device=0, arena_bytes=4 << 30) as ctx:
        bs = [torch.from_numpy(workloads.batch_rhs(m, nx, ny)).cuda()
              for m, (nx, ny) in enumerate(shapes)]
        xs = [torch.zeros_like(b) for b in bs]
        probs = [cg.make_problem(b, x, nx, ny, tol=1e-8, maxit=20000, variant=1)
                 for b, x, (nx, ny) in zip(bs, xs, shapes)]
        say("batch workload sample, 32 solves")
        t0 = time.perf_counter()
        rc, res = ctx.cg_solve_batch(probs)
        tb = time.perf_counter() - t0
        assert rc == cg.CG_OK
        t0 = time.perf_counter()
        for m, (b, (nx, ny)) in enumerate(zip(bs, shapes)):
            xa = torch.zeros_like(b)
            rca, ra = ctx.solve(b, xa, nx, ny, tol=1e-8, maxit=20000, variant=1)
            assert rca == cg.CG_OK and ra.iterations == res[m].iterations
            assert torch.equal(xa, xs[m])
        ts = time.perf_counter() - t0
        say("  batch %.3f s, one-by-one %.3f s" % (tb, ts))


def test_serve_alone_vs_mix():
    """Requests arriving while others run: each result equals its alone solve."""
    probs = mixed_problems(24, 5, refined_every=4)
    with cg.Context(device=0, arena_bytes=2 << 30) as ctx:
        xs = [np.zeros_like(d["b"]) for d in probs]
        tickets = []
        say("serving 24 staggered requests")
        for k, (d, x) in enumerate(zip(probs, xs)):
            tickets.append(ctx.cg_submit(make(d, x)))
            if k % 3 == 2:
                time.sleep(0.003)
        results = {}
        deadline = time.time() + 120
        while len(results) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t in results:
                    continue
                rc, r = ctx.cg_poll(t)
                if rc != cg.CG_PENDING:
                    results[t] = (rc, cg.cg_result.from_buffer_copy(r))
            time.sleep(0.001)
        assert len(results) == len(tickets)
        for d, x, t in zip(probs, xs, tickets):
            rc, r = results[t]
            rca, ra, xa = alone(ctx, d)
            assert rc == rca and r.iterations == ra.iterations
            np.testing.assert_array_equal(x, xa)
            assert r.latency_seconds >= r.device_seconds > 0
        # served results against the oracle: FP64 ones bitwise against its
        # canonical order (the order of the request's plan), refined ones
        # within 1e-9 of the FP64 oracle solution at the same tolerance
        n64 = nref = 0
        for d, x, t in zip(probs, xs, tickets):
            rc, r = results[t]
            nx, ny = d["nx"], d["ny"]
            if d["precision"] == 0 and n64 < 8:
                o = order_of(ctx, nx, ny, d["variant"])
                xo, ro = oracle.cg(d["b"], nx, ny, variant=d["variant"], tol=d["tol"],
                                   maxit=20000, mode=oracle.MODE_CANONICAL, order=o)
                assert rc == ro.status and r.iterations == ro.iterations
                np.testing.assert_array_equal(x, xo)
                n64 += 1
            elif d["precision"] == cg.CG_PREC_FP32_REFINED and nref < 4:
                xo, ro = oracle.cg(d["b"], nx, ny, tol=d["tol"], maxit=20000)
                err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
                say("  served refined %dx%d: err vs FP64 oracle %.2e" % (nx, ny, err))
                assert rc == cg.CG_OK and r.rel_res_true <= d["tol"] and err <= 1e-9
                nref += 1
        assert n64 >= 6 and nref >= 3
        with pytest.raises(cg.CGError) as e:
            ctx.cg_poll(tickets[0])
        assert e.value.code == cg.CG_E_TICKET


def test_serve_rejects_and_unknown_ticket():
    with cg.Context(device=0, arena_bytes=32 << 20) as ctx:
        b = np.ones((2048, 2048))
        x = np.zeros_like(b)
        with pytest.raises(cg.CGError) as e:
            ctx.cg_submit(cg.make_problem(b, x, 2048, 2048))
        assert e.value.code == cg.CG_E_NOMEM
        with pytest.raises(cg.CGError) as e:
            ctx.cg_poll(12345)
        assert e.value.code == cg.CG_E_TICKET


def test_auto_precision_policy_batch_and_served():
    """CG_PREC_AUTO: grids below 20480 unknowns solved in FP64, larger ones
    FP32-refined; in a batch and served, each result is bitwise the solve
    alone in the precision chosen, and the refined ones meet their tol."""
    rng = np.random.default_rng(17)
    shapes = [(100, 100), (143, 143), (144, 143), (300, 200), (64, 64), (513, 257), (17, 3),
              (181, 181)]
    bs = [rng.uniform(-1, 1, (ny, nx)) for nx, ny in shapes]
    with cg.Context(device=0, arena_bytes=2 << 30) as ctx:
        xs = [np.zeros_like(b) for b in bs]
        probs = [cg.make_problem(b, x, nx, ny, tol=1e-8, maxit=20000, variant=k % 2,
                                 precision=cg.CG_PREC_AUTO)
                 for k, (b, x, (nx, ny)) in enumerate(zip(bs, xs, shapes))]
        say("auto precision batch")
        rc, res = ctx.cg_solve_batch(probs)
        assert rc == cg.CG_OK
        xv = [np.zeros_like(b) for b in bs]
        tickets = [ctx.cg_submit(cg.make_problem(b, x, nx, ny, tol=1e-8, maxit=20000,
                                                 variant=k % 2, precision=cg.CG_PREC_AUTO))
                   for k, (b, x, (nx, ny)) in enumerate(zip(bs, xv, shapes))]
        served = {}
        deadline = time.time() + 60
        while len(served) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t not in served:
                    rc2, r2 = ctx.cg_poll(t)
                    if rc2 != cg.CG_PENDING:
                        served[t] = (rc2, cg.cg_result.from_buffer_copy(r2))
            time.sleep(0.001)
        assert len(served) == len(tickets)
        for k, ((nx, ny), b, x, r, t) in enumerate(zip(shapes, bs, xs, res, tickets)):
            chosen = cg.CG_PREC_FP64 if nx * ny < 20480 else cg.CG_PREC_FP32_REFINED
            xa = np.zeros_like(b)
            rca, ra = ctx.cg_solve(cg.make_problem(b, xa, nx, ny, tol=1e-8, maxit=20000,
                                                   variant=k % 2, precision=chosen))
            assert (r.outer_iterations > 0) == (chosen == cg.CG_PREC_FP32_REFINED)
            assert r.status == rca == cg.CG_OK and r.iterations == ra.iterations
            assert r.rel_res_true <= 1e-8 * 1.000001 or chosen == cg.CG_PREC_FP64
            np.testing.assert_array_equal(x, xa)
            rcs, rs = served[t]
            assert rcs == cg.CG_OK and rs.iterations == ra.iterations
            np.testing.assert_array_equal(xv[k], xa)
