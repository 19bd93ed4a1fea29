"""GPU tests of the runtime around the kernels: autotuner and its cache, pinned
tile shapes (the reduction order follows the shape), profiling statistics,
the HBM probe, a caller-provided arena tensor and stream, and the ordering
after the null stream when the caller names none."""
import json
import sys
import time

import numpy as np
import pytest

import oracle
from oracle import MODE_CANONICAL
from paper_1803_03797_amd import cg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def order_of(ctx, nx, ny, variant=0, precision=0):
    info = ctx.cg_plan(nx, ny, variant, precision)
    if info.path == 2:
        return oracle.Order.segments(info.seg_rows, info.lanes, info.seg_waves, info.seg_cols), info
    return oracle.Order(info.cols_per_lane, info.lanes, info.waves, info.rows, info.threads2,
                        alt=info.walk_alt), info


@pytest.mark.parametrize("variant", [0, 1])
def test_tune_cache_and_parity(tmp_path, variant):
    nx, ny = 700, 300
    cache = str(tmp_path / "tune.json")
    with cg.Context(device=0, arena_bytes=1 << 30, tune_cache=cache) as ctx:
        say("tune", nx, ny, variant)
        ctx.cg_tune(nx, ny, variant)
        o, info = order_of(ctx, nx, ny, variant)
        lines = [json.loads(l) for l in open(cache)]
        assert any(d["nx"] == nx and d["ny"] == ny and d["rows"] == info.rows and
                   d["variant"] == variant and d["arch"].startswith("gfx9") and d["hip"] > 0
                   for d in lines)
        b = np.random.default_rng(1).uniform(-1, 1, (ny, nx))
        x = np.zeros_like(b)
        rc, r = ctx.solve(b, x, nx, ny, tol=0.0, maxit=30, variant=variant)
        xo, ro = oracle.cg(b, nx, ny, variant=variant, tol=0.0, maxit=30, mode=MODE_CANONICAL,
                           order=o)
        np.testing.assert_array_equal(x, xo)
    with cg.Context(device=0, arena_bytes=1 << 30, tune_cache=cache) as ctx2:
        info2 = ctx2.cg_plan(nx, ny, variant)
        assert (info2.rows, info2.cols_per_lane, info2.grid) == (info.rows, info.cols_per_lane,
                                                                info.grid)


def test_tune_keeps_variants_apart(tmp_path):
    """Tuning one variant leaves the other variant's pinned shape alone, and
    a cache line of another architecture or HIP runtime is ignored."""
    nx, ny = 600, 260
    cache = str(tmp_path / "tune.json")
    with cg.Context(device=0, arena_bytes=1 << 30, tune_cache=cache) as ctx:
        say("tune both variants", nx, ny)
        ctx.cg_tune(nx, ny, 1)
        p1 = ctx.cg_plan(nx, ny, 1)
        ctx.cg_tune(nx, ny, 0)
        p1b = ctx.cg_plan(nx, ny, 1)
        assert (p1.rows, p1.grid, p1.cols_per_lane) == (p1b.rows, p1b.grid, p1b.cols_per_lane)
        lines = [json.loads(l) for l in open(cache)]
        assert sorted(d["variant"] for d in lines if d["nx"] == nx) == [0, 1]
    # the same lines claimed for another architecture: not loaded
    with open(cache, "w") as f:
        for d in lines:
            d = dict(d, arch="gfx000", rows=1)
            f.write(json.dumps(d) + "\n")
    with cg.Context(device=0, arena_bytes=1 << 30, tune_cache=cache) as ctx2:
        assert ctx2.cg_plan(nx, ny, 1).rows != 1


@pytest.mark.parametrize("rows", [1, 3, 32])
def test_pinned_wide_lanes_classic_bitwise(rows):
    """Classic FP64 with 4 columns per lane: the canonical order with
    cols_per_lane = 4 reproduces it bitwise, alone and in a batch."""
    nx, ny = 513, 130
    with cg.Context(device=0, arena_bytes=1 << 30) as ctx:
        ctx.cg_pin_tile(nx, ny, rows, 0, cg.CG_PREC_FP64, 4)
        o, info = order_of(ctx, nx, ny, 0)
        assert info.cols_per_lane == 4 and info.rows == rows
        b = np.random.default_rng(rows).uniform(-1, 1, (ny, nx))
        x = np.zeros_like(b)
        say("wide lanes rows", rows)
        rc, r = ctx.solve(b, x, nx, ny, tol=1e-8, maxit=5000, variant=0)
        xo, ro = oracle.cg(b, nx, ny, variant=0, tol=1e-8, maxit=5000, mode=MODE_CANONICAL,
                           order=o)
        assert r.iterations == ro.iterations
        np.testing.assert_array_equal(x, xo)
        xb = np.zeros_like(b)
        rc, res = ctx.cg_solve_batch([cg.make_problem(b, xb, nx, ny, tol=1e-8, maxit=5000)])
        np.testing.assert_array_equal(xb, xo)


def test_pin_rejects_bad_shapes():
    with cg.Context(device=0, arena_bytes=64 << 20) as ctx:
        for args in ((10, 10, 0, 0, 0, 3), (10, 10, 0, 0, 0, 0), (10, 10, 4, -1, 0, 0),
                     (10, 10, 4, 0, cg.CG_PREC_FP32_REFINED, 2)):
            nx, ny, rows, grid, prec, cpl = args
            assert ctx.lib.cg_pin_tile(ctx.h, nx, ny, prec, rows, grid, cpl) == cg.CG_E_INVALID


def test_profiling_statistics(torch):
    n = 1024
    with cg.Context(device=0, arena_bytes=1 << 30) as ctx:
        b = torch.rand(n * n, dtype=torch.float64, device="cuda")
        x = torch.zeros_like(b)
        ctx.cg_set_profiling(True)
        ctx.cg_kernel_stats(reset=True)
        say("profiling stats")
        rc, r = ctx.solve(b, x, n, n, tol=0.0, maxit=37, variant=1)
        st = ctx.cg_kernel_stats(reset=True)
        # odd iterations leave x alone (80 B per unknown), even ones update it
        # twice (96 B); the check pass after iteration 37 applies its update
        assert st["pcg_pass_nx"]["launches"] == 19 and st["pcg_pass"]["launches"] == 18
        assert st["final_check"]["launches"] == 1 and st["final_check"]["bytes"] == 0
        assert st["pcg_pass"]["bytes"] == 18 * 96 * n * n
        assert st["pcg_pass_nx"]["bytes"] == 19 * 80 * n * n
        rc, r = ctx.solve(b, x, n, n, tol=0.0, maxit=12, variant=0)
        st = ctx.cg_kernel_stats(reset=False)
        assert st["stencil_dot"]["launches"] == 12
        assert st["update_norm"]["launches"] == 6 and st["update_norm_nx"]["launches"] == 6
        assert st["update_norm"]["bytes"] == 6 * 48 * n * n
        assert st["update_norm_nx"]["bytes"] == 6 * 24 * n * n
        assert ctx.cg_kernel_stats(reset=True) == st
        assert ctx.cg_kernel_stats() == {}


def test_stream_probe():
    with cg.Context(device=0, arena_bytes=2 << 30) as ctx:
        for pat, moved in ((0, 1), (1, 2), (2, 3), (3, 5), (4, 12), (5, 12), (6, 12), (7, 12)):
            t, nbytes = ctx.cg_stream_probe(pat, 1 << 22, 2)
            assert nbytes == moved * (1 << 22) * 8 and t > 0
            say("probe", pat, "%.0f GB/s" % (nbytes / t / 1e9))
        with pytest.raises(cg.CGError):
            ctx.cg_stream_probe(8, 1 << 20, 1)
        with pytest.raises(cg.CGError):
            ctx.cg_stream_probe(7, 4094, 1)  # no whole row of 4096


def test_mul_probe():
    with cg.Context(device=0, arena_bytes=256 << 20) as ctx:
        t, ops = ctx.cg_mul_probe(1024, 2)
        assert t > 0 and ops > 0 and ops % (256 * 8 * 1024) == 0
        say("multiply probe %.1f T/s" % (ops / t / 1e12))
        for bad in ((0, 1), (16, 0)):
            with pytest.raises(cg.CGError):
                ctx.cg_mul_probe(*bad)


def test_caller_arena_and_stream(torch):
    """Workspace carved from a caller's uint8 tensor; work ordered after the
    caller's stream."""
    nx, ny = 300, 200
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(2)
    bh = rng.uniform(-1, 1, (ny, nx))
    with cg.Context(device=0, stream=stream, arena=arena) as ctx:
        with torch.cuda.stream(stream):
            b = torch.from_numpy(bh).cuda()
            b.mul_(2.0)  # pending work on the caller's stream
            x = torch.zeros_like(b)
        rc, r = ctx.solve(b, x, nx, ny, tol=1e-9, maxit=5000, variant=1)
        o, _ = order_of(ctx, nx, ny, 1)
        xo, ro = oracle.cg(2.0 * bh, nx, ny, variant=1, tol=1e-9, maxit=5000,
                           mode=MODE_CANONICAL, order=o)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(x.cpu().numpy(), xo)
    # an arena pointer without a size is rejected
    import ctypes as C
    h = C.c_void_p()
    cfg = cg.cg_config(0, None, arena.data_ptr(), 0, 0, None)
    assert cg.load().cg_create(C.byref(cfg), C.byref(h)) == cg.CG_E_INVALID


def test_null_stream_ordering(torch):
    """A context without a stream orders every call after the null stream:
    inputs that the caller's kernels are still writing (a backlog of products
    queued ahead of the final copy into b) are read only once written, by
    cg_solve, cg_solve_batch and cg_submit alike."""
    nx, ny = 600, 500
    dev = torch.device("cuda:0")
    src = torch.from_numpy(np.random.default_rng(8).uniform(-1, 1, (ny, nx))).to(dev)
    big = torch.randn(4096, 4096, dtype=torch.float64, device=dev)
    with cg.Context(device=0, arena_bytes=1 << 30) as ctx:
        torch.cuda.synchronize()
        want = torch.zeros_like(src)
        ctx.solve(src, want, nx, ny, tol=1e-9, maxit=5000)
        want = want.cpu().numpy()

        def pending_rhs():
            b = torch.zeros_like(src)
            t = big
            for _ in range(24):
                t = t @ big  # about 0.1 s of queued work on the null stream
            b.copy_(src + 0.0 * t[:ny, :nx])
            return b

        b = pending_rhs()
        x = torch.zeros_like(b)
        rc, r = ctx.solve(b, x, nx, ny, tol=1e-9, maxit=5000)
        assert rc == cg.CG_OK
        np.testing.assert_array_equal(x.cpu().numpy(), want)
        b = pending_rhs()
        x = torch.zeros_like(b)
        rc, rs = ctx.cg_solve_batch([cg.make_problem(b, x, nx, ny, tol=1e-9, maxit=5000)])
        assert rc == cg.CG_OK and rs[0].iterations == r.iterations
        np.testing.assert_array_equal(x.cpu().numpy(), want)
        b = pending_rhs()
        x = torch.zeros_like(b)
        t = ctx.cg_submit(cg.make_problem(b, x, nx, ny, tol=1e-9, maxit=5000))
        deadline = time.time() + 60
        while True:
            rc, rp = ctx.cg_poll(t)
            if rc != cg.CG_PENDING or time.time() > deadline:
                break
            time.sleep(0.001)
        assert rc == cg.CG_OK and rp.iterations == r.iterations
        torch.cuda.synchronize()
        np.testing.assert_array_equal(x.cpu().numpy(), want)


def test_interleaved_rows_layout():
    """Pipelined FP64 tile-pass solves lay their vectors out with interleaved
    rows (row stride = padded width x vectors); the other paths keep one
    vector per region.  The results do not depend on it (every pipelined
    parity test on path 0 runs on it)."""
    with cg.Context(device=0, arena_bytes=1 << 30) as ctx:
        n = 1024
        for kw, vecs in ((dict(variant=0), 1), (dict(variant=1), 8),
                         (dict(variant=0, vc=True), 1), (dict(variant=1, vc=True), 12),
                         (dict(variant=1, nz=4), 8), (dict(variant=0, precond=4), 1),
                         (dict(variant=1, precond=4), 10),
                         (dict(variant=0, precision=cg.CG_PREC_FP32_REFINED), 1)):
            info = ctx.cg_plan(n, n, **kw)
            assert info.path == 0
            assert info.row_stride == vecs * info.pitch, (kw, info.row_stride, info.pitch)
        for kw in (dict(variant=0), dict(variant=1), dict(precision=cg.CG_PREC_FIXED)):
            info = ctx.cg_plan(100, 100, **kw)
            assert info.path != 0 and info.row_stride == info.pitch
