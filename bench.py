"""Benchmark of the stencil CG library on one MI355X.

Default (the headline line): CG on the 4096 x 4096 Laplace workload, both
variants.  One step = one solve of A x = b with classic CG (Algorithm 1) plus
one with the pipelined CG (Algorithm 2), each running a fixed 500 iterations
(tol = 0) with b = A x*, x* the lowest grid mode plus 1e-3 uniform noise
(seeded), x0 = 0, FP64.  Inputs are resident in HBM before the timed region.
value = unknowns x iterations per second over the whole step (GDOF-iter/s).

  roofline      the dominant kernel (pcg_pass, the pipelined pass of an even
                iteration, which also brings x up to date): algorithmic bytes
                (96 B per unknown) / its average launch duration, from HIP
                events recorded around each launch on the library's stream
                while the same steps are repeated with profiling on; vs
                8 TB/s.  Odd iterations run pcg_pass_nx (80 B, x untouched).
  cpu_baseline  the CPU oracle (plain C, explicit CSR, one thread) on a
                bounded sample of the same workload.

Other workloads (one JSON line each, not the headline):
  --workload small   100 x 100, both variants, tol 1e-8: solve latency
  --workload batch   256 uneven grids, pipelined, all on the device at once
                     (multi-solve step kernel) vs one-by-one solves
  --workload huge    8192 x 8192: FP32-inner / FP64-outer refinement vs FP64
                     CG, both to a true residual of 1e-10
  --workload serve   request stream with Poisson arrivals: served
                     (continuous batching) FP32-refined and FP64 vs
                     per-request FP64
  --workload fixed   the paper's fixed-point format (Q20.30): solve latency on
                     its synthesized grids and iteration counts, and a batch of
                     256 solves of its largest grid in one launch
  --workload precond 4096 x 4096 to tol 1e-8: classic CG against classic CG
                     preconditioned by s Chebyshev steps (time to solution)
  --workload cube    the 3D 7-point operator on 256^3: both variants, fixed
                     iterations and to tol 1e-8
  --workload vc      the variable-coefficient 5-point operator on 4096^2 (face
                     conductivities log-uniform on [0.1, 10]): both variants,
                     fixed iterations and to tol 1e-8
  --probe            attainable HBM bandwidth of plain streaming kernels, and
                     the attainable rate of 32 x 32 -> 64-bit multiply-adds
"""
import argparse
import json
import math
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BYTES_PER_DOF = {"pcg_pass": 96, "pcg_pass_nx": 80, "stencil_dot": 24, "update_norm": 48,
                 "update_norm_nx": 24}
# algorithmic bytes per unknown and iteration, averaged over an odd/even pair
BYTES_PER_ITER = {"classic": 24 + (48 + 24) / 2, "pipelined": (96 + 80) / 2}
OP_NAMES = {"2d": "", "3d": " on the 7-point operator", "vc": " with variable coefficients"}
# HBM bytes per pcg_pass launch at 4096 x 4096 from two rocprofv3 --pmc runs
# (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, the factors the library's 134 MB
# copy kernel gives for the same counters); set to None whenever pcg_pass
# changes, until the counters are taken again.
PCG_TRAFFIC_BYTES = 1646594743
# The same for pcg_pass of the variable-coefficient operator at 4096 x 4096
# (128 algorithmic bytes per unknown: 96 of vectors, 32 of coefficients).
VC_TRAFFIC_BYTES = 2161653028
# The same for pcg_pass of the 7-point operator at 256^3 (z-march tiles).
CUBE_TRAFFIC_BYTES = 1627106949
# Fixed point (ALU-bound): exact 50 x 50-bit products per unknown and
# iteration (classic: p = r + b p, x += a p, r -= a s, (p, s), (r, r);
# pipelined: the six updates of z, q, p, x, r, w and (r, r), (w, r)), each
# four 32 x 32 -> 64-bit multiplies of two-limb operands.  Peak: 256 CUs x
# 4 SIMDs x 16 lanes per clock x 2.4 GHz, the 64-bit multiply-add at half
# the 32-lane rate of 32-bit VALU operations (a probe kernel of independent
# v_mad_u64_u32 chains reaches 30.3 T/s on the device).
# HBM bytes per Chebyshev-pass launch (classic form) at 4096 x 4096 from the two
# rocprofv3 --pmc runs, by the same calibration: s -> bytes
CHEB_TRAFFIC_BYTES = {8: (120324 * 2 + 131086) * 1024}
FX_PRODUCTS = {"classic": 5, "pipelined": 8}
FX_MULS_PER_PRODUCT = 4
FX_MUL_PEAK_G = 256 * 4 * 16 * 2.4  # Gmul/s
# FP64 vector operations issued per second (256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz; an fma counts once: 78.6 TFLOP/s counting it twice)
FP64_OP_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def emit(line):
    print(json.dumps(line), flush=True)


def setup():
    import torch

    from paper_1803_03797_amd import cg
    if not os.path.exists(cg.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    return torch, cg


def host_info():
    """The host the CPU baseline ran on: logical CPUs, model, OMP_NUM_THREADS."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return {"cpu_count": os.cpu_count(), "model": model,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def cpu_rate(bh, n, variants, k, all_cores):
    """Sequential-mode oracle solves of k iterations each, timed without the
    CSR assembly: (GDOF-iter/s, seconds, threads)."""
    import oracle
    secs, threads = 0.0, 1
    for v in variants:
        r, t, threads = oracle.cg_timed(bh, n, n, v, tol=0.0, maxit=k, all_cores=all_cores)
        assert r.iterations == k
        secs += t
    return len(variants) * n * n * k / secs / 1e9, secs, threads


def kern_table(stats):
    out = {}
    for name, s in stats.items():
        if s["launches"] and s["seconds"] > 0:
            out[name] = dict(launches=s["launches"],
                             avg_us=round(s["seconds"] / s["launches"] * 1e6, 2),
                             GBps=round(s["bytes"] / s["seconds"] / 1e9, 1))
    return out


# ------------------------------------------------------------------ headline --

def headline(args):
    torch, cg = setup()
    from paper_1803_03797_amd import workloads
    dev = torch.device("cuda:0")
    n = args.n
    dof = n * n
    log("bench: %dx%d, %d iterations per variant, steps=%d warmup=%d" %
        (n, n, args.iters, args.steps, args.warmup))
    ctx = cg.Context(device=0, arena_bytes=(64 * dof + (1 << 30)))
    xs = torch.from_numpy(workloads.large_solution(n, n)).to(dev)
    b = torch.zeros_like(xs)
    ctx.cg_apply(xs, b, n, n)  # b = A x* with the library's stencil
    x = torch.zeros_like(b)
    probs = [cg.make_problem(b, x, n, n, tol=0.0, maxit=args.iters, variant=v)
             for v in (cg.CG_VARIANT_CLASSIC, cg.CG_VARIANT_PIPELINED)]

    def step():
        out = []
        for p in probs:
            rc, r = ctx.cg_solve(p)
            assert rc == cg.CG_OK and r.iterations == args.iters, (rc, r.as_dict())
            out.append(r.device_seconds)
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    per_variant = [0.0, 0.0]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s = step()
        per_variant[0] += s[0]
        per_variant[1] += s[1]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = elapsed / args.steps * 1e3
    value = 2 * dof * args.iters * args.steps / elapsed / 1e9
    log("timed: %.2f ms/step, %.2f GDOF-iter/s" % (ms, value))

    # the same steps again with HIP events around every launch
    ctx.cg_set_profiling(True)
    ctx.cg_kernel_stats(reset=True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof_elapsed = time.perf_counter() - tp0
    stats = ctx.cg_kernel_stats(reset=True)
    ctx.cg_set_profiling(False)
    kern = kern_table(stats)
    log("kernels:", json.dumps(kern))
    pk = stats.get("pcg_pass")
    roof = None
    if pk and pk["launches"]:
        avg = pk["seconds"] / pk["launches"]
        per_launch = BYTES_PER_DOF["pcg_pass"] * dof
        ach = per_launch / avg / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": PCG_TRAFFIC_BYTES,
                "kernel": "pcg_pass", "avg_launch_us": round(avg * 1e6, 2),
                "bytes_per_launch": per_launch, "launches": pk["launches"]}

    # the iteration as a whole: each variant's algorithmic bytes of an
    # odd/even iteration pair over the summed average times of its passes
    it_roof = {}
    for name, ks in (("classic", ("stencil_dot", "stencil_dot", "update_norm", "update_norm_nx")),
                     ("pipelined", ("pcg_pass", "pcg_pass_nx"))):
        if all(k in stats and stats[k]["launches"] for k in ks):
            t = sum(stats[k]["seconds"] / stats[k]["launches"] for k in ks)
            by = sum(BYTES_PER_DOF[k] for k in ks) * dof
            it_roof[name] = {"achieved": round(by / t / 1e9, 1),
                             "frac": round(by / t / 1e9 / HBM_PEAK_GBPS, 4),
                             "us_per_iteration_pair": round(t * 1e6, 2)}

    tol_runs = None
    if args.tol_run:
        tol_runs = {}
        for v, name in ((0, "classic"), (1, "pipelined")):
            p = cg.make_problem(b, x, n, n, tol=1e-8, maxit=20000, variant=v)
            rc, r = ctx.cg_solve(p)
            err = ((x - xs).norm() / xs.norm()).item()
            tol_runs[name] = dict(status=cg.cg_status_str(rc), iterations=r.iterations,
                                  seconds=round(r.device_seconds, 4),
                                  rel_res_recursive=r.rel_res_recursive,
                                  rel_res_true=r.rel_res_true, err_vs_xstar=err)
        log("tol 1e-8:", json.dumps(tol_runs))

    cpu = None
    if not args.no_cpu:
        bh = b.cpu().numpy()
        k = args.cpu_iters
        v1, t1, _ = cpu_rate(bh, n, (0, 1), k, False)
        va, ta, tha = cpu_rate(bh, n, (0, 1), k, True)
        cpu = {"value": round(v1, 5), "unit": "GDOF-iter/s", "cores": 1, "kind": "oracle",
               "sample": "classic + pipelined CG, %d iterations each, %dx%d FP64, explicit CSR, "
                         "one thread; the iterations timed without the CSR assembly (%.1f s)"
                         % (k, n, n, t1),
               "host": host_info(),
               "all_cores": {"value": round(va, 5), "unit": "GDOF-iter/s", "threads": tha,
                             "kind": "oracle, OpenMP build of the same CSR code (rows split "
                                     "over the threads, per-thread dot partials added in "
                                     "thread order)",
                             "seconds": round(ta, 2)}}
        log("cpu oracle:", json.dumps(cpu))

    emit({
        "metric": "CG GDOF-iter/s (4096^2 FP64, classic + pipelined, 500 iterations each)",
        "value": round(value, 3), "unit": "GDOF-iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "%dx%d Laplace, b=A(sin*sin+1e-3 noise), x0=0, fixed %d "
                               "iterations per variant" % (n, n, args.iters),
                   "nx": n, "ny": n, "iterations": args.iters,
                   "variants": ["classic", "pipelined"]},
        "per_variant_GDOF_iter_s": {
            "classic": round(dof * args.iters * args.steps / per_variant[0] / 1e9, 3),
            "pipelined": round(dof * args.iters * args.steps / per_variant[1] / 1e9, 3)},
        "algorithmic_GBps": {
            v: round(BYTES_PER_ITER[v] * dof * args.iters * args.steps / per_variant[i] / 1e9, 1)
            for i, v in enumerate(("classic", "pipelined"))},
        "roofline": roof,
        "iteration_roofline": it_roof,
        "kernels": kern,
        "profiled_ms_per_step": round(prof_elapsed / args.steps * 1e3, 3),
        "tol_1e-8": tol_runs,
        "cpu_baseline": cpu,
    })
    ctx.close()


# --------------------------------------------------------------------- small --

def bench_small(args):
    torch, cg = setup()
    import numpy as np

    from paper_1803_03797_amd import workloads
    w = workloads.SMALL
    nx, ny = w["nx"], w["ny"]
    b = workloads.small_problem()
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    ctx = cg.Context(device=0, arena_bytes=256 << 20)
    out = {}
    for v, name in ((0, "classic"), (1, "pipelined")):
        p = cg.make_problem(bd, xd, nx, ny, tol=w["tol"], maxit=w["maxit"], variant=v)
        for _ in range(5):
            ctx.cg_solve(p)
        lat = []
        t0 = time.perf_counter()
        for _ in range(args.count):
            t = time.perf_counter()
            rc, r = ctx.cg_solve(p)
            lat.append(time.perf_counter() - t)
        total = time.perf_counter() - t0
        ctx.cg_set_profiling(True)
        ctx.cg_kernel_stats(reset=True)
        ctx.cg_solve(p)
        ks = kern_table(ctx.cg_kernel_stats(reset=True))
        ctx.cg_set_profiling(False)
        lat = np.array(lat)
        out[name] = dict(status=cg.cg_status_str(rc), iterations=r.iterations,
                         p50_ms=round(float(np.median(lat)) * 1e3, 4),
                         p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 4),
                         solves_per_s=round(args.count / total, 1),
                         us_per_iteration=round(float(np.median(lat)) / r.iterations * 1e6, 3),
                         GDOF_iter_s=round(nx * ny * r.iterations * args.count / total / 1e9, 4),
                         kernel=ks)
        log(name, json.dumps(out[name]))
    cpu = None
    if not args.no_cpu:
        import oracle
        cpu = {}
        for v, name in ((0, "classic"), (1, "pipelined")):
            t = time.perf_counter()
            reps = 3
            for _ in range(reps):
                xo, ro = oracle.cg(b, nx, ny, variant=v, tol=w["tol"], maxit=w["maxit"])
            cpu[name] = dict(ms_per_solve=round((time.perf_counter() - t) / reps * 1e3, 3),
                             iterations=ro.iterations)
        cpu = {"value": cpu, "unit": "ms per solve", "cores": 1, "kind": "oracle",
               "sample": "3 full solves per variant, 100x100, explicit CSR, single thread"}
    emit({"metric": "100x100 solve latency (tol 1e-8)", "workload": "small",
          "config": {"workload": "100x100, b~U[-1,1] seeded, x0=0, tol 1e-8, maxit 2000",
                     "solves": args.count},
          "dtype": "f64", "results": out, "cpu_baseline": cpu,
          "paper_context": "FPGA (Table resNewCG / resCG, N=100, FACTOR 16, 120 iterations, "
                           "RHS/tol not stated): NewCG 1.81 ms, CG 2.66 ms"})
    ctx.close()


# --------------------------------------------------------------------- batch --

def bench_batch(args):
    torch, cg = setup()
    import numpy as np

    from paper_1803_03797_amd import workloads
    w = workloads.BATCH
    op = args.batch_op
    pc = args.batch_precond
    if pc and op != "2d":
        raise SystemExit("--batch-precond applies to the 5-point operator only")
    if op == "3d":
        shapes = workloads.batch_shapes3(w["count"])[:args.count]
        bs = [torch.from_numpy(workloads.batch_rhs3(m, *s)).cuda() for m, s in enumerate(shapes)]
        dof = np.array([nx * ny * nz for nx, ny, nz in shapes], dtype=float)
    else:
        shapes = workloads.batch_shapes(w["count"])[:args.count]
        bs = [torch.from_numpy(workloads.batch_rhs(m, nx, ny)).cuda()
              for m, (nx, ny) in enumerate(shapes)]
        dof = np.array([nx * ny for nx, ny in shapes], dtype=float)
    faces = [None] * len(shapes)
    if op == "vc":
        faces = [tuple(torch.from_numpy(f).cuda() for f in workloads.batch_faces(m, nx, ny))
                 for m, (nx, ny) in enumerate(shapes)]
    xb = [torch.zeros_like(b) for b in bs]
    xs = [torch.zeros_like(b) for b in bs]
    ctx = cg.Context(device=0, arena_bytes=8 << 30)

    def mk(m, x):
        s, f = shapes[m], faces[m]
        return cg.make_problem(bs[m], x, s[0], s[1], tol=w["tol"], maxit=w["maxit"],
                               variant=cg.CG_VARIANT_PIPELINED, precond=pc,
                               nz=s[2] if op == "3d" else 0,
                               kx=f[0] if f else None, ky=f[1] if f else None)
    # warm (graph capture and code paths), then timed
    ctx.cg_solve_batch([mk(m, xb[m]) for m in range(min(8, len(shapes)))])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, res = ctx.cg_solve_batch([mk(m, xb[m]) for m in range(len(shapes))])
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    its = np.array([r.iterations for r in res], dtype=float)
    log("batched: %.3f s, status %s" % (tb, cg.cg_status_str(rc)))
    t0 = time.perf_counter()
    res1 = []
    for m in range(len(shapes)):
        rc1, r1 = ctx.cg_solve(mk(m, xs[m]))
        res1.append(r1)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    log("one-by-one: %.3f s" % ts)
    same = sum(int(torch.equal(a, c)) for a, c in zip(xb, xs))
    same_it = sum(int(r.iterations == r1.iterations) for r, r1 in zip(res, res1))
    work = float(np.sum(dof * its))
    cpu = None
    if not args.no_cpu:
        import oracle
        order = np.argsort(dof)[: args.cpu_solves]
        t = time.perf_counter()
        cw = 0.0
        for m in order:
            nx, ny = shapes[m][:2]
            if pc:
                xo, ro = oracle.pcg(bs[m].cpu().numpy(), nx, ny, pc, tol=w["tol"],
                                    maxit=w["maxit"], variant=1)
            elif op == "3d":
                xo, ro = oracle.cg3(bs[m].cpu().numpy(), nx, ny, shapes[m][2], variant=1,
                                    tol=w["tol"], maxit=w["maxit"])
            elif op == "vc":
                xo, ro = oracle.cg_vc(bs[m].cpu().numpy(), nx, ny, faces[m][0].cpu().numpy(),
                                      faces[m][1].cpu().numpy(), variant=1, tol=w["tol"],
                                      maxit=w["maxit"])
            else:
                xo, ro = oracle.cg(bs[m].cpu().numpy(), nx, ny, variant=1, tol=w["tol"],
                                   maxit=w["maxit"])
            cw += dof[m] * ro.iterations
        ct = time.perf_counter() - t
        cpu = {"value": round(cw / ct / 1e9, 5), "unit": "GDOF-iter/s", "cores": 1,
               "kind": "oracle",
               "sample": "the %d smallest of the solves, pipelined CG%s, explicit CSR, single "
                         "thread (%.1f s)" % (len(order), " + Chebyshev s=%d" % pc if pc else
                                              OP_NAMES[op], ct),
               "extrapolated_batch_seconds": round(work / (cw / ct), 1)}
    recipe = {"2d": "sides i.i.d. from {64..1024} per axis",
              "3d": "3D grids, sides i.i.d. from {16, 32, 48, 64, 96} per axis",
              "vc": "sides i.i.d. from {64..1024} per axis, face conductivities "
                    "i.i.d. U[0.5, 2]"}[op]
    per_iter = BYTES_PER_ITER["pipelined"] + (32 if op == "vc" else 0)
    emit({"metric": "batch solves/s (pipelined FP64, tol 1e-8, multi-solve step kernel)",
          "workload": "batch", "operator": op, "chebyshev_steps": pc,
          "config": {"workload": "%d solves, %s, b~U[-1,1]" % (len(shapes), recipe),
                     "total_dof": int(dof.sum())},
          "dtype": "f64",
          "batched": {"seconds": round(tb, 4), "solves_per_s": round(len(shapes) / tb, 2),
                      "GDOF_iter_s": round(work / tb / 1e9, 3),
                      "algorithmic_GBps": round(per_iter * work / tb / 1e9, 1)},
          "one_by_one": {"seconds": round(ts, 4), "solves_per_s": round(len(shapes) / ts, 2),
                         "GDOF_iter_s": round(work / ts / 1e9, 3)},
          "speedup": round(ts / tb, 3), "status": cg.cg_status_str(rc),
          "iterations": {"min": int(its.min()), "max": int(its.max()),
                         "sum": int(its.sum())},
          "batch_equals_alone": {"bitwise_x": same, "iterations": same_it, "of": len(shapes)},
          "cpu_baseline": cpu})
    ctx.close()


# --------------------------------------------------------------------- fixed --

def bench_fixed(args):
    torch, cg = setup()
    import numpy as np

    from paper_1803_03797_amd import workloads
    W = workloads.FIXED
    FX = cg.CG_PREC_FIXED
    names = ((0, "classic"), (1, "pipelined"))
    ctx = cg.Context(device=0, arena_bytes=2 << 30)
    reps = args.count or 50
    latency = {}
    for n, iters in zip(W["sides"], W["iterations"]):
        b = torch.from_numpy(workloads.fixed_rhs(n)).cuda()
        x = torch.zeros_like(b)
        row = {}
        for v, name in names:
            p = cg.make_problem(b, x, n, n, tol=0.0, maxit=iters, variant=v, precision=FX)
            for _ in range(3):
                ctx.cg_solve(p)
            lat = []
            for _ in range(reps):
                t = time.perf_counter()
                rc, r = ctx.cg_solve(p)
                lat.append(time.perf_counter() - t)
            ctx.cg_set_profiling(True)
            ctx.cg_kernel_stats(reset=True)
            for _ in range(5):
                ctx.cg_solve(p)
            ks = kern_table(ctx.cg_kernel_stats(reset=True))
            ctx.cg_set_profiling(False)
            k_us = ks["solve_fixed"]["avg_us"]
            row[name] = dict(status=cg.cg_status_str(rc), iterations=r.iterations,
                             p50_ms=round(float(np.median(lat)) * 1e3, 4),
                             kernel_us=k_us, us_per_iteration=round(k_us / iters, 3))
        latency["%dx%d/%d it" % (n, n, iters)] = row
        log("fixed latency", n, json.dumps(row))
    # throughput: W["batch"] solves of the largest grid in one launch per variant
    n, iters = W["sides"][-1], W["iterations"][-1]
    count = W["batch"]
    bs = [torch.from_numpy(workloads.fixed_rhs(n, m)).cuda() for m in range(count)]
    xs = [torch.zeros_like(b) for b in bs]
    batch, roof = {}, {}
    for v, name in names:
        probs = [cg.make_problem(b, x, n, n, tol=0.0, maxit=iters, variant=v, precision=FX)
                 for b, x in zip(bs, xs)]
        ctx.cg_solve_batch(probs[:8])
        torch.cuda.synchronize()
        walls = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            rc, res = ctx.cg_solve_batch(probs)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        assert rc == cg.CG_OK and all(r.iterations == iters for r in res)
        ctx.cg_set_profiling(True)
        ctx.cg_kernel_stats(reset=True)
        for _ in range(3):
            ctx.cg_solve_batch(probs)
        ks = kern_table(ctx.cg_kernel_stats(reset=True))
        ctx.cg_set_profiling(False)
        k_s = ks["solve_fixed_many"]["avg_us"] * 1e-6
        wall = float(np.median(walls))
        work = count * n * n * iters
        muls = work * FX_PRODUCTS[name] * FX_MULS_PER_PRODUCT
        batch[name] = dict(solves=count, wall_s=round(wall, 5),
                           solves_per_s=round(count / wall, 1),
                           GDOF_iter_s=round(work / wall / 1e9, 3),
                           kernel_ms=round(k_s * 1e3, 4),
                           GDOF_iter_s_kernel=round(work / k_s / 1e9, 3))
        roof[name] = {"bound": "alu", "achieved": round(muls / k_s / 1e9, 1),
                      "peak": FX_MUL_PEAK_G, "unit": "Gmul/s",
                      "frac": round(muls / k_s / 1e9 / FX_MUL_PEAK_G, 4), "traffic": None}
        log("fixed batch", name, json.dumps(batch[name]))
    cpu = None
    if not args.no_cpu:
        import oracle.oracle as oo
        cpu = {}
        for v, name in names:
            t = time.perf_counter()
            k = 0
            while time.perf_counter() - t < 4.0 and k < 50:
                oo.cg_fixed(bs[k].cpu().numpy(), n, n, variant=v, tol=0.0, maxit=iters)
                k += 1
            dt = time.perf_counter() - t
            cpu[name] = round(k * n * n * iters / dt / 1e9, 5)
        cpu = {"value": cpu, "unit": "GDOF-iter/s", "cores": 1, "kind": "oracle",
               "sample": "consecutive %dx%d solves of %d iterations per variant for about "
                         "4 s, plain C with __int128, single thread" % (n, n, iters)}
    value = sum(batch[nm]["GDOF_iter_s"] for _, nm in names) / 2
    emit({"metric": "fixed-point GDOF-iter/s (batch of %d %dx%d solves, %d iterations)"
                    % (count, n, n, iters),
          "workload": "fixed", "value": round(value, 3), "unit": "GDOF-iter/s",
          "config": {"workload": "Q20.30 fixed point; paper grids %s with %s iterations, "
                                 "b~U[-1,1] seeded, x0=0, tol 0" % (list(W["sides"]),
                                                                     list(W["iterations"])),
                     "batch": count},
          "dtype": "q20.30 (int64)", "latency": latency, "batch": batch, "roofline": roof,
          "cpu_baseline": cpu,
          "paper_context": "FPGA latency at the largest FACTOR (Tables resCG/resNewCG, 100 MHz): "
                           "N=16 CG 0.15 / NewCG 0.10 ms; N=32 0.40 / 0.26 ms; N=40 0.46 / "
                           "0.29 ms; N=100 2.66 / 1.81 ms"})
    ctx.close()


# ------------------------------------------------------------------ precond --

def bench_precond(args):
    torch, cg = setup()
    import numpy as np

    from paper_1803_03797_amd import workloads
    n = args.n
    w = workloads.LARGE
    dev = torch.device("cuda:0")
    xs = torch.from_numpy(workloads.large_solution(n, n)).to(dev)
    b = torch.empty_like(xs)
    ctx = cg.Context(device=0, arena_bytes=8 << 30)
    ctx.cg_apply(xs, b, n, n)  # b = A x* with the library's stencil
    nxs = float(torch.linalg.norm(xs))
    out = {}
    legs = [(0, 0)] + [(0, s) for s in args.steps_list] + \
        [(1, s) for s in args.steps_list if s in (4, 8)]
    for variant, s in legs:
        x = torch.zeros_like(b)
        p = cg.make_problem(b, x, n, n, tol=w["tol"], maxit=w["maxit"], precond=s,
                            variant=variant)
        ctx.cg_solve(p)  # warm: graphs captured
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, r = ctx.cg_solve(p)
        torch.cuda.synchronize()
        tt = time.perf_counter() - t0
        err = float(torch.linalg.norm(x - xs)) / nxs
        # per-pass kernel times over a short fixed run
        ctx.cg_set_profiling(True)
        ctx.cg_kernel_stats(reset=True)
        ctx.cg_solve(cg.make_problem(b, torch.zeros_like(b), n, n, tol=0.0, maxit=20, precond=s,
                                     variant=variant))
        ks = kern_table(ctx.cg_kernel_stats(reset=True))
        ctx.cg_set_profiling(False)
        name = "cg" if s == 0 else ("pcg_s%d" if variant == 0 else "ppcg_s%d") % s
        iter_kernels = ("cheb_precond", "stencil_dot", "update_norm", "update_norm_nx",
                        "cheb_precond_w", "ppcg_pass")
        per_it = sum(v["avg_us"] * v["launches"] for k, v in ks.items() if k in iter_kernels) / 20
        out[name] = dict(status=cg.cg_status_str(rc), iterations=r.iterations,
                         seconds=round(tt, 4), rel_err_vs_xstar=float("%.3g" % err),
                         rel_res_true=float("%.3g" % r.rel_res_true),
                         us_per_iteration=round(per_it, 1),
                         kernels={k: v for k, v in ks.items() if k in iter_kernels})
        log(name, json.dumps(out[name]))
    base = out["cg"]["seconds"]
    best = min((v["seconds"], k) for k, v in out.items())
    # roofline of the Chebyshev pass at the fastest s: FP64 operations per
    # unknown (stage 0 scale and the (r,z) fma, then per stencil step 5 for
    # the stencil, 1 for r, 2 for d, 1 for y) against the FP64 vector issue
    # rate; its HBM view (read r, write z: 16 B per unknown) beside it
    roof = None
    if best[1] != "cg":
        sb = int(best[1].split("_s")[1])
        kb = out[best[1]]["kernels"]
        kc = kb["cheb_precond"] if "cheb_precond" in kb else kb["cheb_precond_w"]
        ops = (2 + 9 * (sb - 1)) * n * n
        ach = ops / (kc["avg_us"] * 1e-6) / 1e12
        roof = {"kernel": "cheb_precond", "s": sb,
                "bound": "alu" if sb >= 6 else "hbm",
                "achieved": round(ach, 2) if sb >= 6 else kc["GBps"],
                "peak": FP64_OP_PEAK_T if sb >= 6 else HBM_PEAK_GBPS,
                "unit": "TOP/s (FP64 ops, fma = 1)" if sb >= 6 else "GB/s",
                "frac": round(ach / FP64_OP_PEAK_T, 4) if sb >= 6
                else round(kc["GBps"] / HBM_PEAK_GBPS, 4),
                "hbm_view": {"achieved": kc["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                             "frac": round(kc["GBps"] / HBM_PEAK_GBPS, 4)},
                "avg_launch_us": kc["avg_us"], "ops_per_launch": ops,
                "traffic": CHEB_TRAFFIC_BYTES.get(sb) if n == 4096 else None}
    cpu = None
    if not args.no_cpu:
        import oracle.oracle as oo
        bh = b.cpu().numpy()
        sb = int(best[1].split("_s")[1]) if best[1] != "cg" else 8
        t = time.perf_counter()
        oo.pcg(bh, n, n, sb, tol=0.0, maxit=2)
        dt = time.perf_counter() - t
        its = out.get("pcg_s%d" % sb, out["cg"])["iterations"]
        cpu = {"value": round(dt / 2 * its, 1), "unit": "s (extrapolated)", "cores": 1,
               "kind": "oracle",
               "sample": "oracle preconditioned CG (explicit CSR, s = %d), 2 iterations at "
                         "%dx%d in %.1f s including CSR assembly, times the GPU's %d "
                         "iterations" % (sb, n, n, dt, its)}
    emit({"metric": "time to solution, %dx%d to tol 1e-8 (classic CG, Chebyshev-preconditioned "
                    "classic and pipelined CG)" % (n, n),
          "workload": "precond", "value": round(best[0], 4), "unit": "s",
          "higher_is_better": False,
          "config": {"workload": "%dx%d Laplace, b=A(sin*sin+1e-3 noise), x0=0, tol 1e-8" % (n, n),
                     "steps": list(args.steps_list)},
          "dtype": "f64", "results": out, "best": best[1],
          "speedup_vs_cg": round(base / best[0], 3), "roofline": roof, "cpu_baseline": cpu})
    ctx.close()


# ------------------------------------------------------------------------ 3d --

def bench_cube(args):
    """The 7-point operator on n^3: both variants, a fixed number of iterations
    (throughput, per-kernel times, the pipelined pass's roofline), then each to
    tol 1e-8."""
    torch, cg = setup()
    from paper_1803_03797_amd import workloads
    w = workloads.CUBE
    n = args.n_cube
    dof = n ** 3
    its = args.cube_iters or w["iterations"]
    b = torch.from_numpy(workloads.cube_rhs(n)).cuda()
    ctx = cg.Context(device=0, arena_bytes=64 * dof + (1 << 30))
    x = torch.zeros_like(b)
    out = {}
    for v, name in ((0, "classic"), (1, "pipelined")):
        p = cg.make_problem(b, x, n, n, tol=0.0, maxit=its, variant=v, nz=n)
        ctx.cg_solve(p)  # warm: graphs captured
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, r = ctx.cg_solve(p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.cg_set_profiling(True)
        ctx.cg_kernel_stats(reset=True)
        ctx.cg_solve(cg.make_problem(b, torch.zeros_like(b), n, n, tol=0.0, maxit=40, variant=v,
                                     nz=n))
        ks = kern_table(ctx.cg_kernel_stats(reset=True))
        ctx.cg_set_profiling(False)
        tol_run = None
        if not args.fixed_only:
            x2 = torch.zeros_like(b)
            p2 = cg.make_problem(b, x2, n, n, tol=w["tol"], maxit=w["maxit"], variant=v, nz=n)
            t1 = time.perf_counter()
            rc2, r2 = ctx.cg_solve(p2)
            dt2 = time.perf_counter() - t1
            tol_run = dict(status=cg.cg_status_str(rc2), iterations=r2.iterations,
                           seconds=round(dt2, 4), rel_res_true=r2.rel_res_true)
        out[name] = dict(GDOF_iter_s=round(dof * its / dt / 1e9, 3),
                         seconds_fixed=round(dt, 4),
                         algorithmic_GBps=round(dof * its * BYTES_PER_ITER[name] / dt / 1e9, 1),
                         kernels={k: vv for k, vv in ks.items() if k != "final_check"},
                         tol_1e8=tol_run)
        log("3d", name, json.dumps(out[name]))
    pk = out["pipelined"]["kernels"].get("pcg_pass")
    roof = None
    if pk:
        ach = BYTES_PER_DOF["pcg_pass"] * dof / (pk["avg_us"] * 1e-6) / 1e9
        roof = {"bound": "hbm", "kernel": "pcg_pass (7-point)", "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4),
                "avg_launch_us": pk["avg_us"], "bytes_per_launch": BYTES_PER_DOF["pcg_pass"] * dof,
                "traffic": CUBE_TRAFFIC_BYTES if n == 256 else None}
    cpu = None
    if not args.no_cpu:
        import oracle
        bh = b.cpu().numpy()
        k = 4
        oracle.cg3(bh, n, n, n, variant=0, tol=0.0, maxit=k)
        ct = oracle.last_solve_seconds()
        cpu = {"value": round(dof * k / ct / 1e9, 5), "unit": "GDOF-iter/s", "cores": 1,
               "kind": "oracle", "host": host_info(),
               "sample": "%d classic iterations of the 3D oracle at %d^3 (explicit 7-point CSR, "
                         "single thread; the iterations timed without the CSR assembly, %.2f s)"
                         % (k, n, ct)}
    value = (out["classic"]["GDOF_iter_s"] + out["pipelined"]["GDOF_iter_s"]) / 2
    emit({"metric": "CG GDOF-iter/s, 3D 7-point Laplacian %d^3 FP64 (classic + pipelined, %d "
                    "iterations each)" % (n, its),
          "workload": "cube", "value": round(value, 3), "unit": "GDOF-iter/s",
          "config": {"workload": "%d^3 7-point Laplacian, b~U[-1,1] seeded, x0=0; fixed %d "
                                 "iterations, then tol 1e-8" % (n, its)},
          "dtype": "f64", "results": out, "roofline": roof, "cpu_baseline": cpu})
    ctx.close()


# ------------------------------------------------------------------------ vc --

def bench_vc(args):
    """The variable-coefficient 5-point operator on n^2 (face conductivities
    log-uniform over [0.1, 10]): both variants, a fixed number of iterations
    (throughput, per-kernel times, the pipelined pass's roofline), then each to
    tol 1e-8."""
    torch, cg = setup()
    from paper_1803_03797_amd import workloads
    w = workloads.VC
    n = args.n_vc
    dof = n * n
    its = w["iterations"]
    kxh, kyh = workloads.vc_faces(n, n, w["k_lo"], w["k_hi"])
    bh = workloads.vc_rhs(n, n)
    b, kx, ky = (torch.from_numpy(a).cuda() for a in (bh, kxh, kyh))
    ctx = cg.Context(device=0, arena_bytes=100 * dof + (1 << 30))
    x = torch.zeros_like(b)
    out = {}
    for v, name in ((0, "classic"), (1, "pipelined")):
        p = cg.make_problem(b, x, n, n, tol=0.0, maxit=its, variant=v, kx=kx, ky=ky)
        ctx.cg_solve(p)  # warm: graphs captured
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, r = ctx.cg_solve(p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.cg_set_profiling(True)
        ctx.cg_kernel_stats(reset=True)
        ctx.cg_solve(cg.make_problem(b, torch.zeros_like(b), n, n, tol=0.0, maxit=40, variant=v,
                                     kx=kx, ky=ky))
        ks = kern_table(ctx.cg_kernel_stats(reset=True))
        ctx.cg_set_profiling(False)
        tol_run = None
        if not args.fixed_only:
            x2 = torch.zeros_like(b)
            p2 = cg.make_problem(b, x2, n, n, tol=w["tol"], maxit=w["maxit"], variant=v, kx=kx,
                                 ky=ky)
            t1 = time.perf_counter()
            rc2, r2 = ctx.cg_solve(p2)
            dt2 = time.perf_counter() - t1
            tol_run = dict(status=cg.cg_status_str(rc2), iterations=r2.iterations,
                           seconds=round(dt2, 4), rel_res_true=r2.rel_res_true)
        # each stencil pass also reads the four coefficients (32 B per unknown):
        # classic applies the stencil in both of its passes, pipelined in one
        per_iter = BYTES_PER_ITER[name] + (32 if name == "pipelined" else 64)
        out[name] = dict(GDOF_iter_s=round(dof * its / dt / 1e9, 3),
                         seconds_fixed=round(dt, 4),
                         algorithmic_GBps=round(dof * its * per_iter / dt / 1e9, 1),
                         kernels={k: vv for k, vv in ks.items() if k != "final_check"},
                         tol_1e8=tol_run)
        log("vc", name, json.dumps(out[name]))
    if not args.fixed_only:
        # the pipelined variant with residual replacement every rr iterations
        rr = args.rr_period
        x3 = torch.zeros_like(b)
        p3 = cg.make_problem(b, x3, n, n, tol=w["tol"], maxit=w["maxit"], variant=1, kx=kx,
                             ky=ky, rr_period=rr)
        t1 = time.perf_counter()
        rc3, r3 = ctx.cg_solve(p3)
        dt3 = time.perf_counter() - t1
        out["pipelined_rr%d" % rr] = dict(tol_1e8=dict(
            status=cg.cg_status_str(rc3), iterations=r3.iterations, seconds=round(dt3, 4),
            rel_res_recursive=r3.rel_res_recursive, rel_res_true=r3.rel_res_true))
        log("vc pipelined rr", json.dumps(out["pipelined_rr%d" % rr]))
    pk = out["pipelined"]["kernels"].get("pcg_pass")
    roof = None
    if pk:
        per_launch = (BYTES_PER_DOF["pcg_pass"] + 32) * dof
        ach = per_launch / (pk["avg_us"] * 1e-6) / 1e9
        roof = {"bound": "hbm", "kernel": "pcg_pass (variable coefficients)",
                "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBPS, 4), "avg_launch_us": pk["avg_us"],
                "bytes_per_launch": per_launch,
                "traffic": VC_TRAFFIC_BYTES if n == 4096 else None}
    cpu = None
    if not args.no_cpu:
        import oracle
        k = 4
        oracle.cg_vc(bh, n, n, kxh, kyh, variant=0, tol=0.0, maxit=k)
        ct = oracle.last_solve_seconds()
        cpu = {"value": round(dof * k / ct / 1e9, 5), "unit": "GDOF-iter/s", "cores": 1,
               "kind": "oracle", "host": host_info(),
               "sample": "%d classic iterations of the variable-coefficient oracle at %d^2 "
                         "(explicit CSR, single thread; the iterations timed without the CSR "
                         "assembly, %.2f s)" % (k, n, ct)}
    value = (out["classic"]["GDOF_iter_s"] + out["pipelined"]["GDOF_iter_s"]) / 2
    emit({"metric": "CG GDOF-iter/s, variable-coefficient 5-point operator %d^2 FP64 (classic "
                    "+ pipelined, %d iterations each)" % (n, its),
          "workload": "vc", "value": round(value, 3), "unit": "GDOF-iter/s",
          "config": {"workload": "%d^2 finite-volume -div(k grad u), face k log-uniform on "
                                 "[%g, %g] seeded, b~U[-1,1] seeded, x0=0; fixed %d "
                                 "iterations, then tol 1e-8" % (n, w["k_lo"], w["k_hi"], its)},
          "dtype": "f64", "results": out, "roofline": roof, "cpu_baseline": cpu})
    ctx.close()


# ---------------------------------------------------------------------- huge --

def bench_huge(args):
    torch, cg = setup()
    from paper_1803_03797_amd import workloads
    w = workloads.HUGE
    n = args.n_huge
    dof = n * n
    b = torch.from_numpy(workloads.huge_rhs(n, n)).cuda()
    ctx = cg.Context(device=0, arena_bytes=48 * dof + (1 << 30))
    out = {}

    def solve(x, **kw):
        """Timed without profiling (the library replays its graph chunks), then
        the kernel table from a profiled run of at most 400 iterations (one pass
        per launch, bracketed by events)."""
        p = cg.make_problem(b, x, n, n, tol=w["tol"], maxit=w["maxit"], **kw)
        t = time.perf_counter()
        rc, r = ctx.cg_solve(p)
        dt = time.perf_counter() - t
        xs = torch.zeros_like(b)
        ps = cg.make_problem(b, xs, n, n, tol=w["tol"], maxit=400, **kw)
        ctx.cg_set_profiling(True)
        ctx.cg_kernel_stats(reset=True)
        ctx.cg_solve(ps)
        kt = kern_table(ctx.cg_kernel_stats(reset=True))
        ctx.cg_set_profiling(False)
        del xs
        return rc, r, dt, kt

    xr = torch.zeros_like(b)
    rc, r, tr, kt = solve(xr, precision=cg.CG_PREC_FP32_REFINED, inner_tol=w["inner_tol"])
    out["refined"] = dict(status=cg.cg_status_str(rc), seconds=round(tr, 3),
                          outer=r.outer_iterations, inner=r.iterations,
                          rel_res_true=r.rel_res_true, kernels=kt)
    log("refined", json.dumps(out["refined"]))
    x64 = torch.zeros_like(b)
    rc, r, t64, kt = solve(x64, variant=0)
    out["fp64_classic"] = dict(status=cg.cg_status_str(rc), seconds=round(t64, 3),
                               iterations=r.iterations, rel_res_true=r.rel_res_true, kernels=kt)
    log("fp64", json.dumps(out["fp64_classic"]))
    if args.huge_precond:
        s_ = args.huge_precond
        # the same solve by classic CG preconditioned with s Chebyshev steps
        xp = torch.zeros_like(b)
        rc, r, tp, kt = solve(xp, variant=0, precond=s_)
        out["fp64_pcg_s%d" % s_] = dict(
            status=cg.cg_status_str(rc), seconds=round(tp, 3), iterations=r.iterations,
            rel_res_true=r.rel_res_true,
            rel_err_vs_fp64_classic=((xp - x64).norm() / x64.norm()).item(), kernels=kt)
        log("fp64 pcg", json.dumps(out["fp64_pcg_s%d" % s_]))
        # and by the refinement whose FP32 inner solve carries the same
        # preconditioner (binary32 Chebyshev steps)
        xq = torch.zeros_like(b)
        tols = [float(v) for v in str(args.huge_pc_inner_tol).split(",")]
        itol = tols[0]
        rc, r, tq, kt = solve(xq, precision=cg.CG_PREC_FP32_REFINED, inner_tol=itol, precond=s_)
        out["refined_pcg_s%d" % s_] = dict(
            status=cg.cg_status_str(rc), seconds=round(tq, 3), inner_tol=itol,
            outer=r.outer_iterations, inner=r.iterations, rel_res_true=r.rel_res_true,
            rel_err_vs_fp64_classic=((xq - x64).norm() / x64.norm()).item(),
            speedup_vs_fp64_pcg=round(tp / tq, 3), kernels=kt)
        log("refined pcg", json.dumps(out["refined_pcg_s%d" % s_]))
        # further inner tolerances (timed only)
        sweep = []
        for itol2 in tols[1:]:
            xq.zero_()
            p = cg.make_problem(b, xq, n, n, tol=w["tol"], maxit=w["maxit"],
                                precision=cg.CG_PREC_FP32_REFINED, inner_tol=itol2, precond=s_)
            t = time.perf_counter()
            rc, r = ctx.cg_solve(p)
            sweep.append(dict(inner_tol=itol2, status=cg.cg_status_str(rc),
                              seconds=round(time.perf_counter() - t, 3),
                              outer=r.outer_iterations, inner=r.iterations,
                              rel_res_true=r.rel_res_true))
            log("refined pcg sweep", json.dumps(sweep[-1]))
        if sweep:
            out["refined_pcg_s%d_inner_tol_sweep" % s_] = sweep
        del xp, xq
    err = ((xr - x64).norm() / x64.norm()).item()
    kappa = (4 - 4 * math.cos(n * math.pi / (n + 1))) / (4 - 4 * math.cos(math.pi / (n + 1)))
    cpu = None
    if not args.no_cpu:
        bh = b.cpu().numpy()
        k = 3
        v1, t1, _ = cpu_rate(bh, n, (0,), k, False)
        cpu = {"value": round(v1, 5), "unit": "GDOF-iter/s", "cores": 1, "kind": "oracle",
               "sample": "%d classic iterations at %dx%d, one thread, timed without the CSR "
                         "assembly (%.1f s); a full solve is extrapolated, not run" % (k, n, n, t1),
               "host": host_info(),
               "extrapolated_fp64_solve_s": round(dof * out["fp64_classic"]["iterations"] /
                                                  (v1 * 1e9), 0)}
    emit({"metric": "8192^2 time to solution, FP32-refined vs FP64 CG (true rel. res 1e-10)",
          "workload": "huge",
          "config": {"workload": "%dx%d, b~N(0,1) seeded, x0=0, outer tol 1e-10 (true FP64 "
                                 "residual), inner tol %g (preconditioned refinement %g)"
                                 % (n, n, w["inner_tol"],
                                    float(str(args.huge_pc_inner_tol).split(",")[0]))},
          "results": out, "speedup_refined_vs_fp64": round(t64 / tr, 3),
          "error_refined_vs_fp64": err, "a_priori_bound_2_tol_kappa": 2 * w["tol"] * kappa,
          "cpu_baseline": cpu})
    ctx.close()


# ---------------------------------------------------------------------- serve --

def bench_serve(args):
    torch, cg = setup()
    import numpy as np

    from paper_1803_03797_amd import workloads
    reqs = workloads.serve_requests(args.count)
    bs = [torch.from_numpy(workloads.serve_rhs(m, nx, ny)).cuda()
          for m, (nx, ny, _) in enumerate(reqs)]
    ctx = cg.Context(device=0, arena_bytes=16 << 30)
    dof = np.array([nx * ny for nx, ny, _ in reqs], dtype=float)

    def prob(m, x, precision, precond=0):
        nx, ny, tol = reqs[m]
        return cg.make_problem(bs[m], x, nx, ny, tol=tol, maxit=200000, variant=0,
                               precision=precision, inner_tol=1e-4, precond=precond)

    def met(rc, r, m):
        # equal accuracy: every result's true FP64 residual meets its tolerance
        return int(rc == cg.CG_OK and r.rel_res_true <= reqs[m][2] * 1.0000001)

    # per-request FP64: one cg_solve after another, all queued at t = 0
    x64 = [torch.zeros_like(b) for b in bs]
    for m in range(min(4, len(reqs))):
        ctx.cg_solve(prob(m, torch.zeros_like(bs[m]), 0))
    svc = np.zeros(len(reqs))
    ok64 = 0
    t0 = time.perf_counter()
    for m in range(len(reqs)):
        t = time.perf_counter()
        rc, r = ctx.cg_solve(prob(m, x64[m], 0))
        svc[m] = time.perf_counter() - t
        ok64 += met(rc, r, m)
        if (m + 1) % 2000 == 0:
            log("per-request FP64: %d done" % (m + 1))
    cap64 = len(reqs) / (time.perf_counter() - t0)
    log("per-request FP64: %.1f solves/s" % cap64)

    def per_request(arrivals):
        # per-request FP64 under the same arrivals, measured: one solver
        # thread takes the requests in arrival order (FIFO) and solves each
        # alone with cg_solve; latency = completion - arrival
        xs = [torch.zeros_like(b) for b in bs]
        lat = np.zeros(len(reqs))
        start = time.perf_counter()
        for m in range(len(reqs)):
            dt = arrivals[m] - (time.perf_counter() - start)
            if dt > 0:
                time.sleep(dt)
            ctx.cg_solve(prob(m, xs[m], 0))
            lat[m] = time.perf_counter() - start - arrivals[m]
            if (m + 1) % 2000 == 0:
                log("per-request FP64 under arrivals: %d done" % (m + 1))
        return lat, time.perf_counter() - start

    iters = [0] * len(reqs)

    def served(precision, arrivals, precond=0):
        xs = [torch.zeros_like(b) for b in bs]
        tickets = [None] * len(reqs)
        results = {}
        start = time.perf_counter()

        def submitter():
            for m in range(len(reqs)):
                if arrivals is not None:
                    dt = arrivals[m] - (time.perf_counter() - start)
                    if dt > 0:
                        time.sleep(dt)
                tickets[m] = ctx.cg_submit(prob(m, xs[m], precision, precond))

        th = threading.Thread(target=submitter)
        th.start()
        pending, nxt, shown = [], 0, 0
        while len(results) < len(reqs):
            # poll only the submitted, unfinished tickets (latency is stamped
            # by the server at completion, so the sweep period does not enter it)
            while nxt < len(reqs) and tickets[nxt] is not None:
                pending.append(nxt)
                nxt += 1
            still = []
            for m in pending:
                rc, r = ctx.cg_poll(tickets[m])
                if rc != cg.CG_PENDING:
                    results[m] = (rc, cg.cg_result.from_buffer_copy(r), time.perf_counter() - start)
                else:
                    still.append(m)
            pending = still
            if len(results) >= shown + 2000:
                shown = len(results) // 2000 * 2000
                log("served: %d done" % len(results))
            time.sleep(0.002 if len(reqs) > 1000 else 0.0005)
        th.join()
        iters[:] = [results[m][1].iterations for m in range(len(reqs))]
        makespan = max(v[2] for v in results.values())
        lat = np.array([results[m][1].latency_seconds for m in range(len(reqs))])
        ok = sum(met(results[m][0], results[m][1], m) for m in range(len(reqs)))
        return xs, dict(solves_per_s=round(len(reqs) / makespan, 2),
                        makespan_s=round(makespan, 3),
                        p50_ms=round(float(np.median(lat)) * 1e3, 3),
                        p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3),
                        met_tolerance=ok)

    # saturated throughput: every request submitted at t = 0
    xs_ref, sat_ref = served(cg.CG_PREC_FP32_REFINED, None)
    log("served FP32-refined, saturated", json.dumps(sat_ref))
    xs_64, sat_64 = served(cg.CG_PREC_FP64, None)
    sat_iters = list(iters)
    log("served FP64, saturated", json.dumps(sat_64))
    # the size-based policy: FP64 below 20480 unknowns, FP32-refined above
    _, sat_auto = served(cg.CG_PREC_AUTO, None)
    log("served auto precision, saturated", json.dumps(sat_auto))
    sat_pc = sat_pca = None
    if args.serve_precond:
        # the same stream served as Chebyshev-preconditioned classic CG (FP64)
        _, sat_pc = served(cg.CG_PREC_FP64, None, args.serve_precond)
        log("served FP64 + Chebyshev s=%d, saturated" % args.serve_precond, json.dumps(sat_pc))
        # and by the size-based policy with the preconditioner (refined
        # requests precondition their FP32 inner solves)
        _, sat_pca = served(cg.CG_PREC_AUTO, None, args.serve_precond)
        log("served auto precision + Chebyshev s=%d, saturated" % args.serve_precond,
            json.dumps(sat_pca))
    same = sum(int(torch.equal(a, c)) for a, c in zip(xs_64, x64))
    # latency under Poisson arrivals at fractions of the per-request capacity
    loads = {}
    for frac in args.loads:
        arr = workloads.poisson_arrivals(len(reqs), frac * cap64, seed_item=int(frac * 100))
        lat64, make64 = per_request(arr)
        entry = {"arrival_rate_per_s": round(frac * cap64, 2),
                 "per_request_fp64": dict(solves_per_s=round(len(reqs) / make64, 2),
                                          p50_ms=round(float(np.median(lat64)) * 1e3, 3),
                                          p99_ms=round(float(np.percentile(lat64, 99)) * 1e3,
                                                       3))}
        _, entry["served_fp32_refined"] = served(cg.CG_PREC_FP32_REFINED, arr)
        _, entry["served_fp64"] = served(cg.CG_PREC_FP64, arr)
        _, entry["served_auto_precision"] = served(cg.CG_PREC_AUTO, arr)
        loads["%.2f" % frac] = entry
        log("load %.2f:" % frac, json.dumps(entry))
    # a 1% sample (every 100th request) on the host: the true residual of the
    # served FP64 and refined solutions with the oracle's explicit CSR
    # matrix, and the oracle's own solve time (one thread, the iterations
    # without the CSR assembly: 20 iterations timed, scaled to the iteration
    # count of the request's served FP64 solve)
    import oracle
    sample = list(range(0, len(reqs), 100))
    host_ok = {"served_fp64": 0, "served_fp32_refined": 0}
    worst = {"served_fp64": 0.0, "served_fp32_refined": 0.0}
    cpu_s = 0.0
    for m in sample:
        nx, ny, tol = reqs[m]
        bh = bs[m].cpu().numpy()
        nb = np.linalg.norm(bh)
        for name, xs in (("served_fp64", xs_64), ("served_fp32_refined", xs_ref)):
            xh = xs[m].cpu().numpy()
            rt = np.linalg.norm(bh - oracle.spmv(xh, nx, ny)) / nb
            worst[name] = max(worst[name], rt / tol)
            host_ok[name] += int(rt <= tol * 1.0001)
        its = sat_iters[m]
        k = min(20, max(its, 1))
        _, t, _ = oracle.cg_timed(bh, nx, ny, 0, tol=0.0, maxit=k)
        cpu_s += t / k * its
    cpu = None if args.no_cpu else {
        "value": round(len(sample) / cpu_s, 3), "unit": "solves/s", "cores": 1, "kind": "oracle",
        "sample": "%d requests (every 100th), classic CG, one thread: 20 iterations each timed "
                  "without the CSR assembly and scaled to the request's iteration count "
                  "(%.1f s extrapolated)" % (len(sample), cpu_s),
        "host": host_info()}
    log("host check:", json.dumps(host_ok), "cpu:", json.dumps(cpu))
    emit({"metric": "served solves/s and p50/p99 latency (FP32-refined vs per-request FP64)",
          "workload": "serve",
          "config": {"workload": "%d requests, sides log-uniform [32,2048] per axis, tol 1e-6 or "
                                 "1e-8, b~U[-1,1]" % len(reqs), "total_dof": int(dof.sum()),
                     "classic CG; refined: inner tol 1e-4": True},
          "saturated_solves_per_s": {"per_request_fp64": round(cap64, 2),
                                     "served_fp32_refined": sat_ref["solves_per_s"],
                                     "served_fp64": sat_64["solves_per_s"],
                                     "served_auto_precision": sat_auto["solves_per_s"]},
          "saturated": {"served_fp32_refined": sat_ref, "served_fp64": sat_64,
                        "served_auto_precision": sat_auto,
                        "per_request_fp64_met_tolerance": ok64,
                        "served_fp64_chebyshev_s%d" % args.serve_precond: sat_pc,
                        "served_auto_chebyshev_s%d" % args.serve_precond: sat_pca},
          "poisson_loads_x_per_request_capacity": loads,
          "per_request_latency": "measured: one thread solves the requests one by one in "
                                 "arrival order (cg_solve each)",
          "host_csr_check_1pct": {"requests": len(sample), "true_res_le_tol": host_ok,
                                  "worst_true_res_over_tol": worst},
          "served_fp64_equals_alone_bitwise": same, "of": len(reqs), "cpu_baseline": cpu})
    ctx.close()


# ------------------------------------------------------------------ precision --

def bench_precision(args):
    """Where FP32 refinement pays on the step engine: batches of k equal
    requests of side S (b~U[-1,1], tol 1e-8, classic CG), solved in FP64,
    FP32-refined (inner tol 1e-4), by the size-based policy, and each of these
    with the Chebyshev preconditioner (s = 4); solves/s of each batch and the
    time of one solve alone."""
    torch, cg = setup()
    import numpy as np
    ctx = cg.Context(device=0, arena_bytes=24 << 30)
    out = {}
    for S, k in ((64, 64), (128, 64), (181, 64), (256, 64), (512, 32), (1024, 16), (2048, 8)):
        rng = np.random.default_rng(S)
        bs = [torch.from_numpy(rng.uniform(-1, 1, (S, S))).cuda() for _ in range(k)]
        row = {}
        for name, prec, pc in (("fp64", 0, 0), ("fp32_refined", 1, 0), ("auto", 3, 0),
                               ("fp64_chebyshev_s4", 0, 4), ("fp32_refined_chebyshev_s4", 1, 4),
                               ("auto_chebyshev_s4", 3, 4)):
            xs = [torch.zeros_like(b) for b in bs]
            probs = [cg.make_problem(b, x, S, S, tol=1e-8, maxit=200000, precision=prec,
                                     inner_tol=1e-4, precond=pc) for b, x in zip(bs, xs)]
            ctx.cg_solve_batch(probs[:2])
            torch.cuda.synchronize()
            t = time.perf_counter()
            rc, r = ctx.cg_solve_batch(probs)
            torch.cuda.synchronize()
            tb = time.perf_counter() - t
            t = time.perf_counter()
            ctx.cg_solve(probs[0])
            torch.cuda.synchronize()
            row[name] = dict(solves_per_s=round(k / tb, 2), batch_s=round(tb, 4),
                             alone_s=round(time.perf_counter() - t, 4), iterations=r[0].iterations,
                             outer=r[0].outer_iterations, true_res=r[0].rel_res_true,
                             met_tol=sum(int(q.rel_res_true <= 1e-8 * 1.000001) for q in r))
        out["%d^2 x %d" % (S, k)] = row
        log("precision", S, json.dumps(row))
    emit({"metric": "batch solves/s by precision (step engine, equal requests, tol 1e-8)",
          "workload": "precision", "results": out})
    ctx.close()


# ----------------------------------------------------------------------- tune --

def bench_tune(args):
    """cg_tune's pick against the unpinned (hand-set) tile shape at 4096^2 and
    8192^2 for both variants: HIP-event time per iteration of the iteration
    passes over a fixed-iteration solve, before and after tuning."""
    torch, cg = setup()
    names = {0: ("stencil_dot", "update_norm", "update_norm_nx"), 1: ("pcg_pass", "pcg_pass_nx")}
    out = {}
    for n in args.tune_sides:
        ctx = cg.Context(device=0, arena_bytes=96 * n * n + (1 << 30))
        b = torch.ones((n, n), dtype=torch.float64, device="cuda")
        for v in (0, 1):
            def per_iter():
                x = torch.zeros_like(b)
                p = cg.make_problem(b, x, n, n, tol=0.0, maxit=64, variant=v)
                ctx.cg_solve(p)
                ctx.cg_set_profiling(True)
                ctx.cg_kernel_stats(reset=True)
                ctx.cg_solve(p)
                st = ctx.cg_kernel_stats(reset=True)
                ctx.cg_set_profiling(False)
                return sum(st[k]["seconds"] for k in names[v] if k in st) / 64 * 1e6

            def shape():
                i = ctx.cg_plan(n, n, v)
                return dict(rows=i.rows, grid=i.grid, cols_per_lane=i.cols_per_lane,
                            tiles=i.tiles)
            before = dict(shape(), us_per_iteration=round(per_iter(), 2))
            t = time.perf_counter()
            ctx.cg_tune(n, n, v)
            tt = time.perf_counter() - t
            after = dict(shape(), us_per_iteration=round(per_iter(), 2))
            key = "%d^2 %s" % (n, "pipelined" if v else "classic")
            out[key] = dict(unpinned=before, tuned=after, tune_seconds=round(tt, 1))
            log("tune", key, json.dumps(out[key]))
        ctx.close()
        del b
    emit({"metric": "autotuner pick vs the unpinned tile shape (us per iteration, HIP events)",
          "workload": "tune", "results": out})


# ---------------------------------------------------------------------- probe --

def bench_probe(args):
    torch, cg = setup()
    ctx = cg.Context(device=0, arena_bytes=8 << 30)
    # 6R6W: in place (the traffic of pcg_pass); 6R6W_out: six other vectors
    # written; 6R6W_nt: in place with non-temporal stores; 6R6W_il: in place
    # with the six vectors' rows interleaved (the pipelined solve's layout)
    names = ["read", "copy", "2R1W", "3R2W", "6R6W", "6R6W_out", "6R6W_nt", "6R6W_il"]
    out = {}
    if args.copy_only:
        # the known-size copy that calibrates the traffic counters: one
        # 4096 x 4096 FP64 vector (134217728 B) read and written, 2 launches
        t, by = ctx.cg_stream_probe(1, 4096 * 4096, 1)
        out["copy_16M"] = round(by / t / 1e9, 1)
    else:
        for elems in (4096 * 4096, 8192 * 8192):
            for pat, nm in enumerate(names):
                t, by = ctx.cg_stream_probe(pat, elems, 5)
                out["%s_%dM" % (nm, elems >> 20)] = round(by / t / 1e9, 1)
    t, ops = ctx.cg_mul_probe(4096, 5)
    emit({"metric": "attainable HBM GB/s of plain streaming kernels", "workload": "probe",
          "results_GBps": out, "peak_GBps": HBM_PEAK_GBPS,
          "mul_probe_Gmul_s": round(ops / t / 1e9, 1), "mul_peak_Gmul_s": FX_MUL_PEAK_G})
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=500)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=48)
    ap.add_argument("--no-tol-run", dest="tol_run", action="store_false",
                    help="skip the tol=1e-8 solves of the headline workload")
    ap.add_argument("--workload",
                    choices=["small", "batch", "huge", "serve", "fixed", "precond", "cube", "vc",
                             "tune", "precision"])
    ap.add_argument("--n-cube", type=int, default=256, help="--workload cube: grid side")
    ap.add_argument("--cube-iters", type=int, default=0,
                    help="--workload cube: fixed iterations (0: the workload's 500)")
    ap.add_argument("--n-vc", type=int, default=4096, help="--workload vc: grid side")
    ap.add_argument("--tune-sides", type=int, nargs="+", default=[4096, 8192],
                    help="--workload tune: grid sides")
    ap.add_argument("--rr-period", type=int, default=100,
                    help="--workload vc: residual replacement period of the pipelined tol run")
    ap.add_argument("--fixed-only", action="store_true",
                    help="--workload cube / vc: only the fixed-iteration runs (no tol solves)")
    ap.add_argument("--huge-pc-inner-tol", default="1e-5",
                    help="huge: inner tolerance of the preconditioned refinement (a comma "
                         "list: the first is reported in full, the others timed)")
    ap.add_argument("--huge-precond", type=int, default=8,
                    help="--workload huge: also solve with s Chebyshev steps (0: skip)")
    ap.add_argument("--steps-list", type=int, nargs="*", default=[2, 4, 6, 8],
                    help="--workload precond: Chebyshev steps to compare with CG")
    ap.add_argument("--probe", action="store_true")
    ap.add_argument("--copy-only", action="store_true",
                    help="with --probe: only the 134 MB copy used for counter calibration")
    ap.add_argument("--count", type=int, default=None)
    ap.add_argument("--cpu-solves", type=int, default=16)
    ap.add_argument("--n-huge", type=int, default=8192)
    ap.add_argument("--loads", type=float, nargs="*", default=[0.5, 0.8, 1.0, 1.5])
    ap.add_argument("--batch-op", choices=("2d", "3d", "vc"), default="2d",
                    help="batch workload: the 5-point operator, 3D grids or variable "
                         "coefficients")
    ap.add_argument("--batch-precond", type=int, default=0,
                    help="--workload batch: Chebyshev steps of every solve (0: none)")
    ap.add_argument("--serve-precond", type=int, default=0,
                    help="--workload serve: also serve the stream preconditioned with s steps")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(multi-GPU sharding is a design note, not an implementation)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.probe:
        return bench_probe(args)
    if args.workload == "small":
        args.count = args.count or 200
        return bench_small(args)
    if args.workload == "batch":
        args.count = args.count or 256
        return bench_batch(args)
    if args.workload == "huge":
        return bench_huge(args)
    if args.workload == "fixed":
        return bench_fixed(args)
    if args.workload == "precond":
        return bench_precond(args)
    if args.workload == "cube":
        return bench_cube(args)
    if args.workload == "precision":
        return bench_precision(args)
    if args.workload == "tune":
        return bench_tune(args)
    if args.workload == "vc":
        return bench_vc(args)
    if args.workload == "serve":
        args.count = args.count or 400
        return bench_serve(args)
    return headline(args)


if __name__ == "__main__":
    main()
