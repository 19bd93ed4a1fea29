"""Benchmark: CG on the 4096 x 4096 Laplace workload, both variants, on one GPU.

One step = one solve of A x = b with classic CG (Algorithm 1) plus one with the
pipelined CG (Algorithm 2), each running a fixed 500 iterations (tol = 0) on
the 4096 x 4096 grid with b = A x*, x* the lowest grid mode plus 1e-3 uniform
noise (seeded), x0 = 0, FP64.  Inputs are resident in HBM before the timed
region.  value = unknowns x iterations per second over the whole step
(GDOF-iter/s).

Also reported:
  roofline      the dominant kernel (pcg_pass) from HIP events recorded
                around each of its launches on the library's stream during a
                profiled repeat of the timed steps: algorithmic bytes
                (96 B per unknown) / average launch duration vs 8 TB/s.
  cpu_baseline  the CPU oracle (plain C, explicit CSR, one thread) on a
                bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BYTES_PER_DOF = {"pcg_pass": 96, "stencil_dot": 24, "update_norm": 40}
# HBM bytes per dispatch measured by rocprofv3 counters for pcg_pass at
# 4096 x 4096 (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel factor);
# None until measured for the current kernel.
PCG_TRAFFIC_BYTES = None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=500)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=12)
    ap.add_argument("--tol-run", action="store_true", help="also time tol=1e-8 solves")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(multi-GPU sharding is a design note, not an implementation)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1803_03797_amd import cg, workloads

    if not os.path.exists(cg.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
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

    # profiled repeat: HIP events around every launch on the library's stream
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
    kern = {}
    for name, s in stats.items():
        if s["launches"] and s["seconds"] > 0:
            kern[name] = dict(launches=s["launches"], avg_us=s["seconds"] / s["launches"] * 1e6,
                              GBps=s["bytes"] / s["seconds"] / 1e9)
    log("kernels:", json.dumps(kern))
    pk = stats.get("pcg_pass")
    roof = None
    if pk and pk["launches"]:
        avg = pk["seconds"] / pk["launches"]
        per_launch = BYTES_PER_DOF["pcg_pass"] * dof
        ach = per_launch / avg / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBPS, 4),
                "traffic": PCG_TRAFFIC_BYTES, "kernel": "pcg_pass",
                "avg_launch_us": round(avg * 1e6, 2), "bytes_per_launch": per_launch}

    tol_runs = None
    if args.tol_run:
        tol_runs = {}
        for v, name in ((0, "classic"), (1, "pipelined")):
            p = cg.make_problem(b, x, n, n, tol=1e-8, maxit=20000, variant=v)
            rc, r = ctx.cg_solve(p)
            err = ((x - xs).norm() / xs.norm()).item()
            tol_runs[name] = dict(status=cg.cg_status_str(rc), iterations=r.iterations,
                                  seconds=round(r.device_seconds, 4),
                                  rel_res_true=r.rel_res_true, err_vs_xstar=err)
        log("tol 1e-8:", json.dumps(tol_runs))

    cpu = None
    if not args.no_cpu:
        import oracle
        bh = b.cpu().numpy()
        t = time.perf_counter()
        k = args.cpu_iters
        oracle.cg(bh, n, n, variant=0, tol=0.0, maxit=k)
        oracle.cg(bh, n, n, variant=1, tol=0.0, maxit=k)
        ct = time.perf_counter() - t
        cpu = {"value": round(2 * dof * k / ct / 1e9, 5), "unit": "GDOF-iter/s", "cores": 1,
               "kind": "oracle",
               "sample": "classic + pipelined CG, %d iterations each, 4096x4096 FP64, explicit "
                         "CSR, single thread (%.1f s, includes CSR assembly)" % (k, ct)}
        log("cpu oracle:", json.dumps(cpu))

    dev_name = torch.cuda.get_device_name(0)
    line = {
        "metric": "CG GDOF-iter/s (4096^2 FP64, classic + pipelined, 500 iterations each)",
        "value": round(value, 3), "unit": "GDOF-iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "4096x4096 Laplace, b=A(sin*sin+1e-3 noise), x0=0, fixed %d "
                               "iterations per variant" % args.iters,
                   "nx": n, "ny": n, "iterations": args.iters,
                   "variants": ["classic", "pipelined"]},
        "per_variant_GDOF_iter_s": {
            "classic": round(dof * args.iters * args.steps / per_variant[0] / 1e9, 3),
            "pipelined": round(dof * args.iters * args.steps / per_variant[1] / 1e9, 3)},
        "algorithmic_GBps": {
            "classic": round(64 * dof * args.iters * args.steps / per_variant[0] / 1e9, 1),
            "pipelined": round(96 * dof * args.iters * args.steps / per_variant[1] / 1e9, 1)},
        "roofline": roof,
        "kernels": kern,
        "profiled_ms_per_step": round(prof_elapsed / args.steps * 1e3, 3),
        "tol_1e-8": tol_runs,
        "cpu_baseline": cpu,
        "device": dev_name,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
