"""Throughput of the back-and-forth iteration on one MI355X.

A step is one full back-and-forth iteration (phi-step and psi-step: four
c-transforms, two pushforwards, two Neumann Poisson solves, the float64
reductions and two step-size updates) on the 4096^2 float32 workload
(8-disk indicator densities, max/mean density 50).  Inputs are resident in
HBM before the timed region; the timed region is one library solve of K
iterations continuing from the W warm-up iterations.

Prints one JSON line: throughput in grid-points x iterations per second,
time to dual gap < 1e-4, the roofline of the dominant kernel (timed live with
HIP events on the library's stream) and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-pts×iters/s & time to dual gap<1e-4 at 4096²; batched+grad vs plain"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--gap-iters", type=int, default=200, help="iteration cap of the time-to-gap run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=20)
    return ap.parse_args()


def kernel_times(plan, phi, reps):
    """Average duration (ms) of each hot kernel class, HIP events on the
    stream the library launches on (the current PyTorch stream).  Inputs are
    what the solver feeds these kernels: the current potential for the first
    c-transform pass, that pass's output for the second."""
    import torch
    s = torch.cuda.current_stream()
    f = phi.contiguous()
    a1 = plan.ctransform_axis(f, 1, -1)
    out = torch.empty_like(f)
    res = {}

    def timeit(fn):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(reps):
            fn()
        b.record(s)
        b.synchronize()
        return a.elapsed_time(b) / reps

    res["ct_axis1"] = timeit(lambda: plan.ctransform_axis(f, 1, -1, out=out))
    res["ct_axis0"] = timeit(lambda: plan.ctransform_axis(a1, 0, 1, out=out))
    return res


def cpu_baseline(n):
    """The float64 oracle, timed on a bounded sample of one iteration at the
    same grid: 64 lines of each c-transform pass (scaled to all lines), one
    full pushforward and one full Poisson solve; the iteration is 8 line
    passes + 2 pushforwards + 2 Poisson solves."""
    import numpy as np
    from oracle import bfm as ob
    from oracle import _native
    from paper_1905_12154_amd import workloads as wl

    mu, nu = wl.config_c3(n)
    xs = ob.centres(mu.shape)
    phi = 0.1 * xs[0] ** 2 - 0.05 * xs[1] + np.zeros(mu.shape)
    t0 = time.perf_counter()
    ob.line_min(-phi[:64], 1)
    t_rows = (time.perf_counter() - t0) * (n / 64)
    t0 = time.perf_counter()
    ob.line_min(np.ascontiguousarray(-phi[:, :64]), 0)
    t_cols = (time.perf_counter() - t0) * (n / 64)
    t0 = time.perf_counter()
    T = ob.transport_map(phi)
    rho = ob.pushforward(mu, T)
    ob.primal_cost(mu, T)
    t_push = time.perf_counter() - t0
    t0 = time.perf_counter()
    ob.poisson_neumann(nu - rho)
    t_pois = time.perf_counter() - t0
    t0 = time.perf_counter()
    ob.dual_value(phi, phi, nu, mu)
    t_dot = time.perf_counter() - t0
    t_iter = 4 * (t_rows + t_cols) + 2 * (t_push + t_pois) + 4 * t_dot
    cores = int(_native.lib().oracle_num_threads())
    return {"value": n * n / t_iter, "unit": "grid-pts*iters/s", "cores": cores, "kind": "oracle",
            "sample": "%d^2 c3 workload, float64: 64 rows + 64 columns of the c-transform line minimum "
                      "(scaled x%d to a full pass, 8 passes/iteration), 2 full map+pushforward, "
                      "2 full DCT Poisson solves, 4 dual sums -> %.1f s per iteration "
                      "(rows %.2f s, cols %.2f s per pass; push %.2f s; poisson %.2f s)"
                      % (n, n // 64, t_iter, t_rows, t_cols, t_push, t_pois),
            "seconds_per_iter": t_iter}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d requested)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1905_12154_amd import bfm, workloads as wl

    dev = torch.device("cuda:0")
    n = args.n
    mu_h, nu_h = wl.config_c3(n)
    mu = torch.tensor(mu_h, dtype=torch.float32, device=dev)
    nu = torch.tensor(nu_h, dtype=torch.float32, device=dev)
    N = n * n

    warm = bfm.Plan((n, n), torch.float32, max_iters=max(args.warmup, 0), check_every=max(args.warmup, 1))
    rw = warm.solve(mu, nu, return_map=False)
    plan = bfm.Plan((n, n), torch.float32, max_iters=args.steps, check_every=max(args.steps, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = plan.solve(mu, nu, phi_init=rw.phi, return_map=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert r.iters == args.steps, (r.iters, args.steps)

    # time to dual gap < 1e-4 from phi_0 = 0 (the trace records every head)
    gplan = bfm.Plan((n, n), torch.float32, max_iters=args.gap_iters, tol=1e-4, check_every=4)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    rg = gplan.solve(mu, nu, return_map=False)
    torch.cuda.synchronize()
    gdt = time.perf_counter() - g0
    tr = gplan.trace(dev)
    min_gap = min(e["gap"] for e in tr) if tr else float("nan")

    # dominant kernel: per-iteration time = launches per iteration x duration
    kt = kernel_times(plan, r.phi, args.kernel_reps)
    per_iter = {"ct_axis1": 4 * kt["ct_axis1"], "ct_axis0": 4 * kt["ct_axis0"]}
    dom = max(per_iter, key=per_iter.get)
    bytes_per_launch = 2 * N * 4          # read u, write the transformed line (float32)
    achieved = bytes_per_launch / (kt[dom] * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": N * args.steps / dt,
        "unit": "grid-pts*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c3: 2D %dx%d grid, float32 fields with float64 sums, 8-disk indicator "
                               "densities (radii U[0.03,0.12], max/mean 50), %d back-and-forth iterations"
                               % (n, n, args.steps),
                   "grid": [n, n]},
        "time_to_gap_1e-4": {"seconds": gdt if rg.converged else None, "iters": rg.iters,
                             "converged": bool(rg.converged), "final_gap": rg.gap, "min_gap": min_gap,
                             "dual": rg.dual, "cap": args.gap_iters},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": dom,
                     "kernel_ms": kt[dom], "algorithmic_bytes_per_launch": bytes_per_launch},
        "kernels_ms": kt,
        "dual": r.dual,
        "gap": r.gap,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
