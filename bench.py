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
COPY_BYTES = 256 << 20     # calibration copy: reads and writes this many bytes
# algorithmic bytes of one whole iteration per grid point, float32: every
# separable sweep reads its input and writes its output once, with the
# fusions of the hot path (19 words per half-step in 2D, 27 in 3D)
ITER_BYTES_PER_POINT = {2: 152, 3: 216}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ct_rows_blocked_sum_c3_4096_f32_traffic.json")
# sources that decide the c-transform kernel's code: counters taken on
# another version of them no longer describe the kernel
TRAFFIC_SOURCES = ["paper_1905_12154_amd/csrc/ctransform.hip", "paper_1905_12154_amd/csrc/common.hpp",
                   "paper_1905_12154_amd/csrc/launch.hpp", "paper_1905_12154_amd/build_lib.py"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, tuning):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs (FETCH_SIZE and WRITE_SIZE, each scaled by the counter's reading on
    a copy of known size), or None when the kernel's sources or launch shape
    differ from those the counters were taken on."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel") != kernel or t.get("source_sha256") != kernel_source_hash():
        return None
    if tuning is not None and [list(x) for x in t.get("launch_shape", [])] != [list(x) for x in tuning]:
        return None
    return t["hbm_bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--gap-iters", type=int, default=200, help="iteration cap of the time-to-gap run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-c5", action="store_true", help="skip the batched 64-pair leg")
    ap.add_argument("--no-c4", action="store_true", help="skip the 3D 384^3 leg")
    ap.add_argument("--c5-iters", type=int, default=400)
    ap.add_argument("--c5-tol", type=float, default=3e-4,
                    help="common stop gap of the batched leg (the smallest at which all 64 pairs converge)")
    ap.add_argument("--c4-iters", type=int, default=20)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-interp", action="store_true", help="skip the 1024^2 displacement-interpolation leg")
    ap.add_argument("--interp-frames", type=int, default=11)
    ap.add_argument("--no-ga", action="store_true",
                    help="skip the back-and-forth versus gradient-ascent leg (two 1024^2 examples, float64)")
    ap.add_argument("--ga-cap", type=int, default=3000, help="iteration cap of the gradient-ascent runs")
    ap.add_argument("--no-pcost", action="store_true", help="skip the power-cost leg (crossing discs, 1024^2)")
    ap.add_argument("--pcost-iters", type=int, default=60)
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the float32-against-float64 comparison on the headline workload")
    ap.add_argument("--precision-iters", type=int, default=200, help="iteration cap of the precision leg")
    ap.add_argument("--tuning", default=None,
                    help="launch shapes of the counter leg instead of autotuning, as C,lines,mode per axis "
                         "separated by ';' (the shapes the bench's own run reported)")
    ap.add_argument("--pmc-leg", nargs="?", const="ct", default=None, choices=["ct", "splat3d", "dct"],
                    help="the program run under rocprofv3 --pmc: 'ct' (default) the dominant kernel's timing "
                         "leg, 'splat3d' three iterations of the 384^3 workload, 'dct' three iterations of the "
                         "4096^2 workload; each followed by a %d MiB copy for counter calibration"
                         % (COPY_BYTES >> 20))
    ap.add_argument("--oracle-c4-iters", type=int, default=3,
                    help="iterations of the 384^3 oracle run of the oracle legs (0 skips it)")
    ap.add_argument("--no-oracle-legs", action="store_true",
                    help="skip the oracle runs at c1, c2, c4 and on c5 pairs (timing and float32 error)")
    return ap.parse_args()


def kernel_times(plan, phi, reps, weight=None):
    """Average duration (ms) of each hot kernel class, HIP events on the
    stream the library launches on (the current PyTorch stream).  Inputs are
    what the solver feeds these kernels: the current potential for the first
    c-transform pass, that pass's output for the second.  When the solver
    runs the column-blocked two-pass transform (2D, persistent shapes), its
    two passes are timed as launched there: the column pass, and the row
    pass with the fused sum against `weight` (as in a gradient step)."""
    import torch
    from paper_1905_12154_amd import bfm
    s = torch.cuda.current_stream()
    f = phi.contiguous()
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

    try:
        mid = plan.ctransform_pass(f, 0)
        out = torch.empty_like(f)
        res["ct_cols_blocked"] = timeit(lambda: plan.ctransform_pass(f, 0, out=mid))
        res["ct_rows_blocked"] = timeit(lambda: plan.ctransform_pass(mid, 1, out=out))
        if weight is not None:
            res["ct_rows_blocked_sum"] = timeit(lambda: plan.ctransform_pass(mid, 1, out=out, weight=weight))
    except bfm.BFMError:
        pass
    a1 = plan.ctransform_axis(f, 1, -1)
    out = torch.empty_like(f)
    res["ct_axis1"] = timeit(lambda: plan.ctransform_axis(f, 1, -1, out=out))
    res["ct_axis0"] = timeit(lambda: plan.ctransform_axis(a1, 0, 1, out=out))
    return res


def dominant_kernel(kt, N, esz=4):
    """The kernel with the largest time per iteration (4 c-transforms) and its
    algorithmic bytes per launch: a pass reads its input and writes its
    output (2 words per point); the row pass with the fused sum also reads
    the weight field (3 words)."""
    if "ct_cols_blocked" in kt:
        rows = kt.get("ct_rows_blocked_sum", kt["ct_rows_blocked"])
        per_iter = {"ct_cols_blocked": 4 * kt["ct_cols_blocked"],
                    "ct_rows_blocked_sum" if "ct_rows_blocked_sum" in kt else "ct_rows_blocked":
                        2 * kt["ct_rows_blocked"] + 2 * rows}
    else:
        per_iter = {"ct_axis1": 4 * kt["ct_axis1"], "ct_axis0": 4 * kt["ct_axis0"]}
    dom = max(per_iter, key=per_iter.get)
    words = 3 if dom == "ct_rows_blocked_sum" else 2
    return dom, words * N * esz


def batched_leg(iters, tol):
    """64 ragged pairs (sides in {128,...,1024}, 2-6 Gaussian components):
    plain solves one after another versus one batched solve (graph replays)
    versus batched solve + W2^2 backward, same stop rule (gap < tol, at most
    `iters` iterations)."""
    import torch
    from paper_1905_12154_amd import bfm, workloads as wl
    dev = torch.device("cuda:0")
    ps = wl.config_c5()
    mus = [torch.tensor(m, dtype=torch.float32, device=dev) for m, _ in ps]
    nus = [torch.tensor(v, dtype=torch.float32, device=dev) for _, v in ps]
    # warm-up: plans, workspaces, first launches
    for m, v in zip(mus, nus):
        bfm.solve(m, v, max_iters=1, tol=tol, return_map=False)
    bfm.solve_batched(mus, nus, max_iters=1, tol=tol)
    torch.cuda.synchronize()

    def timed(fn, reps=3):
        # median of `reps` calls: the first full call of a form can pay
        # one-off costs (graph capture sizes, allocator growth) that vary by run
        ts, out = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[len(ts) // 2], ts, out

    tp, tps, rp = timed(lambda: [bfm.solve(m, v, max_iters=iters, tol=tol, return_map=False)
                                 for m, v in zip(mus, nus)])
    tb, tbs, rb = timed(lambda: bfm.solve_batched(mus, nus, max_iters=iters, tol=tol, iters_per_graph=8))
    gm = [m.clone().requires_grad_(True) for m in mus]
    gn = [v.clone().requires_grad_(True) for v in nus]
    # warm-up of the autograd path (first backward: autograd engine, kernel loads)
    bfm.w2_loss_batched(gm, gn, max_iters=1, tol=tol).sum().backward()
    torch.cuda.synchronize()

    def solve_and_grad():
        for t in gm + gn:
            t.grad = None
        vals = bfm.w2_loss_batched(gm, gn, max_iters=iters, tol=tol)
        vals.sum().backward()

    tg, tgs, _ = timed(solve_and_grad)
    work_p = sum(m.numel() * r.iters for m, r in zip(mus, rp))
    work_b = sum(m.numel() * r.iters for m, r in zip(mus, rb))
    # context: the same two forms at the looser common gap 1e-3, where every
    # pair stops within a few iterations (no long tail of one small pair)
    lp, lps, rp2 = timed(lambda: [bfm.solve(m, v, max_iters=iters, tol=1e-3, return_map=False)
                                  for m, v in zip(mus, nus)])
    lb, lbs, rb2 = timed(lambda: bfm.solve_batched(mus, nus, max_iters=iters, tol=1e-3, iters_per_graph=8))
    w2 = sum(m.numel() * r.iters for m, r in zip(mus, rb2))
    loose = {"tol": 1e-3, "plain_seconds": lp, "batched_seconds": lb,
             "converged": sum(r.converged for r in rb2), "iters_total": sum(r.iters for r in rb2),
             "max_iters_of_a_pair": max(r.iters for r in rb2),
             "plain_pts_iters_per_s": sum(m.numel() * r.iters for m, r in zip(mus, rp2)) / lp,
             "batched_pts_iters_per_s": w2 / lb, "samples_plain": lps, "samples_batched": lbs}
    return {"pairs": len(mus), "total_points": int(sum(m.numel() for m in mus)), "tol": tol, "max_iters": iters,
            "timing": "median of 3 calls per form (samples listed)",
            "plain": {"seconds": tp, "pts_iters_per_s": work_p / tp, "converged": sum(r.converged for r in rp),
                      "iters_total": sum(r.iters for r in rp), "samples": tps},
            "batched": {"seconds": tb, "pts_iters_per_s": work_b / tb, "converged": sum(r.converged for r in rb),
                        "iters_total": sum(r.iters for r in rb), "samples": tbs},
            "batched_plus_grad": {"seconds": tg, "pts_iters_per_s": work_b / tg, "samples": tgs},
            "batched_iteration_frac": ITER_BYTES_PER_POINT[2] * work_b / tb / 1e9 / HBM_PEAK_GBS,
            "max_abs_dual_diff_batched_vs_plain": max(abs(a.dual - b.dual) for a, b in zip(rp, rb)),
            "speedup_batched_vs_plain": tp / tb,
            "at_gap_1e-3": loose}


def c4_leg(iters, autotune):
    """3D 384^3, 6-Gaussian mixtures, float32: iterations per second."""
    import torch
    from paper_1905_12154_amd import bfm, workloads as wl
    dev = torch.device("cuda:0")
    mu_h, nu_h = wl.config_c4()
    mu = torch.tensor(mu_h, dtype=torch.float32, device=dev)
    nu = torch.tensor(nu_h, dtype=torch.float32, device=dev)
    del mu_h, nu_h
    plan = bfm.Plan(mu.shape, torch.float32, max_iters=iters, check_every=max(iters, 1))
    rw = plan.solve(mu, nu, return_map=False)   # warm-up (same work)
    if autotune:
        plan.autotune(dev, sample=rw.phi)
        plan.autotune_deposit(rw.phi, mu)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = plan.solve(mu, nu, return_map=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    N = mu.numel()
    ms = dt / max(r.iters, 1) * 1e3
    gbs = ITER_BYTES_PER_POINT[3] * N / (ms * 1e-3) / 1e9
    return {"workload": "c4: 3D 384^3, 6-Gaussian mixtures, float32", "iters": r.iters, "seconds": dt,
            "ms_per_iter": ms, "pts_iters_per_s": N * r.iters / dt, "gap": r.gap,
            "dual": r.dual, "tuning": plan.tuning(), "deposit_grid": plan.deposit_grid(),
            "roofline": {"bound": "hbm", "model_bytes_per_point_iter": ITER_BYTES_PER_POINT[3],
                         "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "iteration_frac": gbs / HBM_PEAK_GBS}}


def interp_leg(iters, tol, nframes):
    """Displacement interpolation at 1024^2 (c2: ellipses to a 4-Gaussian
    mixture, float32): solve to dual gap < tol (at most `iters` iterations),
    then `nframes` interpolants rho_t = S_t # mu at evenly spaced t."""
    import torch
    from paper_1905_12154_amd import bfm, workloads as wl
    dev = torch.device("cuda:0")
    mu_h, nu_h = wl.config_c2()
    mu = torch.tensor(mu_h, dtype=torch.float32, device=dev)
    nu = torch.tensor(nu_h, dtype=torch.float32, device=dev)
    plan = bfm.Plan(mu.shape, torch.float32, max_iters=iters, tol=tol, check_every=4)
    times = [k / (nframes - 1) for k in range(nframes)]
    plan.solve(mu, nu, return_map=False)                 # warm-up
    plan.interpolate(plan.solve(mu, nu, return_map=False).phi, mu, times[:2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = plan.solve(mu, nu, return_map=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    frames = plan.interpolate(r.phi, mu, times)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    mass = float(mu.double().sum())
    return {"workload": "c2: 1024^2, 5 ellipses to a 4-Gaussian mixture, float32", "tol": tol,
            "iters": r.iters, "converged": bool(r.converged), "gap": r.gap, "solve_seconds": t1 - t0,
            "frames": nframes, "frames_seconds": t2 - t1, "ms_per_frame": (t2 - t1) / nframes * 1e3,
            "total_seconds": t2 - t0,
            "max_frame_mass_error": max(abs(float(f.double().sum()) - mass) / mass for f in frames)}


def ga_leg(cap_bfm, cap_ga, errors=(1e-4, 1e-5, 1e-6)):
    """Back-and-forth iteration against the plain H^1 gradient ascent on the
    two 1024^2 examples of Tables 5 and 6 (float64): iterations and seconds
    until the dual is within `err` of the exact transport cost.  A first solve
    per method records the trace (every head's dual); each error level is
    then timed as a solve of exactly that many iterations."""
    import torch
    from paper_1905_12154_amd import bfm, workloads as wl
    dev = torch.device("cuda:0")
    out = {"workload": "two discs (cost 1/4) and one square to four squares (cost 1/16), 1024^2, float64",
           "measure": "first iteration n with |J(phi_n) - exact cost| < err; seconds = solve of n iterations"}
    for case, exact in (("two_discs", 0.25), ("square_to_four", 1.0 / 16.0)):
        mu_h, nu_h = getattr(wl, case)(1024)
        mu = torch.tensor(mu_h, dtype=torch.float64, device=dev)
        nu = torch.tensor(nu_h, dtype=torch.float64, device=dev)
        res = {}
        for method, cap in (("bfm", cap_bfm), ("ga", cap_ga)):
            plan = bfm.Plan(mu.shape, torch.float64, max_iters=cap, check_every=cap, method=method)
            plan.autotune(dev)
            plan.solve(mu, nu, return_map=False)
            tr = plan.trace(dev)
            row = {"cap": cap}
            for err in errors:
                n = next((int(e["iter"]) for e in tr if abs(e["dual"] - exact) < err), None)
                if n is None:
                    row["%g" % err] = {"iters": None, "seconds": None}
                    continue
                p = bfm.Plan(mu.shape, torch.float64, max_iters=n, check_every=max(n, 1), method=method)
                p.autotune(dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = p.solve(mu, nu, return_map=False)
                torch.cuda.synchronize()
                row["%g" % err] = {"iters": n, "seconds": time.perf_counter() - t0,
                                   "error": abs(r.dual - exact)}
            res[method] = row
        out[case] = res
    return out


def pcost_leg(iters, n=1024):
    """Separable power costs (eq. p_costs) on the Section 4.3 example of two
    pairs of discs at n^2, float32, for the paper's exponent pairs
    (p_0, p_1) per array axis: `iters` iterations from phi = 0, the dual, the
    gap, the motion along each axis, and the c-transform time (HIP events)
    next to the quadratic one.  With (1.1, 3) the exact cost is (1/2)^3/3."""
    import torch
    from paper_1905_12154_amd import bfm, workloads as wl
    dev = torch.device("cuda:0")
    mu_h, nu_h = wl.crossing_discs(n)
    mu = torch.tensor(mu_h, dtype=torch.float32, device=dev)
    nu = torch.tensor(nu_h, dtype=torch.float32, device=dev)
    x = (torch.arange(n, device=dev, dtype=torch.float32) + 0.5) / n
    sup = mu > 0
    rows = []
    ct_ms = {}
    for power in ((2.0, 2.0), (1.75, 2.25), (1.5, 2.5), (1.1, 3.0)):
        plan = bfm.Plan(mu.shape, torch.float32, max_iters=iters, check_every=iters, power=power)
        plan.solve(mu, nu, return_map=False)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = plan.solve(mu, nu)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        move = [float((r.T[0] - x[:, None])[sup].abs().mean()), float((r.T[1] - x[None, :])[sup].abs().mean())]
        row = {"power": list(power), "iters": r.iters, "seconds": dt, "ms_per_iter": dt / max(r.iters, 1) * 1e3,
               "dual": r.dual, "gap": r.gap, "mean_abs_motion_per_axis": move}
        if power == (1.1, 3.0):
            row["abs_error_vs_1_24"] = abs(r.dual - 1.0 / 24.0)
        rows.append(row)
        out = torch.empty_like(mu)
        for _ in range(2):
            plan.ctransform(r.phi, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            plan.ctransform(r.phi, out=out)
        e1.record()
        torch.cuda.synchronize()
        ct_ms["%g,%g" % power] = e0.elapsed_time(e1) / 10
    return {"workload": "two discs to two crossing discs (Section 4.3, general costs), %d^2, float32" % n,
            "runs": rows, "ctransform_ms": ct_ms}


def precision_leg(n, iters, tol=1e-4):
    """The float32 production path against the float64 path of the same
    kernels on the headline workload (c3, n^2): each precision solves from
    phi = 0 to a dual gap below `tol` (at most `iters` iterations), then the
    relative differences of the dual and of W2^2, the map difference in grid
    cells over the support of mu (where the map transports mass) and the
    largest difference of the potential phi.  Agreement of the float64 path
    with the float64 CPU oracle is what the parity tests check, at the sizes
    the oracle finishes."""
    import torch
    from paper_1905_12154_amd import bfm, workloads as wl
    dev = torch.device("cuda:0")
    mu_h, nu_h = wl.config_c3(n)
    res, secs = {}, {}
    for dt in (torch.float64, torch.float32):
        mu = torch.tensor(mu_h, dtype=dt, device=dev)
        nu = torch.tensor(nu_h, dtype=dt, device=dev)
        plan = bfm.Plan((n, n), dt, max_iters=iters, tol=tol, check_every=4)
        plan.solve(mu, nu, return_map=False)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = plan.solve(mu, nu)
        torch.cuda.synchronize()
        secs[dt] = time.perf_counter() - t0
        res[dt] = r
        sup = mu > 0
    r64, r32 = res[torch.float64], res[torch.float32]
    # map difference per source cell in grid cells (largest over the axes);
    # where the transport splits mass the map jumps, and there rounding of
    # phi decides which side a finite difference sees, so the distribution
    # is reported beside the maximum
    d = torch.stack([(r32.T[a].double() - r64.T[a]).abs() for a in range(2)]).amax(0)[sup] * n
    q = torch.quantile(d.float(), torch.tensor([0.5, 0.999], device=dev)).tolist()
    return {"workload": "c3: %d^2, 8-disk indicators; float32 path against the float64 path" % n,
            "tol": tol, "iters_f64": r64.iters, "iters_f32": r32.iters, "gap_f64": r64.gap, "gap_f32": r32.gap,
            "seconds_f64": secs[torch.float64], "seconds_f32": secs[torch.float32],
            "dual_f64": r64.dual, "dual_f32": r32.dual,
            "rel_diff_dual": abs(r32.dual - r64.dual) / abs(r64.dual),
            "rel_diff_w2sq": abs(r32.w2sq - r64.w2sq) / abs(r64.w2sq),
            "map_diff_cells_on_support": {"cells": int(d.numel()), "mean": float(d.mean()), "median": q[0],
                                          "p99_9": q[1], "max": float(d.max()),
                                          "frac_above_0_01": float((d > 0.01).double().mean()),
                                          "frac_above_1": float((d > 1.0).double().mean())},
            "max_phi_diff": float((r32.phi.double() - r64.phi).abs().max()),
            "phi_scale": float(r64.phi.abs().max())}


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


def pmc_leg(n, args):
    """What the counter runs profile: the c3 warm-up potential, the tuned
    launch shapes, `kernel_reps` launches of each c-transform pass, then one
    device copy of COPY_BYTES (the calibration kernel)."""
    import torch
    from paper_1905_12154_amd import bfm, workloads as wl
    dev = torch.device("cuda:0")
    mu_h, nu_h = wl.config_c3(n)
    mu = torch.tensor(mu_h, dtype=torch.float32, device=dev)
    nu = torch.tensor(nu_h, dtype=torch.float32, device=dev)
    warm = bfm.Plan((n, n), torch.float32, max_iters=max(args.warmup, 0), check_every=max(args.warmup, 1))
    rw = warm.solve(mu, nu, return_map=False)
    plan = bfm.Plan((n, n), torch.float32)
    if args.tuning:   # counters slow kernels unevenly: tuning under them would pick other shapes
        plan.set_tuning([tuple(int(x) for x in ax.split(",")) for ax in args.tuning.split(";")])
        tuning = plan.tuning()
    else:
        tuning = plan.autotune(dev, sample=rw.phi) if not args.no_autotune else None
    kt = kernel_times(plan, rw.phi, args.kernel_reps, weight=mu)
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_leg": True, "tuning": tuning, "kernels_ms": kt, "kernel_reps": args.kernel_reps,
                      "copy_bytes": COPY_BYTES, "source_sha256": kernel_source_hash()}), flush=True)


def pmc_splat3d_leg(iters=3):
    """What the 3D deposition counter runs profile: `iters` iterations of the
    384^3 float32 workload from phi = 0 (2 depositions per iteration plus the
    final head's), then one device copy of COPY_BYTES (the calibration
    kernel)."""
    import torch
    from paper_1905_12154_amd import bfm, workloads as wl
    dev = torch.device("cuda:0")
    mu_h, nu_h = wl.config_c4()
    mu = torch.tensor(mu_h, dtype=torch.float32, device=dev)
    nu = torch.tensor(nu_h, dtype=torch.float32, device=dev)
    del mu_h, nu_h
    plan = bfm.Plan(mu.shape, torch.float32, max_iters=iters, check_every=iters)
    r = plan.solve(mu, nu, return_map=False)
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_leg": "splat3d", "iters": r.iters, "dual": r.dual, "copy_bytes": COPY_BYTES}),
          flush=True)


def pmc_dct_leg(n=4096, iters=3):
    """What the Poisson-pass counter runs profile: `iters` iterations of the
    4096^2 float32 headline workload from phi = 0 (per half-step one forward
    row pass, one fused column pass, one inverse row pass), then one device
    copy of COPY_BYTES (the calibration kernel)."""
    import torch
    from paper_1905_12154_amd import bfm, workloads as wl
    dev = torch.device("cuda:0")
    mu_h, nu_h = wl.config_c3(n)
    mu = torch.tensor(mu_h, dtype=torch.float32, device=dev)
    nu = torch.tensor(nu_h, dtype=torch.float32, device=dev)
    del mu_h, nu_h
    plan = bfm.Plan(mu.shape, torch.float32, max_iters=iters, check_every=iters)
    r = plan.solve(mu, nu, return_map=False)
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_leg": "dct", "iters": r.iters, "dual": r.dual, "copy_bytes": COPY_BYTES}), flush=True)


def _map_cells(Tg, To, shape, support):
    """Largest map difference over the axes, in grid cells of each axis, at
    the cells of `support`: mean, median, 99.9th percentile, maximum."""
    import numpy as np
    d = np.max(np.stack([np.abs(Tg[a] - To[a]) * shape[a] for a in range(len(shape))]), axis=0)[support]
    if d.size == 0:
        return None
    q = np.quantile(d, [0.5, 0.999])
    return {"cells": int(d.size), "mean": float(d.mean()), "median": float(q[0]), "p99_9": float(q[1]),
            "max": float(d.max())}


def _f32_vs_oracle(mu_h, nu_h, max_iters, tol):
    """The float32 production path and the float64 CPU oracle on the same
    input (the oracle takes the float32-rounded densities in float64, so both
    solve the same problem): the oracle's wall time and cores, and the
    float32 errors of W2^2 and of the map (grid cells, over supp mu)."""
    import numpy as np
    import torch
    from oracle import bfm as ob
    from oracle import _native
    from paper_1905_12154_amd import bfm
    dev = torch.device("cuda:0")
    mu = torch.tensor(mu_h, dtype=torch.float32, device=dev)
    nu = torch.tensor(nu_h, dtype=torch.float32, device=dev)
    plan = bfm.Plan(mu.shape, torch.float32, max_iters=max_iters, tol=tol, check_every=4)
    r = plan.solve(mu, nu)
    Tg = r.T.double().cpu().numpy()
    gpu = {"iters": r.iters, "converged": bool(r.converged), "w2sq": r.w2sq, "gap": r.gap}
    del mu, nu
    m64 = mu_h.astype(np.float32).astype(np.float64)
    n64 = nu_h.astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    o = ob.solve(m64, n64, ob.Params(max_iters=max_iters, tol=tol))
    secs = time.perf_counter() - t0
    N = m64.size
    return {"oracle": {"iters": o.iters, "converged": bool(o.converged), "w2sq": o.w2sq, "gap": o.gap,
                       "seconds": secs, "pts_iters_per_s": N * max(o.iters, 1) / secs,
                       "cores": int(_native.lib().oracle_num_threads())},
            "gpu_f32": gpu,
            "rel_err_w2sq": abs(r.w2sq - o.w2sq) / abs(o.w2sq),
            "map_err_cells_on_supp_mu": _map_cells(Tg, np.stack(o.T), m64.shape, m64 > 0)}


def oracle_legs(args):
    """The float64 CPU oracle timed on the configurations it finishes (c1 in
    full, c2 to its gap, c4 for a few iterations, c5 pairs to their gap), and
    the float32 GPU path's error against it on each."""
    from paper_1905_12154_amd import workloads as wl
    out = {}
    mu, nu = wl.config_c1()
    out["c1"] = dict(workload="c1: 64^2, 3-Gaussian mixtures, 60 iterations", **_f32_vs_oracle(mu, nu, 60, 0.0))
    mu, nu = wl.config_c2()
    out["c2"] = dict(workload="c2: 1024^2, 5 ellipses to a 4-Gaussian mixture, to gap 1e-5 (cap 2000)",
                     **_f32_vs_oracle(mu, nu, 2000, 1e-5))
    del mu, nu
    if args.oracle_c4_iters > 0:
        mu, nu = wl.config_c4()
        out["c4"] = dict(workload="c4: 384^3, 6-Gaussian mixtures, %d iterations" % args.oracle_c4_iters,
                         **_f32_vs_oracle(mu, nu, args.oracle_c4_iters, 0.0))
        del mu, nu
    sides = wl.c5_sides()
    rows = []
    for pair in range(64):
        if len(rows) == 4:
            break
        if sides[pair] > 256:
            continue
        mu, nu = wl.config_c5_pair(pair, sides[pair])
        rows.append(dict(pair=pair, side=sides[pair], **_f32_vs_oracle(mu, nu, 300, 1e-5)))
    out["c5_pairs"] = {"workload": "c5: the first four pairs of side <= 256, to gap 1e-5 (cap 300)", "pairs": rows}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus %d requested)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1905_12154_amd import bfm, workloads as wl

    dev = torch.device("cuda:0")
    n = args.n
    if args.pmc_leg == "ct":
        pmc_leg(n, args)
        return
    if args.pmc_leg == "dct":
        pmc_dct_leg()
        return
    if args.pmc_leg == "splat3d":
        pmc_splat3d_leg()
        return
    mu_h, nu_h = wl.config_c3(n)
    mu = torch.tensor(mu_h, dtype=torch.float32, device=dev)
    nu = torch.tensor(nu_h, dtype=torch.float32, device=dev)
    N = n * n

    warm = bfm.Plan((n, n), torch.float32, max_iters=max(args.warmup, 0), check_every=max(args.warmup, 1))
    rw = warm.solve(mu, nu, return_map=False)
    plan = bfm.Plan((n, n), torch.float32, max_iters=args.steps, check_every=max(args.steps, 1))
    # launch shapes tuned on the warm-up potential (what the timed solve sees)
    tuning = plan.autotune(dev, sample=rw.phi) if not args.no_autotune else None
    # the deposition's workgroup count, timed on the same potential and mu
    deposit_grid = plan.autotune_deposit(rw.phi, mu) if not args.no_autotune else plan.deposit_grid()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = plan.solve(mu, nu, phi_init=rw.phi, return_map=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert r.iters == args.steps, (r.iters, args.steps)

    # time to dual gap < 1e-4 from phi_0 = 0 (the trace records every head)
    gplan = bfm.Plan((n, n), torch.float32, max_iters=args.gap_iters, tol=1e-4, check_every=4)
    if not args.no_autotune:
        gplan.autotune(dev)   # reuses the table filled above
    gplan.set_deposit_grid(deposit_grid)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    rg = gplan.solve(mu, nu, return_map=False)
    torch.cuda.synchronize()
    gdt = time.perf_counter() - g0
    tr = gplan.trace(dev)
    min_gap = min(e["gap"] for e in tr) if tr else float("nan")

    # dominant kernel: per-iteration time = launches per iteration x duration
    kt = kernel_times(plan, r.phi, args.kernel_reps, weight=mu)
    dom, bytes_per_launch = dominant_kernel(kt, N)
    achieved = bytes_per_launch / (kt[dom] * 1e-3) / 1e9
    traffic = measured_traffic(dom, tuning)

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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                     "kernel_ms": kt[dom], "algorithmic_bytes_per_launch": bytes_per_launch,
                     # the whole iteration against the same peak: ITER_BYTES_PER_POINT per point
                     "iteration_model_bytes_per_point": ITER_BYTES_PER_POINT[2],
                     "iteration_achieved": ITER_BYTES_PER_POINT[2] * N / (dt / args.steps) / 1e9,
                     "iteration_frac": ITER_BYTES_PER_POINT[2] * N / (dt / args.steps) / 1e9 / HBM_PEAK_GBS},
        "kernels_ms": kt,
        "tuning": tuning,
        "deposit_grid": deposit_grid,
        "dual": r.dual,
        "gap": r.gap,
    }
    if not args.no_c5:
        out["batched_c5"] = batched_leg(args.c5_iters, args.c5_tol)
    if not args.no_c4:
        out["c4_3d"] = c4_leg(args.c4_iters, not args.no_autotune)
    if not args.no_interp:
        out["interp_c2"] = interp_leg(2000, 1e-5, max(2, args.interp_frames))
    if not args.no_ga:
        out["bfm_vs_ga"] = ga_leg(40, args.ga_cap)
    if not args.no_pcost:
        out["pcost_crossing_discs"] = pcost_leg(args.pcost_iters)
    if not args.no_precision:
        out["precision_c3"] = precision_leg(n, args.precision_iters)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n)
        if not args.no_oracle_legs:
            out["oracle_legs"] = oracle_legs(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
