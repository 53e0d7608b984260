#!/usr/bin/env python
"""Benchmark of the space-time heat-equation solver on one MI355X.

Metric: PCG unknowns x iterations per second, and time-to-solve at 1e-8
relative residual (sqrt(r^T K_X r) relative to the first residual), for the
largest single solve: FP64, N = 2^12 time intervals and h = 2^-9 (4097 x
261121 = 1,069,812,737 unknowns; seeded Fourier forcing, u0 = sin(pi x)
sin(pi y)).  One step = one complete solve (right-hand side, f-hat, PCG,
u = W w) with the data already resident on the GPU.  The FP32-mixed form of
the same solve is timed beside it.  Timed solves run as in production (each
PCG iteration replayed from a HIP graph); the per-kernel roofline comes from
one more solve run eagerly with HIP events around every hot launch.

Prints one JSON line.  Only one GPU is used; --gpus > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

WORKLOADS = {
    # name: (J, K, nrhs, g seed, u0 kind)
    "heat2d_J10_K9": (10, 9, 1, 2, "sin"),
    "heat2d_J12_K9": (12, 9, 1, 2, "sin"),
    "heat2d_J8_K7_B64": (8, 7, 64, 1000, "random4"),
    "heat2d_J4_K4": (4, 4, 1, None, "sin"),
    # the 3D problem (unit cube, Kuhn mesh) at the shape of the paper's 3D weak
    # scaling row with N_t = 257 time nodes and N_x = 250047: g = 0,
    # u0 = sin(pi x) sin(pi y) sin(pi z)
    "heat3d_J8_K6": (8, 6, 1, None, "sin3"),
    # request stream of uneven sizes (J in 6..11, K in 5..9), see run_serving
    "heat2d_serve": None,
}

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "PCG unknowns\u00b7iters/s + time-to-solve at 1e-8 rel res; FP32-mixed vs FP64"
UNIT = "unknowns\u00b7iters/s"
ROOT = os.path.dirname(os.path.abspath(__file__))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="heat2d_J12_K9", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--nested", type=int, default=0,
                    help="FP64: nested iteration over this many coarser meshes (Section 4.2); "
                         "the comparison run is then the same solve without it")
    ap.add_argument("--lookahead", type=int, default=0, choices=[0, -1],
                    help="0: PCG iterations in batches between flag reads; -1: read after each")
    ap.add_argument("--no-compare", action="store_true", help="skip the other-precision run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-seconds", type=float, default=20.0)
    ap.add_argument("--requests", type=int, default=200, help="serving: open-loop requests")
    ap.add_argument("--calibration-requests", type=int, default=0,
                    help="serving: closed-loop requests that measure the saturated rate "
                         "(0: the measured stream itself, all submitted at once)")
    ap.add_argument("--load", type=float, default=0.8,
                    help="serving: arrival rate as a fraction of the saturated rate")
    ap.add_argument("--budget-gb", type=float, default=180.0, help="serving: device budget")
    ap.add_argument("--slots", type=int, default=4, help="serving: concurrent groups")
    ap.add_argument("--batch", type=int, default=4, help="serving: requests per group")
    ap.add_argument("--serve-baseline", action="store_true",
                    help="serving: also solve the stream one request at a time with plain FP64")
    return ap.parse_args()


def load_inputs(stp, ctx, J, K, nrhs, seed, u0kind, torch):
    import synth

    dev = torch.device("cuda:0")
    for b in range(nrhs):
        if seed is None:
            stp.stp_set_g(ctx, b, None)
        else:
            g = synth.fourier_g_torch(J, K, seed + b if nrhs > 1 else seed, dev)
            stp.stp_set_g(ctx, b, g.reshape(-1))
            del g
        if u0kind == "sin":
            u0 = synth.sine_product(K, 1, 1)
        elif u0kind == "sin3":
            u0 = synth.sine_product_3d(K)
        else:
            u0 = synth.smooth_u0(K, seed + b)
        stp.stp_set_u0(ctx, b, u0.reshape(-1).copy())
    torch.cuda.synchronize()


def _checked(stp, status, st):
    if status != stp.STP_OK:
        bad = [(b, s["status"], s["rel_residual"]) for b, s in enumerate(st) if s["status"] != 0]
        raise SystemExit(f"bench.py: a timed solve did not converge: status {status}, "
                         f"(rhs, status, rel_residual) {bad[:4]}")
    return st


def run_solves(stp, ctx, nrhs, tol, steps, warmup, torch):
    """Mean wall time of `steps` solves after `warmup` untimed ones; every
    solve must converge."""
    for _ in range(warmup):
        _checked(stp, *stp.stp_solve(ctx, tol, nrhs))
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stats.append(_checked(stp, *stp.stp_solve(ctx, tol, nrhs)))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps, stats


def profile_solve(stp, ctx, nrhs, tol, torch):
    """Per-kernel launches, device time and algorithmic bytes of one more
    solve, run eagerly with HIP events around every hot launch."""
    torch.cuda.synchronize()
    stp.stp_profile(ctx, True)
    _checked(stp, *stp.stp_solve(ctx, tol, nrhs))
    kstats = {k: stp.stp_profile_read(ctx, k) for k in stp.STP_KERNEL_NAMES}
    stp.stp_profile(ctx, False)
    return kstats


def kernel_table(stp, kst):
    """Achieved algorithmic GB/s and fraction of the HBM peak per kernel."""
    out = {}
    for k, d in kst.items():
        if d["launches"] == 0:
            continue
        avg_ms = d["total_ms"] / d["launches"]
        per_launch = d["alg_bytes"] / d["launches"]
        gbs = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
        out[stp.STP_KERNEL_NAMES[k]] = {
            "launches": d["launches"], "total_ms": round(d["total_ms"], 3),
            "avg_launch_ms": round(avg_ms, 4), "alg_bytes_per_launch": per_launch,
            "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def measured_traffic(workload, precision, kernel, alg_bytes_per_launch):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel
    calibration), or None when no summary exists for this workload, the
    kernel source has changed since the counters were taken, or the launches
    differ from the measured ones (other algorithmic bytes per launch)."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    src = os.path.join(ROOT, "paper_2009_08875_amd", "csrc", rec["source"])
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if digest != rec["sha256"]:
        return None
    if abs(rec["alg_bytes_per_launch"] - alg_bytes_per_launch) > 1e-3 * alg_bytes_per_launch:
        return None
    return rec["traffic_bytes_per_launch"]


def solo_fp64_sequential(stp, torch, J, K, nrhs, seed, u0kind, tol):
    """The plain FP64 PCG on the same right-hand sides, one solve at a time
    (one single-RHS context reused), inputs resident before each timed solve."""
    import synth

    dev = torch.device("cuda:0")
    ctx = stp.stp_create(J, K, 1, stp.STP_FP64, stream=torch.cuda.current_stream())
    total, its = 0.0, 0
    try:
        for b in range(-1, nrhs):  # b = -1: untimed warm-up (launch tuning, graph capture)
            bb = max(b, 0)
            g = synth.fourier_g_torch(J, K, seed + bb, dev)
            stp.stp_set_g(ctx, 0, g.reshape(-1))
            u0 = synth.sine_product(K, 1, 1) if u0kind == "sin" else synth.smooth_u0(K, seed + bb)
            stp.stp_set_u0(ctx, 0, u0.reshape(-1).copy())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = stp.stp_solve(ctx, tol)
            torch.cuda.synchronize()
            if b >= 0:
                total += time.perf_counter() - t0
                its += st[0]["iterations"]
    finally:
        stp.stp_destroy(ctx)
    return {"time_s": round(total, 4), "solves": nrhs, "iterations_sum": its}


def cpu_baseline(seconds_budget):
    """The oracle (NumPy FP64, unmodified) on a bounded sample of the workload:
    PCG on the same mesh (h = 2^-9) with 2^1 + 1 time rows, seeded Fourier
    forcing, as many iterations as fit in the budget (at least one)."""
    import numpy as np

    import oracle
    import synth
    from oracle.pcg import pcg
    from oracle.schur import Problem

    J, K = 1, 9
    P = Problem(J, K)
    g = synth.fourier_g(J, K, 2)
    u0 = synth.sine_product(K, 1, 1)
    t0 = time.perf_counter()
    fhat = P.WT(P.rhs(g, u0))
    t_rhs = time.perf_counter() - t0
    its = 0
    t0 = time.perf_counter()
    # one iteration to size the run, then more while within the budget
    w, k, _ = pcg(P, fhat, tol=0.0, maxit=1)
    t1 = time.perf_counter() - t0
    per_it = t1
    more = max(0, int((seconds_budget - t_rhs - t1) / max(per_it, 1e-9)) - 1)
    its = 1
    if more > 0:
        t0 = time.perf_counter()
        w, k, _ = pcg(P, fhat, tol=0.0, maxit=1 + more)
        t1 = time.perf_counter() - t0
        its = 1 + more
    unknowns = (2 ** J + 1) * (2 ** K - 1) ** 2
    threads = 1  # NumPy elementwise kernels run on one thread
    return {
        "value": unknowns * its / t1,
        "unit": UNIT,
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle PCG (NumPy FP64) on h=2^-9 with {2 ** J + 1} time rows "
                   f"({unknowns} unknowns), {its} iterations in {t1:.1f} s; rhs+f-hat "
                   f"{t_rhs:.1f} s not counted; host cores available {os.cpu_count()}"),
    }


def serve_stream(stp, torch, server, reqs, prec, rate, window=16):
    """Submit `reqs` at Poisson arrival times of the given rate, or, when rate
    is None, as a closed loop that keeps `window` requests submitted and
    unfinished; wait for all.  Returns per-request results and the span from
    the first submission to the last completion."""
    import synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    arrivals, t = [], 0.0
    for r in reqs:
        t += 0.0 if rate is None else r["gap"] / rate
        arrivals.append(t)
    inflight, results = {}, []
    i = 0
    t0 = time.perf_counter()
    while i < len(reqs) or inflight:
        now = time.perf_counter() - t0
        while i < len(reqs) and now >= arrivals[i] and (rate is not None or len(inflight) < window):
            r = reqs[i]
            g = synth.fourier_g_torch(r["J"], r["K"], r["seed"], dev).reshape(-1)
            u0 = torch.as_tensor(synth.smooth_u0(r["K"], r["seed"]).reshape(-1), device=dev)
            stream.synchronize()  # the server reads g and u0 on its own streams
            rid = stp.stp_server_submit(server, r["J"], r["K"], prec, r["tol"], u0, g, None)
            inflight[rid] = (r, g, u0)
            i += 1
            now = time.perf_counter() - t0
        for rid in list(inflight):
            try:
                res = stp.stp_server_poll(server, rid)
            except stp.StpError as e:  # a failed request is reported, not fatal
                r = inflight.pop(rid)[0]
                print(f"# request J={r['J']} K={r['K']} tol={r['tol']:.2e} seed={r['seed']} "
                      f"failed: {e}", file=sys.stderr, flush=True)
                results.append((r, (e.status, {"iterations": 0}, float("nan"))))
                continue
            if res is not None:
                results.append((inflight.pop(rid)[0], res))
        time.sleep(0.0005)
    return results, time.perf_counter() - t0


def plain_sequential(stp, torch, reqs, _unused=None):
    """The request stream solved one request at a time by plain FP64 PCG
    (a context per shape, reused), each request's inputs resident before its
    timed solve."""
    import synth

    dev = torch.device("cuda:0")
    ctxs, total = {}, 0.0
    try:
        for r in reqs:
            key = (r["J"], r["K"])
            if key not in ctxs:
                ctxs[key] = stp.stp_create(r["J"], r["K"], 1, stp.STP_FP64,
                                           stream=torch.cuda.current_stream())
                warm = True
            else:
                warm = False
            ctx = ctxs[key]
            g = synth.fourier_g_torch(r["J"], r["K"], r["seed"], dev).reshape(-1)
            stp.stp_set_g(ctx, 0, g)
            stp.stp_set_u0(ctx, 0, synth.smooth_u0(r["K"], r["seed"]).reshape(-1).copy())
            torch.cuda.synchronize()
            if warm:  # untimed first solve of a shape: launch tuning and graph capture
                stp.stp_solve(ctx, r["tol"])
                torch.cuda.synchronize()
            t0 = time.perf_counter()
            stp.stp_solve(ctx, r["tol"])
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
            del g
            if len(ctxs) > 6:  # keep device memory bounded
                for k in list(ctxs)[:-1]:
                    stp.stp_destroy(ctxs.pop(k))
    finally:
        for c in ctxs.values():
            stp.stp_destroy(c)
    return {"time_s": round(total, 3), "solves": len(reqs),
            "solves_per_s": round(len(reqs) / total, 3)}


def run_serving(args, stp, torch):
    import numpy as np

    import synth

    prec = stp.STP_MIXED if args.precision == "mixed" else stp.STP_FP64
    warm = synth.serving_stream(12, seed=12343)
    reqs = synth.serving_stream(args.requests, seed=12345)
    cal = reqs if args.calibration_requests <= 0 else synth.serving_stream(
        args.calibration_requests, seed=12344)
    server = stp.stp_server_create(int(args.budget_gb * 1e9), max_slots=args.slots,
                                   max_batch=args.batch, options={"lookahead": args.lookahead})
    try:
        serve_stream(stp, torch, server, warm, prec, None)  # code loading, allocator warm-up
        res_cal, span_cal = serve_stream(stp, torch, server, cal, prec, None)
        saturated = len(res_cal) / span_cal
        rate = args.load * saturated
        print(f"# serving: closed loop {len(res_cal)} requests in {span_cal:.2f} s "
              f"({saturated:.2f} solves/s); open loop at {rate:.2f} requests/s",
              file=sys.stderr, flush=True)
        res, span = serve_stream(stp, torch, server, reqs, prec, rate)
        info = stp.stp_server_info(server)
    finally:
        stp.stp_server_destroy(server)
    def size(q):
        return (2 ** q["J"] + 1) * (2 ** q["K"] - 1) ** 2

    ok = [x for x in res if x[1][0] >= 0]
    lat = np.array([latency for _, (_, _, latency) in ok])
    work = sum(size(q) * st["iterations"] for q, (_, st, _) in res)
    unknowns = sum(size(q) for q, _ in res)
    statuses = sorted({status for _, (status, _, _) in res})
    serving = {
        "requests": len(res),
        "rate_per_s": round(rate, 3),
        "saturated_solves_per_s": round(saturated, 3),
        "closed_loop_span_s": round(span_cal, 3),
        "solves_per_s": round(len(res) / span, 3),
        "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
        "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
        "mean_latency_s": round(float(lat.mean()), 4),
        "span_s": round(span, 3),
        "mean_group_size": round(info["requests_started"] / max(info["groups_started"], 1), 3),
        "peak_device_bytes": info["peak_bytes"],
        "statuses": statuses,
        "failed": len(res) - len(ok),
    }
    if args.serve_baseline:
        serving["plain_fp64_sequential"] = plain_sequential(stp, torch, reqs)
        print(f"# plain FP64, one request at a time: {serving['plain_fp64_sequential']}",
              file=sys.stderr, flush=True)
    line = {
        "metric": METRIC,
        "value": work / span,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": round(span * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == stp.STP_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": "heat2d_serve", "requests": len(res), "unknowns_total": unknowns,
                   "J": "6..11", "K": "5..9", "rel_tol": "1e-10..1e-6", "precision": args.precision,
                   "load": args.load, "slots": args.slots, "batch": args.batch,
                   "budget_gb": args.budget_gb, "lookahead": args.lookahead,
                   "parallelism": "single-gpu"},
        "roofline": None,
        "cpu_baseline": None,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); multi-GPU time "
              "sharding is not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2009_08875_amd as stp

    if args.workload == "heat2d_serve":
        return run_serving(args, stp, torch)

    J, K, nrhs, seed, u0kind = WORKLOADS[args.workload]
    prec = stp.STP_FP64 if args.precision == "fp64" else stp.STP_MIXED
    dim = 3 if u0kind == "sin3" else 2
    opts = {"dim": dim, "lookahead": args.lookahead, "nested": args.nested}
    unknowns = (2 ** J + 1) * (2 ** K - 1) ** dim * nrhs
    print(f"# workload {args.workload} J={J} K={K} nrhs={nrhs} precision={args.precision}",
          file=sys.stderr, flush=True)

    ctx = stp.stp_create(J, K, nrhs, prec, opts, stream=torch.cuda.current_stream())
    load_inputs(stp, ctx, J, K, nrhs, seed, u0kind, torch)
    t_step, stats = run_solves(stp, ctx, nrhs, args.tol, args.steps, args.warmup, torch)
    kst = profile_solve(stp, ctx, nrhs, args.tol, torch)
    its = stats[-1][0]["iterations"]
    iters_sum = sum(s["iterations"] for s in stats[-1])
    u_main = None
    if not args.no_compare:
        u_main = torch.zeros(unknowns // nrhs, dtype=torch.float64, device="cuda:0")
        stp.stp_get_solution(ctx, 0, u_main)
    stp.stp_destroy(ctx)
    print(f"# main: {t_step * 1e3:.1f} ms per solve, iterations {its}", file=sys.stderr, flush=True)

    # roofline of the dominant kernel (largest summed device time), and the
    # achieved rate of every hot kernel
    table = kernel_table(stp, kst)
    dom = max(kst, key=lambda k: kst[k]["total_ms"])
    d = table[stp.STP_KERNEL_NAMES[dom]]
    roofline = {
        "kernel": stp.STP_KERNEL_NAMES[dom],
        "bound": "hbm",
        "achieved": d["achieved_gbs"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": d["frac"],
        "traffic": measured_traffic(args.workload, args.precision, stp.STP_KERNEL_NAMES[dom],
                                    d["alg_bytes_per_launch"]),
        "avg_launch_ms": d["avg_launch_ms"],
        "alg_bytes_per_launch": d["alg_bytes_per_launch"],
        "launches": d["launches"],
        "kernels": table,
    }
    if dim == 3:
        # the 3D multigrid runs as many short launches per level and colour,
        # which the library does not bracket with events
        roofline["scope"] = ("dominant among the timed launches; the 3D multigrid launches are not "
                             "timed here and take most of the solve (kernel trace)")

    compare = None
    if not args.no_compare:
        # the other precision; with nested iteration, the same precision without it
        other = prec if args.nested else (stp.STP_MIXED if prec == stp.STP_FP64 else stp.STP_FP64)
        ctx = stp.stp_create(J, K, nrhs, other, dict(opts, nested=0),
                             stream=torch.cuda.current_stream())
        load_inputs(stp, ctx, J, K, nrhs, seed, u0kind, torch)
        t2, st2 = run_solves(stp, ctx, nrhs, args.tol, 2, 1, torch)
        u2 = torch.zeros_like(u_main)
        stp.stp_get_solution(ctx, 0, u2)
        torch.cuda.synchronize()
        diff = (torch.linalg.vector_norm(u2 - u_main) / torch.linalg.vector_norm(u_main)).item()
        stp.stp_destroy(ctx)
        compare = {
            "precision": "mixed" if other == stp.STP_MIXED else "fp64",
            "nested": 0,
            "time_to_solve_s": round(t2, 4),
            "inner_iterations": st2[-1][0]["iterations"],
            "outer_iterations": st2[-1][0]["outer_iterations"],
            "unknowns_iters_per_s": unknowns * st2[-1][0]["iterations"] / t2,
            "speedup_time_to_solve": round(t_step / t2, 3),
            "rel_l2_diff_vs_main": diff,
        }
        print(f"# compare: {compare}", file=sys.stderr, flush=True)

    solo = None
    if nrhs > 1 and not args.no_compare:
        solo = solo_fp64_sequential(stp, torch, J, K, nrhs, seed, u0kind, args.tol)
        solo["speedup_of_batched"] = round(solo["time_s"] / t_step, 3)
        print(f"# solo FP64, one right-hand side at a time: {solo}", file=sys.stderr, flush=True)

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_sample_seconds)

    line = {
        "metric": METRIC,
        "value": (unknowns // nrhs) * iters_sum / t_step,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == stp.STP_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "J": J, "K": K, "nrhs": nrhs, "dim": dim,
                   "unknowns": unknowns, "precision": args.precision, "rel_tol": args.tol,
                   "iterations": its, "time_to_solve_s": round(t_step, 4),
                   **({"nested": args.nested,
                       "coarse_iterations": stats[-1][0]["coarse_iterations"]}
                      if args.nested else {}),
                   "parallelism": "single-gpu"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "compare": compare,
    }
    if solo is not None:
        line["solo_fp64_sequential"] = solo
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
