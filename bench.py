"""Benchmark: FP64 EGT/as solves of the 1081-hand river endgame on one MI355X.

One step = one complete solve (egt_solve: state creation with the initial-mu
search, then EGT/as iterations until the saddle gap is <= 1e-3 * pot) of a
52-card river endgame with 1081 hands per player, bets {0.5, 1, 2 pot,
all-in} and at most 3 raises (241,063 sequences per player).  The game tables
are built and resident in HBM before timing starts.

Prints one JSON line: solves/s as the value, iterations/s, p50/p99 solve
latency, the roofline of the dominant kernel (HIP-event timing of the same
launch inside this process) and the CPU FP64 oracle timed on a bounded
sample of the same solve.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "EGT iters/sec and endgame solves/sec to gap<=1e-3·pot; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
# HBM bytes per roofline launch (sbr_fused_kernel, egt_smoothed_br without the
# value) on the 1081-hand endgame c1, from two rocprofv3 --pmc passes of
# `bench.py --roofline-only --kernel-reps 50 --copy-calibration-mb 256`:
# FETCH_SIZE 1133.5 KiB and WRITE_SIZE 1895.5 KiB per dispatch, each scaled
# by the same counter on the plain 256 MiB device copy of that run
# (FETCH_SIZE reads 131085 KiB of the 262144 KiB copied: factor 2.0;
# WRITE_SIZE 262144 KiB: factor 1.0).  Valid for this kernel version only.
SBR_TRAFFIC_BYTES = {"c1": (1133.5 * 2.0 + 1895.5 * 1.0) * 1024}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c1")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--variant", default="AS")
    ap.add_argument("--cpu-sample-iters", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large-tree", action="store_true", help="skip the c3 (level path, tiled GEMM) section")
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--mixed-steps", type=int, default=5, help="precision-form solves of the same endgame")
    ap.add_argument("--serve-requests", type=int, default=24, help="requests of the serving trace (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=0.757,
                    help="Poisson arrival rate (requests/s); 0.757 is 0.9 x the saturated precision-form "
                         "throughput of the full 512-request trace")
    ap.add_argument("--serve-shapes", default="c0,c1,c2,c3")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--copy-calibration-mb", type=float, default=0.0,
                    help="run 5 plain device copies of this many MB first (scales HBM counters)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the kernel measurements (for counter runs under a profiler)")
    return ap.parse_args()


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def _timed(torch, fn, reps):
    """Average duration of fn() over reps back-to-back calls, HIP events on
    the current stream (the stream the library launches on)."""
    for _ in range(10):
        fn()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def kernel_roofline(egt, torch, G, reps, config=None):
    """The dominant kernel of an iteration, the single-launch smoothed best
    response (sbr_fused_kernel), launched as egt_smoothed_br without the value
    (one launch per call) on a product A y.  Algorithmic bytes per launch: the
    gradient read and the strategy written, 8-byte doubles over every
    (sequence, hand) of the player: 16 * n_seq * n."""
    y = egt.uniform(G, 1)
    g = egt.gradient(G, 0, y)
    q = G.empty(0)
    mu = 1e-3 * float(g.abs().max()) / 100.0
    avg_s = _timed(torch, lambda: egt.smoothed_br(G, 0, g, mu, q, want_value=False), reps)
    bytes_ = 16.0 * G.n_seq[0] * G.n
    gbs = bytes_ / avg_s / 1e9
    traffic = SBR_TRAFFIC_BYTES.get(config)
    # trees whose tables fit one block's LDS (every workload but c3) take the single-launch pass
    kernel = "level-path passes" if config == "c3" else "sbr_fused_kernel"
    return dict(kernel=kernel, bound="hbm", achieved=round(gbs, 3), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 6), traffic=round(traffic) if traffic else None,
                avg_us=round(avg_s * 1e6, 3), algorithmic_bytes=int(bytes_),
                launch="egt_smoothed_br, player 1, no value")


def gradient_roofline(egt, torch, G, reps):
    """The payoff product (gradient_kernel), A y at a treeplex point.
    Algorithmic bytes: one opponent row per terminal read and one output row
    per sequence written, 8-byte doubles over the n hands."""
    y = egt.uniform(G, 1)
    out = G.empty(0)
    avg_s = _timed(torch, lambda: egt.gradient(G, 0, y, out), reps)
    n_fold, n_show = G.terminals()
    bytes_ = 8.0 * G.n * ((n_fold + n_show) + G.n_seq[0])
    gbs = bytes_ / avg_s / 1e9
    return dict(kernel="gradient_kernel", bound="hbm", achieved=round(gbs, 3), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 6), avg_us=round(avg_s * 1e6, 3), algorithmic_bytes=int(bytes_))


def precision_form(egt, torch, G, steps, fp64_ms, fp64_value, reps):
    """The same endgame in the precision form: FP32 iterates, BF16 hi+lo
    showdown GEMM, FP32 prox with FP64 normalisers, FP64 gap every 10 iters."""
    egt.solve(G, precision="mixed", gap_every=10)  # warm-up (builds W)
    lat, iters, res = [], 0, None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        res, _ = egt.solve(G, precision="mixed", gap_every=10)
        lat.append(time.perf_counter() - ts)
        iters += res["iters"]
        if res["converged"] != 1:
            raise RuntimeError(f"precision-form solve did not converge: {res}")
    elapsed = time.perf_counter() - t0
    # product launch of the precision form: fold kernel + BF16 GEMM
    y32 = egt.uniform(G, 1).float().contiguous()
    out32 = G.empty(0, dtype=torch.float32)
    for _ in range(10):
        egt.gradient_mixed(G, 0, y32, out32)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        egt.gradient_mixed(G, 0, y32, out32)
    e1.record(s)
    e1.synchronize()
    prod_us = e0.elapsed_time(e1) / reps * 1e3
    n_fold, n_show = G.terminals()
    # dense BF16 GEMM of the showdown columns: W (ld x ld) times Y hi and Y lo (ld x n_show)
    flops = 2.0 * G.ld * G.ld * n_show * 2
    ms = elapsed / steps * 1e3
    return dict(
        solves_per_sec=steps / elapsed, iters_per_sec=iters / elapsed, ms_per_solve=ms,
        iters_per_solve=iters / steps, p50_ms=percentile(lat, 50) * 1e3, p99_ms=percentile(lat, 99) * 1e3,
        speedup_vs_fp64=fp64_ms / ms, final_gap_fp64=res["gap"],
        value_minus_fp64=res["value_p1"] - fp64_value,
        product_us=round(prod_us, 3), gemm_dense_gflop=flops / 1e9,
        mfma_util_lower_bound=flops / (prod_us * 1e-6) / 2.5e15,
        note="gap re-measured with FP64 products; mfma_util_lower_bound charges the whole product "
             "launch (fold kernel + GEMM) to the GEMM",
    )


def serving(egt, args):
    """Trace of solve requests (shapes drawn uniformly), continuously batched
    under an HBM budget: all at t = 0 in the precision form (the batched
    capacity over this short trace), then Poisson arrivals at --serve-rate,
    batched in the precision form, batched in FP64, and served one at a time
    in FP64 (the baseline)."""
    from instances import make_instance
    from instances.endgames import serving_trace
    from paper_1810_03063_amd.serve import LibEngine, Request, serve, serve_sequential, summarize

    shapes = tuple(args.serve_shapes.split(","))
    n = args.serve_requests
    budget = int(args.serve_budget_gb * (1 << 30))

    def reqs_for(rate):
        tr = serving_trace(n, rate=rate, seed=11, shapes=shapes)
        return [Request(i, a, make_instance(shape, seed)) for i, (a, shape, seed) in enumerate(tr)]

    def run(rate, precision="mixed"):
        eng = LibEngine(egt, budget, max_slots=64, precision=precision, gap_every=10 if precision == "mixed" else 1)
        out, wall = serve(eng, reqs_for(rate))
        eng.close()
        return summarize(out, wall)

    saturated = run(0.0)  # every request at t = 0
    rate = args.serve_rate
    loaded = run(rate)
    loaded64 = run(rate, "fp64")
    print("serving: batched runs done", file=sys.stderr, flush=True)

    def solve_one(r):
        G = egt.Game(r.payload)
        res, _ = egt.solve(G)
        G.close()
        return res.get("status", "EGT_OK"), res

    seq_out, seq_wall = serve_sequential(solve_one, reqs_for(rate))
    baseline = summarize(seq_out, seq_wall)
    return dict(shapes=list(shapes), requests=n, budget_gb=args.serve_budget_gb, saturated=saturated,
                poisson_rate_per_s=rate, batched=loaded, batched_fp64=loaded64, sequential_fp64=baseline,
                throughput_vs_sequential=loaded["solves_per_sec"] / baseline["solves_per_sec"],
                fp64_batched_vs_sequential=loaded64["solves_per_sec"] / baseline["solves_per_sec"])


def large_tree(egt, torch, args):
    """The 8-bet-size endgame (c3), whose tables exceed one block's LDS so
    every pass runs level by level and whose 3958 showdown columns take the
    tiled GEMM: one FP64 EGT/as solve and one precision-form solve after a
    warm-up of each, and the rooflines of its smoothed best response and
    product."""
    from instances import make_instance

    inst = make_instance("c3", args.seed)
    G = egt.Game(inst)
    egt.solve(G, variant=args.variant)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, _ = egt.solve(G, variant=args.variant)
    fp64_s = time.perf_counter() - t0
    if res["converged"] != 1:
        raise RuntimeError(f"c3 solve did not converge: {res}")
    reps = max(1, args.kernel_reps // 10)
    out = dict(
        workload=f"c3: 52-card river endgame, {G.n} hands/player, bets {list(inst.bet_fracs)} pot + all-in, "
                 f"max {inst.max_raises} raises, {G.n_seq[0] * G.n} sequences/player",
        fp64_ms=fp64_s * 1e3, fp64_iters=res["iters"], fp64_iters_per_sec=res["iters"] / fp64_s,
        roofline=kernel_roofline(egt, torch, G, reps, "c3"),
        roofline_gradient=gradient_roofline(egt, torch, G, reps),
        precision_form=precision_form(egt, torch, G, 1, fp64_s * 1e3, res["value_p1"], reps))
    G.close()
    return out


def cpu_baseline(inst, sample_iters, iters_per_solve, variant):
    import numpy as np  # noqa: F401
    from threadpoolctl import threadpool_info

    from oracle import Problem, solve

    P = Problem(inst)
    t0 = time.perf_counter()
    tr = solve(P, variant, eps=0.0, max_iters=sample_iters)
    dt = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    ips = tr.iters / dt
    return dict(value=ips / iters_per_solve, unit="solves/s", cores=int(threads), kind="oracle",
                sample=f"{tr.iters} EGT/{variant} iterations of the same endgame (incl. start-up) in {dt:.1f} s "
                       f"= {ips:.3f} iters/s, scaled by {iters_per_solve} iterations per solve",
                iters_per_sec=ips)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from instances import make_instance
    from paper_1810_03063_amd import egt

    torch.cuda.set_device(0)
    if args.copy_calibration_mb > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # calibrate the counters of the other kernels
        nbytes = int(args.copy_calibration_mb * (1 << 20)) // 8 * 8
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    inst = make_instance(args.config, args.seed)
    G = egt.Game(inst)
    torch.cuda.synchronize()
    if args.roofline_only:
        y32 = egt.uniform(G, 1).float().contiguous()
        out32 = G.empty(0, dtype=torch.float32)
        prod_s = _timed(torch, lambda: egt.gradient_mixed(G, 0, y32, out32), args.kernel_reps)
        print(json.dumps({"roofline": kernel_roofline(egt, torch, G, args.kernel_reps, args.config),
                          "roofline_gradient": gradient_roofline(egt, torch, G, args.kernel_reps),
                          "mixed_product_us": round(prod_s * 1e6, 3)}), flush=True)
        return
    for _ in range(args.warmup):
        r, _ = egt.solve(G, variant=args.variant)
        print(f"warmup solve: {r['iters']} iters, gap {r['gap']:.4g}, {r['seconds']*1e3:.1f} ms", file=sys.stderr,
              flush=True)
    lat = []
    iters = 0
    res = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        res, _ = egt.solve(G, variant=args.variant)
        lat.append(time.perf_counter() - ts)
        iters += res["iters"]
        if res["converged"] != 1:
            raise RuntimeError(f"solve {k} did not converge: {res}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"timed {args.steps} solves in {elapsed:.3f} s", file=sys.stderr, flush=True)
    roof = kernel_roofline(egt, torch, G, args.kernel_reps, args.config)
    roof_grad = gradient_roofline(egt, torch, G, args.kernel_reps)
    iters_per_solve = iters / args.steps
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.config}: 52-card river endgame, {G.n} hands/player, bets "
                        f"{list(inst.bet_fracs)} pot + all-in, max {inst.max_raises} raises, "
                        f"{G.n_seq[0] * G.n} sequences/player; FP64 EGT/{args.variant} to gap <= 1e-3*pot",
            "seed": args.seed,
            "variant": args.variant,
            "eps": 1e-3 * inst.pot,
        },
        "iters_per_sec": iters / elapsed,
        "iters_per_solve": iters_per_solve,
        "p50_ms": percentile(lat, 50) * 1e3,
        "p99_ms": percentile(lat, 99) * 1e3,
        "final_gap": res["gap"],
        "roofline": roof,
        "roofline_gradient": roof_grad,
    }
    if args.mixed_steps > 0:
        out["precision_form"] = precision_form(egt, torch, G, args.mixed_steps, out["ms_per_step"], res["value_p1"],
                                               args.kernel_reps)
        print(f"precision form: {out['precision_form']['ms_per_solve']:.1f} ms per solve", file=sys.stderr,
              flush=True)
    if not args.no_large_tree and args.config != "c3":
        out["large_tree"] = large_tree(egt, torch, args)
        print(f"large tree: {out['large_tree']['fp64_ms']:.0f} ms FP64, "
              f"{out['large_tree']['precision_form']['ms_per_solve']:.0f} ms precision form", file=sys.stderr,
              flush=True)
    if args.serve_requests > 0:
        out["serving"] = serving(egt, args)
        print("serving done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_sample_iters, iters_per_solve, args.variant)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
