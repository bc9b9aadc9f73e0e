"""Benchmark: FP64 EGT/as solves of the 8-bet-size 1081-hand river endgame on one MI355X.

One step = one complete solve (egt_solve: state creation with the initial-mu
search, then EGT/as iterations until the saddle gap is <= 1e-3 * pot) of a
52-card river endgame with 1081 hands per player, bets {0.25, 0.5, 0.75, 1,
1.5, 2, 3 pot, all-in} and at most 4 raises (6,418,978 sequences per player).
The game tables are built and resident in HBM before timing starts.

Prints one JSON line: solves/s as the value, iterations/s and ms per
iteration, p50/p99 solve latency, the roofline of the dominant kernel (the
payoff product, HIP-event timing of the same launch inside this process), the
same endgame in the precision form, the 241k-sequence endgame (c1) as a second
workload, the serving trace, and the CPU FP64 oracle timed on a bounded sample
of the headline solve.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "EGT iters/sec and endgame solves/sec to gap<=1e-3·pot; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
CSRC = os.path.join(ROOT, "paper_1810_03063_amd", "csrc")

# HBM bytes per launch from two rocprofv3 --pmc passes (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch) of `bench.py --roofline-only --config <c>
# --kernel-reps 50 --copy-calibration-mb 256`, each scaled by the same counter
# on the plain 256 MiB device copy of that run (FETCH_SIZE reads half of the
# bytes copied: factor 2.0; WRITE_SIZE all of them: factor 1.0).  Each entry
# records the SHA-256 of the kernel's source file when the counters were
# taken; a changed source makes the figure stale, and `traffic` is then null.
COUNTERS = {
    ("sbr_fused_kernel", "c1"): dict(fetch_kib=1171.0, write_kib=1895.5, fetch_factor=2.0, write_factor=1.0,
                                     source="egt_kernels.hip",
                                     sha256="81913217080a3eb9a26ab7f61afba20bd5deb50b86c74d123c3ddd81493cd948"),
    ("product_kernel", "c1"): dict(fetch_kib=1516.2, write_kib=1895.5, fetch_factor=2.0, write_factor=1.0,
                                   source="egt_product.hip",
                                   sha256="05488bbbd8d5c5a5f86458629065cd8a37711263bc67d56c718e0d663475b1b2"),
    ("product_kernel", "c3"): dict(fetch_kib=25849.7, write_kib=50474.1, fetch_factor=2.0, write_factor=1.0,
                                   source="egt_product.hip",
                                   sha256="05488bbbd8d5c5a5f86458629065cd8a37711263bc67d56c718e0d663475b1b2"),
}


def source_sha(name):
    with open(os.path.join(CSRC, name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_bytes(kernel, config):
    c = COUNTERS.get((kernel, config))
    if not c or not c["sha256"] or source_sha(c["source"]) != c["sha256"]:
        return None
    return (c["fetch_kib"] * c["fetch_factor"] + c["write_kib"] * c["write_factor"]) * 1024


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed solves of the headline endgame")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", help="headline endgame (c3: 8 bet sizes, 4 raises)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--variant", default="AS")
    ap.add_argument("--cpu-sample-iters", type=int, default=12,
                    help="oracle iterations timed for the CPU baseline (after its start-up)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--mixed-steps", type=int, default=2, help="precision-form solves of the headline endgame")
    ap.add_argument("--second-config", default="c1", help="second workload ('' = skip)")
    ap.add_argument("--second-steps", type=int, default=10)
    ap.add_argument("--serve-requests", type=int, default=32, help="requests of the serving trace (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="Poisson arrival rate (requests/s) of the loaded runs; 0 = 0.9 x the measured "
                         "saturated batched throughput")
    ap.add_argument("--serve-shapes", default="c0,c1,c2,c3")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--serve-small-shapes", default="c0,c1,c2",
                    help="shapes of a second saturated trace without the largest endgame ('' = skip)")
    ap.add_argument("--other-paths", type=int, default=1, help="CFR+, mirror prox and general-game measurements")
    ap.add_argument("--cfr-iters", type=int, default=20000)
    ap.add_argument("--fom-iters", type=int, default=2000)
    ap.add_argument("--fom-step", type=float, default=20.0,
                    help="mirror-prox step (the best of 2e-4 .. 20 in a sweep on the 3-size endgame)")
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
    for _ in range(5):
        fn()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def product_roofline(egt, torch, G, reps, config):
    """The payoff product (product_kernel), A y at the uniform point.
    Algorithmic bytes: one opponent row per terminal read and one output row
    per sequence written, 8-byte doubles over the n hands."""
    y = egt.uniform(G, 1)
    out = G.empty(0)
    avg_s = _timed(torch, lambda: egt.gradient(G, 0, y, out), reps)
    n_fold, n_show = G.terminals()
    bytes_ = 8.0 * G.n * ((n_fold + n_show) + G.n_seq[0])
    gbs = bytes_ / avg_s / 1e9
    traffic = traffic_bytes("product_kernel", config)
    return dict(kernel="product_kernel", bound="hbm", achieved=round(gbs, 3), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 6), traffic=round(traffic) if traffic else None,
                avg_us=round(avg_s * 1e6, 3), algorithmic_bytes=int(bytes_),
                launch="egt_gradient, player 0 (A y): one opponent row read per terminal, one row written per "
                       "sequence")


def sbr_roofline(egt, torch, G, reps, config):
    """The smoothed best response, launched as egt_smoothed_br without the
    value on a product A y.  Algorithmic bytes per launch: the gradient read
    and the strategy written, 8-byte doubles over every (sequence, hand) of the
    player: 16 * n_seq * n.  Trees whose tables fit one block's LDS run it as
    one launch (sbr_fused_kernel), larger ones level by level."""
    y = egt.uniform(G, 1)
    g = egt.gradient(G, 0, y)
    q = G.empty(0)
    mu = 1e-3 * float(g.abs().max()) / 100.0
    avg_s = _timed(torch, lambda: egt.smoothed_br(G, 0, g, mu, q, want_value=False), reps)
    bytes_ = 16.0 * G.n_seq[0] * G.n
    gbs = bytes_ / avg_s / 1e9
    fused = G.n_seq[0] < 1000
    kernel = "sbr_fused_kernel" if fused else "level-path passes"
    traffic = traffic_bytes(kernel, config) if fused else None
    return dict(kernel=kernel, bound="hbm", achieved=round(gbs, 3), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 6), traffic=round(traffic) if traffic else None,
                avg_us=round(avg_s * 1e6, 3), algorithmic_bytes=int(bytes_),
                launch="egt_smoothed_br, player 1, no value")


def timed_solves(egt, torch, G, steps, warmup, **opts):
    for _ in range(warmup):
        r, _ = egt.solve(G, **opts)
        print(f"warmup solve: {r['iters']} iters, gap {r['gap']:.4g}, {r['seconds']*1e3:.1f} ms", file=sys.stderr,
              flush=True)
    lat, iters, res = [], [], None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ts = time.perf_counter()
        res, _ = egt.solve(G, **opts)
        lat.append(time.perf_counter() - ts)
        iters.append(res["iters"])
        if res["converged"] != 1:
            raise RuntimeError(f"solve {k} did not converge: {res}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return dict(elapsed=elapsed, lat=lat, iters=iters, last=res)


def describe(cfg, inst, G):
    return (f"{cfg}: 52-card river endgame, {G.n} hands/player, bets {list(inst.bet_fracs)} pot + all-in, "
            f"max {inst.max_raises} raises, {G.n_seq[0] * G.n} sequences/player; FP64 EGT/AS to gap <= 1e-3*pot")


def precision_form(egt, torch, G, steps, fp64, reps):
    """The same endgame in the precision form: FP32 iterates, BF16 hi+lo
    showdown GEMM, FP32 prox with FP64 normalisers, FP64 gap every 10 iters."""
    r = timed_solves(egt, torch, G, steps, 1, precision="mixed", gap_every=10)
    res = r["last"]
    ms_iter = r["elapsed"] / sum(r["iters"]) * 1e3
    fp64_ms_iter = fp64["elapsed"] / sum(fp64["iters"]) * 1e3
    # FP64 with the same gap cadence (the best responses of the gap run only
    # on the iterations that test it)
    r10 = timed_solves(egt, torch, G, 1, 0, gap_every=10)
    fp64_10_ms_iter = r10["elapsed"] / sum(r10["iters"]) * 1e3
    y32 = egt.uniform(G, 1).float().contiguous()
    out32 = G.empty(0, dtype=torch.float32)
    prod_s = _timed(torch, lambda: egt.gradient_mixed(G, 0, y32, out32), reps)
    n_fold, n_show = G.terminals()
    flops = 2.0 * G.ld * G.ld * n_show * 2  # W (ld x ld) times Y hi and Y lo (ld x showdown columns)
    return dict(
        solves_per_sec=steps / r["elapsed"], iters_per_sec=sum(r["iters"]) / r["elapsed"],
        ms_per_solve=r["elapsed"] / steps * 1e3, ms_per_iteration=ms_iter, iters_per_solve=sum(r["iters"]) / steps,
        p50_ms=percentile(r["lat"], 50) * 1e3, p99_ms=percentile(r["lat"], 99) * 1e3,
        speedup_per_iteration_vs_fp64=fp64_ms_iter / ms_iter,
        fp64_gap_every_10_ms_per_iteration=fp64_10_ms_iter,
        speedup_per_iteration_vs_fp64_same_gap_cadence=fp64_10_ms_iter / ms_iter,
        speedup_per_solve_vs_fp64=(fp64["elapsed"] / len(fp64["lat"])) / (r["elapsed"] / steps),
        final_gap_fp64=res["gap"], value_minus_fp64=res["value_p1"] - fp64["last"]["value_p1"],
        product_us=round(prod_s * 1e6, 3), gemm_dense_gflop=flops / 1e9,
        note="gap measured with FP64 products and FP64 best responses; the product launch is the fold kernel "
             "plus the BF16 GEMM",
    )


def second_workload(egt, torch, args):
    """A second endgame (default c1: 241k sequences per player, whose trees run
    the single-launch smoothed best response)."""
    from instances import make_instance

    cfg = args.second_config
    inst = make_instance(cfg, args.seed)
    G = egt.Game(inst)
    r = timed_solves(egt, torch, G, args.second_steps, 2, variant=args.variant)
    out = dict(workload=describe(cfg, inst, G), solves_per_sec=args.second_steps / r["elapsed"],
               iters_per_sec=sum(r["iters"]) / r["elapsed"], ms_per_iteration=r["elapsed"] / sum(r["iters"]) * 1e3,
               iters_per_solve=sum(r["iters"]) / args.second_steps, p50_ms=percentile(r["lat"], 50) * 1e3,
               p99_ms=percentile(r["lat"], 99) * 1e3,
               roofline_sbr=sbr_roofline(egt, torch, G, args.kernel_reps * 4, cfg),
               roofline_product=product_roofline(egt, torch, G, args.kernel_reps * 4, cfg))
    if args.mixed_steps > 0:
        out["precision_form"] = precision_form(egt, torch, G, max(args.mixed_steps, 5), r, args.kernel_reps * 4)
    G.close()
    return out


def spmv_roofline(egt, torch, G, reps):
    """The general route's CSR product (spmv_kernel), A y.  Algorithmic bytes
    per launch: per nonzero its value, its column and the gathered entry of y
    (8 + 4 + 8), per row its two row pointers and the written output row of ld
    doubles (slot 0 and the zero padding)."""
    y = egt.uniform(G, 1)
    out = G.empty(0)
    avg_s = _timed(torch, lambda: egt.gradient(G, 0, y, out), reps)
    nnz = len(G.inst.entries)
    bytes_ = 20.0 * nnz + (16.0 + 8.0 * G.ld) * G.n_seq[0]
    gbs = bytes_ / avg_s / 1e9
    return dict(kernel="spmv_kernel", bound="hbm", achieved=round(gbs, 3), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 6), traffic=None, avg_us=round(avg_s * 1e6, 3),
                algorithmic_bytes=int(bytes_), nnz=nnz, rows=G.n_seq[0],
                launch="egt_gradient on a general game, player 0 (A y)")


def other_paths(egt, torch, args):
    """The paper's comparison methods and extensions, measured beside the
    headline: CFR+ to the same gap target on the second endgame (gradient
    computations against EGT's, the comparison of Section 7), mirror prox
    there (Section 8), an endgame with Section 7's Libratus-style bet sizes,
    and the general route (Section 6): Leduc hold'em solved to 1e-3 of its
    pot and the CSR product's roofline on a seeded random game tree."""
    from instances import make_instance
    from instances.efg import leduc, random_efg

    cfg = args.second_config or "c1"
    inst = make_instance(cfg, args.seed)
    G = egt.Game(inst)
    eps = 1e-3 * inst.pot
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r_egt, _ = egt.solve(G)
    t1 = time.perf_counter()
    r_cfr = egt.cfr_solve(G, "CFR_PLUS", eps=eps, max_iters=args.cfr_iters, gap_every=10)
    t2 = time.perf_counter()
    F = egt.Fom(G, "MP", args.fom_step)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    F.step(args.fom_iters)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    mp_gap = F.gap()[0]
    F.close()
    G.close()
    out = dict(
        workload=describe(cfg, inst, G),
        egt_as=dict(iters=r_egt["iters"], products=r_egt["products"], gap=r_egt["gap"], seconds=t1 - t0),
        cfr_plus=dict(iters=r_cfr["iters"], products=r_cfr["products"], gap=r_cfr["gap"],
                      converged=r_cfr["converged"], seconds=t2 - t1, iters_per_sec=r_cfr["iters"] / (t2 - t1),
                      note=f"to gap <= 1e-3*pot or {args.cfr_iters} iterations, gap tested every 10"),
        mirror_prox=dict(iters=args.fom_iters, step=args.fom_step, gap=mp_gap, seconds=t4 - t3,
                         iters_per_sec=args.fom_iters / (t4 - t3)),
    )
    li = make_instance("lib", args.seed)
    GL = egt.Game(li)
    r = timed_solves(egt, torch, GL, 3, 1)
    out["libratus_abstraction"] = dict(
        workload=f"lib: 52-card river endgame, {GL.n} hands/player, Section 7's Libratus-style bet sizes with open "
                 f"folds, {GL.n_seq[0] * GL.n} + {GL.n_seq[1] * GL.n} (sequence, hand) pairs; FP64 EGT/AS to gap <= "
                 f"1e-3*pot",
        solves_per_sec=3 / r["elapsed"], iters_per_solve=sum(r["iters"]) / 3,
        ms_per_iteration=r["elapsed"] / sum(r["iters"]) * 1e3, final_gap=r["last"]["gap"], eps=1e-3 * li.pot)
    GL.close()
    lg = leduc()
    GG = egt.GeneralGame(lg)
    r = timed_solves(egt, torch, GG, 3, 1)
    out["general_leduc"] = dict(workload=f"Leduc hold'em, {GG.n_seq[0]} + {GG.n_seq[1]} sequences, "
                                         f"{len(lg.entries)} payoff entries; FP64 EGT/AS to gap <= 1e-3*pot",
                                solves_per_sec=3 / r["elapsed"], iters_per_solve=sum(r["iters"]) / 3,
                                ms_per_iteration=r["elapsed"] / sum(r["iters"]) * 1e3, final_gap=r["last"]["gap"])
    GG.close()
    rg = random_efg(5, depth=8, max_actions=4, n_types=20)
    GR = egt.GeneralGame(rg)
    out["general_spmv"] = dict(workload=f"seeded random game tree, {GR.n_seq[0]} x {GR.n_seq[1]} sequences, "
                                        f"{len(rg.entries)} payoff entries",
                               roofline=spmv_roofline(egt, torch, GR, args.kernel_reps * 4))
    GR.close()
    return out


def serving(egt, args):
    """Trace of solve requests (shapes drawn uniformly), continuously batched
    under an HBM budget: all at t = 0 (the saturated capacity: batched in the
    precision form, batched in FP64, and sequential FP64), then Poisson
    arrivals at 0.9 x the batched capacity, batched in the precision form,
    batched in FP64, and served one at a time in FP64 (the baseline)."""
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

    def solve_one(r):
        G = egt.Game(r.payload)
        res, _ = egt.solve(G)
        G.close()
        return res.get("status", "EGT_OK"), res

    def note(what, res):
        print(f"serving: {what}: {res['solves_per_sec']:.3f} solves/s", file=sys.stderr, flush=True)

    saturated = run(0.0)  # every request at t = 0
    note("saturated, batched", saturated)
    saturated64 = run(0.0, "fp64")
    note("saturated, batched FP64", saturated64)
    seq_sat_out, seq_sat_wall = serve_sequential(solve_one, reqs_for(0.0))
    seq_saturated = summarize(seq_sat_out, seq_sat_wall)
    note("saturated, one at a time", seq_saturated)
    rate = args.serve_rate if args.serve_rate > 0 else 0.9 * saturated["solves_per_sec"]
    loaded = run(rate)
    note("Poisson arrivals, batched precision form", loaded)
    loaded64 = run(rate, "fp64")
    note("Poisson arrivals, batched FP64", loaded64)
    seq_out, seq_wall = serve_sequential(solve_one, reqs_for(rate))
    baseline = summarize(seq_out, seq_wall)
    note("Poisson arrivals, one at a time", baseline)
    out = dict(shapes=list(shapes), requests=n, budget_gb=args.serve_budget_gb, saturated=saturated,
               saturated_sequential_fp64=seq_saturated,
               capacity_vs_sequential=saturated["solves_per_sec"] / seq_saturated["solves_per_sec"],
               saturated_fp64=saturated64,
               capacity_vs_sequential_fp64=saturated64["solves_per_sec"] / seq_saturated["solves_per_sec"],
               poisson_rate_per_s=rate, batched=loaded, batched_fp64=loaded64, sequential_fp64=baseline)
    if args.serve_small_shapes:
        # the same saturated comparison without the 8-size endgame, whose
        # kernels fill the device by themselves
        small = tuple(args.serve_small_shapes.split(","))

        def small_reqs():
            tr = serving_trace(2 * n, rate=0.0, seed=12, shapes=small)
            return [Request(i, a, make_instance(shape, seed)) for i, (a, shape, seed) in enumerate(tr)]

        eng = LibEngine(egt, budget, max_slots=64, precision="fp64", gap_every=1)
        o, w = serve(eng, small_reqs())
        eng.close()
        sb = summarize(o, w)
        so, sw = serve_sequential(solve_one, small_reqs())
        ss = summarize(so, sw)
        note(f"saturated {','.join(small)}, batched FP64", sb)
        note(f"saturated {','.join(small)}, one at a time", ss)
        out["small_shapes"] = dict(shapes=list(small), requests=2 * n, saturated_batched_fp64=sb,
                                   saturated_sequential_fp64=ss,
                                   capacity_vs_sequential=sb["solves_per_sec"] / ss["solves_per_sec"])
    return out


def cpu_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def cpu_baseline(inst, sample_iters, iters_per_solve, variant, mu0):
    """The CPU FP64 oracle on the same endgame: its start-up with the GPU's
    initial mu (no doubling search), then `sample_iters` timed iterations;
    solves/s = iterations/s / iterations per GPU solve (the start-up is left
    out, which favours the CPU)."""
    from threadpoolctl import threadpool_info

    from oracle import Problem, solve

    P = Problem(inst)
    stamps = []
    t0 = time.perf_counter()
    tr = solve(P, variant, eps=0.0, max_iters=sample_iters, mu0=mu0,
               on_iterate=lambda t, *a: stamps.append(time.perf_counter()))
    t1 = time.perf_counter()
    # stamps[t] is taken before iterate t's gap test; iteration t runs until stamps[t + 1]
    it_s = (stamps[-1] - stamps[0]) / max(tr.iters, 1)
    ips = 1.0 / it_s
    blas = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    return dict(value=ips / iters_per_solve, unit="solves/s", cores=int(blas), kind="oracle",
                sample=f"{tr.iters} EGT/{variant} iterations of the same endgame (each with its saddle-gap test) "
                       f"after the start-up at the GPU's initial mu: {it_s:.2f} s per iteration = {ips:.4f} "
                       f"iters/s (extrapolated: x {iters_per_solve:.0f} iterations per GPU solve, start-up "
                       f"{stamps[0] - t0:.1f} s not counted); {t1 - t0:.1f} s in all",
                iters_per_sec=ips, host_cpus=os.cpu_count(), cpu_model=cpu_info(), blas_threads=int(blas))


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
        print(json.dumps({"roofline_sbr": sbr_roofline(egt, torch, G, args.kernel_reps, args.config),
                          "roofline_product": product_roofline(egt, torch, G, args.kernel_reps, args.config),
                          "mixed_product_us": round(prod_s * 1e6, 3)}), flush=True)
        return
    st = egt.State(G, variant=args.variant)
    mu0 = (st.get()["mu_x"], st.get()["mu_y"])
    st.close()
    r = timed_solves(egt, torch, G, args.steps, args.warmup, variant=args.variant)
    elapsed = r["elapsed"]
    print(f"timed {args.steps} solves in {elapsed:.3f} s", file=sys.stderr, flush=True)
    iters_total = sum(r["iters"])
    iters_per_solve = iters_total / args.steps
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
        "config": {"workload": describe(args.config, inst, G), "seed": args.seed, "variant": args.variant,
                   "eps": 1e-3 * inst.pot},
        "iters_per_sec": iters_total / elapsed,
        "ms_per_iteration": elapsed / iters_total * 1e3,
        "iters_per_solve": iters_per_solve,
        "p50_ms": percentile(r["lat"], 50) * 1e3,
        "p99_ms": percentile(r["lat"], 99) * 1e3,
        "final_gap": r["last"]["gap"],
        "roofline": product_roofline(egt, torch, G, args.kernel_reps, args.config),
        "roofline_sbr": sbr_roofline(egt, torch, G, args.kernel_reps, args.config),
    }
    if args.mixed_steps > 0:
        out["precision_form"] = precision_form(egt, torch, G, args.mixed_steps, r, args.kernel_reps)
        print(f"precision form: {out['precision_form']['ms_per_solve']:.1f} ms per solve", file=sys.stderr,
              flush=True)
    G.close()
    if args.second_config:
        out["second_workload"] = second_workload(egt, torch, args)
        print("second workload done", file=sys.stderr, flush=True)
    if args.other_paths:
        out["other_paths"] = other_paths(egt, torch, args)
        print("other paths done", file=sys.stderr, flush=True)
    if args.serve_requests > 0:
        out["serving"] = serving(egt, args)
        print("serving done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_sample_iters, iters_per_solve, args.variant, mu0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
