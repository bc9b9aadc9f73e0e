"""Serve one synthetic request trace end to end and print its latency summary.

    python -m paper_1810_03063_amd.serve_trace --mode batched --precision mixed --rate 0.757 --n 512 --out trace.json

Each request draws one endgame shape uniformly from --shapes with its own seed; arrivals are Poisson at --rate
(requests/s), or all at t = 0 when the rate is 0.  `batched` runs the continuously batched engine (`egt_batch_*`,
one HBM budget); `sequential` solves one request at a time in FP64 in arrival order.  One progress line is printed
per eight finished requests; the summary (throughput, p50/p99/mean latency, the per-shape medians) is printed as one
JSON line and written to --out.
"""
import argparse
import json
import os
import time

from instances import make_instance
from instances.endgames import serving_trace

from . import egt
from .serve import LibEngine, Request, percentile, serve, serve_sequential, summarize


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--mode", choices=["batched", "sequential"], required=True)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--rate", type=float, default=0.0, help="Poisson arrival rate in requests/s; 0 = all at t = 0")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--shapes", default="c0,c1,c2,c3")
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--max-slots", type=int, default=64)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)

    shapes = tuple(a.shapes.split(","))
    trace = serving_trace(a.n, rate=a.rate, seed=a.seed, shapes=shapes)
    reqs = [Request(i, t, make_instance(shape, seed)) for i, (t, shape, seed) in enumerate(trace)]
    count = {s: 0 for s in shapes}
    for _, shape, _ in trace:
        count[shape] += 1
    print("shapes", count, flush=True)

    done = [0]
    t0 = time.perf_counter()

    def progress():
        done[0] += 1
        if done[0] % 8 == 0 or done[0] == a.n:
            print(f"finished {done[0]}/{a.n} at {time.perf_counter() - t0:.1f} s", flush=True)

    if a.mode == "batched":
        class Engine(LibEngine):
            def retire(self, slot):
                super().retire(slot)
                progress()

        eng = Engine(egt, int(a.budget_gb * (1 << 30)), max_slots=a.max_slots, precision=a.precision,
                     gap_every=10 if a.precision == "mixed" else 1)
        out, wall = serve(eng, reqs)
        eng.close()
    else:
        def solve_one(r):
            G = egt.Game(r.payload)
            res, _ = egt.solve(G)
            G.close()
            progress()
            return res.get("status", "EGT_OK"), res

        out, wall = serve_sequential(solve_one, reqs)

    s = summarize(out, wall)
    s.update(mode=a.mode, precision=a.precision if a.mode == "batched" else "fp64", rate=a.rate, n=a.n,
             shapes=count)
    by = {}
    for r, (_, shape, _) in zip(out, trace):
        by.setdefault(shape, []).append(r.latency)
    s["p50_ms_by_shape"] = {k: percentile(v, 50) * 1e3 for k, v in sorted(by.items())}
    if os.path.dirname(a.out):
        os.makedirs(os.path.dirname(a.out), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(s, f)
    print(json.dumps(s), flush=True)


if __name__ == "__main__":
    main()
