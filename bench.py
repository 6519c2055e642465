"""Benchmark: first-come-first-served plan requests per second at 3000 known plans.

Workload: 30 x 30 x 1.5 km airspace, 3000 known straight constant-speed plans,
360 actions (24 headings x 5 climb rates x 3 speeds), dt = 0.5 s, up to 3600
steps per request, 1000 FCFS requests (seeded synthetic inputs).  One bench
step plans and accepts all 1000 requests first-come-first-served with
concurrent slots, starting from the 3000-plan table (rewound between steps,
outside the timed region).  Printed: one JSON line with requests/s, the
planner kernel's roofline against the FP32 vector peak, p50/p99 latency of a
Poisson-arrival serving pass, and the FP64 CPU oracle timed on a bounded
sample of the same requests.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak
FLOPS_PER_PAIR = 8                  # 3 sub + 3 mul + 2 add for one squared distance


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(sc, budget_s: float):
    """FP64 oracle, FCFS with commits, on the first requests until budget_s."""
    from oracle import oracle as O
    orc = O.Oracle(sc.cfg, sc.plans, sc.terrain)
    t0 = time.perf_counter()
    n = 0
    pairs_note = None
    while n < sc.requests.n:
        p = orc.plan(sc.requests.origin[n], sc.requests.goal[n], int(sc.requests.t0[n]))
        if p.status == 0:
            orc.commit(p)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": n / el, "unit": "req/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"first {n} of the {sc.requests.n} FCFS requests (plan + commit, FP64, literal per-peak "
                      f"maximum), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plans", type=int, default=3000)
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--slots", type=int, default=1024)
    ap.add_argument("--steps-per-launch", type=int, default=256)
    ap.add_argument("--planner-threads", type=int, default=0, help="planning workgroup size: 0 or 1024")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrivals [req/s]; 0 disables")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work; 0 disables")
    ap.add_argument("--seed", type=int, default=2)
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    from paper_2008_03518_amd import fastmdp as fm
    from paper_2008_03518_amd import scenario as S

    sc = S.large_actions(seed=args.seed, n_plans=args.plans, n_requests=max(args.requests, args.serve_requests))
    cfg = sc.cfg
    reqs = S.Requests(sc.requests.ident[:args.requests], sc.requests.origin[:args.requests],
                      sc.requests.goal[:args.requests], sc.requests.t0[:args.requests])
    log(f"workload: {sc.plans.n} plans, {cfg.n_actions} actions, {reqs.n} requests, slots {args.slots}")

    ctx = fm.context_for(sc, max_slots=args.slots, steps_per_launch=args.steps_per_launch,
                         planner_threads=args.planner_threads)
    ctx.snapshot()

    def one_step():
        ctx.rewind()
        t = time.perf_counter()
        plans, committed, done = ctx.plan_fcfs(reqs)
        el = time.perf_counter() - t
        return el, plans, committed, done, ctx.stats()

    for w in range(args.warmup):
        el, *_ = one_step()
        log(f"warmup {w}: {el * 1e3:.1f} ms")
    times, pairs, kms, launches, steps, resumes = [], 0, 0.0, 0, 0, 0
    for k in range(args.steps):
        el, plans, committed, done, st = one_step()
        times.append(el)
        pairs += st["pairs"]
        kms += st["kernel_ms"]
        launches += st["launches"]
        steps += st["steps"]
        resumes += st["resumes"]
        log(f"step {k}: {el * 1e3:.1f} ms, committed {int(committed.sum())}/{reqs.n}, "
            f"pairs {st['pairs']:.3e}, planner {st['kernel_ms']:.1f} ms in {st['launches']} launches, "
            f"resumes {st['resumes']}")
    total = sum(times)
    value = args.steps * reqs.n / total
    achieved = FLOPS_PER_PAIR * pairs / (kms * 1e-3) / 1e12
    status = np.array([p.status for p in plans])

    out = {
        "metric": "FCFS plan requests/sec at 3000 known plans",
        "value": value,
        "unit": "req/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{sc.plans.n} known plans, {cfg.n_actions} actions (24 headings x 5 climbs x 3 speeds), "
                        f"dt 0.5 s, {reqs.n} FCFS requests, 30x30x1.5 km",
            "known_plans": sc.plans.n, "actions": cfg.n_actions, "requests_per_step": reqs.n,
            "slots": args.slots, "steps_per_launch": args.steps_per_launch,
            "planner_threads": args.planner_threads,
        },
        "pair_evals_per_s": pairs / (kms * 1e-3),
        "planner_steps": steps,
        "resumes": resumes,
        "committed_per_step": int(committed.sum()),
        "status_counts": {S.STATUS_NAMES[int(k)]: int((status == k).sum()) for k in np.unique(status)},
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": None,
            "kernel": "planner_kernel",
            "avg_launch_ms": kms / max(launches, 1),
            "flops_per_launch": FLOPS_PER_PAIR * pairs / max(launches, 1),
        },
    }

    if args.serve_rate > 0:
        m = args.serve_requests
        sreq = S.Requests(sc.requests.ident[:m], sc.requests.origin[:m], sc.requests.goal[:m], sc.requests.t0[:m])
        arr = S.serving_arrivals(args.serve_rate, m, seed=3)
        ctx.rewind()
        t = time.perf_counter()
        _, scom, sdone = ctx.plan_fcfs(sreq, arrival_s=arr)
        el = time.perf_counter() - t
        lat = (sdone - arr) * 1e3
        out["serving"] = {"rate_req_s": args.serve_rate, "requests": m, "achieved_req_s": m / el,
                          "p50_latency_ms": float(np.percentile(lat, 50)),
                          "p99_latency_ms": float(np.percentile(lat, 99)),
                          "committed": int(scom.sum())}
        out["p50_latency_ms"] = out["serving"]["p50_latency_ms"]
        out["p99_latency_ms"] = out["serving"]["p99_latency_ms"]
        log(f"serving at {args.serve_rate} req/s: p50 {out['p50_latency_ms']:.1f} ms, "
            f"p99 {out['p99_latency_ms']:.1f} ms")
    ctx.close()

    if args.cpu_budget > 0:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
