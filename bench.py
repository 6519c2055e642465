"""Benchmark: first-come-first-served plan requests per second at 3000 known plans.

Workload: 30 x 30 x 1.5 km airspace, 3000 known straight constant-speed plans,
360 actions (24 headings x 5 climb rates x 3 speeds), dt = 0.5 s, up to 3600
steps per request, 1000 FCFS requests (seeded synthetic inputs).  One bench
step plans and accepts all 1000 requests first-come-first-served with
concurrent slots, starting from the 3000-plan table (rewound between steps,
outside the timed region), including the host transfers of requests and
plans.  Timed legs, all committing identical plans:
  * the headline: the exact full sweep with the range query (each step
    sweeps only the plans within reach of the state, Sec. VII) on the
    range-query planner (256-thread workgroups, four requests per compute
    unit, or 512-thread workgroups, one per compute unit, for a launch that
    holds no more requests than compute units), with a memory-side roofline (row bytes streamed); beside it the
    same on the 1024-thread kernel (one request per compute unit);
  * the plain full sweep (every plan, every action), with its roofline
    against the FP32 vector peak;
  * the learned action proposal (trained beforehand, untimed, with the
    library's own kernels on 1M tuples from the plain planner on scenarios of
    seeds 100-109) with its exact certificate, alone and with the range
    query; ablations: goal ranking without a network, an untrained network.
Also: the planners' steady-state step rate without the FCFS order (one
launch planning 1024 departure rows of one request), p50/p99 latency of
Poisson-arrival serving passes, serving on a
20000-plan table, co-simulated batches (the paper's batch-size experiment),
lookahead windows, and the FP64 CPU oracle timed on a bounded sample.
Printed: one JSON line.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak
FP64_VECTOR_PEAK_TFLOPS = 78.6      # MI355X published FP64 vector peak
HBM_PEAK_GBPS = 8000.0              # MI355X published HBM3E bandwidth
FLOPS_PER_PAIR = 8                  # 3 sub + 3 mul + 2 add for one squared distance
ROW_ENTRY_BYTES = 16                # one table row entry read by a 1024-thread step: x, y, z, visibility
RANGE_ENTRY_BYTES = 8               # one row entry read by the range-query planner's box test: x, y

# HBM bytes per planner launch on this workload, from the FETCH_SIZE /
# WRITE_SIZE counter runs in profiles/planner_traffic__*.md (calibrated on a
# copy of known size), valid only for the kernel sources they were taken on.
TRAFFIC_SOURCES = ("planner.hip", "range.hip", "planner.h", "score.h", "proposal.h", "wave.h")
TRAFFIC_SHA256 = "23f389133fa73a82ee227b98009cf74962fa19b1ade96c32f7a36e31e60fd4cc"
# VALU counters per planner launch of an FCFS pass (profiles/planner_valu__*.md),
# valid for the same sources: the share of SIMD cycles issuing VALU work and
# the FLOP the hardware counts (FP32 for the sweep, FP64 for the range-query
# planner's valuation), beside the algorithmic rooflines
VALU_COUNTERS = {"full_sweep": {"valu_busy": 0.582, "hw_fp32_flops_per_launch": 4.64e10},
                 "range_query": {"valu_busy": 0.169, "hw_fp64_flops_per_launch": 2.1e09}}
TRAFFIC_BYTES_PER_LAUNCH = {"range_query": 5.03e08, "range_query_1024": 3.81e08, "proposal": 7.2e08, "full_sweep": 3.57e08}


def _sources_match() -> bool:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2008_03518_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest() == TRAFFIC_SHA256


def _counters(leg: str, avg_launch_ms: float):
    """The leg's VALU counter figures, or None when the sources changed."""
    c = VALU_COUNTERS.get(leg)
    if c is None or not _sources_match():
        return None
    out = {"valu_busy": c["valu_busy"]}
    if "hw_fp32_flops_per_launch" in c:
        out["hw_fp32_tflops"] = c["hw_fp32_flops_per_launch"] / (avg_launch_ms * 1e-3) / 1e12
        out["hw_fp32_frac"] = out["hw_fp32_tflops"] / FP32_VECTOR_PEAK_TFLOPS
    if "hw_fp64_flops_per_launch" in c:
        out["hw_fp64_tflops"] = c["hw_fp64_flops_per_launch"] / (avg_launch_ms * 1e-3) / 1e12
        out["hw_fp64_frac"] = out["hw_fp64_tflops"] / FP64_VECTOR_PEAK_TFLOPS
    return out


def _traffic(leg: str):
    if leg not in TRAFFIC_BYTES_PER_LAUNCH:
        return None
    return TRAFFIC_BYTES_PER_LAUNCH[leg] if _sources_match() else None


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
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "build": "gcc -O3 -fopenmp, no fast-math",
            "sample": f"first {n} of the {sc.requests.n} FCFS requests (plan + commit, FP64, literal per-peak "
                      f"maximum, OpenMP over the actions of a step), {el:.1f} s"}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _leg(ctx, reqs, mode, net, k, steps, warmup, name, refresh=1):
    """Warmup + timed FCFS passes with one proposal mode; returns a dict."""
    from paper_2008_03518_amd import fastmdp as fm
    ctx.set_proposal(mode, k, net, refresh)

    bufs = [fm.Plan(ctx.capacity) for _ in range(reqs.n)]     # output buffers, reused by every pass

    def one():
        ctx.rewind()
        gc.collect()                   # no Python collection inside the timed region
        gc.disable()
        try:
            t = time.perf_counter()
            plans, committed, done = ctx.plan_fcfs(reqs, out=bufs)
            el = time.perf_counter() - t
        finally:
            gc.enable()
        return el, plans, committed, ctx.stats(), ctx.proposal_stats()

    for w in range(warmup):
        el, *_ = one()
        log(f"{name} warmup {w}: {el * 1e3:.1f} ms")
    r = dict(times=[], pairs=0, kms=0.0, launches=0, steps=0, resumes=0, cert=0, fallback=0, entries=0)
    for i in range(steps):
        el, plans, committed, st, ps = one()
        r["times"].append(el)
        for a, b in (("pairs", "pairs"), ("kms", "kernel_ms"), ("launches", "launches"), ("steps", "steps"),
                     ("resumes", "resumes"), ("entries", "row_entries")):
            r[a] += st[b]
        r["cert"] += ps["certified"]
        r["fallback"] += ps["fallbacks"]
        log(f"{name} step {i}: {el * 1e3:.1f} ms, committed {int(committed.sum())}/{reqs.n}, pairs "
            f"{st['pairs']:.3e}, planner {st['kernel_ms']:.1f} ms in {st['launches']} launches, resumes "
            f"{st['resumes']}" + (f", certified {ps['certified']}/{ps['certified'] + ps['fallbacks']} steps"
                                  if mode != fm.PROPOSE_NONE else ""))
    r["plans"], r["committed"] = plans, committed
    r["value"] = steps * reqs.n / sum(r["times"])
    r["ms_per_step"] = sum(r["times"]) / steps * 1e3
    return r


def _roofline(r, leg):
    achieved = FLOPS_PER_PAIR * r["pairs"] / (r["kms"] * 1e-3) / 1e12
    return {
        "bound": "alu",
        "achieved": achieved,
        "peak": FP32_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
        "traffic": _traffic(leg),
        "traffic_unit": "HBM bytes per launch",
        "kernel": "planner_kernel",
        "avg_launch_ms": r["kms"] / max(r["launches"], 1),
        "flops_per_launch": FLOPS_PER_PAIR * r["pairs"] / max(r["launches"], 1),
        "counters": _counters(leg, r["kms"] / max(r["launches"], 1)),
    }


def _roofline_rows(r, leg, entry_bytes=RANGE_ENTRY_BYTES):
    """Memory-side roofline of a leg that sweeps few pairs: the table rows it
    streams per planner-kernel second (entry_bytes per row entry per step:
    x and y for the range-query planner's box test, x, y, z and visibility
    for the 1024-thread kernel), against the HBM peak."""
    achieved = entry_bytes * r["entries"] / (r["kms"] * 1e-3) / 1e9
    return {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBPS,
        "traffic": _traffic(leg),
        "traffic_unit": "HBM bytes per launch",
        "kernel": "planner_kernel",
        "avg_launch_ms": r["kms"] / max(r["launches"], 1),
        "bytes_per_launch": entry_bytes * r["entries"] / max(r["launches"], 1),
        "counters": _counters(leg, r["kms"] / max(r["launches"], 1)),
    }


def _calibrate_copy():
    """A copy of known size for scaling the FETCH_SIZE / WRITE_SIZE counters
    to bytes: 65536 rows of 4096 B gathered by an int64 index, three times
    (256 MiB read plus the 512 KiB index, 256 MiB written, per dispatch)."""
    from paper_2008_03518_amd import fastmdp as fm
    n, row = 65536, 4096
    src = fm.DeviceArray((n, row // 4), np.float32)
    idx = fm.DeviceArray.from_host(np.arange(n, dtype=np.int64))
    for _ in range(3):
        src.gather(idx).free()
    print(json.dumps({"calibration_copy": {"dispatches": 3, "read_bytes": n * row + n * 8,
                                           "written_bytes": n * row}}), flush=True)


def serving_stats(arrival_s, done_s) -> dict:
    """Latency and queue statistics of one open-loop serving pass.

    Latency of a request = its acceptance time minus its scheduled arrival.
    Queue depth = requests in the system (arrived, not yet accepted) seen by
    each arrival, itself included: arrival i finds i + 1 arrivals so far, less
    those already accepted (acceptances never precede their arrival).
    """
    arr = np.asarray(arrival_s, dtype=np.float64)
    done = np.asarray(done_s, dtype=np.float64)
    lat = (done - arr) * 1e3
    gone = np.searchsorted(np.sort(done), arr, side="right")
    depth = np.arange(1, arr.size + 1) - gone
    return {"p50_latency_ms": float(np.percentile(lat, 50)),
            "p99_latency_ms": float(np.percentile(lat, 99)),
            "mean_queue_depth": float(depth.mean()),
            "max_queue_depth": int(depth.max())}


def _serve(ctx, sc, S, rate, m):
    """One Poisson-arrival serving pass of m requests at ``rate`` req/s from
    the rewound table, with the proposal the context has selected."""
    sreq = S.Requests(sc.requests.ident[:m], sc.requests.origin[:m], sc.requests.goal[:m], sc.requests.t0[:m])
    arr = S.serving_arrivals(rate, m, seed=3)
    ctx.rewind()
    t = time.perf_counter()
    _, scom, sdone = ctx.plan_fcfs(sreq, arrival_s=arr)
    el = time.perf_counter() - t
    st = ctx.stats()
    out = {"rate_req_s": rate, "requests": m, "achieved_req_s": m / el}
    out.update(serving_stats(arr, sdone))
    out.update({"committed": int(scom.sum()), "resumes_per_request": st["resumes"] / m})
    return out


def _sequential(ctx, reqs, n, full):
    """The first n requests planned and committed one at a time (one
    workgroup each) with the full sweep, from the rewound table; their plans
    must equal the concurrent pass's."""
    from paper_2008_03518_amd import fastmdp as fm
    ctx.set_proposal(fm.PROPOSE_NONE, 1, None, 1)
    ctx.rewind()
    plans, committed = [], []
    t = time.perf_counter()
    for q in range(n):
        p = ctx.plan_request(reqs.origin[q], reqs.goal[q], int(reqs.t0[q]), int(reqs.ident[q]))
        committed.append(bool(ctx.commit_plan(p)) if p.status == fm.OK else False)
        plans.append(p)
    el = time.perf_counter() - t
    same = _same_plans(plans, full["plans"][:n]) and committed == [bool(c) for c in full["committed"][:n]]
    return {"requests": n, "value": n / el, "ms_per_request": el / n * 1e3,
            "identical_to_concurrent_pass": bool(same)}


def _same_plans(a, b) -> bool:
    for p, q in zip(a, b):
        n = p.n_points
        if p.status != q.status or n != q.n_points:
            return False
        if not (np.array_equal(p.xyz[:n], q.xyz[:n]) and np.array_equal(p.action[:n], q.action[:n])
                and np.array_equal(p.value[:n], q.value[:n])):
            return False
    return len(a) == len(b)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plans", type=int, default=3000)
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--slots", type=int, default=1024)
    ap.add_argument("--steps-per-launch", type=int, default=512)
    ap.add_argument("--planner-threads", type=int, default=0, help="planning workgroup size: 0 or 1024")
    ap.add_argument("--top-k", type=int, default=8)
    ap.add_argument("--refresh", type=int, default=64,
                    help="steps between re-rankings of the proposal (a fallback also re-ranks)")
    ap.add_argument("--train-tuples", type=int, default=1000000)
    ap.add_argument("--train-epochs", type=int, default=4)
    ap.add_argument("--params", default="", help="load trained proposal parameters (.npz) instead of training")
    ap.add_argument("--save-params", default="", help="write the trained parameters (.npz)")
    ap.add_argument("--ablations", type=int, default=1, help="also time goal-ranked and untrained proposals")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrivals [req/s]; 0 disables")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-rates", default="",
                    help="also serve at each of these comma-separated rates [req/s], "
                         "min(--serve-requests, rate * --serve-seconds) arrivals each")
    ap.add_argument("--serve-seconds", type=float, default=20.0)
    ap.add_argument("--serve-large", type=int, default=20000,
                    help="also serve --serve-requests Poisson arrivals at --serve-rate on a table preloaded with "
                         "this many known plans, with the range query; 0 disables")
    ap.add_argument("--growth", type=int, default=0,
                    help="also serve this many Poisson arrivals at --serve-rate from the known-plan table "
                         "as it grows by every accepted plan (a table sized for all of them); 0 disables")
    ap.add_argument("--sequential", type=int, default=0,
                    help="also plan the first N requests one at a time (plan, then commit) with the full "
                         "sweep and compare with the concurrent pass; 0 disables")
    ap.add_argument("--batch-sizes", default="1,5,10,20",
                    help="also plan co-simulated batches of these sizes among 100 known plans in the 10 km box "
                         "(the paper's batch-size experiment); empty disables")
    ap.add_argument("--lookahead", default="2,10",
                    help="also time one FCFS pass with each of these comma-separated scoring windows W "
                         "(full sweep); empty disables")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work; 0 disables")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the copy of known size that scales the HBM byte counters, then exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.calibrate_copy:
        _calibrate_copy()
        return

    from paper_2008_03518_amd import fastmdp as fm
    from paper_2008_03518_amd import proposal as PR
    from paper_2008_03518_amd import scenario as S

    sc = S.large_actions(seed=args.seed, n_plans=args.plans, n_requests=max(args.requests, args.serve_requests))
    cfg = sc.cfg
    A = cfg.n_actions
    reqs = S.Requests(sc.requests.ident[:args.requests], sc.requests.origin[:args.requests],
                      sc.requests.goal[:args.requests], sc.requests.t0[:args.requests])
    log(f"workload: {sc.plans.n} plans, {A} actions, {reqs.n} requests, slots {args.slots}")

    # proposal network: trained (untimed) on the plain planner's choices, seeds 100-109
    train_info = {}
    net = fm.Mlp(A)
    if args.params:
        z = np.load(args.params)
        net.set_params({k: z[k] for k in ("W1", "b1", "W2", "b2", "W3", "b3")})
        train_info = {"loaded": os.path.basename(args.params)}
    else:
        t = time.perf_counter()
        X, y = PR.generate_dataset(range(100, 110), args.train_tuples, n_plans=args.plans, n_requests=1000,
                                   max_slots=args.slots, log=log)
        t_data = time.perf_counter() - t
        net.set_params(PR.init_params(A, seed=0))
        t = time.perf_counter()
        losses = PR.train(net, X, y, epochs=args.train_epochs, batch=4096, lr=2e-3, log=log)
        t_train = time.perf_counter() - t
        train_info = {"tuples": len(X), "seeds": "100-109", "epochs": args.train_epochs, "batch": 4096,
                      "loss_first_epoch": losses[0], "loss_last_epoch": losses[-1],
                      "data_s": t_data, "train_s": t_train}
        del X, y
        if args.save_params:
            np.savez(args.save_params, **net.get_params())

    ctx = fm.context_for(sc, max_slots=args.slots, steps_per_launch=args.steps_per_launch,
                         planner_threads=args.planner_threads)
    ctx.snapshot()
    full = _leg(ctx, reqs, fm.PROPOSE_NONE, None, args.top_k, args.steps, args.warmup, "full sweep")
    prop = _leg(ctx, reqs, fm.PROPOSE_MLP, net, args.top_k, args.steps, args.warmup, "proposal", args.refresh)
    prop_same = _same_plans(prop["plans"], full["plans"]) and np.array_equal(prop["committed"], full["committed"])
    log(f"proposal plans identical to the full sweep: {prop_same}")

    # the headline path: the full sweep with the range query (the same plans)
    import copy
    rsc = copy.deepcopy(sc)
    rsc.cfg.range_query = 1
    rctx = fm.context_for(rsc, max_slots=args.slots, steps_per_launch=args.steps_per_launch,
                          planner_threads=args.planner_threads)
    rctx.snapshot()
    rq = _leg(rctx, reqs, fm.PROPOSE_NONE, None, args.top_k, args.steps, args.warmup, "range query")
    identical = _same_plans(rq["plans"], full["plans"]) and np.array_equal(rq["committed"], full["committed"])
    log(f"range query: {rq['value']:.0f} req/s, plans identical to the full sweep: {identical}")
    status = np.array([p.status for p in rq["plans"]])

    def cert_rate(r):
        return r["cert"] / max(r["cert"] + r["fallback"], 1)

    out = {
        "metric": "FCFS plan requests/sec at 3000 known plans",
        "value": rq["value"],
        "unit": "req/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rq["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{sc.plans.n} known plans, {A} actions (24 headings x 5 climbs x 3 speeds), "
                        f"dt 0.5 s, {reqs.n} FCFS requests, 30x30x1.5 km; exact full sweep with the range query "
                        f"(only plans within reach of the state are swept; plans identical to the full sweep), "
                        f"range-query planner: 256-thread workgroups, four requests per compute unit "
                        f"(512-thread, one per compute unit, in launches of at most one request per CU)",
            "known_plans": sc.plans.n, "actions": A, "requests_per_step": reqs.n,
            "slots": args.slots, "steps_per_launch": args.steps_per_launch,
            "planner_threads": args.planner_threads,
        },
        "identical_to_full_sweep": bool(identical),
        "planner_steps": rq["steps"],
        "resumes": rq["resumes"],
        "committed_per_step": int(rq["committed"].sum()),
        "status_counts": {S.STATUS_NAMES[int(k)]: int((status == k).sum()) for k in np.unique(status)},
        "pairs_swept_per_step": rq["pairs"] / len(rq["times"]),
        "pairs_of_full_sweep_per_step": full["pairs"] / len(full["times"]),
        "roofline": _roofline_rows(rq, "range_query"),
        "full_sweep": {
            "value": full["value"], "ms_per_step": full["ms_per_step"], "planner_steps": full["steps"],
            "pair_evals_per_s": full["pairs"] / (full["kms"] * 1e-3), "resumes": full["resumes"],
            "roofline": _roofline(full, "full_sweep"),
        },
        "proposal": {
            "value": prop["value"], "ms_per_step": prop["ms_per_step"], "identical_to_full_sweep": bool(prop_same),
            "top_k": args.top_k, "refresh": args.refresh, "certified_step_rate": cert_rate(prop),
            "pair_evals_per_s": prop["pairs"] / (prop["kms"] * 1e-3), "resumes": prop["resumes"],
            "roofline": _roofline(prop, "proposal"),
        },
        "training": train_info,
    }
    # the trained proposal with the range query
    rp = _leg(rctx, reqs, fm.PROPOSE_MLP, net, args.top_k, args.steps, args.warmup, "proposal + range query",
              args.refresh)
    same = _same_plans(rp["plans"], full["plans"]) and np.array_equal(rp["committed"], full["committed"])
    out["proposal_with_range_query"] = {
        "value": rp["value"], "ms_per_step": rp["ms_per_step"], "identical_to_full_sweep": bool(same),
        "certified_step_rate": cert_rate(rp), "pairs_swept_per_step": rp["pairs"] / len(rp["times"])}
    log(f"proposal + range query: {rp['value']:.0f} req/s, identical to the full sweep: {same}")

    # the range query on the 1024-thread kernel (one request per compute unit)
    r1 = fm.context_for(rsc, max_slots=args.slots, steps_per_launch=args.steps_per_launch, planner_threads=1024)
    r1.snapshot()
    rq1 = _leg(r1, reqs, fm.PROPOSE_NONE, None, args.top_k, args.steps, args.warmup, "range query, 1024 threads")
    out["range_query_1024_threads"] = {
        "value": rq1["value"], "ms_per_step": rq1["ms_per_step"], "planner_steps": rq1["steps"],
        "resumes": rq1["resumes"],
        "identical_to_full_sweep": bool(_same_plans(rq1["plans"], full["plans"])
                                        and np.array_equal(rq1["committed"], full["committed"])),
        "roofline": _roofline_rows(rq1, "range_query_1024", ROW_ENTRY_BYTES)}
    # the planners alone, without the FCFS order: one launch planning request
    # 3 from 1024 departure rows at once (every CU busy), planner steps per us
    out["kernel_steady_state"] = {}
    for name, kctx in (("range_query_planner", rctx), ("range_query_1024_threads", r1), ("full_sweep", ctx)):
        kctx.set_proposal(fm.PROPOSE_NONE, 1, None, 1)
        kctx.rewind()
        o3, g3 = sc.requests.origin[3], sc.requests.goal[3]
        kctx.plan_departures(o3, g3, list(range(min(1024, args.slots))))
        kctx.plan_departures(o3, g3, list(range(min(1024, args.slots))))
        kst = kctx.stats()
        out["kernel_steady_state"][name] = {"plans": min(1024, args.slots), "planner_ms": kst["kernel_ms"],
                                            "steps": kst["steps"],
                                            "steps_per_us": kst["steps"] / (kst["kernel_ms"] * 1e3)}
        if name == "full_sweep":
            out["kernel_steady_state"][name]["fp32_frac"] = (FLOPS_PER_PAIR * kst["pairs"] / (kst["kernel_ms"] * 1e-3)
                                                             / 1e12 / FP32_VECTOR_PEAK_TFLOPS)
        log(f"steady state {name}: {kst['steps']} steps in {kst['kernel_ms']:.2f} ms")
        kctx.rewind()
    r1.close()

    if args.ablations:
        goal = _leg(ctx, reqs, fm.PROPOSE_GOAL, None, args.top_k, args.steps, 0, "goal-ranked", args.refresh)
        untrained = fm.Mlp(A)
        untrained.set_params(PR.init_params(A, seed=0))
        unt = _leg(ctx, reqs, fm.PROPOSE_MLP, untrained, args.top_k, 1, 0, "untrained", args.refresh)
        out["ablations"] = {
            name: {"value": r["value"], "certified_step_rate": cert_rate(r),
                   "identical_to_full_sweep": bool(_same_plans(r["plans"], full["plans"])),
                   "pair_evals": r["pairs"] / len(r["times"])}
            for name, r in (("goal_ranked_no_network", goal), ("untrained_network", unt))}
        out["ablations"]["trained_network"] = {"value": prop["value"], "certified_step_rate": cert_rate(prop),
                                               "pair_evals": prop["pairs"] / len(prop["times"])}
        untrained.close()

    sizes = [int(x) for x in args.batch_sizes.split(",") if x.strip()]
    if sizes:
        out["batch"] = []
        bsc = S.small(seed=7, n_plans=100, n_requests=max(sizes))
        with fm.context_for(bsc, max_slots=max(sizes)) as bctx:
            for nb in sizes:
                breq = S.Requests(bsc.requests.ident[:nb], bsc.requests.origin[:nb], bsc.requests.goal[:nb],
                                  bsc.requests.t0[:nb])
                bctx.plan_batch(breq)                               # warm-up
                t = time.perf_counter()
                bplans = bctx.plan_batch(breq)
                el = time.perf_counter() - t
                bst = bctx.stats()
                steps = max(p.n_points - 1 for p in bplans)
                bst_status = np.array([p.status for p in bplans])
                out["batch"].append({
                    "batch": nb, "lockstep_steps": steps, "steps_per_s": steps / el,
                    "aircraft_steps_per_s": bst["steps"] / el, "ms": el * 1e3, "gpu_ms": bst["kernel_ms"],
                    "status_counts": {S.STATUS_NAMES[int(k)]: int((bst_status == k).sum())
                                      for k in np.unique(bst_status)}})
                log(f"batch {nb}: {steps} lockstep steps in {el * 1e3:.1f} ms ({steps / el:.0f} steps/s, "
                    f"{bst['steps'] / el:.0f} aircraft-steps/s)")

    windows = [int(x) for x in args.lookahead.split(",") if x.strip() and int(x) > 1]
    if windows:
        import copy
        out["lookahead"] = []
        for W in windows:
            lsc = copy.deepcopy(sc)
            lsc.cfg.lookahead = W
            lctx = fm.context_for(lsc, max_slots=args.slots, steps_per_launch=args.steps_per_launch,
                                  planner_threads=args.planner_threads)
            lctx.snapshot()
            name = f"window {W}"
            r = _leg(lctx, reqs, fm.PROPOSE_NONE, None, args.top_k, 1, 1, name)
            lst = np.array([p.status for p in r["plans"]])
            out["lookahead"].append({
                "window": W, "value": r["value"], "ms_per_step": r["ms_per_step"],
                "planner_steps": r["steps"], "pair_evals_per_s": r["pairs"] / (r["kms"] * 1e-3),
                "resumes": r["resumes"], "committed_per_step": int(r["committed"].sum()),
                "status_counts": {S.STATUS_NAMES[int(k)]: int((lst == k).sum()) for k in np.unique(lst)},
                "roofline": _roofline(r, "lookahead"),
            })
            log(f"{name}: {r['value']:.0f} req/s, committed {int(r['committed'].sum())}/{reqs.n}, "
                f"status {out['lookahead'][-1]['status_counts']}")
            lctx.close()

    if args.sequential > 0:
        out["sequential_full_sweep"] = _sequential(ctx, reqs, min(args.sequential, reqs.n), full)
        q = out["sequential_full_sweep"]
        log(f"sequential full sweep, {q['requests']} requests: {q['value']:.1f} req/s, "
            f"identical to the concurrent pass: {q['identical_to_concurrent_pass']}")

    if args.serve_rate > 0 or args.serve_rates:
        rctx.set_proposal(fm.PROPOSE_NONE, 1, None, 1)
        ctx.set_proposal(fm.PROPOSE_MLP, args.top_k, net, args.refresh)
    if args.serve_rate > 0:
        out["serving"] = _serve(rctx, rsc, S, args.serve_rate, args.serve_requests)
        out["serving"]["method"] = "full sweep with the range query"
        out["p50_latency_ms"] = out["serving"]["p50_latency_ms"]
        out["p99_latency_ms"] = out["serving"]["p99_latency_ms"]
        log(f"serving at {args.serve_rate} req/s: p50 {out['p50_latency_ms']:.1f} ms, "
            f"p99 {out['p99_latency_ms']:.1f} ms")
        out["serving_proposal"] = _serve(ctx, sc, S, args.serve_rate, args.serve_requests)
        out["serving_proposal"]["method"] = "trained proposal"
        log(f"serving with the trained proposal: p50 {out['serving_proposal']['p50_latency_ms']:.1f} ms, "
            f"p99 {out['serving_proposal']['p99_latency_ms']:.1f} ms")
    if args.serve_rates:
        out["serving_sweep"] = []
        for rate in (float(x) for x in args.serve_rates.split(",")):
            m = max(1, min(args.serve_requests, int(rate * args.serve_seconds)))
            r = _serve(rctx, rsc, S, rate, m)
            out["serving_sweep"].append(r)
            log(f"serving at {rate:g} req/s ({m} requests): achieved {r['achieved_req_s']:.1f} req/s, "
                f"p50 {r['p50_latency_ms']:.1f} ms, p99 {r['p99_latency_ms']:.1f} ms, "
                f"queue mean {r['mean_queue_depth']:.2f} max {r['max_queue_depth']}, "
                f"resumes/request {r['resumes_per_request']:.3f}")
    if args.serve_large > 0 and args.serve_rate > 0:
        t = time.perf_counter()
        big = S.large_actions(seed=args.seed, n_plans=args.serve_large, n_requests=args.serve_requests)
        big.cfg.range_query = 1
        bctx = fm.context_for(big, max_slots=args.slots, steps_per_launch=args.steps_per_launch,
                              planner_threads=args.planner_threads)
        bctx.snapshot()
        log(f"serving on {big.plans.n} known plans (drawn and loaded in {time.perf_counter() - t:.1f} s), "
            f"{args.serve_requests} arrivals at {args.serve_rate:g} req/s, range query ...")
        r = _serve(bctx, big, S, args.serve_rate, args.serve_requests)
        r["known_plans"] = int(big.plans.n)
        r["method"] = "full sweep with the range query"
        out["serving_large"] = r
        log(f"serving on {big.plans.n} plans: achieved {r['achieved_req_s']:.1f} req/s, p50 "
            f"{r['p50_latency_ms']:.1f} ms, p99 {r['p99_latency_ms']:.1f} ms, queue mean {r['mean_queue_depth']:.2f} "
            f"max {r['max_queue_depth']}, committed {r['committed']}")
        bctx.close()
        del big

    if args.growth > 0:
        g = S.large_actions(seed=args.seed, n_plans=args.plans, n_requests=args.growth)
        g.cfg.range_query = 1
        gctx = fm.context_for(g, max_slots=args.slots, steps_per_launch=args.steps_per_launch,
                              planner_threads=args.planner_threads)
        gctx.snapshot()
        rate = args.serve_rate if args.serve_rate > 0 else 200.0
        log(f"growth: {args.growth} arrivals at {rate:g} req/s from {g.plans.n} plans ...")
        r = _serve(gctx, g, S, rate, args.growth)
        r["plans_at_start"] = int(g.plans.n)
        r["plans_at_end"] = int(gctx.n_plans)
        out["growth"] = r
        log(f"growth: {r['plans_at_start']} -> {r['plans_at_end']} plans, achieved {r['achieved_req_s']:.1f} req/s, "
            f"p50 {r['p50_latency_ms']:.1f} ms, p99 {r['p99_latency_ms']:.1f} ms, queue mean "
            f"{r['mean_queue_depth']:.2f} max {r['max_queue_depth']}, resumes/request {r['resumes_per_request']:.3f}")
        gctx.close()
    ctx.close()
    rctx.close()
    net.close()

    if args.cpu_budget > 0:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
