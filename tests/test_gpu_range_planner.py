"""The range-query planner (256-thread workgroups, four requests per compute
unit, or 512-thread workgroups alone on a compute unit) through the C ABI.

It must give the plans, actions and values of the 1024-thread range query
and of the full sweep bit for bit (the full sweep is compared with the FP64
oracle by the rest of the suite), and the oracle's trajectories directly.
Cases: every request of the 3000-plan, 360-action workload in the bench's
launch configuration; sequential requests with terrain; a dense shell of
parked plans around the track (hundreds of entries within reach and of
candidates per step: several rounds of staging and of the exact test, rows
of four chunks); rows of ~5000 entries (three DMA chunks); the largest
action sets (two actions per thread); a plan exactly at the well radius of
a successor (the FP64 band recheck); short launches with Poisson arrivals
(stop and resume); departures; degenerate requests; a separation radius
above the well radius (OK plans rejected by the commit validation).
"""
import copy
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import classify_trajectory  # noqa: E402

from oracle.oracle import Oracle, action_index  # noqa: E402
from paper_2008_03518_amd import scenario as S  # noqa: E402

pytestmark = pytest.mark.gpu

# (range_query, planner_threads): the full sweep, the 1024-thread range
# query, the range-query planner on 256-thread workgroups (four per CU), on
# 512-thread workgroups (one per CU), and as the context picks per launch
# (planner_threads 0: 512 threads when a launch holds at most one request
# per CU, else 256)
VARIANTS = {"full": (0, 0), "range1024": (1, 1024), "range256": (1, 256), "range512": (1, 512), "auto": (1, 0)}
RANGE_VARIANTS = [v for v in VARIANTS if v != "full"]
RANGE_MAX_HEADS = 64                # headings the range-query planner takes


@pytest.fixture(scope="module")
def fm():
    from paper_2008_03518_amd import fastmdp
    return fastmdp


def _log(msg):
    print(msg, flush=True)


def _variant(sc, name):
    r = copy.deepcopy(sc)
    r.cfg.range_query = VARIANTS[name][0]
    return r


def _ctx(fm, sc, name, **kw):
    return fm.context_for(_variant(sc, name), planner_threads=VARIANTS[name][1], **kw)


def _same(a, b, q=None):
    assert a.status == b.status and a.n_points == b.n_points, q
    assert np.array_equal(a.points(), b.points()) and np.array_equal(a.actions(), b.actions()), q
    assert np.array_equal(a.values(), b.values()), q


def _fcfs_all(fm, sc, reqs=None, arrivals=None, **kw):
    reqs = sc.requests if reqs is None else reqs
    out = {}
    for name in VARIANTS:
        if VARIANTS[name][1] in (256, 512) and sc.cfg.n_head > RANGE_MAX_HEADS:
            continue                        # the range-query planner's sizes are refused (auto: 1024 threads)
        with _ctx(fm, sc, name, **kw) as ctx:
            plans, committed, _ = ctx.plan_fcfs(reqs, arrival_s=arrivals)
            out[name] = (plans, committed, ctx.stats())
        _log(f"  {name}: {out[name][2]}, committed {int(out[name][1].sum())}/{reqs.n}")
    ref_p, ref_c, _ = out["full"]
    for name in RANGE_VARIANTS:
        if name not in out:
            continue
        p, c, _ = out[name]
        assert np.array_equal(c, ref_c), name
        for q, (a, b) in enumerate(zip(ref_p, p)):
            _same(a, b, (name, q))
    return out


def test_fcfs_full_size_bench_launch_config(fm):
    """All 1000 requests at 3000 plans x 360 actions, 1024 slots, 512 steps
    per launch: identical plans, values and acceptances; the range-query
    planner sweeps a small fraction of the pairs."""
    sc = S.large_actions(seed=2, n_plans=3000, n_requests=1000)
    _log("[range planner, 3000 plans, 1000 requests]")
    out = _fcfs_all(fm, sc, max_slots=1024, steps_per_launch=512)
    assert out["range256"][2]["pairs"] < 0.01 * out["full"][2]["pairs"]


def test_fcfs_separation_wider_than_the_well(fm):
    """R_sep above the well radius: an OK trajectory may pass between R_intr
    and R_sep of a plan, and only the planner's commit validation (every
    point within R_sep + 1 m of a plan checked exactly against its row)
    keeps it out of the table.  Every variant's FCFS acceptances equal the
    oracle's plan-then-commit in request order, and some OK plans are
    rejected, so the rejecting branch of the validation runs."""
    sc = S.large_actions(seed=2, n_plans=300, n_requests=60)
    sc.cfg.R_sep = sc.cfg.R_intr + 20.0
    _log(f"[range planner, R_sep {sc.cfg.R_sep} > R_intr {sc.cfg.R_intr}]")
    out = _fcfs_all(fm, sc, max_slots=1024, steps_per_launch=512)
    plans, committed, _ = out["range256"]
    orc = Oracle(sc.cfg, sc.plans)
    kinds, rejected = {}, 0
    for q in range(sc.requests.n):
        o, g, t = sc.requests.origin[q], sc.requests.goal[q], int(sc.requests.t0[q])
        op = orc.plan(o, g, t)
        k = classify_trajectory(plans[q], op, orc, g)["kind"]
        kinds[k] = kinds.get(k, 0) + 1
        if k != "identical":
            break                       # later requests plan against a different table
        ok_o = op.status == fm.OK and orc.commit(op)
        assert bool(committed[q]) == ok_o, q
        rejected += int(op.status == fm.OK and not ok_o)
    _log(f"  oracle kinds {kinds}, OK plans rejected by the validation: {rejected}")
    assert kinds.get("identical", 0) >= 50 and rejected > 0 and committed.sum() > 0


def test_sequential_with_terrain_against_oracle(fm):
    """Paper-scale box with terrain: requests planned and committed one at a
    time by the range-query planner equal the full sweep's and the oracle's."""
    sc = S.paper_scale(seed=1, n_plans=2000, n_requests=12)
    orc = Oracle(sc.cfg, sc.plans, sc.terrain)
    kinds = {}
    with _ctx(fm, sc, "full") as full, _ctx(fm, sc, "range256") as rq, _ctx(fm, sc, "range512") as r5:
        for q in range(sc.requests.n):
            o, g, t = sc.requests.origin[q], sc.requests.goal[q], int(sc.requests.t0[q])
            a = full.plan_request(o, g, t)
            b = rq.plan_request(o, g, t)
            c = r5.plan_request(o, g, t)
            _same(a, b, q)
            _same(a, c, q)
            op = orc.plan(o, g, t)
            k = classify_trajectory(b, op, orc, g)["kind"]
            kinds[k] = kinds.get(k, 0) + 1
            if op.status == fm.OK:
                ok_o = orc.commit(op)
                if k == "identical":
                    assert full.commit_plan(a) == ok_o and rq.commit_plan(b) == ok_o and r5.commit_plan(c) == ok_o
                else:
                    assert (full.commit_points(op.t0, op.xyz) == ok_o and rq.commit_points(op.t0, op.xyz) == ok_o
                            and r5.commit_points(op.t0, op.xyz) == ok_o)
    _log(f"[range planner, terrain] {kinds}")
    assert kinds.get("identical", 0) >= 10


def test_dense_shell_several_rounds(fm):
    """8000 plans parked on a cylinder of radius 165 m around a straight
    track: every step has ~300 entries within reach (two rounds of staging)
    and ~1000 box-test candidates (several rounds of the exact test), rows
    of 8000 entries (four chunks).  No successor on the axis is inside a
    well, so every variant and the oracle fly the axis exactly."""
    cfg = S.cfg_large_actions()
    n = 8000
    cfg.plan_capacity = 8192
    rng = np.random.default_rng(5)
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    pts = np.stack([rng.uniform(1500.0, 4000.0, n), 15000.0 + 165.0 * np.cos(th), 700.0 + 165.0 * np.sin(th)], 1)
    rows = 200
    plans = S.Plans(t0=np.zeros(n, np.int32), length=np.full(n, rows, np.int32),
                    xyz=np.repeat(pts[:, None, :], rows, axis=1).reshape(-1, 3).astype(np.float32))
    o, g = np.array([2000.0, 15000.0, 700.0]), np.array([3500.0, 15000.0, 700.0])
    res = {}
    for name in VARIANTS:
        c = copy.deepcopy(cfg)
        c.range_query = VARIANTS[name][0]
        with fm.Context(c, planner_threads=VARIANTS[name][1]) as ctx:
            ctx.load_plans(plans)
            res[name] = (ctx.plan_request(o, g, 0), ctx.stats())
        _log(f"[shell] {name}: status {res[name][0].status}, {res[name][0].n_points} points, {res[name][1]}")
    for name in RANGE_VARIANTS:
        _same(res["full"][0], res[name][0], name)
    p, st = res["range256"]
    assert p.status == fm.OK and p.n_points - 1 == int(np.ceil(1500.0 / cfg.ell - 1.0))
    assert np.all(p.points()[:, 1] == 15000.0) and np.all(p.points()[:, 2] == 700.0)
    assert st["pairs"] > 256 * cfg.n_actions * (p.n_points - 1)          # > 256 staged per step on average
    orc = Oracle(cfg, plans)
    op = orc.plan(o, g, 0)
    assert classify_trajectory(p, op, orc, g)["kind"] == "identical"


def test_rows_of_several_chunks(fm):
    """5000 known plans: the first rows hold ~5000 entries (three chunks of
    the range-query planner, two tiles of the 1024-thread kernel)."""
    sc = S.large_actions(seed=31, n_plans=5000, n_requests=24)
    assert int(np.sum(sc.plans.t0 == 0)) > 4096
    _log("[range planner, rows of ~5000 entries]")
    _fcfs_all(fm, sc, max_slots=32, steps_per_launch=512)


@pytest.mark.parametrize("n_head,climb,speed", [(34, (-5.0, -2.5, 0.0, 2.5, 5.0), (20.0, 30.0, 40.0)),
                                                 (128, (-5.0, 0.0, 5.0), (30.0,))])
def test_largest_action_sets(fm, n_head, climb, speed):
    """510 actions (two actions on most threads of the range-query planner)
    and 128 headings x 3 climbs (384 actions: more headings than the
    range-query planner takes, so the range query runs on the 1024-thread
    kernel)."""
    sc = S.small(seed=21, n_plans=200, n_requests=10)
    sc.cfg.n_head, sc.cfg.climb, sc.cfg.speed = n_head, climb, speed
    sc.cfg.plan_capacity = 512
    _log(f"[range planner, {sc.cfg.n_actions} actions]")
    _fcfs_all(fm, sc, max_slots=8, steps_per_launch=64)


def test_band_recheck_at_the_well_radius(fm):
    """A plan parked exactly R_intr from the straight action's first
    successor: its FP32 nearest distance lands in the band and is recomputed
    in FP64 (exactly R_intr: outside the well).  Identical to both other
    variants and to the oracle."""
    cfg = S.cfg_large_actions()
    o, g = np.array([1000.0, 5000.0, 300.0]), np.array([9000.0, 5000.0, 300.0])
    step = max(cfg.speed) * cfg.dt
    rows = 50
    x = np.repeat(np.array([[1000.0 + step, 5000.0 + cfg.R_intr, 300.0]], np.float32), rows, axis=0)
    plans = S.Plans(np.zeros(1, np.int32), np.array([rows], np.int32), x)
    straight = action_index(cfg, 0, len(cfg.climb) // 2, len(cfg.speed) - 1)
    res = {}
    for name in VARIANTS:
        c = copy.deepcopy(cfg)
        c.range_query = VARIANTS[name][0]
        with fm.Context(c, planner_threads=VARIANTS[name][1]) as ctx:
            ctx.load_plans(plans)
            res[name] = ctx.plan_request(o, g, 0)
    for name in RANGE_VARIANTS:
        _same(res["full"], res[name], name)
    p = res["range256"]
    assert p.actions()[1] == straight and p.status == fm.OK
    orc = Oracle(cfg, plans)
    op = orc.plan(o, g, 0)
    assert classify_trajectory(p, op, orc, g)["kind"] == "identical"


@pytest.mark.parametrize("steps_per_launch", [1, 16])
def test_short_launches_with_arrivals(fm, steps_per_launch):
    """Launches of 1 and 16 steps and Poisson arrivals on the dense 10 km
    box: every launch stops and resumes requests mid-trajectory."""
    sc = S.small(seed=12, n_plans=150, n_requests=40)
    sc.cfg.plan_capacity = 1024
    arr = S.serving_arrivals(300.0, sc.requests.n, seed=5)
    _log(f"[range planner, {steps_per_launch} steps per launch, arrivals]")
    _fcfs_all(fm, sc, arrivals=arr, max_slots=16, steps_per_launch=steps_per_launch)


def test_departures(fm):
    """Candidate departure rows planned in one launch: every candidate and
    the choice equal the full sweep's."""
    sc = S.small(seed=9, n_plans=200, n_requests=6)
    t0s = [0, 15, 30, 45]
    for name in ("range256", "auto"):                    # four per CU; one per CU on 512 threads
        with _ctx(fm, sc, "full", max_slots=4) as full, _ctx(fm, sc, name, max_slots=4) as rq:
            for q in range(sc.requests.n):
                o, g = sc.requests.origin[q], sc.requests.goal[q]
                a, ca = full.plan_departures(o, g, t0s)
                b, cb = rq.plan_departures(o, g, t0s)
                assert ca == cb, (name, q)
                for x, y in zip(a, b):
                    _same(x, y, (name, q))
                if ca >= 0:
                    assert full.commit_plan(a[ca]) and rq.commit_plan(b[cb])


def test_many_departures_in_one_launch(fm):
    """640 departure rows of one request in one launch: more workgroups than
    two per CU, so the range-query planner runs four per CU (at most 128
    VGPRs); every candidate equals the full sweep's and the per-launch
    choice's."""
    sc = S.large_actions(seed=2, n_plans=3000, n_requests=1)
    t0s = np.arange(640, dtype=np.int32)
    o, g = sc.requests.origin[0], sc.requests.goal[0]
    res = {}
    for name in ("full", "range256", "auto"):
        with _ctx(fm, sc, name, max_slots=640) as ctx:
            res[name] = ctx.plan_departures(o, g, t0s)
    for name in ("range256", "auto"):
        assert res[name][1] == res["full"][1], name
        for k, (x, y) in enumerate(zip(res["full"][0], res[name][0])):
            _same(x, y, (name, k))
    _log(f"[departures] chosen {res['full'][1]}")


def test_degenerate_requests(fm):
    """Capture at the origin, a goal straight above the origin, an origin
    inside a plan's separation radius, an origin outside the box."""
    sc = S.small(seed=22, n_plans=100, n_requests=1)
    o = np.array([300.0, 9700.0, 500.0])
    p0 = sc.plans.xyz[0].astype(np.float64)
    cases = [(o, o + [5.0, -5.0, 3.0], 0), (o, o + [0.0, 0.0, 300.0], 0),
             (p0 + [20.0, 0.0, 0.0], np.array([5000.0, 5000.0, 500.0]), int(sc.plans.t0[0])),
             (np.array([-50.0, 500.0, 500.0]), np.array([5000.0, 5000.0, 500.0]), 0)]
    with _ctx(fm, sc, "full") as full, _ctx(fm, sc, "range256") as rq, _ctx(fm, sc, "range512") as r5:
        for k, (a, g, t) in enumerate(cases):
            x, y, z = full.plan_request(a, g, t), rq.plan_request(a, g, t), r5.plan_request(a, g, t)
            _log(f"[degenerate {k}] status {x.status}, {x.n_points} points")
            _same(x, y, k)
            _same(x, z, k)


@pytest.mark.parametrize("threads", [256, 512])
def test_config_rejects_range_threads_without_range_query(fm, threads):
    cfg = S.cfg_small()
    with pytest.raises(fm.FastMDPError):
        fm.Context(cfg, planner_threads=threads)
    cfg.range_query, cfg.lookahead = 1, 2
    with pytest.raises(fm.FastMDPError):
        fm.Context(cfg, planner_threads=threads)
    cfg.lookahead = 1
    with fm.Context(cfg, planner_threads=threads) as ctx:
        assert ctx.n_plans == 0
    cfg.n_head = 65                                          # beyond the range-query planner's headings
    with pytest.raises(fm.FastMDPError):
        fm.Context(cfg, planner_threads=threads)
    cfg.n_head = 24
    with pytest.raises(fm.FastMDPError):
        fm.Context(cfg, planner_threads=384)
