"""The lookahead window on the GPU against the FP64 oracle, through the C ABI.

Action a held for w = 1..W steps reaches s + w * Delta_a at row t + w; its
value is the largest value along the window (Alg. 1's one- and ten-step
forward projections; "Forward project" and "Compute value" kernels).
Cases: the hand case of the oracle's pin (a plan appearing at row 8),
single steps near plans, trajectories, the concurrent engine against
sequential planning bit for bit (all at once and with Poisson arrivals),
and the 3000-plan, 360-action workload.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import classify_trajectory, compare_eval  # noqa: E402

from oracle.oracle import Oracle, action_index  # noqa: E402
from paper_2008_03518_amd import scenario as S  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fm():
    from paper_2008_03518_amd import fastmdp
    return fastmdp


def _log(msg):
    print(msg, flush=True)


def _with_window(sc, W):
    sc.cfg.lookahead = W
    return sc


def _near_plan_states(sc, n, seed):
    rng = np.random.default_rng(seed)
    off = sc.plans.offsets()
    out = []
    while len(out) < n:
        j = int(rng.integers(sc.plans.n))
        L = int(sc.plans.length[j])
        if L < 14:
            continue
        k = int(rng.integers(0, L - 12))
        p = sc.plans.xyz[off[j] + k + 3].astype(np.float64)
        s = p + rng.uniform(-250, 250, 3) * np.array([1.0, 1.0, 0.4])
        lo, hi = np.array(sc.cfg.box_min), np.array(sc.cfg.box_max)
        s = np.clip(s, lo + 1.0, hi - 1.0)
        g = np.array([rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]), rng.uniform(100, 900)])
        out.append((s, g, int(sc.plans.t0[j]) + k))
    return out


def test_window_hand_case(fm):
    """The oracle pin's geometry: a plan at (1400, 5000, 300) from row 8 on
    makes the straight action's value the goal term at w = 7, 0.99^43."""
    cfg = S.cfg_small()
    cfg.lookahead = 10
    rows = 40
    x = np.repeat(np.array([[9000.0, 9000.0, 900.0]], np.float32), rows, axis=0)
    x[8:] = [1400.0, 5000.0, 300.0]
    plans = S.Plans(np.zeros(1, np.int32), np.array([rows], np.int32), x)
    o, g = np.array([1000.0, 5000.0, 300.0]), np.array([3000.0, 5000.0, 300.0])
    straight = action_index(cfg, 0, 1, 2)
    with fm.Context(cfg) as ctx:
        ctx.load_plans(plans)
        r = ctx.eval_step(o, g, 0)
    assert abs(r["V"][straight] - 0.649102628368402432993856004081) <= 1e-5 * 0.65
    compare_eval(r, Oracle(cfg, plans).eval_step(o, g, 0))


@pytest.mark.parametrize("W", [2, 10])
def test_window_eval_near_plans(fm, W):
    sc = _with_window(S.small(seed=0, n_plans=200, n_requests=1), W)
    orc = Oracle(sc.cfg, sc.plans)
    n_cmp = n_in = 0
    with fm.context_for(sc) as ctx:
        for s, g, t in _near_plan_states(sc, 60, 13):
            o = orc.eval_step(s, g, t)
            n, _, _, _, _ = compare_eval(ctx.eval_step(s, g, t), o)
            n_cmp += n
            n_in += int(np.sum(o["I"] > 0))
    _log(f"[window {W}] compared {n_cmp} actions, {n_in} scored inside a well")
    assert n_in > 50


def test_window_trajectories(fm):
    """Requests planned one after another with commits, W = 10, against the
    oracle planning the same requests on its own table."""
    sc = _with_window(S.small(seed=4, n_plans=200, n_requests=8), 10)
    orc = Oracle(sc.cfg, sc.plans)
    kinds = {}
    with fm.context_for(sc) as ctx:
        for q in range(sc.requests.n):
            goal = sc.requests.goal[q]
            op = orc.plan(sc.requests.origin[q], goal, 0)
            gp = ctx.plan_request(sc.requests.origin[q], goal, 0)
            r = classify_trajectory(gp, op, orc, goal)
            kinds[r["kind"]] = kinds.get(r["kind"], 0) + 1
            if op.status == fm.OK:
                ok_o = orc.commit(op)
                ok_g = ctx.commit_plan(gp) if r["kind"] == "identical" else ctx.commit_points(op.t0, op.xyz)
                assert ok_o == ok_g
            _log(f"[window 10] request {q}: status {op.status}, {op.n_points} points, {r['kind']}")
    assert kinds.get("identical", 0) >= 6


@pytest.mark.parametrize("arrivals", [False, True])
def test_window_fcfs_equals_sequential(fm, arrivals):
    """The concurrent engine with the window (its interaction check covers
    every window row) gives bit for bit the sequential plan-then-commit
    result; with Poisson arrivals as well."""
    sc = _with_window(S.small(seed=12, n_plans=150, n_requests=60), 10)     # dense: requests interact
    sc.cfg.plan_capacity = 1024                  # withdrawn tentative entries keep their columns
    seq = []
    with fm.context_for(sc) as ctx:
        for q in range(sc.requests.n):
            p = ctx.plan_request(sc.requests.origin[q], sc.requests.goal[q], 0)
            seq.append((p, ctx.commit_plan(p) if p.status == fm.OK else False))
    arr = S.serving_arrivals(300.0, sc.requests.n, seed=5) if arrivals else None
    with fm.context_for(sc, max_slots=32, steps_per_launch=32) as ctx:
        plans, committed, _ = ctx.plan_fcfs(sc.requests, arrival_s=arr)
        st = ctx.stats()
    _log(f"[window fcfs] arrivals {arrivals}: {st}, committed {int(committed.sum())}")
    for q, ((p, c), b, cb) in enumerate(zip(seq, plans, committed)):
        assert p.status == b.status and p.n_points == b.n_points, q
        assert np.array_equal(p.points(), b.points()) and np.array_equal(p.actions(), b.actions()), q
        assert np.array_equal(p.values(), b.values()), q
        assert c == cb, q


def test_window_full_size(fm):
    """3000 plans, 360 actions, W = 10: the first requests against the oracle,
    and 200 requests through the concurrent engine against sequential."""
    sc = _with_window(S.large_actions(seed=2, n_plans=3000, n_requests=1000), 10)
    orc = Oracle(sc.cfg, sc.plans)
    m = 200
    reqs = S.Requests(sc.requests.ident[:m], sc.requests.origin[:m], sc.requests.goal[:m], sc.requests.t0[:m])
    seq = []
    with fm.context_for(sc) as ctx:
        for q in range(m):
            p = ctx.plan_request(reqs.origin[q], reqs.goal[q], 0)
            if q < 2:
                op = orc.plan(reqs.origin[q], reqs.goal[q], 0)
                r = classify_trajectory(p, op, orc, reqs.goal[q])
                _log(f"[window full size] request {q}: {op.n_points} points, status {op.status}, {r['kind']}")
                assert r["kind"] == "identical"
                if op.status == fm.OK:
                    orc.commit(op)
            seq.append((p, ctx.commit_plan(p) if p.status == fm.OK else False))
    with fm.context_for(sc, max_slots=1024, steps_per_launch=512) as ctx:
        plans, committed, _ = ctx.plan_fcfs(reqs)
        _log(f"[window full size] concurrent: {ctx.stats()}, committed {int(committed.sum())}/{m}")
    for q, ((p, c), b, cb) in enumerate(zip(seq, plans, committed)):
        assert p.status == b.status and np.array_equal(p.points(), b.points()), q
        assert np.array_equal(p.values(), b.values()) and c == cb, q


def test_window_rejects_proposal(fm):
    sc = _with_window(S.small(seed=0, n_plans=20, n_requests=1), 4)
    with fm.context_for(sc) as ctx:
        with pytest.raises(fm.FastMDPError):
            ctx.set_proposal(fm.PROPOSE_GOAL, 8)
