"""Range query on the GPU: the same values and plans as the full sweep.

With range_query on, a step sweeps only the row entries within reach of the
state (Sec. VII: range queries restrict the trajectories considered to the
relevant volume).  The oracle's range-query pin shows on the CPU that no
value changes; here the GPU's single steps (W = 1 and W = 4) and its
concurrent FCFS passes on the 3000-plan, 360-action workload are compared
bit for bit with the full sweep, which the rest of the suite compares with
the oracle.
"""
import copy
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from paper_2008_03518_amd import scenario as S  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fm():
    from paper_2008_03518_amd import fastmdp
    return fastmdp


def _log(msg):
    print(msg, flush=True)


def _ranged(sc):
    r = copy.deepcopy(sc)
    r.cfg.range_query = 1
    return r


def _near_plan_states(sc, n, seed):
    rng = np.random.default_rng(seed)
    off = sc.plans.offsets()
    out = []
    while len(out) < n:
        j = int(rng.integers(sc.plans.n))
        L = int(sc.plans.length[j])
        if L < 10:
            continue
        k = int(rng.integers(0, L - 8))
        s = sc.plans.xyz[off[j] + k + 1].astype(np.float64) + rng.uniform(-200, 200, 3) * np.array([1, 1, 0.4])
        lo, hi = np.array(sc.cfg.box_min), np.array(sc.cfg.box_max)
        s = np.clip(s, lo + 1.0, hi - 1.0)
        g = np.array([rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]), rng.uniform(100, 900)])
        out.append((s, g, int(sc.plans.t0[j]) + k))
    return out


@pytest.mark.parametrize("name,W", [("small", 1), ("small", 4), ("large", 1)])
def test_range_query_single_steps(fm, name, W):
    sc = S.small(seed=0, n_plans=200, n_requests=1) if name == "small" else S.large_actions(2, 3000, 10)
    sc.cfg.lookahead = W
    rs = _ranged(sc)
    n_in = 0
    with fm.context_for(sc) as full, fm.context_for(rs) as ranged:
        for s, g, t in _near_plan_states(sc, 40, 21):
            a, b = full.eval_step(s, g, t), ranged.eval_step(s, g, t)
            pa, pb = full.stats()["pairs"], ranged.stats()["pairs"]
            for k in ("V", "G", "I", "T"):
                assert np.array_equal(a[k], b[k]), k
            assert a["best"] == b["best"] and pb <= pa
            n_in += int(np.sum(a["I"] > 0))
    _log(f"[range query {name}, W {W}] {n_in} actions scored inside a well, all identical")
    assert n_in > 20


def test_range_query_fcfs_full_size(fm):
    """All 1000 requests at 3000 plans x 360 actions, concurrent engine in the
    benchmark's launch configuration: plans, values and acceptances equal to
    the full sweep's bit for bit, with a small fraction of the pairs swept."""
    sc = S.large_actions(seed=2, n_plans=3000, n_requests=1000)
    out = {}
    for tag, scen in (("full", sc), ("ranged", _ranged(sc))):
        with fm.context_for(scen, max_slots=1024, steps_per_launch=512) as ctx:
            plans, committed, _ = ctx.plan_fcfs(scen.requests)
            out[tag] = (plans, committed, ctx.stats())
            _log(f"[range query fcfs] {tag}: {out[tag][2]}, committed {int(committed.sum())}")
    (p1, c1, s1), (p2, c2, s2) = out["full"], out["ranged"]
    assert np.array_equal(c1, c2)
    for q, (a, b) in enumerate(zip(p1, p2)):
        assert a.status == b.status and a.n_points == b.n_points, q
        assert np.array_equal(a.points(), b.points()) and np.array_equal(a.actions(), b.actions()), q
        assert np.array_equal(a.values(), b.values()), q
    assert s2["pairs"] < 0.1 * s1["pairs"]


def test_range_query_window_fcfs(fm):
    """Window W = 4 with the range query (radius grown by the window) through
    the concurrent engine: equal to the window's full sweep."""
    sc = S.small(seed=12, n_plans=150, n_requests=40)
    sc.cfg.lookahead = 4
    sc.cfg.plan_capacity = 1024
    res = []
    for scen in (sc, _ranged(sc)):
        with fm.context_for(scen, max_slots=16, steps_per_launch=32) as ctx:
            res.append(ctx.plan_fcfs(scen.requests)[:2])
    (p1, c1), (p2, c2) = res
    assert np.array_equal(c1, c2)
    for a, b in zip(p1, p2):
        assert a.status == b.status and np.array_equal(a.points(), b.points())
        assert np.array_equal(a.values(), b.values())


def test_range_query_with_proposal(fm):
    """The proposal path with the range query (its k-action sweep and its
    full-sweep fallbacks see only the plans within reach; ranking steps of a
    network still stage every plan for the features): plans equal to the
    full sweep's bit for bit, with the goal ranking and with a network; the
    single-step features and ranking are those without the range query."""
    from paper_2008_03518_amd import proposal as PR
    sc = S.large_actions(seed=2, n_plans=3000, n_requests=300)
    A = sc.cfg.n_actions
    net = fm.Mlp(A)
    net.set_params(PR.init_params(A, seed=3))
    rs = _ranged(sc)
    with fm.context_for(sc, max_slots=1024, steps_per_launch=512) as ctx:
        ref, com, _ = ctx.plan_fcfs(sc.requests)
        s0, g0 = sc.requests.origin[0], sc.requests.goal[0]
        ctx.set_proposal(fm.PROPOSE_MLP, 8, net, 64)
        e_full = ctx.eval_proposal(s0, g0, 0)
    with fm.context_for(rs, max_slots=1024, steps_per_launch=512) as ctx:
        ctx.snapshot()
        for mode, nt in ((fm.PROPOSE_GOAL, None), (fm.PROPOSE_MLP, net)):
            ctx.rewind()
            ctx.set_proposal(mode, 8, nt, 64)
            plans, c2, _ = ctx.plan_fcfs(rs.requests)
            _log(f"[range query + proposal {mode}] {ctx.stats()}, {ctx.proposal_stats()}")
            assert np.array_equal(c2, com)
            for q, (a, b) in enumerate(zip(ref, plans)):
                assert a.status == b.status and np.array_equal(a.points(), b.points()), q
                assert np.array_equal(a.values(), b.values()), q
        e_rq = ctx.eval_proposal(s0, g0, 0)
    assert np.array_equal(e_full["features"], e_rq["features"]) and np.array_equal(e_full["topk"], e_rq["topk"])
    net.close()
