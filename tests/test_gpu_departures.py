"""Candidate departure times (ground delay) on the GPU against the oracle.

One request planned from several departure rows at once (fastmdp_plan_departures):
every candidate equals the oracle's plan from that row, and the chosen one
is the earliest departure whose plan the oracle also accepts (Sec. V:
parallel scheduling at different departure times; the planned evaluation
of candidate flight plans with different ground delay).
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import classify_trajectory  # noqa: E402

from oracle.oracle import Oracle  # noqa: E402
from paper_2008_03518_amd import scenario as S  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fm():
    from paper_2008_03518_amd import fastmdp
    return fastmdp


def _log(msg):
    print(msg, flush=True)


def _oracle_choice(orc, origin, goal, t0s):
    """Plans from every row; the earliest one that reaches the goal and that
    the oracle's commit accepts (appended to its table)."""
    plans = [orc.plan(origin, goal, int(t)) for t in t0s]
    for i in sorted(range(len(t0s)), key=lambda i: (t0s[i], i)):
        if plans[i].status == 0 and orc.commit(plans[i]):
            return plans, i
    return plans, -1


def test_ground_delay_clears_a_crossing():
    """A plan that sits across the straight path until row 60 and then
    leaves: departing at rows 0 and 30 the request has to go around (or is
    rejected), departing at 60 or later it flies the straight track, whose
    step count is ceil(D / ell - 1).  Every candidate equals the oracle's."""
    from paper_2008_03518_amd import fastmdp as fm
    cfg = S.cfg_small()
    rows = 200
    x = np.repeat(np.array([[3000.0, 5000.0, 300.0]], np.float32), rows, axis=0)
    x[60:] = [9500.0, 9500.0, 950.0]
    plans = S.Plans(np.zeros(1, np.int32), np.array([rows], np.int32), x)
    o, g = np.array([1000.0, 5000.0, 300.0]), np.array([9030.0, 5000.0, 300.0])
    t0s = [0, 30, 60, 90]
    orc = Oracle(cfg, plans)
    with fm.Context(cfg, max_slots=8) as ctx:
        ctx.load_plans(plans)
        got, chosen = ctx.plan_departures(o, g, t0s)
    want, ochosen = _oracle_choice(orc, o, g, t0s)
    for i, (gp, op) in enumerate(zip(got, want)):
        r = classify_trajectory(gp, op, orc, g)
        _log(f"[departures] t0 {t0s[i]}: status {op.status}, {op.n_points} points, {r['kind']}")
        assert r["kind"] == "identical"
    assert chosen == ochosen
    D = 8030.0
    straight = int(np.ceil(D / cfg.ell - 1.0))
    for i in (2, 3):
        assert got[i].status == fm.OK and got[i].n_points - 1 == straight
        assert np.max(np.abs(got[i].points()[:, 1] - 5000.0)) < 1e-6
    assert got[0].n_points - 1 != straight or got[0].status != fm.OK


def test_departures_against_oracle(fm):
    """Twelve requests of the small scenario, four departure rows each,
    committed first come first served with their chosen departure."""
    sc = S.small(seed=9, n_plans=200, n_requests=12)
    orc = Oracle(sc.cfg, sc.plans)
    t0s = [0, 15, 30, 45]
    n_delay = 0
    with fm.context_for(sc, max_slots=4) as ctx:
        for q in range(sc.requests.n):
            o, g = sc.requests.origin[q], sc.requests.goal[q]
            got, chosen = ctx.plan_departures(o, g, t0s)
            want = [orc.plan(o, g, t) for t in t0s]
            for gp, op in zip(got, want):
                assert classify_trajectory(gp, op, orc, g)["kind"] == "identical"
            ochosen = -1
            for i in range(len(t0s)):
                if want[i].status == 0 and orc.commit(want[i]):
                    ochosen = i
                    break
            assert chosen == ochosen, q
            if chosen >= 0:
                assert ctx.commit_plan(got[chosen])
                n_delay += int(chosen > 0)
            assert ctx.n_plans == orc.n_plans
    _log(f"[departures] {n_delay} of {sc.requests.n} requests accepted only with a delayed departure")
