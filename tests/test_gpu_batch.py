"""Co-simulated batches on the GPU against the FP64 oracle (Sec. V; the peak
table: five risk wells per other aircraft along its extrapolated track;
"Process negative rewards").  The oracle's own pins fix the head-on pair
(14 straight steps, then point-symmetric avoidance) and reduce a batch of
one to the single-request plan."""
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


def _requests(origins, goals, t0=0):
    n = len(origins)
    return S.Requests(np.arange(1, n + 1, dtype=np.uint64), np.asarray(origins, np.float64),
                      np.asarray(goals, np.float64), np.full(n, t0, np.int32))


def test_batch_head_on_pair(fm):
    cfg = S.cfg_small()
    o = np.array([[1000.0, 5000.0, 300.0], [3000.0, 5000.0, 300.0]])
    g = o[::-1].copy()
    with fm.Context(cfg, max_slots=2) as ctx:
        got = ctx.plan_batch(_requests(o, g))
    orc = Oracle(cfg)
    want = orc.plan_batch(o, g, 0)
    for i in range(2):
        r = classify_trajectory(got[i], want[i], orc, g[i])
        assert r["kind"] == "identical", (i, r)
    assert np.max(np.abs(got[0].points()[:15, 1] - 5000.0)) < 1e-9 and abs(got[0].points()[15, 1] - 5000.0) > 1.0


@pytest.mark.parametrize("n", [1, 5, 12])
def test_batch_against_oracle(fm, n):
    """A batch from the small scenario (200 known plans, 81 actions): every
    aircraft's trajectory equals the oracle's co-simulated plan (a batch of
    one also equals the single-request plan)."""
    sc = S.small(seed=31, n_plans=200, n_requests=n)
    reqs = sc.requests
    with fm.context_for(sc, max_slots=32) as ctx:
        got = ctx.plan_batch(reqs)
        st = ctx.stats()
        single = ctx.plan_request(reqs.origin[0], reqs.goal[0], 0) if n == 1 else None
    orc = Oracle(sc.cfg, sc.plans)
    want = orc.plan_batch(reqs.origin, reqs.goal, 0)
    kinds = []
    for i in range(n):
        # inside a batch any difference changes what the others see: every
        # trajectory must equal the oracle's (no excused divergence)
        try:
            r = classify_trajectory(got[i], want[i], orc if n == 1 else _NoEval(), reqs.goal[i])
            kinds.append(r["kind"])
        except AssertionError as e:
            g, w = got[i], want[i]
            m = min(g.n_points, w.n_points)
            d = [k for k in range(m) if np.max(np.abs(g.points()[k] - w.xyz[k])) > 1e-6]
            kinds.append(f"differs: {e}; status gpu {g.status} oracle {w.status}, points {g.n_points} / "
                         f"{w.n_points}, first differing point {d[0] if d else None}")
    _log(f"[batch {n}] statuses {[p.status for p in got]}, {kinds}, {st}")
    assert all(k == "identical" for k in kinds)
    if single is not None:
        assert np.array_equal(single.points(), got[0].points()) and np.array_equal(single.values(), got[0].values())


class _NoEval:
    """Inside a batch the oracle's single-aircraft step is not the batch's:
    any action difference is reported, not excused."""

    def eval_step(self, *a, **k):
        raise AssertionError("batch trajectories differ")
