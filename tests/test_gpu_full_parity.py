"""Every request of the two benchmark-sized workloads against the FP64 oracle.

Workloads (seeded, as the benchmark draws them):
  * paper scale: 30 x 30 x 1.5 km, 2000 known plans, 256 x 256 terrain of
    50 hills, 81 actions, dt 1 s, all 200 FCFS requests;
  * 3000 known plans, 360 actions, dt 0.5 s, all 1000 FCFS requests.

Lockstep: the GPU (through the C ABI, full sweep, one request at a time)
and the oracle plan each request against identical tables, in request
order (Sec. V: first come, first served).  While the two trajectories are
identical each side commits its own plan; after an excused divergence both
receive the oracle's plan, so that the next request again starts from
identical tables.  Before each commit the GPU's single step is compared
with the oracle's at every TEACH-th state of the oracle's trajectory
(teacher forcing).  Counted and asserted: identical trajectories, excused
divergences (near tie / boundary band), zero unexcused differences, value
errors within 1e-5 relative, and the stored-table separation invariant
(R_sep less the FP32 rounding bound) over the final tables.

Then the concurrent engine in the benchmark's launch configuration (1024
slots, at most one request per compute unit, 512 steps per launch; full
sweep and goal-ranked proposal) plans all requests of the workload at once:
its plans equal GPU sequential planning bit for bit, so when the lockstep
found no divergence they are the oracle's plans.

The oracle runs on every host core (OpenMP over the actions of a step);
the larger workload is split into request ranges, one test each, which
continue the same tables in order.
"""
import os
import sys
import time

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import classify_trajectory, compare_eval, fp32_rounding_bound, separation_report, stored  # noqa: E402

from oracle.oracle import Oracle  # noqa: E402
from paper_2008_03518_amd import scenario as S  # noqa: E402

pytestmark = pytest.mark.gpu

C2_CHUNK = 200


def _log(msg):
    print(msg, flush=True)


class Lockstep:
    def __init__(self, fm, sc, teach):
        self.fm, self.sc, self.teach = fm, sc, teach
        self.ctx = fm.context_for(sc)
        self.orc = Oracle(sc.cfg, sc.plans, sc.terrain)
        self.q = 0
        self.counts = dict(requests=0, identical=0, near_tie=0, band=0, committed=0, points=0,
                           teacher_steps=0, teacher_actions=0, teacher_band_actions=0)
        self.max_rel = 0.0
        self.accepted = []           # (t0, FP64 points) in acceptance order
        self.gpu_plans = []          # the GPU's own plan of every request (lockstep)
        self.divergences = []

    def run(self, upto):
        sc, fm = self.sc, self.fm
        t = time.perf_counter()
        while self.q < upto:
            q = self.q
            goal = sc.requests.goal[q]
            t0 = int(sc.requests.t0[q])
            op = self.orc.plan(sc.requests.origin[q], goal, t0)
            gp = self.ctx.plan_request(sc.requests.origin[q], goal, t0)
            r = classify_trajectory(gp, op, self.orc, goal)
            self.counts[r["kind"]] += 1
            self.counts["points"] += min(gp.n_points, op.n_points)
            self.max_rel = max(self.max_rel, r["max_rel"])
            if r["kind"] != "identical":
                self.divergences.append((q, r["kind"], r["at"]))
                _log(f"[lockstep] request {q}: excused divergence ({r['kind']}) at point {r['at']}")
            for k in range(0, op.n_points - 1, self.teach):
                o = self.orc.eval_step(op.xyz[k], goal, t0 + k)
                n_cmp, n_band, mx, _, _ = compare_eval(self.ctx.eval_step(op.xyz[k], goal, t0 + k), o)
                self.counts["teacher_steps"] += 1
                self.counts["teacher_actions"] += n_cmp
                self.counts["teacher_band_actions"] += n_band
                self.max_rel = max(self.max_rel, mx)
            if op.status == fm.OK:
                ok_o = self.orc.commit(op)
                if r["kind"] == "identical":
                    ok_g = self.ctx.commit_plan(gp)
                else:
                    ok_g = self.ctx.commit_points(op.t0, op.xyz)
                assert ok_g == ok_o, q
                if ok_o:
                    self.accepted.append((op.t0, op.xyz.copy()))
                    self.counts["committed"] += 1
            assert self.ctx.n_plans == self.orc.n_plans
            self.gpu_plans.append((gp.status, gp.n_points, gp.points().copy(), gp.actions().copy(),
                                   gp.values().copy()))
            self.counts["requests"] += 1
            self.q += 1
        _log(f"[lockstep {self.sc.name}] requests {self.q}: {self.counts}, max value rel err {self.max_rel:.2e}, "
             f"{time.perf_counter() - t:.1f} s")

    def separation(self):
        sc = self.sc
        off = sc.plans.offsets()
        known = [(int(sc.plans.t0[j]), sc.plans.xyz[off[j]:off[j + 1]]) for j in range(sc.plans.n)]
        delta = fp32_rounding_bound(sc.cfg.box_min, sc.cfg.box_max)
        bad, gap = separation_report(known, [stored(t0, x) for t0, x in self.accepted], sc.cfg.R_sep, delta)
        _log(f"[lockstep {sc.name}] separation: {bad} pairs below R_sep - {delta:.2e} m, minimum stored gap "
             f"{gap:.4f} m over {len(self.accepted)} accepted plans")
        return bad, gap, delta

    def close(self):
        self.ctx.close()


@pytest.fixture(scope="module")
def fm():
    from paper_2008_03518_amd import fastmdp
    return fastmdp


@pytest.fixture(scope="module")
def c2(fm):
    ls = Lockstep(fm, S.large_actions(seed=2, n_plans=3000, n_requests=1000), teach=200)
    yield ls
    ls.close()


def _concurrent_equals(fm, ls, n):
    """The concurrent engine (benchmark launch configuration, full sweep and
    goal-ranked proposal) against GPU sequential planning of all n requests."""
    sc = ls.sc
    with fm.context_for(sc, max_slots=1024, steps_per_launch=512) as ctx:
        ctx.snapshot()
        out = {}
        for mode in (fm.PROPOSE_NONE, fm.PROPOSE_GOAL):
            ctx.rewind()
            ctx.set_proposal(mode, 8, None, 64)
            plans, committed, _ = ctx.plan_fcfs(sc.requests)
            out[mode] = (plans, committed)
            _log(f"[concurrent {sc.name}] mode {mode}: {ctx.stats()}, committed {int(committed.sum())}/{n}")
    if ls.divergences:
        # the lockstep tables took the oracle's plan after a divergence:
        # compare with a plain GPU sequential pass instead
        seq = []
        with fm.context_for(sc) as ctx:
            for q in range(n):
                p = ctx.plan_request(sc.requests.origin[q], sc.requests.goal[q], int(sc.requests.t0[q]))
                if p.status == fm.OK:
                    ctx.commit_plan(p)
                seq.append((p.status, p.n_points, p.points().copy(), p.actions().copy(), p.values().copy()))
    else:
        seq = ls.gpu_plans
    for mode, (plans, committed) in out.items():
        for q, (st, npt, x, a, v) in enumerate(seq):
            b = plans[q]
            assert b.status == st and b.n_points == npt, (mode, q)
            assert np.array_equal(b.points(), x) and np.array_equal(b.actions(), a), (mode, q)
            assert np.array_equal(b.values(), v), (mode, q)
    return out


def test_paper_scale_every_request(fm):
    sc = S.paper_scale(seed=1, n_plans=2000, n_requests=200)
    ls = Lockstep(fm, sc, teach=50)
    try:
        ls.run(sc.requests.n)
        c = ls.counts
        assert c["requests"] == 200 and c["identical"] + c["near_tie"] + c["band"] == 200
        assert c["committed"] >= 100
        bad, gap, delta = ls.separation()
        assert bad == 0 and gap >= sc.cfg.R_sep - delta
        out = _concurrent_equals(fm, ls, sc.requests.n)
        if not ls.divergences:
            for plans, committed in out.values():
                assert int(committed.sum()) == c["committed"]
    finally:
        ls.close()


@pytest.mark.parametrize("upto", list(range(C2_CHUNK, 1000 + 1, C2_CHUNK)))
def test_large_actions_every_request(fm, c2, upto):
    c2.run(upto)
    assert c2.q == upto


def test_large_actions_separation_and_concurrent(fm, c2):
    assert c2.q == 1000, "the request ranges above ran first"
    c = c2.counts
    assert c["identical"] + c["near_tie"] + c["band"] == 1000
    bad, gap, delta = c2.separation()
    assert bad == 0 and gap >= c2.sc.cfg.R_sep - delta
    out = _concurrent_equals(fm, c2, 1000)
    if not c2.divergences:
        for plans, committed in out.values():
            assert int(committed.sum()) == c["committed"]
