"""HIP planner versus the FP64 oracle, through the C ABI.

Sizes: the 50/200-plan 10 km box (81 actions), the paper-scale 2000-plan box
with terrain (81 actions), and the 3000-plan, 360-action workload at full
size on sampled requests; plus ragged multi-tile rows, outcomes, commit,
checkpoint and the first-come-first-served batch against sequential
planning.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import compare_eval, compare_trajectory, fp32_rounding_bound, separation_report, stored  # noqa: E402

from oracle.oracle import Oracle  # noqa: E402
from paper_2008_03518_amd import scenario as S  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fm():
    from paper_2008_03518_amd import fastmdp
    return fastmdp


def _log(msg):
    print(msg, flush=True)


def _states_near_plans(sc, n, seed):
    rng = np.random.default_rng(seed)
    off = sc.plans.offsets()
    out = []
    while len(out) < n:
        j = int(rng.integers(sc.plans.n))
        L = int(sc.plans.length[j])
        if L < 3:
            continue
        k = int(rng.integers(0, L - 1))
        p = sc.plans.xyz[off[j] + k + 1].astype(np.float64)
        s = p + rng.uniform(-170, 170, 3) * np.array([1.0, 1.0, 0.4])
        lo, hi = np.array(sc.cfg.box_min), np.array(sc.cfg.box_max)
        s = np.clip(s, lo + 1.0, hi - 1.0)
        g = np.array([rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]), rng.uniform(100, 900)])
        out.append((s, g, int(sc.plans.t0[j]) + k))
    return out


# ---------------------------------------------------------------------------
def test_eval_step_small_near_plans(fm):
    sc = S.small(seed=0, n_plans=200, n_requests=1)
    orc = Oracle(sc.cfg, sc.plans)
    n_cmp = n_in = 0
    with fm.context_for(sc) as ctx:
        for s, g, t in _states_near_plans(sc, 80, 11):
            o = orc.eval_step(s, g, t)
            r = ctx.eval_step(s, g, t)
            n, _, mx, _, _ = compare_eval(r, o)
            n_cmp += n
            n_in += int(np.sum(o["I"] > 0))
    _log(f"[eval small] compared {n_cmp} actions, {n_in} inside wells")
    assert n_in > 200


def test_eval_step_small_teacher_forced(fm):
    sc = S.small(seed=0, n_plans=200, n_requests=3)
    orc = Oracle(sc.cfg, sc.plans)
    with fm.context_for(sc) as ctx:
        for q in range(sc.requests.n):
            op = orc.plan(sc.requests.origin[q], sc.requests.goal[q], 0)
            for k in range(op.n_points - 1):
                o = orc.eval_step(op.xyz[k], sc.requests.goal[q], k)
                r = ctx.eval_step(op.xyz[k], sc.requests.goal[q], k)
                compare_eval(r, o)
            _log(f"[teacher small] request {q}: {op.n_points - 1} steps ok (status {op.status})")


def test_plan_request_small(fm):
    sc = S.small(seed=4, n_plans=200, n_requests=6)
    orc = Oracle(sc.cfg, sc.plans)
    with fm.context_for(sc) as ctx:
        for q in range(sc.requests.n):
            op = orc.plan(sc.requests.origin[q], sc.requests.goal[q], 0)
            gp = ctx.plan_request(sc.requests.origin[q], sc.requests.goal[q], 0)
            same, diverged = compare_trajectory(gp, op, orc, sc.requests.goal[q])
            _log(f"[plan small] request {q}: {same} identical points, diverged={diverged}, status {op.status}")


def _fcfs_sync(fm, sc, n_req, teacher_every=0):
    """Plan requests in order on both sides; commit each plan to both tables.

    While the GPU and oracle trajectories are identical the GPU commits its
    own plan; after an excused divergence both tables receive the oracle's
    plan, so that the next request starts from identical tables.
    """
    orc = Oracle(sc.cfg, sc.plans, sc.terrain)
    stats = dict(identical=0, diverged=0, committed=0)
    with fm.context_for(sc) as ctx:
        for q in range(n_req):
            goal = sc.requests.goal[q]
            op = orc.plan(sc.requests.origin[q], goal, int(sc.requests.t0[q]))
            gp = ctx.plan_request(sc.requests.origin[q], goal, int(sc.requests.t0[q]))
            same, diverged = compare_trajectory(gp, op, orc, goal)
            if teacher_every:
                for k in range(0, op.n_points - 1, teacher_every):
                    compare_eval(ctx.eval_step(op.xyz[k], goal, op.t0 + k), orc.eval_step(op.xyz[k], goal, op.t0 + k))
            ok_o = orc.commit(op) if op.status == 0 else False
            if op.status == 0:
                if diverged:
                    ok_g = ctx.commit_points(op.t0, op.xyz)
                else:
                    ok_g = ctx.commit_plan(gp)
                assert ok_g == ok_o
            assert ctx.n_plans == orc.n_plans
            stats["diverged" if diverged else "identical"] += 1
            stats["committed"] += int(ok_o)
            _log(f"[fcfs sync] request {q}: status {op.status}, {op.n_points} points, "
                 f"identical {same}, diverged {diverged}")
    return stats


def test_fcfs_sync_small(fm):
    st = _fcfs_sync(fm, S.small(seed=5, n_plans=120, n_requests=12), 12, teacher_every=5)
    _log(f"[fcfs small] {st}")
    assert st["committed"] >= 6


def test_paper_scale_terrain(fm):
    sc = S.paper_scale(seed=1, n_plans=2000, n_requests=200)
    st = _fcfs_sync(fm, sc, 6, teacher_every=25)
    _log(f"[paper scale] {st}")


def test_large_actions_full_size_sampled(fm):
    sc = S.large_actions(seed=2, n_plans=3000, n_requests=1000)
    st = _fcfs_sync(fm, sc, 2, teacher_every=40)
    _log(f"[3000 plans x 360 actions] {st}")


def test_fcfs_full_size_bench_launch_config(fm):
    """The 3000-plan, 360-action workload through the concurrent engine in the
    benchmark's launch configuration (1024 slots, at most one request per
    compute unit, 512 steps per launch, early end), on more requests than
    compute units: every result equals sequential plan-then-commit bitwise,
    and the first requests equal the oracle's own sequential planning."""
    sc = S.large_actions(seed=2, n_plans=3000, n_requests=1000)
    m = 300
    reqs = S.Requests(sc.requests.ident[:m], sc.requests.origin[:m], sc.requests.goal[:m], sc.requests.t0[:m])
    with fm.context_for(sc, max_slots=1024, steps_per_launch=512) as ctx:
        ctx.snapshot()
        plans, committed, _ = ctx.plan_fcfs(reqs)
        st = ctx.stats()
        _log(f"[fcfs full size] {st}, committed {int(committed.sum())}/{m}")
        ctx.rewind()
        seq = []
        for q in range(m):
            p = ctx.plan_request(reqs.origin[q], reqs.goal[q], int(reqs.t0[q]))
            seq.append((p, ctx.commit_plan(p) if p.status == 0 else False))
    assert st["launches"] > 1
    for q, ((p, c), b, cb) in enumerate(zip(seq, plans, committed)):
        assert p.status == b.status and p.n_points == b.n_points, q
        assert np.array_equal(p.points(), b.points()) and np.array_equal(p.actions(), b.actions()), q
        assert np.array_equal(p.values(), b.values()), q
        assert c == cb, q
    assert _separation_violations(sc, plans, committed) == 0
    orc = Oracle(sc.cfg, sc.plans)
    for q in range(2):
        goal = reqs.goal[q]
        op = orc.plan(reqs.origin[q], goal, int(reqs.t0[q]))
        same, diverged = compare_trajectory(plans[q], op, orc, goal)
        _log(f"[fcfs full size] request {q}: oracle status {op.status}, {op.n_points} points, "
             f"identical {same}, diverged {diverged}")
        if diverged:
            break                 # the tables differ from here on
        assert (orc.commit(op) if op.status == 0 else False) == bool(committed[q])


def test_multi_tile_ragged_rows(fm):
    """Rows far larger than one LDS tile, with a ragged tail."""
    cfg = S.cfg_large_actions()
    cfg.plan_capacity = 6000
    rng = np.random.default_rng(9)
    n = 5000 + 37
    s = np.array([15000.0, 15000.0, 700.0])
    pts = s[None, :] + rng.uniform(-2000, 2000, (n, 3)) * np.array([1, 1, 0.15])
    pts[:50] = s[None, :] + rng.uniform(-170, 170, (50, 3))
    L = 8
    plans = S.Plans(t0=np.zeros(n, np.int32), length=np.full(n, L, np.int32),
                    xyz=np.repeat(pts[:, None, :], L, axis=1).reshape(-1, 3).astype(np.float32))
    orc = Oracle(cfg, plans)
    with fm.Context(cfg) as ctx:
        ctx.load_plans(plans)
        for q, g in enumerate([np.array([29000.0, 15000.0, 700.0]), np.array([100.0, 29000.0, 300.0])]):
            for t in range(3):
                o = orc.eval_step(s + [3.0 * t, -2.0 * t, 1.0], g, t)
                r = ctx.eval_step(s + [3.0 * t, -2.0 * t, 1.0], g, t)
                compare_eval(r, o)
        st = ctx.stats()
        assert st["pairs"] == cfg.n_actions * n


@pytest.mark.parametrize("n_head,climb,speed", [(34, (-5.0, -2.5, 0.0, 2.5, 5.0), (20.0, 30.0, 40.0)),
                                                 (128, (-5.0, 0.0, 5.0), (30.0,))])
def test_largest_action_sets(fm, n_head, climb, speed):
    """The largest action sets the kernels take: 510 actions (34 headings x 5
    climbs x 3 speeds) and 128 headings (x 3 climbs, one speed: 384
    actions).  Per-action values
    near plans and trajectories against the oracle; the proposal path's
    plans against the full sweep's."""
    sc = S.small(seed=21, n_plans=200, n_requests=6)
    sc.cfg.n_head, sc.cfg.climb, sc.cfg.speed = n_head, climb, speed
    sc.cfg.plan_capacity = 512                               # room for tentative entries
    A = sc.cfg.n_actions
    assert A in (510, 384)
    orc = Oracle(sc.cfg, sc.plans)
    with fm.context_for(sc) as ctx:
        for s, g, t in _states_near_plans(sc, 6, seed=4):
            compare_eval(ctx.eval_step(s, g, t), orc.eval_step(s, g, t))
    st = _fcfs_sync(fm, sc, 3, teacher_every=0)
    _log(f"[{A} actions] {st}")
    with fm.context_for(sc, max_slots=8) as ctx:
        ctx.snapshot()
        ctx.set_proposal(fm.PROPOSE_NONE, 1)
        ref, com, _ = ctx.plan_fcfs(sc.requests)
        ctx.rewind()
        ctx.set_proposal(fm.PROPOSE_GOAL, 8, None, 4)
        got, com2, _ = ctx.plan_fcfs(sc.requests)
        ps = ctx.proposal_stats()
    _log(f"[{A} actions] proposal: {ps}")
    assert np.array_equal(com, com2)
    for p, q in zip(ref, got):
        assert p.status == q.status and np.array_equal(p.points(), q.points())
        assert np.array_equal(p.actions(), q.actions()) and np.array_equal(p.values(), q.values())


def test_degenerate_requests(fm):
    """Capture at the origin (one point), a goal straight above the origin
    (no horizontal bearing: heading offsets from 0), and an empty batch."""
    sc = S.small(seed=22, n_plans=100, n_requests=1)
    orc = Oracle(sc.cfg, sc.plans)
    o = np.array([300.0, 9700.0, 500.0])
    cases = [(o, o + [5.0, -5.0, 3.0]), (o, o + [0.0, 0.0, 300.0])]
    with fm.context_for(sc) as ctx:
        n0 = ctx.n_plans
        for k, (a, g) in enumerate(cases):
            gp = ctx.plan_request(a, g, 0)
            op = orc.plan(a, g, 0)
            same, diverged = compare_trajectory(gp, op, orc, g)
            _log(f"[degenerate {k}] status {op.status}, {op.n_points} points, identical {same}")
            assert not diverged
            if k == 0:
                assert op.status == fm.OK and op.n_points == 1 and gp.n_points == 1
        empty = S.Requests(np.zeros(0, np.uint64), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, np.int32))
        plans, committed, done = ctx.plan_fcfs(empty)
        assert len(plans) == 0 and committed.size == 0 and done.size == 0 and ctx.n_plans == n0


def test_planning_rows_beyond_one_tile(fm):
    """Planning (not only single steps) on rows of more plans than one LDS
    tile holds: 5000 known plans, so the first rows hold ~5000 entries.  The
    concurrent full sweep equals sequential plan-then-commit bitwise, the
    proposal path (which sweeps such rows in full) equals it too, and the
    first request equals the oracle's."""
    sc = S.large_actions(seed=31, n_plans=5000, n_requests=24)
    assert int(np.sum(sc.plans.t0 == 0)) > 4096
    seq = []
    with fm.context_for(sc) as ctx:
        for q in range(sc.requests.n):
            p = ctx.plan_request(sc.requests.origin[q], sc.requests.goal[q], int(sc.requests.t0[q]))
            seq.append((p, ctx.commit_plan(p) if p.status == 0 else False))
    with fm.context_for(sc, max_slots=32, steps_per_launch=512) as ctx:
        ctx.snapshot()
        for mode in (fm.PROPOSE_NONE, fm.PROPOSE_GOAL):
            ctx.rewind()
            ctx.set_proposal(mode, 8, None, 64)
            plans, committed, _ = ctx.plan_fcfs(sc.requests)
            _log(f"[rows beyond one tile] mode {mode}: {ctx.stats()}, committed {int(committed.sum())}")
            for q, ((p, c), b, cb) in enumerate(zip(seq, plans, committed)):
                assert p.status == b.status and p.n_points == b.n_points, q
                assert np.array_equal(p.points(), b.points()) and np.array_equal(p.actions(), b.actions()), q
                assert np.array_equal(p.values(), b.values()), q
                assert c == cb, q
    orc = Oracle(sc.cfg, sc.plans)
    goal = sc.requests.goal[0]
    op = orc.plan(sc.requests.origin[0], goal, int(sc.requests.t0[0]))
    same, diverged = compare_trajectory(seq[0][0], op, orc, goal)
    _log(f"[rows beyond one tile] request 0: {op.n_points} points, identical {same}, diverged {diverged}")


def test_terrain_well_own_constants(fm):
    """Terrain well with r_T = 2.5, gamma_T = 0.95, R_T = 90 m (intruder
    well 1, 0.99, 150 m) over flat ground at 40 m: per-action values against
    the oracle, and the terrain term against the hand values the oracle's
    pin uses (clearances 55 / 60 / 65 m by climb rate; none inside 90 m at
    125-135 m; the full magnitude below the surface)."""
    from test_oracle_pins import TERRAIN_WELL_HAND, plane_terrain, terrain_constants_cfg
    cfg = terrain_constants_cfg()
    ter = plane_terrain(0.0, 0.0, 40.0)
    orc = Oracle(cfg, terrain=ter)
    g = np.array([3000.0, 2000.0, 100.0])
    with fm.Context(cfg) as ctx:
        ctx.set_terrain(ter)
        for z in (100.0, 170.0, 38.0):
            s = np.array([3000.0, 7000.0, z])
            r = ctx.eval_step(s, g, 0)
            compare_eval(r, orc.eval_step(s, g, 0))
            for a in range(cfg.n_actions):
                c = (a // len(cfg.speed)) % len(cfg.climb)
                clr = z - 40.0 + (c - 1) * 5.0
                if clr in TERRAIN_WELL_HAND or clr >= cfg.R_terr or clr < 0:
                    want = TERRAIN_WELL_HAND[clr] if clr in TERRAIN_WELL_HAND else (2.5 if clr < 0 else 0.0)
                    assert abs(r["T"][a] - want) <= 1e-5 * max(want, 1e-300), (z, a, r["T"][a], want)


def test_empty_table_straight_track(fm):
    cfg = S.cfg_large_actions()
    o, g = np.array([1000.0, 5000.0, 300.0]), np.array([9030.0, 5000.0, 300.0])
    with fm.Context(cfg) as ctx:
        p = ctx.plan_request(o, g, 0)
    D = 8030.0
    assert p.status == 0 and p.n_points - 1 == int(np.ceil(D / cfg.ell - 1.0))
    assert np.max(np.abs(p.points()[:, 1] - 5000.0)) < 1e-6 and np.max(np.abs(p.points()[:, 2] - 300.0)) < 1e-9


def test_outcomes(fm):
    cfg = S.cfg_small()
    o = np.array([5000.0, 5000.0, 500.0])
    goal = np.array([9000.0, 5000.0, 500.0])
    # every successor inside a well
    x = np.repeat(o[None, :], 64, axis=0)
    x[0] += [0.0, 0.0, 400.0]
    with fm.Context(cfg) as ctx:
        ctx.load_plans(S.Plans(np.zeros(1, np.int32), np.array([64], np.int32), x.astype(np.float32)))
        p = ctx.plan_request(o, goal, 0)
        assert p.status == fm.REJECT_SEPARATION and p.n_points == 2
        p = ctx.plan_request(o, goal, 1)        # the plan sits on the origin at row 1
        assert p.status == fm.REJECT_ORIGIN and p.n_points == 1
    c2 = S.cfg_small()
    c2.max_steps = 5
    with fm.Context(c2) as ctx:
        p = ctx.plan_request([1000.0, 1000.0, 500.0], [9000.0, 9000.0, 500.0], 0)
        assert p.status == fm.TIMEOUT and p.n_points == 6
    tiny = S.cfg_small()
    tiny.box_min, tiny.box_max = (0.0, 0.0, 0.0), (10.0, 10.0, 1000.0)
    with fm.Context(tiny) as ctx:
        p = ctx.plan_request([5.0, 5.0, 500.0], [9.0, 9.0, 900.0], 0)
        assert p.status == fm.NO_VALID_ACTION and p.n_points == 1
    c3 = S.cfg_small()
    c3.climb = (-5.0,)
    xs = np.arange(17) * 625.0
    X, Y = np.meshgrid(xs, xs)
    ter = S.Terrain(17, 17, np.full(X.shape, 497.0, np.float32), 0.0, 0.0, 625.0, np.zeros((0, 4)))
    with fm.Context(c3) as ctx:
        ctx.set_terrain(ter)
        p = ctx.plan_request(o, goal, 0)
        assert p.status == fm.REJECT_TERRAIN and p.n_points == 2


def test_commit_validates_and_appends(fm):
    cfg = S.cfg_small()
    base = np.repeat(np.array([[5000.0, 5000.0, 500.0]], np.float32), 30, axis=0)
    with fm.Context(cfg) as ctx:
        ctx.load_plans(S.Plans(np.zeros(1, np.int32), np.array([30], np.int32), base))
        near = np.repeat(np.array([[5100.0, 5000.0, 500.0]]), 10, axis=0)
        assert ctx.commit_points(5, near) is False and ctx.n_plans == 1
        assert ctx.commit_points(31, near) is True and ctx.n_plans == 2
        far = np.repeat(np.array([[5151.0, 5000.0, 500.0]]), 10, axis=0)
        assert ctx.commit_points(0, far) is True and ctx.n_plans == 3
        assert ctx.commit_points(28, far) is False and ctx.n_plans == 3
        far2 = np.repeat(np.array([[5000.0, 5000.0, 650.5]]), 10, axis=0)
        assert ctx.commit_points(60, far2) is True and ctx.n_plans == 4
        assert ctx.commit_points(0, far2 - [0.0, 0.0, 1.0]) is False
        with pytest.raises(fm.FastMDPError):
            ctx.commit_points(cfg.max_rows - 3, near)          # runs past the last row


def test_checkpoint_roundtrip(fm, tmp_path):
    sc = S.small(seed=6, n_plans=100, n_requests=3)
    path = str(tmp_path / "table.bin")
    with fm.context_for(sc) as ctx:
        p0 = ctx.plan_request(sc.requests.origin[0], sc.requests.goal[0], 0)
        assert p0.status == 0 and ctx.commit_plan(p0)
        ctx.save_table(path)
        p1 = ctx.plan_request(sc.requests.origin[1], sc.requests.goal[1], 0)
    with fm.Context(sc.cfg) as ctx2:
        ctx2.load_table(path)
        assert ctx2.n_plans == sc.plans.n + 1
        p2 = ctx2.plan_request(sc.requests.origin[1], sc.requests.goal[1], 0)
    assert p1.n_points == p2.n_points and np.array_equal(p1.points(), p2.points())


def test_determinism(fm):
    sc = S.large_actions(seed=8, n_plans=600, n_requests=2)
    with fm.context_for(sc) as ctx:
        a = ctx.plan_request(sc.requests.origin[0], sc.requests.goal[0], 0)
        b = ctx.plan_request(sc.requests.origin[0], sc.requests.goal[0], 0)
    assert a.n_points == b.n_points and np.array_equal(a.points(), b.points()) and np.array_equal(a.values(), b.values())


def _separation_violations(sc, plans, committed):
    """Stored-versus-stored separation of the accepted plans against the
    known plans and each other: pairs closer than R_sep less the FP32
    rounding bound of a stored point (the invariant the oracle suite checks
    with the same function)."""
    off = sc.plans.offsets()
    known = [(int(sc.plans.t0[j]), sc.plans.xyz[off[j]:off[j + 1]]) for j in range(sc.plans.n)]
    acc = [stored(p.t0, p.points()) for p, c in zip(plans, committed) if c]
    delta = fp32_rounding_bound(sc.cfg.box_min, sc.cfg.box_max)
    bad, gap = separation_report(known, acc, sc.cfg.R_sep, delta)
    _log(f"[separation] {len(acc)} accepted plans, minimum stored gap {gap:.4f} m, bound {sc.cfg.R_sep - delta:.4f} m")
    return bad


def test_fcfs_batch_equals_sequential(fm):
    """Alone versus in the mix: concurrent FCFS gives bitwise the sequential result."""
    sc = S.large_actions(seed=12, n_plans=400, n_requests=48)
    cfg = sc.cfg
    seq = []
    with fm.context_for(sc) as ctx:
        for q in range(sc.requests.n):
            p = ctx.plan_request(sc.requests.origin[q], sc.requests.goal[q], 0)
            c = ctx.commit_plan(p) if p.status == 0 else False
            seq.append((p, c))
    with fm.context_for(sc, max_slots=16) as ctx:
        plans, committed, _ = ctx.plan_fcfs(sc.requests)
        st = ctx.stats()
    _log(f"[fcfs batch] stats {st}")
    for q, ((p, c), b, cb) in enumerate(zip(seq, plans, committed)):
        assert p.status == b.status and p.n_points == b.n_points, q
        assert np.array_equal(p.points(), b.points()) and np.array_equal(p.actions(), b.actions()), q
        assert np.array_equal(p.values(), b.values()), q
        assert c == cb, q
    assert _separation_violations(sc, plans, committed) == 0
    assert committed.sum() >= sc.requests.n // 2


def test_serving_arrivals_equal_sequential(fm):
    """Poisson arrivals (admitted as they arrive, planned while others are in
    flight) give bitwise the sequential result; acceptance follows arrival."""
    sc = S.large_actions(seed=13, n_plans=400, n_requests=40)
    seq = []
    with fm.context_for(sc) as ctx:
        for q in range(sc.requests.n):
            p = ctx.plan_request(sc.requests.origin[q], sc.requests.goal[q], 0)
            seq.append((p, ctx.commit_plan(p) if p.status == 0 else False))
    arr = S.serving_arrivals(400.0, sc.requests.n, seed=5)
    with fm.context_for(sc, max_slots=32, steps_per_launch=64) as ctx:
        plans, committed, done = ctx.plan_fcfs(sc.requests, arrival_s=arr)
    for q, ((p, c), b, cb) in enumerate(zip(seq, plans, committed)):
        assert p.status == b.status and np.array_equal(p.points(), b.points()), q
        assert c == cb, q
    assert np.all(done >= arr) and np.all(np.diff(done) >= 0)


def test_fcfs_then_checkpoint(fm, tmp_path):
    """After a concurrent batch the table holds exactly the accepted plans
    (withdrawn tentative entries are not saved) and planning continues
    identically from a reloaded checkpoint."""
    sc = S.large_actions(seed=14, n_plans=300, n_requests=30)
    path = str(tmp_path / "t.bin")
    with fm.context_for(sc, max_slots=30) as ctx:
        plans, committed, _ = ctx.plan_fcfs(sc.requests, limit=25)
        assert ctx.n_plans == sc.plans.n + int(committed.sum())
        ctx.save_table(path)
        nxt = ctx.plan_request(sc.requests.origin[27], sc.requests.goal[27], 0)
    live = int(sc.plans.length.sum()) + sum(p.n_points for p, c in zip(plans, committed) if c)
    import struct
    with open(path, "rb") as f:
        f.read(8)
        rows, cap, n_plans = struct.unpack("3i", f.read(12))
        counts = np.frombuffer(f.read(4 * rows), dtype=np.int32)
    assert int(counts.sum()) == live and n_plans == sc.plans.n + int(committed.sum())
    with fm.Context(sc.cfg) as ctx2:
        ctx2.load_table(path)
        again = ctx2.plan_request(sc.requests.origin[27], sc.requests.goal[27], 0)
    assert nxt.n_points == again.n_points and np.array_equal(nxt.points(), again.points())
