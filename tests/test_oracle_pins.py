"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage it rests on.  None re-derives the oracle's own
expression for the value: the expected numbers come from the paper's worked
risk-well example, from brute-force value iteration, from geometry built so
that distances are known exactly, from invariances, or from a second
formulation (nearest-plan distance via a library distance routine).
"""
import json
import math
import os
import sys

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle.oracle import Oracle, action_index, run_fcfs
from oracle.vi import greedy_chain, value_iteration_chain
from paper_2008_03518_amd import scenario as S

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import fp32_rounding_bound, separation_report, stored  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def line_cfg(**kw):
    """1-D chain along x: two headings (towards / away from the goal), one speed."""
    base = dict(box_min=(-100.0, -1.0, -1.0), box_max=(100.0, 1.0, 1.0), dt=1.0, n_head=2,
                climb=(0.0,), speed=(1.0,), max_steps=1000, plan_capacity=64, max_rows=2048)
    base.update(kw)
    return S.Config(**base)


def parked(x, n_rows=2048):
    """A plan that sits at point x for rows 0..n_rows-1."""
    return np.repeat(np.asarray(x, dtype=np.float32)[None, :], n_rows, axis=0)


# ---------------------------------------------------------------------------
# Fig. "riskwell": the worked risk well -2 * 0.7^|x-5| * (2 < x < 8)
# ---------------------------------------------------------------------------
def test_riskwell_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "riskwell.json")))
    w = g["well"]
    cfg = line_cfg(r_goal=0.0, r_intr=w["magnitude"], gamma_intr=w["decay"], R_intr=w["radius"], R_sep=w["radius"])
    orc = Oracle(cfg)
    orc.add_plan(0, parked([w["center"], 0.0, 0.0]))
    for p in g["points"]:
        # from x-1 the action towards a far goal at +x lands on x
        r = orc.eval_step([p["x"] - 1.0, 0.0, 0.0], [90.0, 0.0, 0.0], 0)
        assert r["V"][0] == pytest.approx(p["value"], abs=1e-12), p


# ---------------------------------------------------------------------------
# Sec. II / III: value iteration on a tiny chain; FastMDP is exact with one
# positive reward and no wells.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("gamma,goal,n", [(0.9, 7, 12), (0.99, 0, 9), (0.5, 10, 11)])
def test_value_iteration_chain(gamma, goal, n):
    cfg = line_cfg(box_min=(0.0, -0.5, -0.5), box_max=(n - 1.0, 0.5, 0.5), gamma=gamma)
    orc = Oracle(cfg)
    Vvi = value_iteration_chain(n, goal, 1.0, gamma)
    for x in range(n):
        if x == goal:
            continue
        r = orc.eval_step([float(x), 0.0, 0.0], [float(goal), 0.0, 0.0], 0)
        toward = 1 if goal > x else -1
        for a, mv in ((0, toward), (1, -toward)):       # heading 0 points at the goal
            y = x + mv
            if 0 <= y < n:
                assert r["V"][a] == pytest.approx(Vvi[y], rel=1e-12, abs=1e-300)
            else:
                assert r["V"][a] == -np.inf
        mv_best = toward if r["best"] == 0 else -toward
        assert mv_best == greedy_chain(Vvi, x)


# ---------------------------------------------------------------------------
# No intruders: straight track to the goal, closed-form step count and value.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mk", [S.cfg_small, S.cfg_large_actions])
@pytest.mark.parametrize("o,g", [((1000.0, 2000.0, 500.0), (8000.0, 6500.0, 500.0)),
                                 ((1000.0, 5000.0, 300.0), (9030.0, 5000.0, 300.0))])
def test_no_intruder_straight_level_track(mk, o, g):
    """Capture within one step of the goal (ell): ceil(D/ell - 1) straight moves."""
    cfg = mk()
    orc = Oracle(cfg)
    o, g = np.array(o), np.array(g)
    D = float(np.linalg.norm(g - o))
    ell = max(cfg.speed) * cfg.dt
    p = orc.plan(o, g, 0)
    assert p.status == 0
    steps = p.n_points - 1
    assert steps == max(0, math.ceil(D / ell - 1.0))
    straight = action_index(cfg, 0, list(cfg.climb).index(0.0), len(cfg.speed) - 1)
    assert np.all(p.action[1:] == straight)
    u = (g - o) / D
    rel = p.xyz - o[None, :]
    cross = rel - np.outer(rel @ u, u)
    assert np.max(np.abs(cross)) < 1e-6
    # progress is one full step per move, and the value is the goal reward
    # discounted by the remaining distance in steps
    k = np.arange(1, p.n_points)
    assert np.allclose(rel[1:] @ u, k * ell, atol=1e-6)
    assert np.allclose(p.value[1:], cfg.r_goal * cfg.gamma ** ((D - k * ell) / ell), rtol=1e-12)
    assert np.linalg.norm(g - p.xyz[-1]) <= ell


def test_no_intruder_climbing_track_is_vertical_plane():
    cfg = S.cfg_small()
    orc = Oracle(cfg)
    o = np.array([500.0, 9000.0, 150.0])
    g = np.array([9500.0, 1000.0, 850.0])
    p = orc.plan(o, g, 0)
    assert p.status == 0
    u = (g - o)[:2] / np.linalg.norm((g - o)[:2])
    rel = p.xyz[:, :2] - o[None, :2]
    cross = rel[:, 0] * u[1] - rel[:, 1] * u[0]
    assert np.max(np.abs(cross)) < 1e-6
    d = np.linalg.norm(p.xyz - g[None, :], axis=1)
    assert np.all(np.diff(d) < 0)
    assert d[-1] <= max(cfg.speed) * cfg.dt


def test_step_displacements_follow_the_action_set():
    """Each move covers one of the speeds times dt horizontally and one of the
    climb rates times dt vertically (dt = 0.5 s, 360 actions)."""
    sc = S.large_actions(seed=7, n_plans=300, n_requests=2)
    cfg = sc.cfg
    orc = Oracle(cfg, sc.plans)
    for k in range(2):
        p = orc.plan(sc.requests.origin[k], sc.requests.goal[k], 0)
        assert p.n_points > 50
        d = np.diff(p.xyz, axis=0)
        hz = np.hypot(d[:, 0], d[:, 1])
        sp = np.array(cfg.speed) * cfg.dt
        cl = np.array(cfg.climb) * cfg.dt
        assert np.all(np.min(np.abs(hz[:, None] - sp[None, :]), axis=1) < 1e-9)
        assert np.all(np.min(np.abs(d[:, 2][:, None] - cl[None, :]), axis=1) < 1e-9)
        v_idx = p.action[1:] % len(cfg.speed)
        c_idx = (p.action[1:] // len(cfg.speed)) % len(cfg.climb)
        assert np.allclose(hz, sp[v_idx], atol=1e-9) and np.allclose(d[:, 2], cl[c_idx], atol=1e-9)


# ---------------------------------------------------------------------------
# Per-peak maximum versus nearest-plan distance (the two formulations of the
# intruder term agree because gamma^d is decreasing in d).
# ---------------------------------------------------------------------------
def _successors(cfg, s, g):
    beta = math.atan2(g[1] - s[1], g[0] - s[0])
    out = []
    for h in range(cfg.n_head):
        th = beta + 2.0 * math.pi * h / cfg.n_head
        for c in cfg.climb:
            for v in cfg.speed:
                out.append([s[0] + v * cfg.dt * math.cos(th), s[1] + v * cfg.dt * math.sin(th), s[2] + c * cfg.dt])
    return np.array(out)


def _active_points(plans, row, extra=()):
    off = plans.offsets()
    pts = [plans.xyz[off[j] + row - plans.t0[j]] for j in range(plans.n)
           if plans.t0[j] <= row < plans.t0[j] + plans.length[j]]
    pts += [x[row - t0] for (t0, x) in extra if t0 <= row < t0 + len(x)]
    return np.asarray(pts, dtype=np.float64).reshape(-1, 3)


def test_intruder_term_equals_nearest_plan_well():
    sc = S.small(seed=0, n_plans=200)
    cfg = sc.cfg
    orc = Oracle(cfg, sc.plans)
    ell = cfg.ell
    rng = np.random.default_rng(5)
    n_in = 0
    for trial in range(60):
        t = int(rng.integers(0, 200))
        pts = _active_points(sc.plans, t + 1)
        # put the state next to an active plan so that some wells are hit
        s = pts[rng.integers(len(pts))] + rng.uniform(-120, 120, 3) * np.array([1, 1, 0.5])
        g = np.array([rng.uniform(0, 1e4), rng.uniform(0, 1e4), rng.uniform(100, 900)])
        r = orc.eval_step(s, g, t)
        sp = _successors(cfg, s, g)
        dmin = cdist(sp, pts).min(axis=1)
        expect = np.where(dmin < cfg.R_intr, cfg.r_intr * cfg.gamma_intr ** (dmin / ell), 0.0)
        assert np.allclose(r["dmin"], dmin, rtol=1e-12, atol=1e-9)
        assert np.allclose(r["I"], expect, rtol=1e-12, atol=0.0)
        n_in += int(np.sum(expect > 0))
    assert n_in > 100


# ---------------------------------------------------------------------------
# Invariances: plan order, mirror symmetry.
# ---------------------------------------------------------------------------
def test_permutation_invariance():
    sc = S.small(seed=0, n_plans=120)
    orc1 = Oracle(sc.cfg, sc.plans)
    perm = np.random.default_rng(1).permutation(sc.plans.n)
    off = sc.plans.offsets()
    orc2 = Oracle(sc.cfg)
    for j in perm:
        orc2.add_plan(int(sc.plans.t0[j]), sc.plans.xyz[off[j]:off[j + 1]])
    p = orc1.plan(sc.requests.origin[0], sc.requests.goal[0], 0)
    for k in range(0, p.n_points - 1, 7):
        a = orc1.eval_step(p.xyz[k], sc.requests.goal[0], k)
        b = orc2.eval_step(p.xyz[k], sc.requests.goal[0], k)
        assert np.array_equal(a["V"], b["V"]) and a["best"] == b["best"]


def test_mirror_symmetry():
    sc = S.small(seed=0, n_plans=150)
    cfg = sc.cfg
    L = cfg.box_max[0]
    # snap x to multiples of 1/512 so that L - x is exact in FP32 and the
    # mirrored table is the exact mirror image
    base = S.Plans(t0=sc.plans.t0.copy(), length=sc.plans.length.copy(), xyz=sc.plans.xyz.copy())
    base.xyz[:, 0] = np.round(base.xyz[:, 0] * 512.0) / 512.0
    mir = S.Plans(t0=base.t0.copy(), length=base.length.copy(), xyz=base.xyz.copy())
    mir.xyz[:, 0] = np.float32(L) - mir.xyz[:, 0]
    assert np.array_equal(np.float32(L) - mir.xyz[:, 0], base.xyz[:, 0])
    o1, o2 = Oracle(cfg, base), Oracle(cfg, mir)
    H, Cn, Sn = cfg.n_head, len(cfg.climb), len(cfg.speed)
    mirror_a = np.array([action_index(cfg, (H - h) % H, c, v) for h in range(H) for c in range(Cn) for v in range(Sn)])
    rng = np.random.default_rng(2)
    for _ in range(40):
        t = int(rng.integers(0, 150))
        s = np.array([rng.uniform(500, 9500), rng.uniform(500, 9500), rng.uniform(150, 850)])
        g = np.array([rng.uniform(0, 1e4), rng.uniform(0, 1e4), rng.uniform(100, 900)])
        sm, gm = s.copy(), g.copy()
        sm[0], gm[0] = L - s[0], L - g[0]
        a = o1.eval_step(s, g, t)
        b = o2.eval_step(sm, gm, t)
        fin = np.isfinite(a["V"])
        assert np.array_equal(fin, np.isfinite(b["V"][mirror_a]))
        assert np.allclose(a["V"][fin], b["V"][mirror_a][fin], rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------------------
# Hand case: one plan parked 185 m ahead on the straight path.
# ---------------------------------------------------------------------------
def test_hand_case_detour():
    cfg = S.cfg_small()
    orc = Oracle(cfg)
    s = np.array([1000.0, 5000.0, 500.0])
    g = np.array([9000.0, 5000.0, 500.0])
    orc.add_plan(0, parked(s + [185.0, 0.0, 0.0], 64))
    r = orc.eval_step(s, g, 0)
    ell, gam = cfg.ell, cfg.gamma
    c0 = list(cfg.climb).index(0.0)
    # straight at 40 m/s lands 145 m from the plan: inside the well
    a_fast = action_index(cfg, 0, c0, 2)
    assert r["I"][a_fast] == pytest.approx(cfg.r_intr * gam ** (145.0 / ell), rel=1e-14)
    # straight at 30 m/s lands 155 m away and at 20 m/s 165 m away: outside
    assert r["I"][action_index(cfg, 0, c0, 1)] == 0.0
    assert r["I"][action_index(cfg, 0, c0, 0)] == 0.0
    # the two 40-degree headings at 40 m/s tie; the lower index (+40 deg) wins
    best = action_index(cfg, 1, c0, 2)
    assert r["best"] == best
    D, th = 8000.0, math.radians(40.0)
    Dp = math.sqrt(D * D + ell * ell - 2.0 * D * ell * math.cos(th))   # law of cosines
    assert r["V"][best] == pytest.approx(cfg.r_goal * gam ** (Dp / ell), rel=1e-12)
    assert r["V"][action_index(cfg, cfg.n_head - 1, c0, 2)] == pytest.approx(r["V"][best], rel=1e-12)
    # and its distance to the plan is 156.49 m (outside the well)
    q = np.array([ell * math.cos(th), ell * math.sin(th)])
    assert math.hypot(185.0 - q[0], q[1]) > cfg.R_intr and r["I"][best] == 0.0


# ---------------------------------------------------------------------------
# Terrain: bilinear interpolation reproduces a plane exactly, and the value
# subtracts the larger of the intruder and terrain penalties (Compute value).
# ---------------------------------------------------------------------------
def plane_terrain(a, b, c, n=17, cell=625.0):
    xs = np.arange(n) * cell
    X, Y = np.meshgrid(xs, xs)
    h = (a * X + b * Y + c).astype(np.float32)
    return S.Terrain(nx=n, ny=n, h=h, x0=0.0, y0=0.0, cell=cell, hills=np.zeros((0, 4)))


def test_terrain_plane_clearance():
    cfg = S.cfg_small()
    a, b, c = 0.0125, 0.005, 40.0     # FP32-exact plane over the grid
    ter = plane_terrain(a, b, c)
    orc = Oracle(cfg, terrain=ter)
    s = np.array([3000.0, 7000.0, 0.0])
    s[2] = a * s[0] + b * s[1] + c + 148.0
    g = np.array([3000.0, 2000.0, s[2]])
    r = orc.eval_step(s, g, 0)
    sp = _successors(cfg, s, g)
    clr = sp[:, 2] - (a * sp[:, 0] + b * sp[:, 1] + c)
    expect = np.where(clr < cfg.R_terr, cfg.r_terr * cfg.gamma_terr ** (np.maximum(clr, 0) / cfg.ell), 0.0)
    assert np.allclose(r["T"], expect, rtol=1e-12, atol=1e-12)
    assert np.any(expect > 0) and np.any(expect == 0)


# Terrain well constants (r_T, gamma_T, R_T) distinct from the intruder
# well's (Sec. III: each negative peak carries its own reward, discount and
# radius; "Process negative terrain rewards").  Hand values, 40 decimal
# digits: 2.5 * 0.95^(55/40) = 2.329753462960785240871...,
# 2.5 * 0.95^(60/40) = 2.314863656892128927874...,
# 2.5 * 0.95^(65/40) = 2.300069013821741297421...
TERRAIN_WELL_HAND = {55.0: 2.329753462960785240871, 60.0: 2.314863656892128927874,
                     65.0: 2.300069013821741297421}


def terrain_constants_cfg():
    cfg = S.cfg_small()
    cfg.r_terr, cfg.R_terr, cfg.gamma_terr = 2.5, 90.0, 0.95     # intruder well stays 1, 150 m, 0.99
    return cfg


def test_terrain_well_own_constants():
    cfg = terrain_constants_cfg()
    assert (cfg.r_intr, cfg.R_intr, cfg.gamma_intr) == (1.0, 150.0, 0.99)
    ter = plane_terrain(0.0, 0.0, 40.0)                          # flat ground at 40 m
    orc = Oracle(cfg, terrain=ter)
    g = np.array([3000.0, 2000.0, 100.0])
    # clearance 60 m at the state; climb rates -5, 0, +5 m/s over 1 s give
    # clearances 55, 60, 65 m at every heading and speed (ell = 40 m)
    r = orc.eval_step(np.array([3000.0, 7000.0, 100.0]), g, 0)
    for a in range(cfg.n_actions):
        clr = {0: 55.0, 1: 60.0, 2: 65.0}[(a // len(cfg.speed)) % len(cfg.climb)]
        assert abs(r["T"][a] - TERRAIN_WELL_HAND[clr]) <= 1e-14 * TERRAIN_WELL_HAND[clr]
        assert r["I"][a] == 0.0
        assert r["V"][a] == r["G"][a] - r["T"][a]
    # clearances 125-135 m: outside R_T = 90 m (inside the intruder radius 150 m)
    r = orc.eval_step(np.array([3000.0, 7000.0, 170.0]), g, 0)
    assert np.all(r["T"] == 0.0)
    # below the surface: the well's full magnitude r_T (gamma_T^0)
    r = orc.eval_step(np.array([3000.0, 7000.0, 38.0]), g, 0)
    assert np.all(r["T"][[a for a in range(cfg.n_actions) if (a // 3) % 3 == 1]] == 2.5)


def test_value_subtracts_larger_penalty():
    cfg = S.cfg_small()
    ter = plane_terrain(0.0, 0.0, 400.0)
    orc = Oracle(cfg, terrain=ter)
    s = np.array([5000.0, 5000.0, 500.0])          # 100 m above flat ground
    g = np.array([9000.0, 5000.0, 500.0])
    orc.add_plan(0, parked(s + [40.0, 0.0, 60.0], 64))   # 60 m above the straight successor
    r = orc.eval_step(s, g, 0)
    c0 = list(cfg.climb).index(0.0)
    a = action_index(cfg, 0, c0, 2)                 # lands 100 m above ground, 60 m from the plan
    Iv = cfg.gamma_intr ** (60.0 / cfg.ell)
    Tv = cfg.gamma_terr ** (100.0 / cfg.ell)
    assert r["I"][a] == pytest.approx(Iv, rel=1e-13) and r["T"][a] == pytest.approx(Tv, rel=1e-13)
    assert r["V"][a] == pytest.approx(r["G"][a] - max(Iv, Tv), rel=1e-12)
    assert r["V"][a] != pytest.approx(r["G"][a] - Iv - Tv, rel=1e-6)


# ---------------------------------------------------------------------------
# Outcomes (Sec. V): stop at the first collision; only collision-free plans
# are accepted.
# ---------------------------------------------------------------------------
def test_reject_separation_when_every_action_is_in_a_well():
    cfg = S.cfg_small()
    orc = Oracle(cfg)
    o = np.array([5000.0, 5000.0, 500.0])
    x = np.repeat(o[None, :], 64, axis=0)
    x[0] += [0.0, 0.0, 400.0]                       # away at row 0, parked on the origin from row 1
    orc.add_plan(0, x)
    p = orc.plan(o, [9000.0, 5000.0, 500.0], 0)
    assert p.status == 1 and p.n_points == 2


def test_reject_origin():
    cfg = S.cfg_small()
    orc = Oracle(cfg)
    o = np.array([5000.0, 5000.0, 500.0])
    orc.add_plan(0, parked(o + [100.0, 0.0, 0.0], 8))
    p = orc.plan(o, [9000.0, 5000.0, 500.0], 0)
    assert p.status == 3 and p.n_points == 1


def test_timeout_and_no_valid_action():
    cfg = S.cfg_small()
    cfg.max_steps = 5
    p = Oracle(cfg).plan([1000.0, 1000.0, 500.0], [9000.0, 9000.0, 500.0], 0)
    assert p.status == 4 and p.n_points == 6
    tiny = S.cfg_small()
    tiny.box_min, tiny.box_max = (0.0, 0.0, 0.0), (10.0, 10.0, 1000.0)
    p = Oracle(tiny).plan([5.0, 5.0, 500.0], [9.0, 9.0, 900.0], 0)
    assert p.status == 5 and p.n_points == 1


def test_reject_terrain():
    cfg = S.cfg_small()
    cfg.climb = (-5.0,)
    ter = plane_terrain(0.0, 0.0, 497.0)
    p = Oracle(cfg, terrain=ter).plan([5000.0, 5000.0, 500.0], [9000.0, 5000.0, 500.0], 0)
    assert p.status == 2 and p.n_points == 2


def test_commit_validates_and_appends():
    cfg = S.cfg_small()
    orc = Oracle(cfg)
    base = parked([5000.0, 5000.0, 500.0], 30)
    orc.add_plan(0, base)
    near = np.repeat(np.array([[5100.0, 5000.0, 500.0]]), 10, axis=0)
    assert orc.commit(5, near) is False and orc.n_plans == 1
    assert orc.commit(31, near) is True and orc.n_plans == 2     # after the parked plan ends
    far = np.repeat(np.array([[5151.0, 5000.0, 500.0]]), 10, axis=0)
    assert orc.commit(0, far) is True and orc.n_plans == 3       # 151 m from the parked plan
    assert orc.commit(28, far) is False and orc.n_plans == 3     # 51 m from the plan committed at row 31
    far2 = np.repeat(np.array([[5000.0, 5000.0, 650.5]]), 10, axis=0)
    assert orc.commit(60, far2) is True and orc.n_plans == 4     # no plan active at rows 60..69
    assert orc.commit(0, far2 - [0.0, 0.0, 1.0]) is False         # 149.5 m above the parked plan


# ---------------------------------------------------------------------------
# Separation invariant over a first-come-first-served sequence.
# ---------------------------------------------------------------------------
def test_fcfs_separation_invariant():
    """Stored versus stored: every pair of table points at a common row, one
    of them from an accepted plan, is at least R_sep - delta apart, delta
    the FP32 rounding bound of a stored point (the invariant the GPU suite
    checks with the same function)."""
    sc = S.small(seed=3, n_plans=80, n_requests=12)
    cfg = sc.cfg
    orc = Oracle(cfg, sc.plans)
    res = run_fcfs(orc, sc.requests)
    committed = [stored(p.t0, p.xyz) for p, ok in res if ok]
    assert len(committed) >= 8
    off = sc.plans.offsets()
    known = [(int(sc.plans.t0[j]), sc.plans.xyz[off[j]:off[j + 1]]) for j in range(sc.plans.n)]
    delta = fp32_rounding_bound(cfg.box_min, cfg.box_max)
    assert 0.0 < delta < 1e-3                      # half a spacing of 10 km in FP32, two axes
    bad, gap = separation_report(known, committed, cfg.R_sep, delta)
    print(f"[separation] minimum stored gap {gap:.4f} m (bound {cfg.R_sep - delta:.4f} m)")
    assert bad == 0 and gap >= cfg.R_sep - delta
    # every rejection is a stated outcome
    for p, ok in res:
        assert ok == (p.status == 0)


def test_separation_report_finds_planted_violation():
    """The checker itself: a stored point moved to R_sep - 2 delta from a
    known plan is reported; moving it to R_sep exactly is not."""
    delta = fp32_rounding_bound((0, 0, 0), (10000.0, 10000.0, 1000.0))
    a = np.array([[5000.0, 5000.0, 500.0]] * 3)
    for shift, want in ((150.0 - 2 * delta, 1), (150.0, 0)):
        b = a + [shift, 0.0, 0.0]
        bad, gap = separation_report([(0, a)], [(0, b)], 150.0, delta)
        assert bad == 3 * want and abs(gap - shift) < 1e-9


# ---------------------------------------------------------------------------
# Lookahead window (Alg. 1: one-step and ten-step forward projections;
# "Forward project": W future points per action; "Compute value": the
# largest value along the window).  Hand values, 30 digits:
# 0.99^190.75 = 0.147032509431998899816819048270
# 0.99^40 = 0.668971758569680513938338598804
# 0.99^43 = 0.649102628368402432993856004081
# ---------------------------------------------------------------------------
def _window_cfg(W):
    cfg = S.cfg_small()
    cfg.lookahead = W
    return cfg


def test_lookahead_no_intruder_straight_value():
    """No plans: the straight, level, fastest action's farthest window point
    is W * ell nearer the goal, so its value is r * gamma^(D/ell - W), the
    largest of all actions; the track stays straight while the goal is
    farther than the window."""
    cfg = _window_cfg(10)
    orc = Oracle(cfg)
    o, g = np.array([1000.0, 5000.0, 300.0]), np.array([9030.0, 5000.0, 300.0])   # D / ell = 200.75
    r = orc.eval_step(o, g, 0)
    straight = action_index(cfg, 0, 1, 2)
    assert r["best"] == straight
    assert abs(r["V"][straight] - 0.147032509431998899816819048270) <= 1e-14
    p = orc.plan(o, g, 0)
    assert p.status == 0
    far = p.xyz[: 180]                                   # the goal still beyond the window
    assert np.all(p.action[1:180] == straight)
    assert np.max(np.abs(far[:, 1] - 5000.0)) < 1e-9 and np.max(np.abs(far[:, 2] - 300.0)) < 1e-9
    assert np.allclose(np.diff(far[:, 0]), cfg.ell, rtol=0, atol=1e-9)


def test_lookahead_takes_the_window_maximum_at_its_own_rows():
    """A plan that appears at (1400, 5000, 300) from row 8 on (before that it
    is far away): the straight action's window points 1040 .. 1400 m meet it
    at rows 8, 9, 10 only, so its value is the goal term at w = 7,
    0.99^43 (scoring every point against row t+1 would give 0.99^40, against
    row t+w-1 0.99^42).  Without the window the same action scores its
    successor alone: 0.99^49."""
    o, g = np.array([1000.0, 5000.0, 300.0]), np.array([3000.0, 5000.0, 300.0])   # D = 2000 m = 50 ell
    rows = 40
    x = np.repeat(np.array([[9000.0, 9000.0, 900.0]], np.float32), rows, axis=0)
    x[8:] = [1400.0, 5000.0, 300.0]
    plans = S.Plans(np.zeros(1, np.int32), np.array([rows], np.int32), x)
    straight = action_index(S.cfg_small(), 0, 1, 2)
    r = Oracle(_window_cfg(10), plans).eval_step(o, g, 0)
    assert abs(r["V"][straight] - 0.649102628368402432993856004081) <= 1e-14
    assert r["I"][straight] == 0.0 and r["T"][straight] == 0.0 and r["V"][straight] == r["G"][straight]
    r1 = Oracle(_window_cfg(1), plans).eval_step(o, g, 0)
    assert abs(r1["V"][straight] - 0.99 ** 49) <= 1e-15
    # a plan parked 100 m ahead at every row: points w = 1..6 lie inside its
    # well, w = 7..10 outside, so the value is the goal term at w = 10
    parked_ahead = S.Plans(np.zeros(1, np.int32), np.array([rows], np.int32),
                           np.repeat(np.array([[1100.0, 5000.0, 300.0]], np.float32), rows, axis=0))
    r = Oracle(_window_cfg(10), parked_ahead).eval_step(o, g, 0)
    assert abs(r["V"][straight] - 0.668971758569680513938338598804) <= 1e-14
    # the chosen successor's own well decides a rejection, whatever the window
    # scored: parked 175 m ahead (the origin clear of its well), the straight
    # action still wins on its clear points w = 9, 10 and its successor lies
    # 135 m from the plan
    ahead175 = S.Plans(np.zeros(1, np.int32), np.array([rows], np.int32),
                       np.repeat(np.array([[1175.0, 5000.0, 300.0]], np.float32), rows, axis=0))
    orc = Oracle(_window_cfg(10), ahead175)
    assert orc.eval_step(o, g, 0)["best"] == straight
    p = orc.plan(o, g, 0)
    assert p.status == 1 and p.n_points == 2 and p.action[1] == straight


def test_lookahead_equals_nearest_plan_window_maximum():
    """Second formulation: window points built here, nearest plan per row by
    a library distance routine (the monotone well makes the per-peak maximum
    the nearest plan's), maximum over the window."""
    cfg = _window_cfg(6)
    sc = S.small(seed=17, n_plans=150, n_requests=1)
    orc = Oracle(cfg, sc.plans)
    off = sc.plans.offsets()
    rng = np.random.default_rng(5)
    A = cfg.n_actions
    for trial in range(6):
        j = int(rng.integers(sc.plans.n))
        t = int(rng.integers(0, max(1, int(sc.plans.length[j]) - 8)))
        s = sc.plans.xyz[off[j] + t].astype(np.float64) + rng.uniform(-200, 200, 3) * [1, 1, 0.3]
        s[2] = min(max(s[2], 50.0), 950.0)
        g = np.array([rng.uniform(0, 10000), rng.uniform(0, 10000), rng.uniform(100, 900)])
        r = orc.eval_step(s, g, t)
        beta = math.atan2(g[1] - s[1], g[0] - s[0])
        best = np.full(A, -np.inf)
        for a in range(A):
            h, c, v = a // 9, (a // 3) % 3, a % 3
            th = beta + 2 * math.pi * h / cfg.n_head
            for w in range(1, cfg.lookahead + 1):
                p = s + w * np.array([cfg.speed[v] * cfg.dt * math.cos(th), cfg.speed[v] * cfg.dt * math.sin(th),
                                      cfg.climb[c] * cfg.dt])
                inside = np.all(p >= cfg.box_min) and np.all(p <= cfg.box_max)
                if w == 1 and not inside:
                    break
                if not inside:
                    continue
                act = [k for k in range(sc.plans.n) if sc.plans.t0[k] <= t + w < sc.plans.t0[k] + sc.plans.length[k]]
                pts = np.array([sc.plans.xyz[off[k] + t + w - sc.plans.t0[k]] for k in act], np.float64)
                d = cdist(p[None, :], pts).min() if len(act) else np.inf
                well = cfg.r_intr * cfg.gamma_intr ** (d / cfg.ell) if d < cfg.R_intr else 0.0
                val = cfg.r_goal * cfg.gamma ** (np.linalg.norm(g - p) / cfg.ell) - well
                best[a] = max(best[a], val)
        fin = np.isfinite(best)
        assert np.array_equal(fin, np.isfinite(r["V"]))
        assert np.allclose(r["V"][fin], best[fin], rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------
# Range query (Sec. VII: restrict the trajectories considered to the volume
# relevant to the flight).  A plan farther than max(R_I, R_sep) + 1 m + W
# longest steps from the state is farther than the well radius from every
# point scored in the step (triangle inequality), so skipping it changes no
# value; a ball any smaller does change values near plans.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("W", [1, 4])
def test_range_query_changes_no_value(W):
    sc = S.small(seed=17, n_plans=150, n_requests=1)
    cfg = sc.cfg
    cfg.lookahead = W
    step = math.hypot(max(cfg.speed), max(abs(c) for c in cfg.climb)) * cfg.dt
    radius = max(cfg.R_intr, cfg.R_sep) + 1.0 + W * step
    full = Oracle(cfg, sc.plans)
    cut = S.Config(**{**cfg.__dict__})
    cut.range_radius = radius
    ranged = Oracle(cut, sc.plans)
    small = S.Config(**{**cfg.__dict__})
    small.range_radius = cfg.R_intr - 10.0
    too_small = Oracle(small, sc.plans)
    off = sc.plans.offsets()
    rng = np.random.default_rng(3)
    differs = 0
    for trial in range(40):
        j = int(rng.integers(sc.plans.n))
        t = int(rng.integers(0, max(1, int(sc.plans.length[j]) - 6)))
        s = sc.plans.xyz[off[j] + t].astype(np.float64) + rng.uniform(-220, 220, 3) * [1, 1, 0.3]
        s[2] = min(max(s[2], 50.0), 950.0)
        g = np.array([rng.uniform(0, 10000), rng.uniform(0, 10000), rng.uniform(100, 900)])
        a, b = full.eval_step(s, g, t), ranged.eval_step(s, g, t)
        for k in ("V", "G", "I", "T"):
            assert np.array_equal(a[k], b[k]), (trial, k)
        assert a["best"] == b["best"]
        c = too_small.eval_step(s, g, t)
        differs += int(not np.array_equal(a["I"], c["I"]))
    assert differs > 5


# ---------------------------------------------------------------------------
# Co-simulated batch (Sec. V; Table "Peaks created in the environment": five
# risk wells per other aircraft at p + v*tau, tau in {-5, 0, 5, 10, 15} s,
# radius R + 10*tau; "Build peaks"; "Process negative rewards").
# ---------------------------------------------------------------------------
def test_batch_of_one_is_the_single_plan():
    sc = S.small(seed=5, n_plans=120, n_requests=3)
    orc = Oracle(sc.cfg, sc.plans)
    for q in range(3):
        p = orc.plan(sc.requests.origin[q], sc.requests.goal[q], 0)
        b = orc.plan_batch(sc.requests.origin[q:q + 1], sc.requests.goal[q:q + 1], 0)[0]
        assert b.status == p.status and np.array_equal(b.xyz, p.xyz) and np.array_equal(b.action, p.action)
        assert np.array_equal(b.value, p.value)


def test_batch_head_on_pair():
    """Two aircraft fly head-on along y = 5000 m (origins 2 km apart, each
    one's goal the other's origin, no known plans).  Both fly straight until
    the other's tau = 15 s peak -- 600 m ahead of it, radius 150 + 150 =
    300 m -- reaches the straight successor: with both at 40 m/s that gap is
    2000 - 600 - 40 - 80k m at step k, first below 300 m at k = 14, so
    points 1..14 are straight and point 15 turns away.  Every later point
    mirrors the other aircraft's through the midpoint (the action set is
    relative to the goal bearing, so the pair is point-symmetric)."""
    cfg = S.cfg_small()
    o = np.array([[1000.0, 5000.0, 300.0], [3000.0, 5000.0, 300.0]])
    g = o[::-1].copy()
    a, b = Oracle(cfg).plan_batch(o, g, 0)
    assert np.allclose(a.xyz[:15, 0], 1000.0 + 40.0 * np.arange(15), rtol=0, atol=1e-9)
    assert np.max(np.abs(a.xyz[:15, 1] - 5000.0)) < 1e-9
    assert abs(a.xyz[15, 1] - 5000.0) > 1.0
    n = min(a.n_points, b.n_points)
    mid = np.array([2000.0, 5000.0, 300.0])
    assert np.allclose(a.xyz[:n, :2] - mid[:2], -(b.xyz[:n, :2] - mid[:2]), rtol=0, atol=1e-6)
    assert a.status == b.status == 0 and a.n_points == b.n_points
    # they keep R_sep apart at every common row
    assert np.min(np.linalg.norm(a.xyz[:n] - b.xyz[:n], axis=1)) >= cfg.R_sep
    # without each other (planned alone) both fly the straight track
    solo = Oracle(cfg).plan(o[0], g[0], 0)
    assert np.max(np.abs(solo.xyz[:, 1] - 5000.0)) < 1e-9


def test_batch_far_apart_equals_solo():
    """Aircraft whose tracks stay kilometres apart do not see each other's
    wells: each batch plan equals the plan of the aircraft alone."""
    cfg = S.cfg_small()
    o = np.array([[1000.0, 1000.0, 300.0], [1000.0, 9000.0, 300.0]])
    g = np.array([[9000.0, 1000.0, 300.0], [9000.0, 9000.0, 300.0]])
    orc = Oracle(cfg)
    batch = orc.plan_batch(o, g, 0)
    for i in range(2):
        solo = orc.plan(o[i], g[i], 0)
        assert np.array_equal(batch[i].xyz, solo.xyz) and batch[i].status == solo.status
