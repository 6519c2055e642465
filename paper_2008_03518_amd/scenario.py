"""Seeded synthetic workloads for FCFS pre-departure planning.

This module only draws inputs: the airspace box, the action set, the known
flight plans (straight, level, constant-speed tracks sampled every ``dt``),
the terrain heightmap (sum of Gaussian hills) and the stream of requests
(aircraft id, source, destination), as in the paper's problem statement
(Sec. I and Sec. V).  It holds none of the planner's arithmetic: no value,
no discount, no argmax.  Both the FP64 CPU oracle and the HIP library read
exactly these arrays.

The paper's own scenario (vertiports, terrain peaks, its accepted-plan file)
was never published, so every workload is synthetic; the recipe of each
preset is stated in its docstring.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Plan-outcome codes shared by the tests' bookkeeping (the numbers are a data
# convention: each side defines them itself).
STATUS_NAMES = {
    0: "OK",
    1: "REJECT_SEPARATION",
    2: "REJECT_TERRAIN",
    3: "REJECT_ORIGIN",
    4: "TIMEOUT",
    5: "NO_VALID_ACTION",
}


@dataclasses.dataclass
class Config:
    """Problem constants (peak tuples of Sec. III, action set, table sizes)."""

    box_min: tuple = (0.0, 0.0, 0.0)
    box_max: tuple = (10000.0, 10000.0, 1000.0)
    dt: float = 1.0
    gamma: float = 0.99          # goal (positive peak) discount
    r_goal: float = 1.0          # goal reward
    r_intr: float = 1.0          # intruder risk-well magnitude
    R_intr: float = 150.0        # intruder risk-well radius [m]
    gamma_intr: float = 0.99     # intruder risk-well discount
    R_sep: float = 150.0         # separation radius checked at commit [m]
    r_terr: float = 1.0          # terrain risk-well magnitude
    R_terr: float = 150.0        # terrain clearance radius [m]
    gamma_terr: float = 0.99     # terrain risk-well discount
    n_head: int = 9
    climb: tuple = (-5.0, 0.0, 5.0)        # m/s
    speed: tuple = (20.0, 30.0, 40.0)      # m/s
    max_steps: int = 3600        # steps per request (trajectory <= max_steps+1 points)
    plan_capacity: int = 4096    # plans per time row
    max_rows: int = 3601         # time rows in the table
    lookahead: int = 1           # steps W of the scoring window (Alg. 1 forward projections)
    range_query: int = 0         # 1: sweep only the plans within reach of the state (exact)
    peak_growth: float = 10.0    # co-simulated batch: peak radius R_intr + peak_growth * tau [m/s]

    @property
    def n_climb(self) -> int:
        return len(self.climb)

    @property
    def n_speed(self) -> int:
        return len(self.speed)

    @property
    def n_actions(self) -> int:
        return self.n_head * self.n_climb * self.n_speed

    @property
    def ell(self) -> float:
        """Metres covered per step at the fastest action speed."""
        return max(self.speed) * self.dt


@dataclasses.dataclass
class Terrain:
    nx: int
    ny: int
    h: np.ndarray        # float32 [ny, nx]; h[j, i] is the height at (x0 + i*cell, y0 + j*cell)
    x0: float
    y0: float
    cell: float
    hills: np.ndarray    # float64 [K, 4]: (cx, cy, amplitude, sigma), for the generator's own checks


@dataclasses.dataclass
class Plans:
    t0: np.ndarray       # int32 [n]
    length: np.ndarray   # int32 [n]
    xyz: np.ndarray      # float32 [sum(length), 3], plan-major

    @property
    def n(self) -> int:
        return int(self.t0.shape[0])

    def points(self, j: int) -> np.ndarray:
        off = int(self.length[:j].sum())
        return self.xyz[off: off + int(self.length[j])]

    def offsets(self) -> np.ndarray:
        off = np.zeros(self.n + 1, dtype=np.int64)
        np.cumsum(self.length, out=off[1:])
        return off


@dataclasses.dataclass
class Requests:
    ident: np.ndarray    # uint64 [m]
    origin: np.ndarray   # float64 [m, 3]
    goal: np.ndarray     # float64 [m, 3]
    t0: np.ndarray       # int32 [m]
    arrival_s: Optional[np.ndarray] = None   # float64 [m] scheduled arrival (serving only)

    @property
    def n(self) -> int:
        return int(self.t0.shape[0])


@dataclasses.dataclass
class Scenario:
    name: str
    cfg: Config
    plans: Plans
    requests: Requests
    terrain: Optional[Terrain] = None
    seed: int = 0


# ---------------------------------------------------------------------------
# drawing helpers
# ---------------------------------------------------------------------------

def _hill_height(hills: np.ndarray, x, y):
    """Analytic height of the summed Gaussian hills (generator-side only)."""
    x = np.asarray(x, dtype=np.float64)[..., None]
    y = np.asarray(y, dtype=np.float64)[..., None]
    cx, cy, amp, sig = hills[:, 0], hills[:, 1], hills[:, 2], hills[:, 3]
    r2 = (x - cx) ** 2 + (y - cy) ** 2
    return (amp * np.exp(-r2 / (2.0 * sig * sig))).sum(axis=-1)


def make_terrain(rng: np.random.Generator, cfg: Config, n: int = 256, k_hills: int = 50,
                 amp=(50.0, 600.0), sigma=(500.0, 3000.0)) -> Terrain:
    """n x n FP32 heightmap of k summed Gaussian hills spanning the box."""
    lo, hi = np.asarray(cfg.box_min), np.asarray(cfg.box_max)
    cx = rng.uniform(lo[0], hi[0], k_hills)
    cy = rng.uniform(lo[1], hi[1], k_hills)
    a = rng.uniform(amp[0], amp[1], k_hills)
    s = rng.uniform(sigma[0], sigma[1], k_hills)
    hills = np.stack([cx, cy, a, s], axis=1)
    cell = (hi[0] - lo[0]) / (n - 1)
    xs = lo[0] + cell * np.arange(n)
    ys = lo[1] + cell * np.arange(n)
    X, Y = np.meshgrid(xs, ys)           # [ny, nx]
    h = _hill_height(hills, X, Y).astype(np.float32)
    return Terrain(nx=n, ny=n, h=h, x0=float(lo[0]), y0=float(lo[1]), cell=float(cell), hills=hills)


def _straight_track(o: np.ndarray, e: np.ndarray, v: float, dt: float, max_pts: int) -> np.ndarray:
    """Points o + (e-o)*min(k*v*dt/D, 1), k = 0..ceil(D/(v*dt)), at most max_pts of them."""
    D = float(np.linalg.norm(e - o))
    K = int(math.ceil(D / (v * dt))) if D > 0 else 0
    k = np.arange(min(K + 1, max_pts), dtype=np.float64)
    f = np.minimum(k * v * dt / D, 1.0) if D > 0 else np.zeros_like(k)
    return o[None, :] + f[:, None] * (e - o)[None, :]


def make_known_plans(rng: np.random.Generator, cfg: Config, n: int, terrain: Optional[Terrain] = None,
                     alt=(100.0, 900.0), vel=(20.0, 40.0), terrain_margin: float = 50.0) -> Plans:
    """n straight, level, constant-speed tracks starting at t0 = 0.

    Origin and destination uniform over the square, altitude U[alt], speed
    U[vel].  With terrain, a track whose altitude is not at least
    ``terrain_margin`` above the analytic hill surface at every point is
    drawn again.
    """
    lo, hi = np.asarray(cfg.box_min), np.asarray(cfg.box_max)
    max_pts = min(cfg.max_steps + 1, cfg.max_rows)
    tracks = []
    while len(tracks) < n:
        o = np.array([rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]), 0.0])
        e = np.array([rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]), 0.0])
        z = rng.uniform(alt[0], alt[1])
        v = rng.uniform(vel[0], vel[1])
        o[2] = e[2] = z
        pts = _straight_track(o, e, v, cfg.dt, max_pts)
        if terrain is not None:
            hz = _hill_height(terrain.hills, pts[:, 0], pts[:, 1])
            if np.any(pts[:, 2] < hz + terrain_margin):
                continue
        tracks.append(pts)
    length = np.array([len(p) for p in tracks], dtype=np.int32)
    xyz = np.concatenate(tracks, axis=0).astype(np.float32)
    return Plans(t0=np.zeros(n, dtype=np.int32), length=length, xyz=xyz)


def make_requests(rng: np.random.Generator, cfg: Config, m: int, plans: Plans,
                  terrain: Optional[Terrain] = None, alt=(100.0, 900.0),
                  terrain_margin: float = 150.0, t0: int = 0,
                  arrival_s: Optional[np.ndarray] = None) -> Requests:
    """m requests (id, source, destination), departure row ``t0``.

    Source and destination are uniform over the square with altitude U[alt]
    each.  A source closer than ``R_sep`` (3-D) to a known plan's point at
    the departure row is drawn again; with terrain, sources and destinations
    lower than ``terrain_margin`` above the analytic hill surface are drawn
    again.
    """
    lo, hi = np.asarray(cfg.box_min), np.asarray(cfg.box_max)
    off = plans.offsets()
    # positions of the known plans at the departure row (plain indexing, no method arithmetic)
    act = [(off[j] + (t0 - plans.t0[j])) for j in range(plans.n)
           if plans.t0[j] <= t0 < plans.t0[j] + plans.length[j]]
    at_t0 = plans.xyz[np.asarray(act, dtype=np.int64)].astype(np.float64) if act else np.zeros((0, 3))

    def draw_point(check_plans: bool) -> np.ndarray:
        while True:
            p = np.array([rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]), rng.uniform(alt[0], alt[1])])
            if terrain is not None:
                if p[2] < float(_hill_height(terrain.hills, p[0], p[1])) + terrain_margin:
                    continue
            if check_plans and at_t0.shape[0]:
                if np.min(np.sum((at_t0 - p[None, :]) ** 2, axis=1)) < cfg.R_sep ** 2:
                    continue
            return p

    origin = np.zeros((m, 3))
    goal = np.zeros((m, 3))
    for k in range(m):
        origin[k] = draw_point(True)
        goal[k] = draw_point(False)
    return Requests(ident=np.arange(1, m + 1, dtype=np.uint64), origin=origin, goal=goal,
                    t0=np.full(m, t0, dtype=np.int32), arrival_s=arrival_s)


# ---------------------------------------------------------------------------
# presets
# ---------------------------------------------------------------------------

def cfg_small() -> Config:
    """10 x 10 x 1 km, dt 1 s, 81 actions (9 headings x 3 climbs x 3 speeds)."""
    return Config(box_min=(0.0, 0.0, 0.0), box_max=(10000.0, 10000.0, 1000.0), dt=1.0,
                  n_head=9, climb=(-5.0, 0.0, 5.0), speed=(20.0, 30.0, 40.0),
                  max_steps=3600, plan_capacity=256, max_rows=3601)


def cfg_paper_scale() -> Config:
    """30 x 30 x 1.5 km, dt 1 s, 81 actions, terrain."""
    return Config(box_min=(0.0, 0.0, 0.0), box_max=(30000.0, 30000.0, 1500.0), dt=1.0,
                  n_head=9, climb=(-5.0, 0.0, 5.0), speed=(20.0, 30.0, 40.0),
                  max_steps=3600, plan_capacity=2304, max_rows=3601)


def cfg_large_actions() -> Config:
    """30 x 30 x 1.5 km, dt 0.5 s, 360 actions (24 headings x 5 climbs x 3 speeds)."""
    return Config(box_min=(0.0, 0.0, 0.0), box_max=(30000.0, 30000.0, 1500.0), dt=0.5,
                  n_head=24, climb=(-5.0, -2.5, 0.0, 2.5, 5.0), speed=(20.0, 30.0, 40.0),
                  max_steps=3600, plan_capacity=4096, max_rows=3601)


def small(seed: int = 0, n_plans: int = 50, n_requests: int = 1) -> Scenario:
    """50 known plans in a 10 x 10 x 1 km box, one request (seed 0)."""
    cfg = cfg_small()
    rng = np.random.default_rng(seed)
    plans = make_known_plans(rng, cfg, n_plans)
    req = make_requests(rng, cfg, n_requests, plans)
    return Scenario("small-50plans-81actions", cfg, plans, req, None, seed)


def paper_scale(seed: int = 1, n_plans: int = 2000, n_requests: int = 200) -> Scenario:
    """2000 known plans, 256 x 256 terrain of 50 hills, 200 FCFS requests (seed 1)."""
    cfg = cfg_paper_scale()
    cfg.plan_capacity = max(cfg.plan_capacity, (n_plans + n_requests + 64 + 3) // 4 * 4)
    rng = np.random.default_rng(seed)
    terrain = make_terrain(rng, cfg)
    plans = make_known_plans(rng, cfg, n_plans, terrain)
    req = make_requests(rng, cfg, n_requests, plans, terrain)
    return Scenario("paper-scale-2000plans-terrain", cfg, plans, req, terrain, seed)


def large_actions(seed: int = 2, n_plans: int = 3000, n_requests: int = 1000) -> Scenario:
    """3000 known plans, 360 actions, dt 0.5 s, 1000 FCFS requests (seed 2)."""
    cfg = cfg_large_actions()
    cfg.plan_capacity = max(cfg.plan_capacity, (n_plans + n_requests + 64 + 3) // 4 * 4)
    rng = np.random.default_rng(seed)
    plans = make_known_plans(rng, cfg, n_plans)
    req = make_requests(rng, cfg, n_requests, plans)
    return Scenario("3000plans-360actions", cfg, plans, req, None, seed)


def serving_arrivals(rate_hz: float, n: int, seed: int = 3) -> np.ndarray:
    """Poisson arrival times [s] at ``rate_hz`` (open loop)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))


PRESETS = {
    "small": small,
    "paper_scale": paper_scale,
    "large_actions": large_actions,
}
