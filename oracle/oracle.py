"""ctypes wrapper of the FP64 CPU oracle (``fastmdp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  The HIP product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fastmdp_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

MAX_ACT_DIM = 32
TIE_REL = 1e-9        # argmax tie band (relative to the maximum value)
AMB_BAND = 1e-3       # metres: a distance this close to a radius is boundary-ambiguous


def build(openmp: bool = True) -> str:
    """Compile the oracle (plain C, -O3, no fast-math) into liboracle.so."""
    cmd = ["gcc", "-O3", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-fno-fast-math", SRC, "-o", LIB + ".tmp", "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Cfg(C.Structure):
    _fields_ = [
        ("box_min", C.c_double * 3), ("box_max", C.c_double * 3),
        ("dt", C.c_double),
        ("gamma", C.c_double), ("r_goal", C.c_double),
        ("r_intr", C.c_double), ("R_intr", C.c_double), ("gamma_intr", C.c_double),
        ("R_sep", C.c_double),
        ("r_terr", C.c_double), ("R_terr", C.c_double), ("gamma_terr", C.c_double),
        ("n_head", C.c_int32), ("n_climb", C.c_int32), ("n_speed", C.c_int32),
        ("climb", C.c_double * MAX_ACT_DIM), ("speed", C.c_double * MAX_ACT_DIM),
        ("max_steps", C.c_int32),
        ("tie_rel", C.c_double),
        ("amb_band", C.c_double),
        ("lookahead", C.c_int32),
        ("range_radius", C.c_double),
        ("peak_growth", C.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = C.CDLL(LIB)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        fp = C.POINTER(C.c_float)
        lib.orc_create.argtypes = [C.POINTER(_Cfg), C.POINTER(P)]
        lib.orc_destroy.argtypes = [P]
        lib.orc_destroy.restype = None
        lib.orc_add_plan.argtypes = [P, C.c_int32, C.c_int32, fp]
        lib.orc_num_plans.argtypes = [P]
        lib.orc_set_terrain.argtypes = [P, C.c_int32, C.c_int32, fp, C.c_double, C.c_double, C.c_double]
        lib.orc_eval_step.argtypes = [P, dp, dp, C.c_int32, dp, dp, dp, dp, dp, ip, ip]
        lib.orc_plan.argtypes = [P, dp, dp, C.c_int32, C.c_int32, dp, ip, dp, ip, ip]
        lib.orc_commit.argtypes = [P, C.c_int32, C.c_int32, dp]
        lib.orc_plan_batch.argtypes = [P, C.c_int32, dp, dp, C.c_int32, C.c_int32, dp, ip, dp, ip, ip]
        lib.orc_num_threads.argtypes = []
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def make_cfg(cfg) -> _Cfg:
    """Translate a scenario Config (or any object with the same fields)."""
    c = _Cfg()
    for k in range(3):
        c.box_min[k] = float(cfg.box_min[k])
        c.box_max[k] = float(cfg.box_max[k])
    for name in ("dt", "gamma", "r_goal", "r_intr", "R_intr", "gamma_intr", "R_sep",
                 "r_terr", "R_terr", "gamma_terr"):
        setattr(c, name, float(getattr(cfg, name)))
    c.n_head = int(cfg.n_head)
    c.n_climb = len(cfg.climb)
    c.n_speed = len(cfg.speed)
    for i, v in enumerate(cfg.climb):
        c.climb[i] = float(v)
    for i, v in enumerate(cfg.speed):
        c.speed[i] = float(v)
    c.max_steps = int(cfg.max_steps)
    c.tie_rel = float(getattr(cfg, "tie_rel", TIE_REL))
    c.amb_band = float(getattr(cfg, "amb_band", AMB_BAND))
    c.lookahead = int(getattr(cfg, "lookahead", 1))
    c.range_radius = float(getattr(cfg, "range_radius", 0.0))
    c.peak_growth = float(getattr(cfg, "peak_growth", 10.0))
    return c


class OraclePlan:
    def __init__(self, status, t0, xyz, act, val):
        self.status = int(status)
        self.t0 = int(t0)
        self.xyz = xyz          # float64 [n, 3]
        self.action = act       # int32 [n]   (-1 for the origin)
        self.value = val        # float64 [n]

    @property
    def n_points(self):
        return self.xyz.shape[0]


class Oracle:
    """One known-plan table plus terrain, planned in FP64 on the CPU."""

    def __init__(self, cfg, plans=None, terrain=None):
        self.lib = _load()
        self.cfg = cfg
        self._c = make_cfg(cfg)
        self.A = int(cfg.n_head) * len(cfg.climb) * len(cfg.speed)
        self.ell = max(cfg.speed) * cfg.dt
        h = C.c_void_p()
        rc = self.lib.orc_create(C.byref(self._c), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_create failed: {rc}")
        self._h = h
        if plans is not None:
            self.add_plans(plans)
        if terrain is not None:
            self.set_terrain(terrain)

    def close(self):
        if self._h:
            self.lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- table ---------------------------------------------------------------
    def add_plan(self, t0: int, xyz) -> None:
        xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
        rc = self.lib.orc_add_plan(self._h, int(t0), int(xyz.shape[0]), _fptr(xyz))
        if rc != 0:
            raise ValueError(f"orc_add_plan failed: {rc}")

    def add_plans(self, plans) -> None:
        off = plans.offsets()
        for j in range(plans.n):
            self.add_plan(int(plans.t0[j]), plans.xyz[off[j]:off[j + 1]])

    def set_terrain(self, terrain) -> None:
        h = np.ascontiguousarray(terrain.h, dtype=np.float32)
        rc = self.lib.orc_set_terrain(self._h, int(terrain.nx), int(terrain.ny), _fptr(h),
                                      float(terrain.x0), float(terrain.y0), float(terrain.cell))
        if rc != 0:
            raise ValueError(f"orc_set_terrain failed: {rc}")

    @property
    def n_plans(self) -> int:
        return int(self.lib.orc_num_plans(self._h))

    # -- method --------------------------------------------------------------
    def eval_step(self, s, g, t):
        A = self.A
        s = np.ascontiguousarray(s, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        V, G, I, T, D = (np.zeros(A) for _ in range(5))
        amb = np.zeros(A, dtype=np.int32)
        best = np.zeros(1, dtype=np.int32)
        rc = self.lib.orc_eval_step(self._h, _dptr(s), _dptr(g), int(t), _dptr(V), _dptr(G), _dptr(I),
                                    _dptr(T), _dptr(D), _iptr(amb), _iptr(best))
        if rc != 0:
            raise ValueError(f"orc_eval_step failed: {rc}")
        return dict(V=V, G=G, I=I, T=T, dmin=D, amb=amb.astype(bool), best=int(best[0]))

    def plan(self, origin, goal, t0: int = 0, cap: Optional[int] = None) -> OraclePlan:
        cap = int(cap or (self.cfg.max_steps + 1))
        origin = np.ascontiguousarray(origin, dtype=np.float64)
        goal = np.ascontiguousarray(goal, dtype=np.float64)
        xyz = np.zeros((cap, 3))
        act = np.zeros(cap, dtype=np.int32)
        val = np.zeros(cap)
        n = np.zeros(1, dtype=np.int32)
        st = np.zeros(1, dtype=np.int32)
        rc = self.lib.orc_plan(self._h, _dptr(origin), _dptr(goal), int(t0), cap, _dptr(xyz), _iptr(act),
                               _dptr(val), _iptr(n), _iptr(st))
        if rc != 0:
            raise ValueError(f"orc_plan failed: {rc}")
        k = int(n[0])
        return OraclePlan(int(st[0]), t0, xyz[:k].copy(), act[:k].copy(), val[:k].copy())

    def plan_batch(self, origins, goals, t0: int = 0, cap: Optional[int] = None):
        """Plan n aircraft co-simulated in lockstep (see orc_plan_batch)."""
        cap = int(cap or (self.cfg.max_steps + 1))
        origins = np.ascontiguousarray(origins, dtype=np.float64).reshape(-1, 3)
        goals = np.ascontiguousarray(goals, dtype=np.float64).reshape(-1, 3)
        n = origins.shape[0]
        xyz = np.zeros((n, cap, 3))
        act = np.zeros((n, cap), dtype=np.int32)
        val = np.zeros((n, cap))
        npts = np.zeros(n, dtype=np.int32)
        st = np.zeros(n, dtype=np.int32)
        rc = self.lib.orc_plan_batch(self._h, n, _dptr(origins), _dptr(goals), int(t0), cap, _dptr(xyz), _iptr(act),
                                     _dptr(val), _iptr(npts), _iptr(st))
        if rc != 0:
            raise ValueError(f"orc_plan_batch failed: {rc}")
        return [OraclePlan(int(st[i]), t0, xyz[i, :npts[i]].copy(), act[i, :npts[i]].copy(), val[i, :npts[i]].copy())
                for i in range(n)]

    def commit(self, plan_or_t0, xyz=None) -> bool:
        """Validate and append; False (table unchanged) on a separation conflict."""
        if xyz is None:
            t0, xyz = plan_or_t0.t0, plan_or_t0.xyz
        else:
            t0 = plan_or_t0
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        rc = self.lib.orc_commit(self._h, int(t0), int(xyz.shape[0]), _dptr(xyz))
        if rc == -4:
            return False
        if rc != 0:
            raise ValueError(f"orc_commit failed: {rc}")
        return True


def run_fcfs(oracle: Oracle, requests, limit: Optional[int] = None, commit: bool = True):
    """Plan requests in arrival order, committing every accepted plan (FCFS)."""
    out = []
    m = requests.n if limit is None else min(limit, requests.n)
    for k in range(m):
        p = oracle.plan(requests.origin[k], requests.goal[k], int(requests.t0[k]))
        committed = False
        if commit and p.status == 0:
            committed = oracle.commit(p)
        out.append((p, committed))
    return out


def num_threads() -> int:
    """Threads the oracle's per-action loop uses."""
    return int(_load().orc_num_threads())


def action_index(cfg, h: int, c: int, v: int) -> int:
    return (h * len(cfg.climb) + c) * len(cfg.speed) + v
