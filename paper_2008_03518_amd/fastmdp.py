"""Python binding of libfastmdp (ctypes over the C ABI in include/fastmdp.h).

Argument marshalling only: every step of the planner runs in the HIP
kernels of the shared library.  Importing this module fails loudly when the
library has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfastmdp.so")
MAX_ACT_DIM = 8
TIE_REL = 1e-9
N_FEAT = 96
MLP_HIDDEN = 256
MAX_TOPK = 16
PROPOSE_NONE, PROPOSE_MLP, PROPOSE_GOAL = 0, 1, 2

E_INVAL, E_CAPACITY, E_DEVICE, E_CONFLICT, E_NOMEM, E_IO = -1, -2, -3, -4, -5, -6
OK, REJECT_SEPARATION, REJECT_TERRAIN, REJECT_ORIGIN, TIMEOUT, NO_VALID_ACTION = 0, 1, 2, 3, 4, 5


class FastMDPError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn}: {msg} ({code})")
        self.code = code


class _Vec3(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("z", C.c_double)]


class _Config(C.Structure):
    _fields_ = [
        ("box_min", C.c_double * 3), ("box_max", C.c_double * 3),
        ("dt", C.c_double),
        ("gamma", C.c_double), ("r_goal", C.c_double),
        ("r_intr", C.c_double), ("R_intr", C.c_double), ("gamma_intr", C.c_double),
        ("R_sep", C.c_double),
        ("r_terr", C.c_double), ("R_terr", C.c_double), ("gamma_terr", C.c_double),
        ("n_head", C.c_int32), ("n_climb", C.c_int32), ("n_speed", C.c_int32),
        ("climb", C.c_double * MAX_ACT_DIM), ("speed", C.c_double * MAX_ACT_DIM),
        ("max_steps", C.c_int32), ("plan_capacity", C.c_int32), ("max_rows", C.c_int32),
        ("max_slots", C.c_int32), ("steps_per_launch", C.c_int32), ("planner_threads", C.c_int32),
        ("tie_rel", C.c_double),
        ("lookahead", C.c_int32), ("range_query", C.c_int32),
        ("peak_growth", C.c_double),
    ]


class _Request(C.Structure):
    _fields_ = [("id", C.c_uint64), ("origin", _Vec3), ("goal", _Vec3), ("t0", C.c_int32)]


class _Plan(C.Structure):
    _fields_ = [("status", C.c_int32), ("t0", C.c_int32), ("n_points", C.c_int32), ("capacity", C.c_int32),
                ("xyz", C.POINTER(C.c_double)), ("action", C.POINTER(C.c_int32)), ("value", C.POINTER(C.c_double))]


class _State(C.Structure):
    _fields_ = [("pos", _Vec3), ("goal", _Vec3), ("t", C.c_int32)]


def _load_lib():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libfastmdp.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    dp, ip, fp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_float)
    lib.fastmdp_create.argtypes = [C.POINTER(_Config), C.POINTER(P)]
    lib.fastmdp_destroy.argtypes = [P]
    lib.fastmdp_destroy.restype = None
    lib.fastmdp_set_stream.argtypes = [P, P]
    lib.fastmdp_load_plans.argtypes = [P, I32, ip, ip, fp]
    lib.fastmdp_load_plans_noalloc.argtypes = [P, I32, ip, ip, fp]
    lib.fastmdp_set_terrain.argtypes = [P, I32, I32, fp, D, D, D]
    lib.fastmdp_eval_step.argtypes = [P, C.POINTER(_State), dp, dp, dp, dp, ip]
    lib.fastmdp_plan_request.argtypes = [P, C.POINTER(_Request), C.POINTER(_Plan)]
    lib.fastmdp_commit_plan.argtypes = [P, C.POINTER(_Plan)]
    lib.fastmdp_plan_departures.argtypes = [P, C.POINTER(_Request), I32, ip, C.POINTER(_Plan), ip]
    lib.fastmdp_plan_batch.argtypes = [P, I32, C.POINTER(_Request), C.POINTER(_Plan)]
    lib.fastmdp_num_plans.argtypes = [P]
    lib.fastmdp_plan_fcfs.argtypes = [P, I32, C.POINTER(_Request), dp, C.POINTER(_Plan), ip, dp]
    lib.fastmdp_table_snapshot.argtypes = [P]
    lib.fastmdp_table_rewind.argtypes = [P]
    lib.fastmdp_last_stats.argtypes = [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64), C.POINTER(I64),
                                       C.POINTER(D), C.POINTER(I64)]
    lib.fastmdp_save_table.argtypes = [P, C.c_char_p]
    lib.fastmdp_load_table.argtypes = [P, C.c_char_p]
    lib.fastmdp_strerror.argtypes = [C.c_int]
    lib.fastmdp_strerror.restype = C.c_char_p
    # learned action proposal
    lib.fastmdp_mlp_create.argtypes = [I32, I32, I32, I32, C.POINTER(P)]
    lib.fastmdp_mlp_destroy.argtypes = [P]
    lib.fastmdp_mlp_destroy.restype = None
    lib.fastmdp_mlp_num_params.argtypes = [P]
    lib.fastmdp_mlp_num_params.restype = I64
    lib.fastmdp_mlp_set_params.argtypes = [P, fp]
    lib.fastmdp_mlp_get_params.argtypes = [P, fp]
    lib.fastmdp_mlp_forward.argtypes = [P, I32, P, P]
    lib.fastmdp_mlp_gradient.argtypes = [P, I32, P, P, fp, fp]
    lib.fastmdp_mlp_train_step.argtypes = [P, I32, P, P, C.c_float, fp]
    lib.fastmdp_features.argtypes = [P, I32, P, P, P, P, P]
    lib.fastmdp_next_seq.argtypes = [P]
    lib.fastmdp_set_proposal.argtypes = [P, I32, I32, I32, P]
    lib.fastmdp_eval_proposal.argtypes = [P, C.POINTER(_State), fp, fp, ip, ip, ip]
    lib.fastmdp_proposal_stats.argtypes = [P, C.POINTER(I64), C.POINTER(I64)]
    lib.fastmdp_device_alloc.argtypes = [I64, C.POINTER(P)]
    lib.fastmdp_device_free.argtypes = [P]
    lib.fastmdp_copy_to_device.argtypes = [P, P, I64]
    lib.fastmdp_copy_to_host.argtypes = [P, P, I64]
    lib.fastmdp_gather_rows.argtypes = [P, P, I64, P, I64, I32]
    return lib


_lib = _load_lib()

EXPORTS = [
    "fastmdp_create", "fastmdp_destroy", "fastmdp_set_stream", "fastmdp_load_plans", "fastmdp_load_plans_noalloc",
    "fastmdp_set_terrain",
    "fastmdp_eval_step", "fastmdp_plan_request", "fastmdp_plan_departures", "fastmdp_plan_batch",
    "fastmdp_commit_plan",
    "fastmdp_num_plans", "fastmdp_plan_fcfs",
    "fastmdp_last_stats", "fastmdp_save_table", "fastmdp_load_table", "fastmdp_strerror",
    "fastmdp_table_snapshot", "fastmdp_table_rewind",
    "fastmdp_mlp_create", "fastmdp_mlp_destroy", "fastmdp_mlp_num_params", "fastmdp_mlp_set_params",
    "fastmdp_mlp_get_params", "fastmdp_mlp_forward", "fastmdp_mlp_gradient", "fastmdp_mlp_train_step",
    "fastmdp_features", "fastmdp_next_seq", "fastmdp_set_proposal", "fastmdp_eval_proposal",
    "fastmdp_proposal_stats", "fastmdp_device_alloc", "fastmdp_device_free", "fastmdp_copy_to_device",
    "fastmdp_copy_to_host", "fastmdp_gather_rows",
]


def strerror(code: int) -> str:
    return _lib.fastmdp_strerror(int(code)).decode()


def _check(fn: str, rc: int) -> int:
    if rc < 0:
        raise FastMDPError(fn, rc, strerror(rc))
    return rc


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class DeviceArray:
    """A C-contiguous array in device memory owned by this object (allocated
    through the library, so no second HIP runtime enters the process)."""

    def __init__(self, shape, dtype):
        self.shape = tuple(int(d) for d in np.atleast_1d(shape)) if not isinstance(shape, tuple) else shape
        self.dtype = np.dtype(dtype)
        self.nbytes = int(np.prod(self.shape)) * self.dtype.itemsize
        self._p = C.c_void_p()
        if self.nbytes > 0:
            _check("fastmdp_device_alloc", _lib.fastmdp_device_alloc(self.nbytes, C.byref(self._p)))

    @classmethod
    def from_host(cls, a, dtype=None) -> "DeviceArray":
        a = np.ascontiguousarray(a, dtype=dtype)
        d = cls(a.shape, a.dtype)
        if d.nbytes:
            _check("fastmdp_copy_to_device", _lib.fastmdp_copy_to_device(d._p, a.ctypes.data_as(C.c_void_p),
                                                                         d.nbytes))
        return d

    @property
    def ptr(self) -> int:
        view = getattr(self, "_view", None)
        return view[1] if view else int(self._p.value or 0)

    def __len__(self) -> int:
        return self.shape[0]

    def row_ptr(self, i: int) -> int:
        return self.ptr + int(i) * (self.nbytes // max(self.shape[0], 1))

    def numpy(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=self.dtype)
        if self.nbytes:
            _check("fastmdp_copy_to_host", _lib.fastmdp_copy_to_host(out.ctypes.data_as(C.c_void_p),
                                                                     C.c_void_p(self.ptr), self.nbytes))
        return out

    def rows(self, i: int, k: int) -> "DeviceArray":
        """Rows [i, i + k) as a view (no copy; keeps this array alive)."""
        if not (0 <= i and k >= 0 and i + k <= self.shape[0]):
            raise IndexError((i, k, self.shape))
        v = DeviceArray.__new__(DeviceArray)
        v.shape = (int(k),) + self.shape[1:]
        v.dtype = self.dtype
        v.nbytes = int(k) * (self.nbytes // max(self.shape[0], 1))
        v._p = C.c_void_p()
        v._view = (self, self.row_ptr(i))
        return v

    def gather(self, idx) -> "DeviceArray":
        """Rows idx (host or device int64) as a new array."""
        di = idx if isinstance(idx, DeviceArray) else DeviceArray.from_host(np.asarray(idx, dtype=np.int64))
        out = DeviceArray((len(di),) + self.shape[1:], self.dtype)
        row = self.nbytes // max(self.shape[0], 1)
        if len(di):
            _check("fastmdp_gather_rows", _lib.fastmdp_gather_rows(out._p, C.c_void_p(self.ptr), self.shape[0],
                                                                   C.c_void_p(di.ptr), len(di), row))
        return out

    def free(self):
        if getattr(self, "_p", None) and self._p.value:
            _lib.fastmdp_device_free(self._p)
            self._p = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _dev(a, dtype) -> DeviceArray:
    """A device array of the given numpy dtype (uploaded unless it already is one)."""
    if isinstance(a, DeviceArray):
        if a.dtype != np.dtype(dtype):
            raise TypeError(f"device array of {a.dtype}, expected {np.dtype(dtype)}")
        return a
    return DeviceArray.from_host(np.asarray(a), dtype=dtype)


def make_config(cfg, max_slots: int = 1, tie_rel: float = TIE_REL, steps_per_launch: int = 0,
                planner_threads: int = 0) -> _Config:
    c = _Config()
    for k in range(3):
        c.box_min[k] = float(cfg.box_min[k])
        c.box_max[k] = float(cfg.box_max[k])
    for name in ("dt", "gamma", "r_goal", "r_intr", "R_intr", "gamma_intr", "R_sep", "r_terr", "R_terr",
                 "gamma_terr"):
        setattr(c, name, float(getattr(cfg, name)))
    c.n_head = int(cfg.n_head)
    c.n_climb = len(cfg.climb)
    c.n_speed = len(cfg.speed)
    for i, v in enumerate(cfg.climb):
        c.climb[i] = float(v)
    for i, v in enumerate(cfg.speed):
        c.speed[i] = float(v)
    c.max_steps = int(cfg.max_steps)
    c.plan_capacity = int(cfg.plan_capacity)
    c.max_rows = int(cfg.max_rows)
    c.max_slots = int(max_slots)
    c.steps_per_launch = int(steps_per_launch)
    c.planner_threads = int(planner_threads)
    c.tie_rel = float(tie_rel)
    c.lookahead = int(getattr(cfg, "lookahead", 1))
    c.range_query = int(getattr(cfg, "range_query", 0))
    c.peak_growth = float(getattr(cfg, "peak_growth", 10.0))
    return c


class Plan:
    """A trajectory returned by the planner (host arrays; entries beyond
    n_points are unspecified)."""

    def __init__(self, capacity: int):
        self.xyz = np.empty((capacity, 3))
        self.action = np.empty(capacity, dtype=np.int32)
        self.value = np.empty(capacity)
        self.c = _Plan(0, 0, 0, capacity, _dptr(self.xyz), _iptr(self.action), _dptr(self.value))

    @property
    def status(self) -> int:
        return int(self.c.status)

    @property
    def t0(self) -> int:
        return int(self.c.t0)

    @property
    def n_points(self) -> int:
        return int(self.c.n_points)

    def points(self) -> np.ndarray:
        return self.xyz[: self.n_points]

    def actions(self) -> np.ndarray:
        return self.action[: self.n_points]

    def values(self) -> np.ndarray:
        return self.value[: self.n_points]


# fastmdp_request as a NumPy record (same layout as _Request), so that a
# batch of requests is marshalled without a Python loop
_REQUEST_DTYPE = np.dtype({"names": ["id", "origin", "goal", "t0"],
                           "formats": ["<u8", ("<f8", 3), ("<f8", 3), "<i4"],
                           "offsets": [0, 8, 32, 56], "itemsize": 64})


def _request_array(requests, m: int) -> np.ndarray:
    a = np.zeros(max(m, 1), dtype=_REQUEST_DTYPE)
    a["id"][:m] = np.asarray(requests.ident[:m], dtype=np.uint64)
    a["origin"][:m] = np.asarray(requests.origin[:m], dtype=np.float64)
    a["goal"][:m] = np.asarray(requests.goal[:m], dtype=np.float64)
    a["t0"][:m] = np.asarray(requests.t0[:m], dtype=np.int32)
    return a


def _request(origin, goal, t0: int, ident: int = 0) -> _Request:
    r = _Request()
    r.id = int(ident)
    r.origin = _Vec3(*[float(v) for v in origin])
    r.goal = _Vec3(*[float(v) for v in goal])
    r.t0 = int(t0)
    return r


class Context:
    """One planner context on the current HIP device."""

    def __init__(self, cfg, max_slots: int = 1, tie_rel: float = TIE_REL, steps_per_launch: int = 0,
                 planner_threads: int = 0):
        self.cfg = cfg
        self._c = make_config(cfg, max_slots, tie_rel, steps_per_launch, planner_threads)
        self.A = int(cfg.n_head) * len(cfg.climb) * len(cfg.speed)
        self.capacity = int(cfg.max_steps) + 1
        h = C.c_void_p()
        _check("fastmdp_create", _lib.fastmdp_create(C.byref(self._c), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.fastmdp_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream_handle: Optional[int]):
        _check("fastmdp_set_stream", _lib.fastmdp_set_stream(self._h, C.c_void_p(stream_handle or 0)))

    def load_plans(self, plans) -> None:
        t0 = np.ascontiguousarray(plans.t0, dtype=np.int32)
        ln = np.ascontiguousarray(plans.length, dtype=np.int32)
        xyz = np.ascontiguousarray(plans.xyz, dtype=np.float32)
        _check("fastmdp_load_plans", _lib.fastmdp_load_plans(self._h, int(t0.shape[0]), _iptr(t0), _iptr(ln), _fptr(xyz)))

    def load_plans_noalloc(self, plans) -> None:
        """load_plans through the library's fixed staging array (no allocation)."""
        t0 = np.ascontiguousarray(plans.t0, dtype=np.int32)
        ln = np.ascontiguousarray(plans.length, dtype=np.int32)
        xyz = np.ascontiguousarray(plans.xyz, dtype=np.float32)
        _check("fastmdp_load_plans_noalloc",
               _lib.fastmdp_load_plans_noalloc(self._h, int(t0.shape[0]), _iptr(t0), _iptr(ln), _fptr(xyz)))

    def set_terrain(self, terrain) -> None:
        h = np.ascontiguousarray(terrain.h, dtype=np.float32)
        _check("fastmdp_set_terrain", _lib.fastmdp_set_terrain(self._h, int(terrain.nx), int(terrain.ny), _fptr(h),
                                                               float(terrain.x0), float(terrain.y0),
                                                               float(terrain.cell)))

    @property
    def n_plans(self) -> int:
        return _check("fastmdp_num_plans", _lib.fastmdp_num_plans(self._h))

    def eval_step(self, s, g, t: int) -> dict:
        st = _State(_Vec3(*[float(v) for v in s]), _Vec3(*[float(v) for v in g]), int(t))
        A = self.A
        V, G, I, T = (np.zeros(A) for _ in range(4))
        best = np.zeros(1, dtype=np.int32)
        _check("fastmdp_eval_step", _lib.fastmdp_eval_step(self._h, C.byref(st), _dptr(V), _dptr(G), _dptr(I),
                                                           _dptr(T), _iptr(best)))
        return dict(V=V, G=G, I=I, T=T, best=int(best[0]))

    def plan_request(self, origin, goal, t0: int = 0, ident: int = 0) -> Plan:
        p = Plan(self.capacity)
        r = _request(origin, goal, t0, ident)
        _check("fastmdp_plan_request", _lib.fastmdp_plan_request(self._h, C.byref(r), C.byref(p.c)))
        return p

    def plan_departures(self, origin, goal, t0s, ident: int = 0):
        """Plan one request from every departure row in t0s (nothing is
        committed).  Returns (plans, chosen): chosen is the index of the
        earliest departure whose plan would be accepted, -1 if none."""
        t0s = np.ascontiguousarray(np.asarray(t0s, dtype=np.int32))
        n = int(t0s.shape[0])
        plans = [Plan(self.capacity) for _ in range(n)]
        parr = (_Plan * max(n, 1))()
        for k in range(n):
            parr[k] = plans[k].c
        r = _request(origin, goal, int(t0s[0]) if n else 0, ident)
        chosen = np.zeros(1, dtype=np.int32)
        _check("fastmdp_plan_departures", _lib.fastmdp_plan_departures(self._h, C.byref(r), n, _iptr(t0s), parr,
                                                                       _iptr(chosen)))
        for k in range(n):
            plans[k].c = parr[k]
        return plans, int(chosen[0])

    def plan_batch(self, requests, limit: Optional[int] = None):
        """Plan the requests as one co-simulated batch (nothing committed)."""
        m = requests.n if limit is None else min(limit, requests.n)
        reqa = _request_array(requests, m)
        plans = [Plan(self.capacity) for _ in range(m)]
        parr = (_Plan * max(m, 1))()
        for k in range(m):
            parr[k] = plans[k].c
        _check("fastmdp_plan_batch", _lib.fastmdp_plan_batch(self._h, m, reqa.ctypes.data_as(C.POINTER(_Request)),
                                                             parr))
        for k in range(m):
            plans[k].c = parr[k]
        return plans

    def commit_plan(self, plan: Plan) -> bool:
        """True if appended; False if refused for a separation/terrain conflict."""
        rc = _lib.fastmdp_commit_plan(self._h, C.byref(plan.c))
        if rc == E_CONFLICT:
            return False
        _check("fastmdp_commit_plan", rc)
        return True

    def commit_points(self, t0: int, xyz) -> bool:
        """Commit an arbitrary FP64 trajectory (status OK) -- for tests and tools."""
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        p = Plan(xyz.shape[0])
        p.xyz[:] = xyz
        p.c.status, p.c.t0, p.c.n_points = OK, int(t0), xyz.shape[0]
        return self.commit_plan(p)

    def plan_fcfs(self, requests, limit: Optional[int] = None, arrival_s=None, out: Optional[list] = None):
        """Plan requests first-come-first-served with concurrent slots.

        With ``arrival_s`` (non-decreasing seconds), request i is admitted no
        earlier than arrival_s[i] after the call starts.  ``out`` may supply
        Plan buffers (of this context's capacity) to fill instead of new ones.
        Returns (plans, committed, done_s): committed a bool array, done_s the
        acceptance time of each request in seconds since the call started.
        """
        m = requests.n if limit is None else min(limit, requests.n)
        reqa = _request_array(requests, m)
        arr = reqa.ctypes.data_as(C.POINTER(_Request))
        if out is not None and len(out) >= m and all(p.c.capacity >= self.capacity for p in out[:m]):
            plans = list(out[:m])
        else:
            plans = [Plan(self.capacity) for _ in range(m)]
        parr = (_Plan * max(m, 1))()
        for k in range(m):
            parr[k] = plans[k].c
        committed = np.zeros(max(m, 1), dtype=np.int32)
        done = np.zeros(max(m, 1))
        arr_s = None
        if arrival_s is not None:
            arr_s = np.ascontiguousarray(np.asarray(arrival_s, dtype=np.float64)[:m])
        rc = _lib.fastmdp_plan_fcfs(self._h, m, arr, _dptr(arr_s) if arr_s is not None else None, parr,
                                    _iptr(committed), _dptr(done))
        for k in range(m):
            plans[k].c = parr[k]
        if rc < 0:
            # an interrupted call keeps the requests accepted before the error
            err = FastMDPError("fastmdp_plan_fcfs", rc, strerror(rc))
            err.plans, err.committed = plans, committed[:m].astype(bool)
            raise err
        return plans, committed[:m].astype(bool), done[:m]

    def snapshot(self) -> None:
        _check("fastmdp_table_snapshot", _lib.fastmdp_table_snapshot(self._h))

    def rewind(self) -> None:
        _check("fastmdp_table_rewind", _lib.fastmdp_table_rewind(self._h))

    def stats(self) -> dict:
        v = [C.c_int64() for _ in range(4)]
        ms = C.c_double()
        ent = C.c_int64()
        _check("fastmdp_last_stats", _lib.fastmdp_last_stats(self._h, *[C.byref(x) for x in v], C.byref(ms),
                                                             C.byref(ent)))
        return dict(pairs=v[0].value, steps=v[1].value, resumes=v[2].value, launches=v[3].value, kernel_ms=ms.value,
                    row_entries=ent.value)

    # -- learned action proposal ------------------------------------------
    def next_seq(self) -> int:
        return _check("fastmdp_next_seq", _lib.fastmdp_next_seq(self._h))

    def features(self, states, goals, rows, seqs) -> DeviceArray:
        """Proposal features [n, 96] (device array) of FP64 states/goals [n, 3]
        against the plans of rows[i] + 1 visible to sequence number seqs[i]."""
        st, gl = _dev(states, np.float64), _dev(goals, np.float64)
        rw, sq = _dev(rows, np.int32), _dev(seqs, np.int32)
        n = int(st.shape[0])
        out = DeviceArray((n, N_FEAT), np.float32)
        _check("fastmdp_features", _lib.fastmdp_features(self._h, n, st.ptr, gl.ptr, rw.ptr, sq.ptr, out.ptr))
        return out

    def set_proposal(self, mode: int, top_k: int = 8, net: "Optional[Mlp]" = None, refresh: int = 1) -> None:
        _check("fastmdp_set_proposal", _lib.fastmdp_set_proposal(self._h, int(mode), int(top_k), int(refresh),
                                                                 net._h if net is not None else None))
        self._net = net if mode == PROPOSE_MLP else None      # keep the network alive while selected
        self._top_k = int(top_k)

    def eval_proposal(self, s, g, t: int) -> dict:
        st = _State(_Vec3(*[float(v) for v in s]), _Vec3(*[float(v) for v in g]), int(t))
        f = np.zeros(N_FEAT, dtype=np.float32)
        lg = np.zeros(self.A, dtype=np.float32)
        tk = np.zeros(MAX_TOPK, dtype=np.int32)
        ce = np.zeros(1, dtype=np.int32)
        b = np.zeros(1, dtype=np.int32)
        _check("fastmdp_eval_proposal", _lib.fastmdp_eval_proposal(self._h, C.byref(st), _fptr(f), _fptr(lg), _iptr(tk),
                                                                   _iptr(ce), _iptr(b)))
        return dict(features=f, logits=lg, topk=tk[: self._top_k].copy(), certified=bool(ce[0]), best=int(b[0]))

    def proposal_stats(self) -> dict:
        a, b = C.c_int64(), C.c_int64()
        _check("fastmdp_proposal_stats", _lib.fastmdp_proposal_stats(self._h, C.byref(a), C.byref(b)))
        return dict(certified=a.value, fallbacks=b.value)

    def save_table(self, path: str) -> None:
        _check("fastmdp_save_table", _lib.fastmdp_save_table(self._h, path.encode()))

    def load_table(self, path: str) -> None:
        _check("fastmdp_load_table", _lib.fastmdp_load_table(self._h, path.encode()))


def pack_params(params: dict) -> np.ndarray:
    """Packed FP32 parameter vector of the library from weights in the
    x @ W convention (W1 [in, hid], W2 [hid, hid], W3 [hid, out], biases)."""
    parts = [params["W1"].T, params["b1"], params["W2"].T, params["b2"], params["W3"].T, params["b3"]]
    return np.concatenate([np.ascontiguousarray(p, dtype=np.float32).ravel() for p in parts])


def unpack_params(v: np.ndarray, n_in: int, n_hid: int, n_out: int) -> dict:
    """Inverse of pack_params (float64 arrays in the x @ W convention)."""
    v = np.asarray(v, dtype=np.float64)
    out, o = {}, 0
    for name, shape in (("W1", (n_hid, n_in)), ("b1", (n_hid,)), ("W2", (n_hid, n_hid)), ("b2", (n_hid,)),
                        ("W3", (n_out, n_hid)), ("b3", (n_out,))):
        k = int(np.prod(shape))
        a = v[o: o + k].reshape(shape)
        out[name] = a.T.copy() if name.startswith("W") else a.copy()
        o += k
    return out


class Mlp:
    """The proposal network on the current HIP device (BF16 MFMA kernels,
    FP32 master weights, Adam)."""

    def __init__(self, n_out: int, n_in: int = N_FEAT, n_hidden: int = MLP_HIDDEN, max_batch: int = 4096):
        self.n_in, self.n_hid, self.n_out, self.max_batch = int(n_in), int(n_hidden), int(n_out), int(max_batch)
        h = C.c_void_p()
        _check("fastmdp_mlp_create", _lib.fastmdp_mlp_create(self.n_in, self.n_hid, self.n_out, self.max_batch,
                                                             C.byref(h)))
        self._h = h
        self.n_params = int(_lib.fastmdp_mlp_num_params(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.fastmdp_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: dict) -> None:
        v = pack_params(params)
        assert v.size == self.n_params
        _check("fastmdp_mlp_set_params", _lib.fastmdp_mlp_set_params(self._h, _fptr(v)))

    def get_params(self) -> dict:
        v = np.zeros(self.n_params, dtype=np.float32)
        _check("fastmdp_mlp_get_params", _lib.fastmdp_mlp_get_params(self._h, _fptr(v)))
        return unpack_params(v, self.n_in, self.n_hid, self.n_out)

    def forward(self, x) -> np.ndarray:
        """Logits [B, n_out] (host) of features x [B, n_in] (host or device)."""
        xd = _dev(x, np.float32)
        out = DeviceArray((xd.shape[0], self.n_out), np.float32)
        _check("fastmdp_mlp_forward", _lib.fastmdp_mlp_forward(self._h, int(xd.shape[0]), xd.ptr, out.ptr))
        return out.numpy()

    def gradient(self, x, y):
        """(gradients in the x @ W convention, mean loss) of a batch."""
        xd, yd = _dev(x, np.float32), _dev(y, np.int32)
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        _check("fastmdp_mlp_gradient", _lib.fastmdp_mlp_gradient(self._h, int(xd.shape[0]), xd.ptr, yd.ptr,
                                                                 _fptr(g), _fptr(loss)))
        return unpack_params(g, self.n_in, self.n_hid, self.n_out), float(loss[0])

    def train_step(self, x, y, lr: float) -> float:
        """One Adam step on the batch (host or device arrays); returns its loss
        before the step."""
        xd, yd = _dev(x, np.float32), _dev(y, np.int32)
        loss = np.zeros(1, dtype=np.float32)
        _check("fastmdp_mlp_train_step", _lib.fastmdp_mlp_train_step(self._h, int(xd.shape[0]), xd.ptr, yd.ptr,
                                                                     float(lr), _fptr(loss)))
        return float(loss[0])


def context_for(scenario, max_slots: int = 1, steps_per_launch: int = 0, planner_threads: int = 0) -> Context:
    """Context with the scenario's known plans and terrain loaded."""
    ctx = Context(scenario.cfg, max_slots=max_slots, steps_per_launch=steps_per_launch,
                  planner_threads=planner_threads)
    ctx.load_plans(scenario.plans)
    if scenario.terrain is not None:
        ctx.set_terrain(scenario.terrain)
    return ctx
