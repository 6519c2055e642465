"""Comparison rules between the HIP planner and the FP64 oracle.

Value parity: for every action not in the boundary band (a plan distance or
terrain clearance within 1e-3 m of its radius, where FP32 and FP64 may fall
on different sides of a strict well boundary), the GPU value is within
1e-5 relative of the oracle's, relative to the largest of |V|, G, I, T (so
that cancellation between the goal term and a penalty cannot blow the
relative error up); -inf box masks match exactly.

Action parity: the chosen action matches, unless the oracle's two best
values lie within that tolerance of each other or a boundary-band action is
involved (an excused divergence).
"""
from __future__ import annotations

import numpy as np

REL_TOL = 1e-5


def scale(o):
    return np.maximum.reduce([np.abs(np.where(np.isfinite(o["V"]), o["V"], 0.0)), o["G"], o["I"], o["T"],
                              np.full_like(o["G"], 1e-300)])


def compare_eval(g, o, rel=REL_TOL):
    """Assert value parity; return (n_compared, n_band, max_rel_err, action_ok, excused)."""
    band = o["amb"]
    fin_o = np.isfinite(o["V"])
    fin_g = np.isfinite(g["V"])
    assert np.array_equal(fin_o, fin_g), "box mask differs"
    sel = fin_o & ~band
    sc = scale(o)
    err = np.abs(g["V"][sel] - o["V"][sel]) / sc[sel]
    mx = float(err.max()) if err.size else 0.0
    assert mx <= rel, f"value error {mx:.3e}"
    for key in ("G", "I", "T"):
        e = np.abs(g[key] - o[key])[~band] / np.maximum(o[key][~band], 1e-300)
        e = np.where(o[key][~band] == 0, np.abs(g[key][~band]), e)
        assert (e.max() if e.size else 0.0) <= rel, f"{key} error {e.max():.3e}"
    action_ok = g["best"] == o["best"]
    excused = False
    if not action_ok:
        v = np.where(fin_o, o["V"], -np.inf)
        top = np.sort(v)[::-1]
        near_tie = top.size > 1 and np.isfinite(top[1]) and (top[0] - top[1]) <= rel * max(sc.max(), 1e-300)
        in_band = bool(band[o["best"]]) or (g["best"] >= 0 and bool(band[g["best"]]))
        excused = near_tie or in_band
        assert excused, f"chosen action {g['best']} != oracle {o['best']}"
    return int(sel.sum()), int(band.sum()), mx, action_ok, excused


def compare_trajectory(gp, op, orc, goal, pos_tol=1e-6, rel=REL_TOL):
    """Compare GPU and oracle trajectories up to the first excused divergence.

    Returns the number of identical steps, or raises on a real mismatch.
    A divergence is excused when the oracle's eval at the diverging state
    shows a near-tie or a boundary-band action.
    """
    n = min(gp.n_points, op.n_points)
    ga, oa = gp.actions(), op.action
    gx = gp.points()
    k = 0
    while k < n:
        assert np.max(np.abs(gx[k] - op.xyz[k])) <= pos_tol, f"point {k} differs"
        if k > 0:
            assert abs(gp.values()[k] - op.value[k]) <= rel * max(abs(op.value[k]), 1e-300) or \
                _value_band(orc, op, goal, k), f"value at point {k}"
        if k + 1 < n and ga[k + 1] != oa[k + 1]:
            o = orc.eval_step(op.xyz[k], goal, op.t0 + k)
            v = np.where(np.isfinite(o["V"]), o["V"], -np.inf)
            top = np.sort(v)[::-1]
            sc = scale(o).max()
            near_tie = top.size > 1 and (top[0] - top[1]) <= rel * sc
            in_band = bool(o["amb"][oa[k + 1]]) or bool(o["amb"][ga[k + 1]])
            assert near_tie or in_band, f"action at point {k + 1}: gpu {ga[k + 1]} oracle {oa[k + 1]}"
            return k + 1, True
        k += 1
    assert gp.n_points == op.n_points, f"length {gp.n_points} vs {op.n_points}"
    assert gp.status == op.status, f"status {gp.status} vs {op.status}"
    return n, False


def classify_trajectory(gp, op, orc, goal, pos_tol=1e-6, rel=REL_TOL):
    """Compare a GPU trajectory with the oracle's; never silent on a real mismatch.

    Returns a dict: kind 'identical' (same status, points within pos_tol,
    actions equal, values within rel), or an excused divergence at step
    `at` -- 'near_tie' (the oracle's two best values at the diverging state
    lie within the value tolerance) or 'band' (the oracle's or the GPU's
    choice has a plan distance or clearance within the boundary band); plus
    the largest relative value error over the compared points.  Raises
    AssertionError on any other difference.
    """
    n = min(gp.n_points, op.n_points)
    ga, oa = gp.actions(), op.action
    gx, gv = gp.points(), gp.values()
    mx = 0.0
    for k in range(n):
        assert np.max(np.abs(gx[k] - op.xyz[k])) <= pos_tol, f"point {k} differs"
        if k > 0:
            e = abs(gv[k] - op.value[k]) / max(abs(op.value[k]), 1e-300)
            if e > rel:
                assert _value_band(orc, op, goal, k), f"value at point {k}: rel error {e:.3e}"
            else:
                mx = max(mx, e)
        if k + 1 < n and ga[k + 1] != oa[k + 1]:
            o = orc.eval_step(op.xyz[k], goal, op.t0 + k)
            v = np.where(np.isfinite(o["V"]), o["V"], -np.inf)
            top = np.sort(v)[::-1]
            near_tie = top.size > 1 and (top[0] - top[1]) <= rel * scale(o).max()
            in_band = bool(o["amb"][oa[k + 1]]) or bool(o["amb"][ga[k + 1]])
            assert near_tie or in_band, f"action at point {k + 1}: gpu {ga[k + 1]} oracle {oa[k + 1]}"
            return dict(kind="near_tie" if near_tie else "band", at=k + 1, max_rel=mx)
    assert gp.n_points == op.n_points, f"length {gp.n_points} vs {op.n_points}"
    assert gp.status == op.status, f"status {gp.status} vs {op.status}"
    return dict(kind="identical", at=-1, max_rel=mx)


def _value_band(orc, op, goal, k):
    o = orc.eval_step(op.xyz[k - 1], goal, op.t0 + k - 1)
    return bool(o["amb"][op.action[k]])


# ---------------------------------------------------------------------------
# Separation invariant of the stored table (Sec. V: only collision-free plans
# are accepted).  A plan is validated as planned (FP64) against the earlier
# plans as stored (FP32) and then stored rounded to FP32.  Rounding moves a
# point by at most half an FP32 spacing per axis, so any two stored points
# at a common row, one of them from an accepted plan, are at least
# R_sep - delta apart, with delta the length of that per-axis bound at the
# box's largest coordinates.
# ---------------------------------------------------------------------------

def fp32_rounding_bound(box_min, box_max) -> float:
    """Largest distance between an FP64 point of the box and its FP32 rounding."""
    m = np.maximum(np.abs(np.asarray(box_min, np.float64)), np.abs(np.asarray(box_max, np.float64)))
    half = np.spacing(m.astype(np.float32)).astype(np.float64) / 2.0
    return float(np.sqrt(np.sum(half * half)))


def separation_report(known, accepted, R_sep, delta, probe=50.0):
    """Stored-versus-stored separation over every row.

    known: [(t0, points)] loaded plans (their mutual distances are not
    checked: they were never validated); accepted: [(t0, points)] accepted
    plans as stored (FP32 values), in acceptance order.  Returns the number
    of pairs closer than R_sep - delta and the smallest distance of a pair
    involving an accepted plan (inf when none is within R_sep + probe).
    """
    from scipy.spatial import cKDTree
    R, P, T = [], [], []
    for tag, plans in ((0, known), (1, accepted)):
        for t0, x in plans:
            x = np.asarray(x, np.float64).reshape(-1, 3)
            R.append(int(t0) + np.arange(x.shape[0]))
            P.append(x)
            T.append(np.full(x.shape[0], tag, np.int8))
    if not R:
        return 0, np.inf
    R, P, T = np.concatenate(R), np.concatenate(P), np.concatenate(T)
    order = np.argsort(R, kind="stable")
    R, P, T = R[order], P[order], T[order]
    cuts = np.flatnonzero(np.diff(R)) + 1
    rows = zip(np.split(P, cuts), np.split(T, cuts))
    gap, bad = np.inf, 0
    for pts, tags in rows:
        if not tags.any() or len(tags) < 2:
            continue
        pairs = cKDTree(pts).query_pairs(R_sep + probe, output_type="ndarray")
        if pairs.size == 0:
            continue
        pairs = pairs[(tags[pairs[:, 0]] == 1) | (tags[pairs[:, 1]] == 1)]
        if pairs.size == 0:
            continue
        d = np.linalg.norm(pts[pairs[:, 0]] - pts[pairs[:, 1]], axis=1)
        gap = min(gap, float(d.min()))
        bad += int(np.sum(d < R_sep - delta))
    return bad, gap


def stored(t0, xyz):
    """An accepted plan as the table stores it (FP32 values)."""
    return int(t0), np.asarray(xyz, np.float64).astype(np.float32).astype(np.float64)
