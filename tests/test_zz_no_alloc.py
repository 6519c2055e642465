"""fastmdp_load_plans_noalloc against fastmdp_load_plans, through the C ABI.

Two calls in a row on each side (the second with fewer plans, so that the
shared staging array still holds the first call's larger contents): after
each call the two tables are byte-identical checkpoints, and single steps
and plans computed from them are bitwise identical.  A load beyond the
staging array's limits is refused and leaves the table unchanged.
"""
import numpy as np
import pytest

from paper_2008_03518_amd import scenario as S

pytestmark = pytest.mark.gpu


def _staggered(plans, lo, hi, rows, seed):
    """Plans lo..hi-1 with departure rows 0..39, cut to end by the last row."""
    rng = np.random.default_rng(seed)
    off = plans.offsets()
    t0 = rng.integers(0, 40, hi - lo).astype(np.int32)
    pts = [plans.xyz[off[j]:off[j + 1]][: rows - t] for j, t in zip(range(lo, hi), t0)]
    return S.Plans(t0, np.array([len(p) for p in pts], np.int32), np.concatenate(pts).astype(np.float32))


def _same_tables(a, b, tmp_path, tag):
    pa, pb = str(tmp_path / f"a{tag}.bin"), str(tmp_path / f"b{tag}.bin")
    a.save_table(pa)
    b.save_table(pb)
    with open(pa, "rb") as fa, open(pb, "rb") as fb:
        return fa.read() == fb.read()


def test_load_plans_noalloc_equals_load_plans(tmp_path):
    from paper_2008_03518_amd import fastmdp as fm
    sc = S.large_actions(seed=41, n_plans=550, n_requests=3)
    rows = sc.cfg.max_rows
    first, second = _staggered(sc.plans, 0, 400, rows, 7), _staggered(sc.plans, 400, 550, rows, 8)
    assert int(first.length.sum()) > int(second.length.sum())
    with fm.Context(sc.cfg) as ref, fm.Context(sc.cfg) as na:
        for tag, part in (("1", first), ("2", second)):
            ref.load_plans(part)
            na.load_plans_noalloc(part)
            print(f"[no-alloc] call {tag}: {part.n} plans, {int(part.length.sum())} points", flush=True)
            assert na.n_plans == ref.n_plans
            assert _same_tables(ref, na, tmp_path, tag)
            for q in range(sc.requests.n):
                o, g = sc.requests.origin[q], sc.requests.goal[q]
                er, en = ref.eval_step(o, g, 3), na.eval_step(o, g, 3)
                for k in ("V", "G", "I", "T"):
                    assert np.array_equal(er[k], en[k])
                assert er["best"] == en["best"]
            pr = ref.plan_request(sc.requests.origin[0], sc.requests.goal[0], 0)
            pn = na.plan_request(sc.requests.origin[0], sc.requests.goal[0], 0)
            assert pr.status == pn.status and pr.n_points == pn.n_points
            assert np.array_equal(pr.points(), pn.points()) and np.array_equal(pr.values(), pn.values())
        # beyond the staging array: refused, table unchanged
        n_big = 700
        big = S.Plans(np.zeros(n_big, np.int32), np.full(n_big, 1000, np.int32),
                      np.zeros((n_big * 1000, 3), np.float32))
        with pytest.raises(fm.FastMDPError) as ei:
            na.load_plans_noalloc(big)
        assert ei.value.code == fm.E_CAPACITY
        assert na.n_plans == ref.n_plans and _same_tables(ref, na, tmp_path, "3")
