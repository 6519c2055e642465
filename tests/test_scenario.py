"""Seeded workload generator: deterministic, the stated shapes and ranges."""
import numpy as np

from paper_2008_03518_amd import scenario as S


def test_small_is_deterministic_and_in_range():
    a, b = S.small(seed=0), S.small(seed=0)
    assert np.array_equal(a.plans.xyz, b.plans.xyz) and np.array_equal(a.requests.origin, b.requests.origin)
    assert a.plans.n == 50 and a.cfg.n_actions == 81 and a.plans.xyz.dtype == np.float32
    z = a.plans.xyz[:, 2]
    assert z.min() >= 100.0 and z.max() <= 900.0
    assert a.plans.xyz[:, :2].min() >= 0.0 and a.plans.xyz[:, :2].max() <= 10000.0
    # level, constant-speed tracks: consecutive points at most 40 m apart
    off = a.plans.offsets()
    for j in range(a.plans.n):
        p = a.plans.xyz[off[j]:off[j + 1]].astype(np.float64)
        step = np.linalg.norm(np.diff(p, axis=0), axis=1)
        assert np.all(step <= 40.0 + 1e-3) and np.ptp(p[:, 2]) == 0.0


def test_large_actions_shapes():
    sc = S.large_actions(n_plans=40, n_requests=5)
    assert sc.cfg.n_actions == 360 and sc.cfg.dt == 0.5 and sc.cfg.ell == 20.0
    assert sc.plans.length.max() <= sc.cfg.max_steps + 1
    assert sc.requests.n == 5 and np.all(sc.requests.t0 == 0)


def test_paper_scale_terrain_grid():
    rng = np.random.default_rng(1)
    cfg = S.cfg_paper_scale()
    ter = S.make_terrain(rng, cfg)
    assert ter.h.shape == (256, 256) and ter.h.dtype == np.float32
    assert abs(ter.x0 + ter.cell * 255 - cfg.box_max[0]) < 1e-6
