"""Pins of the FP64 proposal reference: backprop against central finite
differences, the features against hand-built geometry."""
import math

import numpy as np

from oracle import mlp
from paper_2008_03518_amd import scenario as S


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    A = 12
    params = mlp.init_params(rng, A, hidden=16)
    X = rng.normal(size=(5, mlp.N_FEAT))
    y = rng.integers(0, A, 5)
    g = mlp.backward(params, X, y)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        P = params[name]
        flat = P.reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = mlp.loss(params, X, y)
            flat[i] = old - h
            lm = mlp.loss(params, X, y)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, i, fd, an)


def test_softmax_loss_uniform_logits():
    """Zero last layer: every action equally likely, loss = log A."""
    rng = np.random.default_rng(1)
    A = 7
    params = mlp.init_params(rng, A, hidden=8)
    params["W3"][:] = 0.0
    X = rng.normal(size=(3, mlp.N_FEAT))
    assert abs(mlp.loss(params, X, np.array([0, 3, 6])) - math.log(A)) < 1e-12


def test_features_hand_geometry():
    cfg = S.cfg_large_actions()
    s = np.array([1000.0, 1000.0, 500.0])
    g = np.array([1000.0, 9000.0, 500.0])          # goal due +y: along = +y, cross = -x
    plans = np.array([[1000.0, 1300.0, 600.0],     # 300 m ahead, above: phi = 0 -> sector 8, upper
                      [1200.0, 1000.0, 400.0],     # 200 m to +x (right of track, cross < 0), below
                      [1000.0, 2000.0, 500.0]])    # 1000 m ahead: outside the feature radius
    f = mlp.features(s, g, plans, cfg)
    d1 = math.sqrt(300.0 ** 2 + 100.0 ** 2)
    assert abs(f[2 * 8 + 0] - (1.0 - d1 / 600.0)) < 1e-12 and f[32 + 16] == 0.25
    d2 = math.sqrt(200.0 ** 2 + 100.0 ** 2)
    # phi = atan2(cross=-200, along=0) = -pi/2 -> sector floor((pi/2) * 16 / (2 pi)) = 4, lower half
    assert abs(f[2 * 4 + 1] - (1.0 - d2 / 600.0)) < 1e-12 and f[32 + 9] == 0.25
    assert np.count_nonzero(f[:64]) == 4
    assert f[74] == 2.0 / 16.0 and abs(f[75] - d2 / 600.0) < 1e-12
    assert f[72] == 0.0 and f[73] == 1.0 and abs(f[64] - 0.8) < 1e-12
