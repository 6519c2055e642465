"""FP64 reference of the learned action proposal (features and MLP).

TEST INFRASTRUCTURE ONLY (imported by tests; never by the product path).

The proposal is not part of the paper: it ranks actions so that only a few
are scored exactly; a certificate (the exact best of the few beats every
other action's goal-only upper bound) keeps the chosen actions identical
to the full sweep.  This module is the plain reference of the two pieces
whose numerics the HIP path must reproduce:

* ``features``: the 96 inputs at a state, from the goal and the visible
  plans at the successor's time (definition in the design notes);
* ``forward`` / ``backward``: a 96 -> 256 -> 256 -> A ReLU network with a
  softmax cross-entropy loss on the chosen action, written out in FP64.
  ``backward`` is pinned by central finite differences in the tests.
"""
from __future__ import annotations

import math

import numpy as np

N_FEAT = 96
SECTORS = 16
R_FEAT = 600.0      # metres: plans nearer than this enter the traffic features


def features(s, g, plans_xyz, cfg) -> np.ndarray:
    """The 96 proposal features at state s (FP64), goal g, with the visible
    plan positions at the successor's time (array [n, 3])."""
    s = np.asarray(s, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    f = np.zeros(N_FEAT)
    bx, by = g[0] - s[0], g[1] - s[1]
    rh = math.hypot(bx, by)
    ux, uy = (bx / rh, by / rh) if rh > 0 else (1.0, 0.0)
    near = np.zeros(2 * SECTORS)
    cnt = np.zeros(2 * SECTORS)
    n_close, dmin = 0, R_FEAT
    for p in np.asarray(plans_xyz, dtype=np.float64).reshape(-1, 3):
        q = p - s
        d = math.sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2])
        if d >= R_FEAT:
            continue
        along = q[0] * ux + q[1] * uy
        cross = -q[0] * uy + q[1] * ux
        phi = math.atan2(cross, along)
        k = min(SECTORS - 1, int(math.floor((phi + math.pi) * SECTORS / (2.0 * math.pi))))
        idx = 2 * k + (0 if q[2] >= 0.0 else 1)
        near[idx] = max(near[idx], 1.0 - d / R_FEAT)
        cnt[idx] += 1.0
        n_close += 1
        dmin = min(dmin, d)
    f[0:32] = near
    f[32:64] = np.minimum(cnt, 4.0) / 4.0
    ell = max(cfg.speed) * cfg.dt
    d3 = float(np.linalg.norm(g - s))
    lo, hi = np.asarray(cfg.box_min, dtype=np.float64), np.asarray(cfg.box_max, dtype=np.float64)
    f[64] = rh / 10000.0
    f[65] = (g[2] - s[2]) / 500.0
    f[66] = d3 / ell / 1000.0
    f[67] = math.log1p(d3 / ell) / 8.0
    f[68] = s[2] / 1000.0
    f[69] = (s[2] - lo[2]) / (hi[2] - lo[2])
    f[70] = (s[0] - lo[0]) / (hi[0] - lo[0])
    f[71] = (s[1] - lo[1]) / (hi[1] - lo[1])
    f[72] = ux
    f[73] = uy
    f[74] = min(n_close / 16.0, 1.0)
    f[75] = dmin / R_FEAT
    return f


def init_params(rng, n_out, hidden=256, n_in=N_FEAT):
    """He-uniform weights, zero biases (float64)."""
    def lin(fan_in, fan_out):
        lim = math.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, (fan_in, fan_out)), np.zeros(fan_out)
    W1, b1 = lin(n_in, hidden)
    W2, b2 = lin(hidden, hidden)
    W3, b3 = lin(hidden, n_out)
    return dict(W1=W1, b1=b1, W2=W2, b2=b2, W3=W3, b3=b3)


def forward(params, X):
    """Logits and the cache for backward.  X: [B, 96]."""
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ params["W1"] + params["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ params["W2"] + params["b2"]
    h2 = np.maximum(z2, 0.0)
    logits = h2 @ params["W3"] + params["b3"]
    return logits, (X, z1, h1, z2, h2)


def loss(params, X, y):
    """Mean softmax cross-entropy of the chosen actions y [B]."""
    logits, _ = forward(params, X)
    m = logits.max(axis=1, keepdims=True)
    lse = m[:, 0] + np.log(np.exp(logits - m).sum(axis=1))
    return float(np.mean(lse - logits[np.arange(len(y)), y]))


def backward(params, X, y):
    """Gradients of ``loss`` with respect to every parameter (float64)."""
    logits, (X, z1, h1, z2, h2) = forward(params, X)
    B = X.shape[0]
    m = logits.max(axis=1, keepdims=True)
    p = np.exp(logits - m)
    p /= p.sum(axis=1, keepdims=True)
    d3 = p
    d3[np.arange(B), y] -= 1.0
    d3 /= B
    g = {}
    g["W3"] = h2.T @ d3
    g["b3"] = d3.sum(axis=0)
    dh2 = d3 @ params["W3"].T
    dz2 = dh2 * (z2 > 0.0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ params["W2"].T
    dz1 = dh1 * (z1 > 0.0)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return g
