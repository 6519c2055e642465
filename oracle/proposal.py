"""FP64 reference of the proposal certificate and of the optimiser step.

TEST INFRASTRUCTURE ONLY (imported by tests; never by the product path).

The proposal is an addition to the method (the paper scores every action
at every step).  Its exactness rests on one fact of the value of Sec. III:
an action's value is its goal term minus the largest of its penalties, and
the penalties are non-negative, so no action's value exceeds its goal term.
``certify`` states the resulting test in plain form: given the exact values
of a proposed set K and the goal terms of all actions, the argmax over all
actions (largest value, then the lowest index within tie_rel of it) is
decided inside K whenever every action outside K has a goal term below
the tie threshold of K's best value.
"""
from __future__ import annotations

import numpy as np


def argmax_tie(V, tie_rel):
    """Chosen action of a full sweep: the lowest index whose value is within
    tie_rel*|max| of the maximum; -1 if every value is -inf."""
    V = np.asarray(V, dtype=np.float64)
    vm = V.max()
    if vm == -np.inf:
        return -1
    thr = vm - tie_rel * abs(vm)
    return int(np.flatnonzero(V >= thr)[0])


def certify(V_K, K, G, tie_rel):
    """(certified, chosen action) from the exact values V_K of the actions K
    and the goal terms G of all actions (-inf outside the box)."""
    K = [int(a) for a in K]
    V_K = np.asarray(V_K, dtype=np.float64)
    vm = V_K.max()
    if vm == -np.inf:
        return False, -1
    thr = vm - tie_rel * abs(vm)
    others = np.ones(len(G), dtype=bool)
    others[K] = False
    tau = np.max(np.asarray(G, dtype=np.float64)[others]) if others.any() else -np.inf
    if not tau < thr:
        return False, -1
    chosen = min(a for a, v in zip(K, V_K) if v >= thr)
    return True, chosen


def top_k(keys, k):
    """Indices of the k largest keys, lowest index first among equal keys."""
    keys = np.asarray(keys, dtype=np.float64)
    order = sorted(range(len(keys)), key=lambda a: (-keys[a], a))
    return order[:k]


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (step number t >= 1); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
