"""Brute-force value iteration on tiny deterministic grids.

TEST INFRASTRUCTURE ONLY.  The paper contrasts FastMDP with the table-based
value iteration of Bellman's dynamic programming (Sec. II) and states that the
peak construction closely approximates the value function value iteration
produces (Sec. III, Fig. "compare").  With a single positive reward and no
risk wells the construction is exact, which is what the oracle is pinned to.
"""
from __future__ import annotations

import numpy as np


def value_iteration_chain(n: int, goal: int, reward: float, gamma: float, moves=(-1, 1),
                          penalty=None, tol: float = 0.0, max_iter: int = 100000) -> np.ndarray:
    """Optimal values of a deterministic chain x = 0..n-1.

    The goal state is absorbing and worth ``reward`` on arrival; every other
    state takes one of ``moves`` (moves that leave the chain are not
    available) and V(x) = max_a [gamma * V(x + a) - penalty(x + a)], with
    ``penalty`` an optional per-state cost paid on entering a state.
    Iterates the Bellman backup to a fixed point.
    """
    V = np.zeros(n)
    pen = np.zeros(n) if penalty is None else np.asarray(penalty, dtype=np.float64)
    for _ in range(max_iter):
        Vn = np.full(n, -np.inf)
        for x in range(n):
            if x == goal:
                Vn[x] = reward
                continue
            for a in moves:
                y = x + a
                if 0 <= y < n:
                    Vn[x] = max(Vn[x], gamma * V[y] - pen[y])
        if np.max(np.abs(Vn - V)) <= tol:
            return Vn
        V = Vn
    return V


def greedy_chain(V: np.ndarray, x: int, moves=(-1, 1)) -> int:
    """Move that leads to the most valuable neighbour (first on ties)."""
    best, arg = -np.inf, None
    for a in moves:
        y = x + a
        if 0 <= y < V.shape[0] and V[y] > best:
            best, arg = V[y], a
    return arg
