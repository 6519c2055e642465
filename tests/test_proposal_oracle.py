"""Pins of the proposal certificate and the Adam reference (CPU)."""
import numpy as np

from oracle import proposal as P


def _instance(rng, A):
    """Goal terms in (0, 1], some actions outside the box (-inf), values =
    goal term minus a non-negative penalty (zero for most actions)."""
    G = rng.uniform(0.0, 1.0, A) ** 3
    G[rng.random(A) < 0.1] = -np.inf
    pen = np.where(rng.random(A) < 0.4, rng.uniform(0.0, 1.0, A), 0.0)
    V = G - pen
    V[G == -np.inf] = -np.inf
    # a few exact and near ties
    if A > 4:
        V[3] = V[1]
        G[3] = max(G[3], V[3])
    return V, G


def test_certificate_reproduces_full_argmax():
    rng = np.random.default_rng(0)
    hits = 0
    for trial in range(3000):
        A = int(rng.integers(2, 40))
        V, G = _instance(rng, A)
        k = int(rng.integers(1, min(A, 8) + 1))
        K = rng.choice(A, size=k, replace=False) if trial % 2 else P.top_k(G, k)
        ok, a = P.certify(V[K], K, G, 1e-9)
        if ok:
            hits += 1
            assert a == P.argmax_tie(V, 1e-9), (trial, V, G, K)
    assert hits > 500


def test_goal_ordering_certifies_whenever_any_set_does():
    """If some k-set is certified, the top-k goal terms are certified too."""
    rng = np.random.default_rng(1)
    for trial in range(2000):
        A = int(rng.integers(2, 30))
        V, G = _instance(rng, A)
        k = int(rng.integers(1, min(A, 6) + 1))
        K = rng.choice(A, size=k, replace=False)
        ok, a = P.certify(V[K], K, G, 1e-9)
        if ok:
            Kg = P.top_k(G, k)
            okg, ag = P.certify(V[Kg], Kg, G, 1e-9)
            assert okg and ag == a, (trial, V, G, K, Kg)


def test_certificate_refuses_when_an_outside_bound_reaches_the_threshold():
    V = np.array([0.5, 0.4, 0.3])
    G = np.array([0.5, 0.6, 0.3])
    assert P.certify(V[[0]], [0], G, 1e-9) == (False, -1)       # action 1 could still win
    assert P.certify(V[[0, 1]], [0, 1], G, 1e-9) == (True, 0)
    # outside bound inside the tie band: refused (it might be chosen on the index rule)
    G2 = np.array([0.5, 0.5 * (1 - 1e-12), 0.1])
    assert P.certify(V[[0]], [0], G2, 1e-9)[0] is False


def test_adam_first_step_moves_by_lr_times_sign():
    """Bias correction makes the first step lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p, m, v = P.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # constant gradient: every step has m_hat = g, v_hat = g^2
    for t in range(2, 6):
        p2, m, v = P.adam_step(p, g, m, v, t, lr=0.01)
        assert np.allclose(p2 - p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
        p = p2
