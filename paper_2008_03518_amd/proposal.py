"""Training driver of the learned action proposal.

Tuples (features of the state, action the plain planner chose there) are
taken from first-come-first-served runs of the full-sweep planner on
seeded synthetic traffic; the network is trained with the library's own
BF16 MFMA forward / backward kernels and Adam on FP32 master weights.
Everything here is argument marshalling around the C ABI: the planning,
the features and every training step run in the HIP kernels.
"""
from __future__ import annotations

import math
from typing import Iterable, Optional

import numpy as np

from . import fastmdp as fm
from . import scenario as S


def trajectory_tuples(plans, requests, seq0: int):
    """States, goals, rows, sequence numbers and chosen actions of every
    step of every planned trajectory (host arrays).  Step k of request i
    went from point k (row t0 + k) by action[k + 1]."""
    st, gl, rw, sq, ac = [], [], [], [], []
    for i, p in enumerate(plans):
        n = p.n_points
        if n < 2:
            continue
        st.append(p.xyz[: n - 1])
        gl.append(np.repeat(np.asarray(requests.goal[i], dtype=np.float64)[None, :], n - 1, axis=0))
        rw.append(p.t0 + np.arange(n - 1, dtype=np.int32))
        sq.append(np.full(n - 1, seq0 + i, dtype=np.int32))
        ac.append(p.action[1:n].astype(np.int32))
    if not st:
        z = np.zeros((0, 3))
        return z, z, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32)
    return (np.concatenate(st), np.concatenate(gl), np.concatenate(rw), np.concatenate(sq), np.concatenate(ac))


def generate_dataset(seeds: Iterable[int], n_tuples: int, n_plans: int = 3000, n_requests: int = 1000,
                     max_slots: int = 1024, sample_seed: int = 0, log=None):
    """(X [N, 96] FP32, y [N] int32) as device arrays: N = n_tuples drawn
    evenly over the seeds, each seed one FCFS run of the plain planner on
    its own synthetic scenario of the 3000-plan, 360-action kind."""
    seeds = list(seeds)
    per = int(math.ceil(n_tuples / len(seeds)))
    rng = np.random.default_rng(sample_seed)
    Xs, ys = [], []
    for sd in seeds:
        sc = S.large_actions(seed=sd, n_plans=n_plans, n_requests=n_requests)
        ctx = fm.context_for(sc, max_slots=max_slots)
        seq0 = ctx.next_seq()
        plans, _, _ = ctx.plan_fcfs(sc.requests)
        st, gl, rw, sq, ac = trajectory_tuples(plans, sc.requests, seq0)
        take = np.sort(rng.choice(st.shape[0], size=min(per, st.shape[0]), replace=False))
        Xs.append(ctx.features(st[take], gl[take], rw[take], sq[take]).numpy())
        ys.append(ac[take])
        ctx.close()
        if log:
            log(f"dataset seed {sd}: {st.shape[0]} steps, {take.size} taken")
    X = np.concatenate(Xs)[:n_tuples]
    y = np.concatenate(ys)[:n_tuples]
    return fm.DeviceArray.from_host(X, np.float32), fm.DeviceArray.from_host(y, np.int32)


def init_params(n_out: int, seed: int, n_in: int = fm.N_FEAT, n_hidden: int = fm.MLP_HIDDEN) -> dict:
    """He-uniform weights, zero biases (x @ W convention)."""
    rng = np.random.default_rng(seed)

    def lin(fi, fo):
        lim = math.sqrt(6.0 / fi)
        return rng.uniform(-lim, lim, (fi, fo)), np.zeros(fo)

    W1, b1 = lin(n_in, n_hidden)
    W2, b2 = lin(n_hidden, n_hidden)
    W3, b3 = lin(n_hidden, n_out)
    return dict(W1=W1, b1=b1, W2=W2, b2=b2, W3=W3, b3=b3)


def train(net: "fm.Mlp", X, y, epochs: int = 4, batch: int = 4096, lr: float = 2e-3, seed: int = 0,
          log=None) -> list:
    """Adam on shuffled batches (batch a multiple of 32; the tail is dropped).
    X, y are device arrays.  Returns the mean loss of each epoch."""
    n = len(X)
    batch = min(batch, net.max_batch) // 32 * 32
    rng = np.random.default_rng(seed)
    out = []
    for ep in range(epochs):
        perm = fm.DeviceArray.from_host(rng.permutation(n).astype(np.int64))
        Xp, yp = X.gather(perm), y.gather(perm)
        tot, cnt = 0.0, 0
        for i in range(0, n - batch + 1, batch):
            tot += net.train_step(_rows(Xp, i, batch), _rows(yp, i, batch), lr)
            cnt += 1
        out.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {out[-1]:.4f}")
    return out


def _rows(a: "fm.DeviceArray", i: int, k: int) -> "fm.DeviceArray":
    return a.rows(i, k)


def accuracy(net: "fm.Mlp", X, y, batch: Optional[int] = None) -> float:
    """Fraction of tuples whose largest logit is the chosen action."""
    batch = batch or net.max_batch
    n = len(X)
    yh = y.numpy()
    hit = 0
    for i in range(0, n, batch):
        k = min(batch, n - i)
        lg = net.forward(_rows(X, i, k))
        hit += int((lg.argmax(axis=1) == yh[i: i + k]).sum())
    return hit / max(n, 1)
