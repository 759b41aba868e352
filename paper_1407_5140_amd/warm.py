"""Warm start of REWL from a network trained on REWL results of smaller systems.

The pipeline (an extension of the method of arXiv:1407.5140, not part of it):

1. REWL runs smaller instances to convergence (one batched handle); the
   concatenated, normalised ln g of each (Sec. II.B) becomes training rows
   x = (E/N, 1/L, q), t = ln g(E)/N over the energy levels that occur.
2. The network of include/rewl_mlp.h is trained on those rows on the device.
3. For a larger target, the network's table N * net(E/N, 1/L, q) (rounded to
   2^-16) replaces the flat starting ln g, and the run begins its ln f schedule
   at 2^-k0 instead of 1 (Sec. II.A).  Everything else of the method is unchanged.

This module only arranges data and calls; every step runs in the library.
"""
from __future__ import annotations

import time

import numpy as np

from . import Mlp, Rewl, make_config, make_tune

# instance types of the training set: Ising L <= 48 and Potts q in {4, 8, 10}, L <= 32
TRAIN_TYPES = [("ising", 2, 16), ("ising", 2, 24), ("ising", 2, 32), ("ising", 2, 48),
               ("potts", 4, 16), ("potts", 4, 24), ("potts", 4, 32), ("potts", 8, 16),
               ("potts", 8, 24), ("potts", 8, 32), ("potts", 10, 16), ("potts", 10, 24),
               ("potts", 10, 32)]


def n_windows_for(L: int) -> int:
    N = L * L
    return 8 if N <= 576 else (16 if N <= 1024 else 32)


def training_workload(types=TRAIN_TYPES, m: int = 32, kfinal: int = 16, X: int = 10000,
                      seed0: int = 2000) -> list[dict]:
    """One plain REWL instance per type (overlap 3/4, flatness 4/5, ln f 1 -> 2^-kfinal)."""
    return [dict(model=mo, q=q, L=L, n_windows=n_windows_for(L), m=m, kfinal=kfinal, X=X,
                 seed=seed0 + i) for i, (mo, q, L) in enumerate(types)]


def run_to_convergence(kws: list[dict], max_seconds: float, tune=None, poll: int = 50,
                       warm_tables=None, log=None):
    """Run the instances in one batch until all converge or time runs out.

    Returns (handle, per-instance dict with converged flag, intervals and seconds
    at convergence, the latter at `poll`-interval resolution)."""
    cfgs = [make_config(**kw) for kw in kws]
    g = Rewl(cfgs, tune=tune if tune is not None else make_tune(poll_every=poll))
    if warm_tables is not None:
        for i, tab in enumerate(warm_tables):
            if tab is not None:
                g.set_initial_lng(tab, i)
    n = len(cfgs)
    done_at = [None] * n
    t0 = time.perf_counter()
    last = t0
    while True:
        all_done = g.run(poll)
        now = time.perf_counter() - t0
        for i in range(n):
            if done_at[i] is None:
                st = g.stats(i)
                if st["windows_done"] == kws[i]["n_windows"]:
                    done_at[i] = (st["intervals"], now)
        if all_done or now > max_seconds:
            break
        if log and now - (last - t0) > 10:
            log(f"{now:.0f} s: {sum(d is not None for d in done_at)}/{n} instances done")
            last = time.perf_counter()
    res = []
    for i in range(n):
        st = g.stats(i)
        res.append(dict(converged=done_at[i] is not None,
                        intervals=done_at[i][0] if done_at[i] else st["intervals"],
                        seconds=done_at[i][1] if done_at[i] else None,
                        min_k=st["min_k"]))
    return g, res


def training_rows(g: Rewl, kws: list[dict], which=None):
    """Rows (E/N, 1/L, q) -> ln g / N from converged instances of handle g."""
    xs, ts = [], []
    for i, kw in enumerate(kws):
        if which is not None and not which[i]:
            continue
        lng, _ = g.concat(i)
        L = kw["L"]
        N = L * L
        b = np.arange(lng.size, dtype=np.float64)
        E = 4.0 * b - 2.0 * N if kw["model"] == "ising" else b - 2.0 * N
        ok = np.isfinite(lng)
        q = 2.0 if kw["model"] == "ising" else float(kw["q"])
        xs.append(np.stack([E[ok] / N, np.full(ok.sum(), 1.0 / L), np.full(ok.sum(), q)], axis=1))
        ts.append(lng[ok] / N)
    return np.concatenate(xs).astype(np.float32), np.concatenate(ts).astype(np.float32)


def train(x, t, steps: int = 4000, batch: int = 4096, lr: float = 1e-3, seed: int = 1,
          hidden: int = 256, layers: int = 3, decay_every: int = 0) -> tuple[Mlp, dict]:
    """Fit the network on the rows; lr is divided by 10 every `decay_every` steps
    (0: constant).  Returns the network and a summary."""
    net = Mlp(3, hidden, layers, max_batch=max(batch, 32), seed=seed)
    t0 = time.perf_counter()
    done = 0
    cur = lr
    chunk = decay_every or steps
    loss = float("nan")
    while done < steps:
        n = min(chunk, steps - done)
        loss = net.fit(x, t, n, batch=batch, lr=cur, seed=seed)
        done += n
        cur *= 0.1
    secs = time.perf_counter() - t0
    y = net.infer(x)
    err = y - t
    return net, dict(steps=steps, seconds=secs, last_batch_loss=loss, rms=float(np.sqrt(np.mean(err ** 2))),
                     max_abs=float(np.max(np.abs(err))), rows=int(len(t)))


def warm_table(net: Mlp, kw: dict) -> np.ndarray:
    return net.warm_table(kw["model"], kw["q"], kw["L"])


def suggest_k0(rms_s: float, N: int, k_max: int = 10) -> int:
    """Initial ln f = 2^-k0 for a warm table whose error in ln g/N is about rms_s.

    The table's error in ln g is about delta = rms_s N.  Measured on 10-state Potts
    L=16 with smooth table errors of known size: up to delta ~ 1 a start at 2^-10
    needs a third of plain WL's intervals, and at delta = 10 a start at 2^-6 beats
    one at 2^-10.  So k0 = k_max - log2(delta) for delta > 1, floored, within
    0..k_max."""
    delta = max(float(rms_s) * float(N), 1.0)
    return int(min(k_max, max(0, np.floor(k_max - np.log2(delta)))))
