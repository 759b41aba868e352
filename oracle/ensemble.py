"""n-run mean, bootstrap and canonical thermodynamics of REWL results.

TEST INFRASTRUCTURE ONLY (part of the oracle): it checks the GPU library and
the product never imports it.

* Error analysis of Sec. II.B: n independent runs give n pieces per window.
  The mean global ln g averages, window by window, the n pieces bin by bin and
  then concatenates the mean pieces (the joining of Sec. II.B).  A bootstrap
  resample draws n pieces per window with repetition (draws: ``boot_picks``)
  and does the same; the spread over resamples is the statistical error.
  Reading: the mean is taken over ln g values (the quantity each run
  estimates); each run's arbitrary additive constant only shifts the mean
  piece, which the joining removes.
* Canonical averages from a density of states (the specific heat of the
  Potts study, Sec. IV.A): for k_B = J = 1 and temperature T,
  Z = sum_E g(E) e^{-E/T}, u = <E>/N, c = (<E^2> - <E>^2) / (N T^2) written as
  the mean square deviation <(E - <E>)^2>, and f = -T ln Z / N.
"""
from __future__ import annotations

import numpy as np

from . import boot_picks, concat


def mean_pieces(runs: np.ndarray, picks: np.ndarray) -> np.ndarray:
    """runs: (n, h, WB) pieces; picks: (h, n) run per draw.  Per window, the sum
    over draws in draw order, divided by n."""
    n, h, WB = runs.shape
    out = np.empty((h, WB))
    for a in range(h):
        acc = np.zeros(WB)
        for j in range(n):
            acc = acc + runs[picks[a, j], a]
        out[a] = acc / n
    return out


def ensemble(cfg, mask: np.ndarray, runs: np.ndarray, R: int, seed: int):
    """Mean global ln g (row 0) and R bootstrap resamples (rows 1..R), each
    joined and normalised like a single run; joins per row."""
    n, h, _ = runs.shape
    picks = boot_picks(seed, R, h, n)
    rows, joins = [], []
    for r in range(R + 1):
        out, join = concat(cfg, mask, mean_pieces(runs, picks[r]))
        rows.append(out)
        joins.append(join)
    return np.array(rows), np.array(joins).reshape(R + 1, max(h - 1, 0))


def energies(model: str, L: int) -> np.ndarray:
    """Energy of every bin: Ising E = 4b - 2N, Potts E = b - 2N."""
    N = L * L
    W = N + 1 if model == "ising" else 2 * N + 1
    b = np.arange(W, dtype=np.float64)
    return 4.0 * b - 2.0 * N if model == "ising" else b - 2.0 * N


def canonical(model: str, L: int, lng: np.ndarray, T) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """u(T), c(T), f(T) per spin for ln g over the model's bins (-inf: absent)."""
    N = L * L
    E = energies(model, L)
    ok = np.isfinite(lng)
    E, s = E[ok], lng[ok]
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    u = np.empty(T.size)
    c = np.empty(T.size)
    f = np.empty(T.size)
    for i, t in enumerate(T):
        x = s - E / t
        m = x.max()
        w = np.exp(x - m)
        Z = w.sum()
        U = (w * E).sum() / Z
        V = (w * (E - U) ** 2).sum() / Z
        u[i] = U / N
        c[i] = V / (N * t * t)
        f[i] = -t * (m + np.log(Z)) / N
    return u, c, f
