"""Workload definitions (problem statements only, no arithmetic of the method).

Each workload is a list of keyword dicts accepted by `make_config` of the binding
and of the oracle: model, q, L, n_windows, overlap, m, flat, k0, kfinal, X, seed.
"""
from __future__ import annotations

_BATCH_TYPES = [("ising", 2, 16), ("ising", 2, 24), ("ising", 2, 32), ("ising", 2, 48),
                ("ising", 2, 64), ("potts", 4, 16), ("potts", 4, 24), ("potts", 4, 32),
                ("potts", 8, 16), ("potts", 8, 24), ("potts", 8, 32), ("potts", 10, 16),
                ("potts", 10, 24), ("potts", 10, 32)]


def single(name: str) -> dict:
    """The single-instance workloads: Ising L=8 (4 windows, 1 walker each, ln f to 2^-20),
    Ising L=32 (8 windows x 16 walkers, ln f to 2^-20), 10-state Potts L=100 (the paper's
    77 windows of 1001 bins, 8 walkers each),
    Ising L=64 (16 windows x 64 walkers) and 10-state Potts L=32 (32 windows x 128
    walkers), both to ln f = 2^-27, and the larger targets Ising L=128 (32 x 64) and 10-state
    Potts L=64 (32 x 128); 75% overlap, flatness 4/5, X = 10^4, seed 1."""
    table = {
        "ising8": dict(model="ising", q=2, L=8, n_windows=4, m=1, kfinal=20, X=10000, seed=1),
        "ising32": dict(model="ising", q=2, L=32, n_windows=8, m=16, kfinal=20, X=10000, seed=1),
        "ising64": dict(model="ising", q=2, L=64, n_windows=16, m=64, kfinal=27, X=10000, seed=1),
        "potts32": dict(model="potts", q=10, L=32, n_windows=32, m=128, kfinal=27, X=10000, seed=1),
        # the paper's smallest Potts lattice (Sec. IV.A): 77 windows of 1001 bins, 75 % overlap
        "potts100": dict(model="potts", q=10, L=100, n_windows=77, m=8, kfinal=27, X=10000, seed=1),
        # the warm start's larger targets: Ising L=128 (h=32, m=64) and 10-state Potts L=64
        # (h=32, m=128), both to ln f = 2^-27
        "ising128": dict(model="ising", q=2, L=128, n_windows=32, m=64, kfinal=27, X=10000, seed=1),
        "potts64": dict(model="potts", q=10, L=64, n_windows=32, m=128, kfinal=27, X=10000, seed=1),
    }
    return dict(table[name])


def batch(n: int = 64, X: int = 10000) -> list[dict]:
    """n independent instances of uneven size: instance i takes type i mod 14 of
    Ising L in {16, 24, 32, 48, 64} and Potts q in {4, 8, 10} x L in {16, 24, 32};
    h = 8 windows if N <= 576, 16 if N <= 1024, else 32; m = 32, 64, 128 by i mod 3;
    overlap 3/4, flatness 4/5, ln f 1 -> 2^-27, seed 1000 + i."""
    out = []
    for i in range(n):
        model, q, L = _BATCH_TYPES[i % len(_BATCH_TYPES)]
        N = L * L
        h = 8 if N <= 576 else (16 if N <= 1024 else 32)
        out.append(dict(model=model, q=q, L=L, n_windows=h, m=(32, 64, 128)[i % 3], kfinal=27,
                        X=X, seed=1000 + i))
    return out
