"""Seeded synthetic inputs for the density-of-states network (parameters, rows,
targets).  Shared by the oracle tests and the GPU parity tests; holds none of
the network's arithmetic.  Every value is a float32 number (the GPU path's
parameter and input type) returned as float64, so both sides see it exactly."""
import numpy as np


def params(in_dim: int, hidden: int, layers: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Weights uniform in +-scale/sqrt(fan_in), biases uniform in +-0.1 (flat order
    W1, b1, (W, b) per further hidden layer, w_out, b_out)."""
    rng = np.random.default_rng(seed)
    parts = []
    fan = in_dim
    for _ in range(layers):
        parts.append(rng.uniform(-1, 1, fan * hidden) * scale / np.sqrt(fan))
        parts.append(rng.uniform(-0.1, 0.1, hidden))
        fan = hidden
    parts.append(rng.uniform(-1, 1, hidden) * scale / np.sqrt(hidden))
    parts.append(rng.uniform(-0.1, 0.1, 1))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def rows(B: int, in_dim: int, seed: int):
    """x[B][in_dim], t[B].  With in_dim = 3 the rows look like the warm-start
    encoding: E/N in [-2, 2], 1/L for L in 8..48, q in {2, 4, 8, 10}; targets of the
    size of ln g / N (0 .. ln 10)."""
    rng = np.random.default_rng(seed)
    if in_dim == 3:
        x = np.stack([rng.uniform(-2, 2, B), 1.0 / rng.integers(8, 49, B),
                      rng.choice([2.0, 4.0, 8.0, 10.0], B)], axis=1)
    else:
        x = rng.uniform(-1, 1, (B, in_dim))
    t = rng.uniform(0, np.log(10.0), B)
    return x.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)
