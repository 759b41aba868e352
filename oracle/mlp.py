"""Plain FP64 reference of the density-of-states network used for warm starts.

TEST INFRASTRUCTURE ONLY.  The test suite may import this module; the product
path never does, and nothing here is shared with the GPU library.

The warm start is an extension of the method of arXiv:1407.5140, not part of the
paper: a multilayer perceptron maps x = (E/N, 1/L, q) to ln g(E)/N and its
output, scaled by N, becomes the starting ln g of a larger REWL run that begins
its modification-factor schedule (Sec. II.A) below ln f = 1.  Everything here
is the textbook definition written out in float64:

* hidden units  a = GELU(z) = z * Phi(z) with Phi the standard normal CDF,
  Phi(z) = (1 + erf(z / sqrt 2)) / 2 (Hendrycks & Gimpel's exact form);
* output        y = a_last . w_out + b_out (linear);
* loss          (1/B) sum_r (y_r - t_r)^2;
* gradient      the chain rule applied layer by layer (reverse mode);
* optimiser     Adam (Kingma & Ba 2015, Algorithm 1) with bias correction.

The flat parameter vector is ordered W1[in][H], b1[H], then (W[H][H], b[H]) per
further hidden layer, then w_out[H], b_out; W[i][j] connects input i to unit j.

Pins (tests/test_mlp_oracle.py): the gradient against central finite
differences of the loss; GELU against tabulated values of the normal CDF and
its symmetry; a network whose hidden weights vanish against its closed form;
the first Adam steps against their closed form.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z), phi the standard normal density."""
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def n_params(in_dim: int, hidden: int, layers: int) -> int:
    return in_dim * hidden + hidden + (layers - 1) * (hidden * hidden + hidden) + hidden + 1


def unpack(p, in_dim: int, hidden: int, layers: int):
    """Views (W_l, b_l) for each hidden layer, then (w_out, b_out), of the flat vector."""
    p = np.asarray(p, dtype=np.float64)
    assert p.size == n_params(in_dim, hidden, layers)
    out, o = [], 0
    fan_in = in_dim
    for _ in range(layers):
        W = p[o:o + fan_in * hidden].reshape(fan_in, hidden)
        o += fan_in * hidden
        b = p[o:o + hidden]
        o += hidden
        out.append((W, b))
        fan_in = hidden
    w_out = p[o:o + hidden]
    b_out = p[o + hidden]
    return out, w_out, b_out


def forward(p, x, in_dim: int, hidden: int, layers: int):
    """y[B] and the per-layer pre-activations z_l and activations a_l."""
    hid, w_out, b_out = unpack(p, in_dim, hidden, layers)
    a = np.asarray(x, dtype=np.float64).reshape(-1, in_dim)
    zs, acts = [], [a]
    for W, b in hid:
        z = a @ W + b
        a = gelu(z)
        zs.append(z)
        acts.append(a)
    y = a @ w_out + b_out
    return y, zs, acts


def loss(p, x, t, in_dim: int, hidden: int, layers: int) -> float:
    y, _, _ = forward(p, x, in_dim, hidden, layers)
    d = y - np.asarray(t, dtype=np.float64)
    return float(np.mean(d * d))


def grad(p, x, t, in_dim: int, hidden: int, layers: int):
    """(dloss/dp as a flat vector, loss) by reverse-mode differentiation."""
    y, zs, acts = forward(p, x, in_dim, hidden, layers)
    t = np.asarray(t, dtype=np.float64)
    B = y.shape[0]
    hid, w_out, _ = unpack(p, in_dim, hidden, layers)
    dy = 2.0 * (y - t) / B                                   # dloss/dy_r
    g_wout = acts[-1].T @ dy
    g_bout = dy.sum()
    da = np.outer(dy, w_out)                                 # dloss/da_last
    gW, gb = [None] * layers, [None] * layers
    for l in range(layers - 1, -1, -1):
        dz = da * gelu_grad(zs[l])                           # through the activation
        gW[l] = acts[l].T @ dz                               # acts[l] is the layer's input
        gb[l] = dz.sum(axis=0)
        da = dz @ hid[l][0].T                                # to the previous layer
    parts = []
    for l in range(layers):
        parts += [gW[l].ravel(), gb[l]]
    parts += [g_wout, np.array([g_bout])]
    d = y - t
    return np.concatenate(parts), float(np.mean(d * d))


def adam_step(p, g, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def encode_bins(model: str, q: int, L: int) -> np.ndarray:
    """Network inputs (E/N, 1/L, q) for every global energy bin (q = 2 for Ising).

    Bins follow the REWL convention: Ising E = 4b - 2N for b in [0, N], Potts
    E = b - 2N for b in [0, 2N] (E = -sum over bonds of delta(s_i, s_j), Eq. (2)).
    """
    N = L * L
    if model == "ising":
        E = 4.0 * np.arange(N + 1) - 2.0 * N
        qq = 2
    else:
        E = np.arange(2 * N + 1) - 2.0 * N
        qq = q
    return np.stack([E / N, np.full(E.shape, 1.0 / L), np.full(E.shape, float(qq))], axis=1)


def warm_table(p, model: str, q: int, L: int, hidden: int, layers: int) -> np.ndarray:
    """N * net(E/N, 1/L, q) at every bin (unrounded; the library rounds to 2^-16)."""
    y, _, _ = forward(p, encode_bins(model, q, L), 3, hidden, layers)
    return (L * L) * y
