"""Pins of the FP64 network oracle (oracle/mlp.py) against facts that do not come
from its own code: tabulated normal-CDF values, central finite differences of the
loss, a closed form when the hidden weights vanish, the closed form of the first
Adam steps, and an independent library implementation of the same network
(torch.nn in float64 on the CPU)."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from mlp_inputs import params, rows


def test_gelu_is_z_times_normal_cdf():
    # standard normal CDF table values
    table = {0.5: 0.6914624612740131, 1.0: 0.8413447460685429, 2.0: 0.9772498680518208,
             -1.0: 0.15865525393145707, -2.5: 0.006209665325776132}
    for z, phi in table.items():
        assert M.gelu(np.float64(z)) == pytest.approx(z * phi, rel=1e-14, abs=1e-16)
    z = np.linspace(-6, 6, 101)
    assert np.allclose(M.gelu(z) - M.gelu(-z), z, rtol=0, atol=1e-14)   # Phi(z) + Phi(-z) = 1
    assert M.gelu(np.float64(0.0)) == 0.0


def test_gelu_grad_matches_finite_differences():
    z = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.allclose(M.gelu_grad(z), fd, rtol=1e-8, atol=1e-9)
    assert M.gelu_grad(np.float64(0.0)) == 0.5


@pytest.mark.parametrize("in_dim,hidden,layers", [(3, 4, 3), (2, 5, 1), (3, 3, 2)])
def test_gradient_matches_central_differences(in_dim, hidden, layers):
    p = params(in_dim, hidden, layers, seed=7, scale=0.8)
    x, t = rows(9, in_dim, seed=8)
    g, loss = M.grad(p, x, t, in_dim, hidden, layers)
    assert loss == pytest.approx(M.loss(p, x, t, in_dim, hidden, layers), rel=1e-15)
    h = 1e-6
    fd = np.empty_like(g)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (M.loss(p + e, x, t, in_dim, hidden, layers) - M.loss(p - e, x, t, in_dim, hidden, layers)) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_vanishing_hidden_weights_closed_form():
    in_dim, hidden, layers = 3, 6, 3
    p = params(in_dim, hidden, layers, seed=3)
    hid, w_out, b_out = M.unpack(p, in_dim, hidden, layers)
    q = p.copy()
    o = 0
    fan = in_dim
    for _ in range(layers):
        q[o:o + fan * hidden] = 0.0          # weights off, biases kept
        o += fan * hidden + hidden
        fan = hidden
    x, _ = rows(5, in_dim, seed=4)
    y, _, _ = M.forward(q, x, in_dim, hidden, layers)
    last_b = hid[-1][1]
    want = sum(w_out[j] * 0.5 * last_b[j] * (1 + math.erf(last_b[j] / math.sqrt(2))) for j in range(hidden)) + b_out
    assert np.allclose(y, want, rtol=1e-14, atol=1e-14)


def test_adam_first_steps_closed_form():
    # with a constant gradient the bias-corrected moments are g and g^2 exactly,
    # so every step moves each parameter by lr * g / (|g| + eps)
    g = np.array([3.0, -0.5, 0.0, 1e-3])
    p = np.array([1.0, 2.0, 3.0, 4.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-2, 1e-8
    for step in (1, 2, 3):
        p_new, m, v = M.adam_step(p, g, m, v, step, lr, eps=eps)
        assert np.allclose(p - p_new, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
        p = p_new


def test_matches_torch_nn_reference():
    torch = pytest.importorskip("torch")
    in_dim, hidden, layers = 3, 8, 3
    p = params(in_dim, hidden, layers, seed=11)
    x, t = rows(13, in_dim, seed=12)
    hid, w_out, b_out = M.unpack(p, in_dim, hidden, layers)
    mods = []
    fan = in_dim
    for W, b in hid:
        lin = torch.nn.Linear(fan, hidden).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W.T.copy()))    # torch stores [out][in]
            lin.bias.copy_(torch.from_numpy(b.copy()))
        mods += [lin, torch.nn.GELU(approximate="none")]
        fan = hidden
    out = torch.nn.Linear(hidden, 1).double()
    with torch.no_grad():
        out.weight.copy_(torch.from_numpy(w_out.reshape(1, -1).copy()))
        out.bias.fill_(float(b_out))
    net = torch.nn.Sequential(*mods, out)
    xt = torch.from_numpy(x)
    yt = net(xt).squeeze(1)
    loss = torch.mean((yt - torch.from_numpy(t)) ** 2)
    loss.backward()
    y, _, _ = M.forward(p, x, in_dim, hidden, layers)
    assert np.allclose(y, yt.detach().numpy(), rtol=1e-13, atol=1e-14)
    g, lo = M.grad(p, x, t, in_dim, hidden, layers)
    parts = []
    for lin in net[0:2 * layers:2]:
        parts += [lin.weight.grad.numpy().T.ravel(), lin.bias.grad.numpy()]
    parts += [out.weight.grad.numpy().ravel(), out.bias.grad.numpy()]
    assert lo == pytest.approx(float(loss.detach()), rel=1e-13)
    assert np.allclose(g, np.concatenate(parts), rtol=1e-11, atol=1e-13)


def test_bin_encoding_spans_the_energy_range():
    x = M.encode_bins("ising", 2, 4)
    assert x.shape == (17, 3)
    assert tuple(x[0]) == (-2.0, 0.25, 2.0) and tuple(x[-1]) == (2.0, 0.25, 2.0)
    assert np.allclose(np.diff(x[:, 0]), 4 / 16)
    x = M.encode_bins("potts", 10, 4)
    assert x.shape == (33, 3)
    assert tuple(x[0]) == (-2.0, 0.25, 10.0) and tuple(x[-1]) == (0.0, 0.25, 10.0)
