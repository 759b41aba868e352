"""GPU parity of the density-of-states network (BF16 matrix-core kernels, FP32
accumulation) against the FP64 oracle (oracle/mlp.py).

Tolerance.  The device multiplies with BF16 copies of the hidden weights, so
the oracle is evaluated at those weight values (rounded to nearest even by a
library conversion on the CPU); what remains is the rounding of activations and
back-propagated errors to BF16 (unit roundoff u = 2^-8), FP32 accumulation and
the device's erff/expf (a few ulp).  These elementary roundings are independent
of one another (probabilistic rounding-error analysis, Higham & Mary, SIAM J.
Sci. Comput. 41 (2019)); a rounding of a value v is an error uniform within
+-u|v| (variance at most (u v)^2 / 3).
* Outputs: every elementary rounding is carried to y by the network's exact
  Jacobian (back-propagation of dy = 1 through the FP64 oracle), which gives the
  first-order standard deviation sigma of each y exactly under that model.
* Gradients: the same model is propagated by Monte Carlo: the FP64 forward and
  backward pass is repeated with every BF16-rounded quantity multiplied by
  (1 + u xi), xi uniform in [-1, 1], and sigma is the spread of the results.
The tests allow 6 sigma (8 for the 64-sample Monte Carlo estimate) plus a floor
of 2^-20 of the largest magnitude (FP32 effects).
"""
import numpy as np
import pytest

from oracle import mlp as M
from mlp_inputs import params, rows

pytestmark = pytest.mark.gpu

U = 2.0 ** -8          # BF16 unit roundoff (8-bit significand, round to nearest even)
E32 = 2.0 ** -24       # FP32 unit roundoff
V3 = 1.0 / 3.0         # variance of a rounding error uniform in [-1, 1] ulp/2 units
K_SIGMA = 6.0


@pytest.fixture(scope="module")
def rw():
    import paper_1407_5140_amd as rw
    return rw


def gelu2(z):
    return np.exp(-0.5 * z * z) / np.sqrt(2 * np.pi) * (2.0 - z * z)


def bf16_round(a):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, np.float32))
    return t.to(torch.bfloat16).float().numpy().astype(np.float64)


def device_weights(p, in_dim, hidden, layers):
    """The parameter vector with every hidden x hidden matrix rounded to BF16."""
    q = np.array(p, dtype=np.float64)
    o = in_dim * hidden + hidden
    for _ in range(1, layers):
        q[o:o + hidden * hidden] = bf16_round(q[o:o + hidden * hidden])
        o += hidden * hidden + hidden
    return q


def forward_sigma(pw, x, in_dim, hidden, layers):
    """(y, sigma of y per row) at weights pw."""
    hid, w_out, b_out = M.unpack(pw, in_dim, hidden, layers)
    y, zs, acts = M.forward(pw, x, in_dim, hidden, layers)
    fn = 16 * E32 ** 2                                   # erff / expf: a few ulp
    var = (hidden + 1) * E32 ** 2 * V3 * ((acts[-1] ** 2) @ w_out ** 2 + b_out ** 2)
    J = np.broadcast_to(w_out, acts[-1].shape)          # dy / da of the last hidden layer
    for l in range(layers - 1, -1, -1):
        var = var + (U ** 2 + fn) * V3 * np.sum(J ** 2 * acts[l + 1] ** 2, axis=1)   # a_l to BF16
        Jz = J * M.gelu_grad(zs[l])                                                # dy / dz_l
        W, b = hid[l]
        K = in_dim if l == 0 else hidden
        var = var + np.sum(Jz ** 2 * ((K + 1) * E32 ** 2 * V3 * ((acts[l] ** 2) @ W ** 2 + b ** 2)), axis=1)
        J = Jz @ W.T
    return y, np.sqrt(var)


def _rounded(v, rng):
    return v * (1.0 + U * rng.uniform(-1.0, 1.0, v.shape))


def _perturbed_grad(pw, x, t, in_dim, hidden, layers, rng):
    """FP64 gradient with every quantity the device rounds to BF16 perturbed by one
    rounding (activations, and the errors that feed the two matrix products)."""
    hid, w_out, b_out = M.unpack(pw, in_dim, hidden, layers)
    a = x
    zs, acts = [], [x]
    for W, b in hid:
        z = a @ W + b
        a = _rounded(M.gelu(z), rng)
        zs.append(z)
        acts.append(a)
    y = a @ w_out + b_out
    dy = 2.0 * (y - t) / x.shape[0]
    g_wout, g_bout = a.T @ dy, dy.sum()
    D = np.outer(dy, w_out) * M.gelu_grad(zs[-1])
    gW, gb = [None] * layers, [None] * layers
    for l in range(layers - 1, 0, -1):
        D16 = _rounded(D, rng)
        gW[l] = acts[l].T @ D16
        gb[l] = D.sum(axis=0)
        D = (D16 @ hid[l][0].T) * M.gelu_grad(zs[l - 1])
    gW[0] = x.T @ D
    gb[0] = D.sum(axis=0)
    parts = []
    for l in range(layers):
        parts += [gW[l].ravel(), gb[l]]
    return np.concatenate(parts + [g_wout, np.array([g_bout])])


def grad_sigma(pw, x, t, in_dim, hidden, layers, samples=64, seed=0):
    rng = np.random.default_rng(seed)
    g0, _ = M.grad(pw, x, t, in_dim, hidden, layers)
    acc = np.zeros_like(g0)
    for _ in range(samples):
        acc += (_perturbed_grad(pw, x, t, in_dim, hidden, layers, rng) - g0) ** 2
    return g0, np.sqrt(acc / samples)


def within(dev, ref, sigma, k=K_SIGMA):
    return np.abs(dev - ref) <= k * sigma + 2 ** -20 * np.max(np.abs(ref))


# ------------------------------------------------------------ matrix cores
def test_gemm_lane_layout_exact(rw):
    # small integers over 8 are exact in BF16 and every partial sum is exact in
    # FP32, so the product must match bit for bit: this pins the operand and
    # accumulator lane layout of the matrix instruction
    rng = np.random.default_rng(5)
    for M_, N_, K in [(64, 64, 32), (128, 192, 96), (128, 64, 256)]:
        A = rng.integers(-8, 9, (M_, K)) / 8.0
        B = rng.integers(-8, 9, (K, N_)) / 8.0
        C = rw.mlp_probe_gemm(A, B)
        assert np.array_equal(C.astype(np.float64), A @ B), (M_, N_, K)


def test_gemm_rounds_operands_to_bf16(rw):
    rng = np.random.default_rng(6)
    A = rng.standard_normal((128, 256))
    B = rng.standard_normal((256, 64))
    C = rw.mlp_probe_gemm(A, B).astype(np.float64)
    Ar, Br = bf16_round(A), bf16_round(B)
    ref = Ar @ Br
    bound = 256 * E32 * (np.abs(Ar) @ np.abs(Br))
    assert np.all(np.abs(C - ref) <= bound)
    # and not the unrounded product: the BF16 rounding is visible
    assert np.max(np.abs(C - A @ B)) > 10 * np.max(bound)


def test_gemm_rejects_ragged_shapes(rw):
    with pytest.raises(rw.MlpError):
        rw.mlp_probe_gemm(np.ones((30, 32)), np.ones((32, 64)))
    with pytest.raises(rw.MlpError):
        rw.mlp_probe_gemm(np.ones((64, 16)), np.ones((16, 64)))


# ------------------------------------------------------------ network
SHAPE = (3, 256, 3)


@pytest.fixture(scope="module")
def net(rw):
    n = rw.Mlp(*SHAPE, max_batch=512, seed=1)
    yield n
    n.close()


def test_parameter_count_and_roundtrip(net):
    assert net.n_params == M.n_params(*SHAPE) == 132865
    p = params(*SHAPE, seed=21)
    net.set_params(p)
    assert np.array_equal(net.params().astype(np.float64), p)


@pytest.mark.parametrize("B", [1, 31, 300, 1100])
def test_forward_matches_oracle(net, B):
    p = params(*SHAPE, seed=22)
    net.set_params(p)
    x, t = rows(B, 3, seed=23 + B)
    y = net.infer(x).astype(np.float64)
    yo, sy = forward_sigma(device_weights(p, *SHAPE), x, *SHAPE)
    assert within(y, yo, sy).all()


@pytest.mark.parametrize("B,seed", [(200, 31), (512, 32), (64, 33), (7, 34)])
def test_gradient_matches_oracle(net, B, seed):
    p = params(*SHAPE, seed=seed)
    net.set_params(p)
    x, t = rows(B, 3, seed=seed + 100)
    g, loss = net.grad(x, t)
    pw = device_weights(p, *SHAPE)
    _, lo = M.grad(pw, x, t, *SHAPE)
    go, sg = grad_sigma(pw, x, t, *SHAPE)
    ok = within(g.astype(np.float64), go, sg, k=8.0)
    assert ok.all(), f"{(~ok).sum()} of {g.size} gradient entries outside the bound"
    assert np.median(sg / np.maximum(np.abs(go), 1e-300)) < 1e-2     # the bound is tight
    assert loss == pytest.approx(lo, rel=1e-2)


def test_adam_steps_match_oracle(rw):
    # one repeated row makes every minibatch the same, so each device step uses
    # the gradient mlp_grad reports at the same parameters; the FP64 Adam update
    # of that gradient must match the device's FP32 update to rounding
    net = rw.Mlp(*SHAPE, max_batch=64, seed=2)
    try:
        p = params(*SHAPE, seed=41)
        net.set_params(p)
        x, t = rows(1, 3, seed=42)
        X, T = np.repeat(x, 64, axis=0), np.repeat(t, 64)
        lr = 1e-3
        m = np.zeros_like(p)
        v = np.zeros_like(p)
        po = p.copy()
        for step in (1, 2, 3):
            g, _ = net.grad(X, T)
            net.fit(X, T, steps=1, batch=64, lr=lr, seed=7)
            po_new, m, v = M.adam_step(po, g.astype(np.float64), m, v, step, lr)
            pd = net.params().astype(np.float64)
            assert np.all(np.abs(pd - po_new) <= 1e-4 * lr + 2 ** -23 * np.abs(po_new))
            assert np.abs(pd - po).max() > 0.5 * lr                      # the step was taken
            po = pd
    finally:
        net.close()


def test_training_fits_exact_ising_entropy(rw, golden):
    # ln g / N of the exact Ising DOS at L = 16, 24, 32: the network must learn
    # it to a small error within a few thousand device steps
    xs, ts = [], []
    for L in (16, 24, 32):
        lng = golden.lng(f"ising_L{L}_lng.txt")
        ok = np.isfinite(lng)
        enc = M.encode_bins("ising", 2, L)[ok]
        xs.append(enc)
        ts.append(lng[ok] / (L * L))
    x = np.concatenate(xs).astype(np.float32).astype(np.float64)
    t = np.concatenate(ts).astype(np.float32).astype(np.float64)
    net = rw.Mlp(*SHAPE, max_batch=1024, seed=3)
    try:
        l0 = float(np.mean((net.infer(x) - t) ** 2))
        net.fit(x, t, steps=1500, batch=512, lr=1e-3, seed=1)
        y = net.infer(x).astype(np.float64)
        l1 = float(np.mean((y - t) ** 2))
        print(f"[mlp fit] loss {l0:.3e} -> {l1:.3e}, rms {np.sqrt(l1):.3e}, max {np.max(np.abs(y - t)):.3e}")
        assert l1 < 1e-3 * l0 and np.sqrt(l1) < 1e-2
        pw = device_weights(net.params(), *SHAPE)            # trained weights, FP64 forward
        yo, sy = forward_sigma(pw, x, *SHAPE)
        assert within(y, yo, sy).all()
        assert np.median(K_SIGMA * sy / np.abs(yo)) < 1e-2
    finally:
        net.close()


@pytest.mark.parametrize("model,q,L", [("ising", 2, 16), ("potts", 10, 12), ("ising", 2, 128)])
def test_warm_table_matches_oracle(net, model, q, L):
    p = params(*SHAPE, seed=51)
    net.set_params(p)
    tab = net.warm_table(model, q, L)
    N = L * L
    assert tab.shape == ((N + 1) if model == "ising" else (2 * N + 1),)
    assert np.array_equal(tab * 65536, np.round(tab * 65536))        # multiples of 2^-16
    x = M.encode_bins(model, q, L).astype(np.float32).astype(np.float64)
    yo, sy = forward_sigma(device_weights(p, *SHAPE), x, *SHAPE)
    assert (np.abs(tab - N * yo) <= N * (K_SIGMA * sy + 2 ** -20 * np.max(np.abs(yo))) + 2 ** -17).all()
