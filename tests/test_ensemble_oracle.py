"""Pins of the oracle's n-run error analysis and canonical averages.

The bootstrap of Sec. II.B is pinned by what it must reproduce: exact pieces
with arbitrary per-run constants give the exact ln g in every row, and the
spread of a within-piece difference over resamples equals the closed-form
bootstrap variance of a mean of n values.  The canonical averages are pinned
by direct Boltzmann sums over every microstate of small lattices, by the
infinite- and zero-temperature limits, and by Onsager's exact solution (the
exact 64 x 64 torus DOS away from T_c).
"""
import numpy as np
import pytest

import oracle as O
from oracle import ensemble as EN
from oracle import exact_dos as X


# ------------------------------------------------------------ bootstrap draws
def test_boot_picks_shape_identity_and_range():
    p = O.boot_picks(seed=11, R=50, h=3, n=5)
    assert p.shape == (51, 3, 5)
    assert np.array_equal(p[0], np.tile(np.arange(5), (3, 1)))
    assert p.min() >= 0 and p.max() < 5
    assert np.array_equal(O.boot_picks(11, 50, 3, 5), p)          # deterministic
    assert not np.array_equal(O.boot_picks(12, 50, 3, 5)[1:], p[1:])
    assert np.all(O.boot_picks(3, 10, 2, 1) == 0)                  # one run: always run 0
    with pytest.raises(ValueError):
        O.boot_picks(1, -1, 2, 2)
    with pytest.raises(ValueError):
        O.boot_picks(1, 2, 2, 0)


def test_boot_picks_uniform_and_independent():
    n, R, h = 7, 3000, 4
    p = O.boot_picks(seed=5, R=R, h=h, n=n)[1:]
    cnt = np.bincount(p.ravel(), minlength=n)
    exp = p.size / n
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert chi2 < 35.0                              # 6 degrees of freedom, p ~ 1e-5
    # windows draw independently: equal picks in windows 0 and 1 at rate 1/n
    same = np.mean(p[:, 0, :] == p[:, 1, :])
    sd = np.sqrt((1 / n) * (1 - 1 / n) / p[:, 0, :].size)
    assert abs(same - 1 / n) < 6 * sd
    # draws of one window are independent of each other
    same = np.mean(p[:, 2, 0] == p[:, 2, 1])
    sd = np.sqrt((1 / n) * (1 - 1 / n) / R)
    assert abs(same - 1 / n) < 6 * sd


def test_boot_pick_is_the_stated_philox_word():
    seed, n = 0x1234_5678_9ABC, 9
    p = O.boot_picks(seed, 3, 2, n)
    for r in (1, 3):
        for a in (0, 1):
            for j in (0, 8):
                x0 = O.philox((r, j, a, 4), (seed & 0xFFFFFFFF, seed >> 32))[0]
                assert p[r, a, j] == (x0 * n) >> 32


# ------------------------------------------------------------ mean + joining
def _exact_pieces(lg, c, mask, consts):
    lo, hi = O.layout(c)
    WB = int((hi - lo).max()) + 1
    h = c.n_windows
    runs = np.zeros((len(consts), h, WB))
    for j, cj in enumerate(consts):
        for a in range(h):
            seg = np.where(mask[lo[a]:hi[a] + 1] > 0, lg[lo[a]:hi[a] + 1], 0.0)
            runs[j, a, :seg.size] = seg + cj[a]
    return runs, lo, hi


def test_ensemble_of_exact_pieces_is_exact(golden):
    """Any per-run, per-window constants: every row (mean and resamples) is exact."""
    lg = golden.lng("ising_L16_lng.txt")
    rng = np.random.default_rng(8)
    for h, n in ((2, 1), (5, 4), (8, 3)):
        c = O.make_config("ising", L=16, n_windows=h)
        mask = O.mask_rule(c)
        runs, _, _ = _exact_pieces(lg, c, mask, rng.uniform(-60, 60, size=(n, h)))
        rows, joins = EN.ensemble(c, mask, runs, R=6, seed=2)
        ok = mask > 0
        assert rows.shape == (7, lg.size) and joins.shape == (7, h - 1)
        assert np.max(np.abs(rows[:, ok] - lg[ok])) < 1e-9
        assert np.all(np.isneginf(rows[:, ~ok]))


def test_mean_row_equals_single_run_concat_for_n1(golden):
    lg = golden.lng("ising_L16_lng.txt")
    c = O.make_config("ising", L=16, n_windows=4)
    mask = O.mask_rule(c)
    runs, _, _ = _exact_pieces(lg, c, mask, [[1.5, -3.0, 7.25, 0.5]])
    runs[0] += np.random.default_rng(1).normal(0, 0.01, runs.shape[1:])
    rows, joins = EN.ensemble(c, mask, runs, R=3, seed=9)
    one, j1 = O.concat(c, mask, runs[0])
    for r in range(4):                                    # n = 1: every resample is the run
        assert np.array_equal(rows[r], one) and np.array_equal(joins[r], j1)


def test_bootstrap_variance_matches_closed_form(golden):
    """A difference of two bins below the first overlap moves by the mean of the
    picked perturbations: over resamples its variance is sum (d - mean d)^2 / n^2."""
    lg = golden.lng("ising_L16_lng.txt")
    c = O.make_config("ising", L=16, n_windows=3)
    mask = O.mask_rule(c)
    n, R = 6, 4000
    rng = np.random.default_rng(21)
    runs, lo, hi = _exact_pieces(lg, c, mask, rng.uniform(-20, 20, size=(n, 3)))
    b1, b2 = int(lo[1]) - 3, int(lo[1]) - 9            # window 0 only, outside every stencil
    b3, b4 = int(hi[1]) + 3, int(hi[1]) + 9            # last window only
    assert mask[b1] and mask[b2] and mask[b3] and mask[b4]
    d = rng.normal(0, 1, n)
    e = rng.normal(0, 1, n)
    runs[:, 0, b1 - lo[0]] += d
    runs[:, 2, b3 - lo[2]] += e
    rows, _ = EN.ensemble(c, mask, runs, R=R, seed=4)
    D = rows[:, b1] - rows[:, b2]
    Dp = rows[:, b3] - rows[:, b4]
    base = lg[b1] - lg[b2]
    assert abs(D[0] - (base + d.mean())) < 1e-9            # the ensemble row
    V = np.sum((d - d.mean()) ** 2) / n ** 2
    assert abs(np.var(D[1:]) / V - 1) < 0.15                 # sd of the ratio ~ sqrt(2/R) = 0.022
    assert abs(D[1:].mean() - D[0]) < 6 * np.sqrt(V / R)
    assert abs(np.corrcoef(D[1:], Dp[1:])[0, 1]) < 6 / np.sqrt(R)   # windows resample apart


# ------------------------------------------------------------ canonical averages
def _microstate_energies(model, q, L):
    qq = 2 if model == "ising" else q
    N = L * L
    idx = np.arange(qq ** N, dtype=np.int64)
    s = np.empty((qq ** N, N), np.int8)
    for i in range(N):
        s[:, i] = idx % qq
        idx //= qq
    g = s.reshape(-1, L, L)
    if model == "ising":
        spin = 2 * g.astype(np.int64) - 1
        E = -(spin * np.roll(spin, 1, axis=1)).sum(axis=(1, 2)) - (spin * np.roll(spin, 1, axis=2)).sum(axis=(1, 2))
    else:
        E = -(g == np.roll(g, 1, axis=1)).sum(axis=(1, 2)) - (g == np.roll(g, 1, axis=2)).sum(axis=(1, 2))
    return E.astype(np.float64)


@pytest.mark.parametrize("model,q,L", [("ising", 2, 4), ("potts", 3, 3), ("ising", 2, 3)])
def test_canonical_matches_boltzmann_sum_over_microstates(golden, model, q, L):
    E = _microstate_energies(model, q, L)
    N = L * L
    lg = X.ln_g(X.brute_force(model, q, L))
    T = np.array([0.3, 0.9, 1.5, 2.269, 4.0, 30.0])
    u, c, f = EN.canonical(model, L, lg, T)
    for i, t in enumerate(T):
        x = -E / t
        m = x.max()
        w = np.exp(x - m)
        Z = w.sum()
        U = (w * E).sum() / Z
        V = (w * E * E).sum() / Z - U * U
        assert abs(u[i] - U / N) <= 1e-11 * max(1.0, abs(U / N))
        assert abs(c[i] - V / (N * t * t)) <= 1e-9 * max(1e-3, V / (N * t * t))
        assert abs(f[i] + t * (m + np.log(Z)) / N) <= 1e-11 * max(1.0, abs(f[i]))


@pytest.mark.parametrize("model,q,L,name", [("ising", 2, 8, "ising_q2_L8_counts.txt"),
                                            ("potts", 3, 5, "potts_q3_L5_counts.txt")])
def test_canonical_limits(golden, model, q, L, name):
    """T -> infinity: bonds are pairwise uncorrelated, so <E>/N -> -2/q (Ising 0) and
    c T^2 -> 2 p (1 - p) with p = 1/q (Ising: 2); f/T -> -ln q.  T -> 0: the
    ground level (energy -2N, degeneracy q) gives u -> -2, f -> -2 - T ln q / N."""
    lg = X.ln_g(golden.counts(name))
    N = L * L
    hi_T, lo_T = 1e5, 0.05
    u, c, f = EN.canonical(model, L, lg, [hi_T, lo_T])
    p = 1.0 / q
    var = 2.0 if model == "ising" else 2 * p * (1 - p)
    assert abs(c[0] * hi_T ** 2 / var - 1) < 1e-3
    assert abs(u[0] - (0.0 if model == "ising" else -2 * p)) < 1e-3
    assert abs(f[0] / hi_T + np.log(q)) < 1e-5
    assert abs(u[1] + 2.0) < 1e-12
    assert c[1] < 1e-30
    assert abs(f[1] - (-2.0 - lo_T * np.log(q) / N)) < 1e-12


def test_canonical_shift_invariance(golden):
    lg = golden.lng("ising_L16_lng.txt")
    T = np.linspace(1.0, 4.0, 13)
    u0, c0, f0 = EN.canonical("ising", 16, lg, T)
    u1, c1, f1 = EN.canonical("ising", 16, lg + 123.0, T)
    assert np.allclose(u1, u0, rtol=1e-12, atol=1e-13)
    assert np.allclose(c1, c0, rtol=1e-9)
    assert np.allclose(f1, f0 - T * 123.0 / 256, rtol=1e-12, atol=1e-12)


def _onsager_u(T):
    """Onsager's internal energy per spin of the infinite square lattice (J = 1)."""
    from scipy.special import ellipk
    K = 1.0 / T
    kap = 2 * np.sinh(2 * K) / np.cosh(2 * K) ** 2
    t2 = np.tanh(2 * K) ** 2
    return -(1 + 2 / np.pi * (2 * t2 - 1) * ellipk(kap ** 2)) / np.tanh(2 * K)


def _onsager_f(T):
    """Onsager's free energy per spin: -T [ln 2 + (1 / 2 pi^2) of the double integral
    over [0, pi]^2 of ln(cosh^2 2K - sinh 2K (cos a + cos b))]."""
    from scipy import integrate
    K = 1.0 / T
    g = lambda a, b: np.log(np.cosh(2 * K) ** 2 - np.sinh(2 * K) * (np.cos(a) + np.cos(b)))
    I, _ = integrate.dblquad(g, 0, np.pi, 0, np.pi, epsabs=1e-13, epsrel=1e-13)
    return -T * (np.log(2) + I / (2 * np.pi ** 2))


def test_canonical_of_exact_L64_matches_onsager(golden):
    """Away from T_c a 64 x 64 torus is the infinite lattice up to terms ~ e^{-L/xi}:
    u equals Onsager's closed form, c its temperature derivative, and f Onsager's
    free energy above T_c; below T_c the two ordered states of the finite torus add
    -T ln 2 / N to f."""
    lg = golden.lng("ising_L64_lng.txt")
    N = 64 * 64
    T = np.array([1.0, 1.5, 1.8, 3.0, 4.0, 6.0])
    u, c, f = EN.canonical("ising", 64, lg, T)
    assert np.max(np.abs(u - _onsager_u(T))) < 1e-12
    h = 1e-4
    dudT = (_onsager_u(T + h) - _onsager_u(T - h)) / (2 * h)
    assert np.max(np.abs(c / dudT - 1)) < 1e-6
    for i, t in enumerate(T):
        shift = -t * np.log(2) / N if t < 2.269 else 0.0
        assert abs(f[i] - (_onsager_f(t) + shift)) < 1e-9
