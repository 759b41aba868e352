"""Pins of the CPU oracle against facts fixed outside it (not GPU tests).

Each test names what it pins: published known answers (Philox), the paper's
worked window example, exact enumeration, closed forms and invariants.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O
from oracle import exact_dos as X


# ---------------------------------------------------------------- Philox (R4)
def test_philox_known_answers(golden):
    with open(os.path.join(golden.dir, "philox_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert O.philox(v[0:4], v[4:6]) == tuple(v[6:10])


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_host(golden):
    """rocRAND's Philox4x32-10, built for the host, on 3000 (seed, T, slot, tag) counters."""
    tmp = tempfile.mkdtemp()
    exe = os.path.join(tmp, "ref")
    subprocess.check_call(["hipcc", "-O1", os.path.join(golden.dir, "rocrand_philox_ref.cpp"),
                           "-o", exe], stderr=subprocess.DEVNULL)
    rng = np.random.default_rng(7)
    cases = []
    for i in range(3000):
        seed = int(rng.integers(0, 2**63))
        T = int(rng.integers(0, 2**62)) if i % 2 else int(rng.integers(0, 10**6))
        cases.append((seed, T, int(rng.integers(0, 2**31)), int(rng.integers(0, 4))))
    inp = "".join(f"{s} {T} {sl} {tg}\n" for s, T, sl, tg in cases)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for (seed, T, sl, tg), line in zip(cases, out):
        ref = tuple(int(x, 16) for x in line.split())
        got = O.philox([T & 0xFFFFFFFF, T >> 32, sl, tg], [seed & 0xFFFFFFFF, seed >> 32])
        assert got == ref
    shutil.rmtree(tmp)


# ------------------------------------------------------ acceptance test (R6)
def test_accept_exact_predicate_vs_mpmath():
    """accept(delta, u) == [u < 2^53 e^delta] decided at 60 digits, incl. near-ties."""
    import mpmath as mp
    mp.mp.dps = 60
    rng = np.random.default_rng(3)
    cases = []
    for _ in range(4000):
        d = -float(rng.uniform(0, 40)) if rng.random() < 0.9 else -float(rng.uniform(0, 1e-6))
        d = math.ldexp(round(math.ldexp(d, 30)), -30)        # dyadic, as on the path
        y = mp.ldexp(mp.exp(mp.mpf(d)), 53)
        base = int(mp.floor(y))
        for off in (-3, -1, 0, 1, 2, 5, -20, 20):             # straddle the exact boundary
            u = base + off
            if 0 <= u < 2**53:
                cases.append((d, u, bool(mp.mpf(u) < y)))
        u = int(rng.integers(0, 2**53))
        cases.append((d, u, bool(mp.mpf(u) < y)))
    for d, u, want in cases:
        assert O.accept(d, u) == want, (d, u)
    # special cases
    assert O.accept(0.0, 2**53 - 1) and O.accept(3.5, 2**53 - 1)
    assert O.accept(-1e5, 0) and not O.accept(-1e5, 1)
    assert not O.accept(-37.0, 1)        # 2^53 e^-37 ~ 0.77 < 1
    assert O.accept(-36.0, 1)            # 2^53 e^-36 ~ 2.09 > 1


# ---------------------------------------------------------------- layout (R2)
def test_layout_reproduces_paper_window_counts(golden):
    """Potts Q=10, width 1000, o = 75%: 77/317/717/1277 pieces (paper Sec. IV.A)."""
    with open(os.path.join(golden.dir, "paper_windows.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for L, pieces, width, on, od in (map(int, r) for r in rows):
        c = O.make_config("potts", q=10, L=L, n_windows=pieces, overlap=(on, od), m=1)
        lo, hi = O.layout(c)
        assert np.all(hi - lo == width)
        shift = width * (od - on) // od
        assert np.array_equal(lo, shift * np.arange(pieces))
        assert hi[-1] == 2 * L * L and lo[0] == 0
        # one window fewer cannot cover the range at this width and overlap
        c2 = O.make_config("potts", q=10, L=L, n_windows=pieces - 1, overlap=(on, od), m=1)
        lo2, hi2 = O.layout(c2)
        assert (hi2 - lo2)[0] > width


def test_layout_properties():
    rng = np.random.default_rng(11)
    for _ in range(300):
        L = int(rng.integers(4, 40)) * 2
        h = int(rng.integers(1, 40))
        den = int(rng.integers(2, 9))
        num = int(rng.integers(0, den))
        c = O.make_config("ising", L=L, n_windows=h, overlap=(num, den))
        S = O.n_bins(c) - 1
        w = (S * den + (den + (h - 1) * (den - num)) - 1) // (den + (h - 1) * (den - num))
        if h > 1 and w >= S:
            continue
        lo, hi = O.layout(c)
        assert lo[0] == 0 and hi[-1] == S
        assert np.all(np.diff(lo) >= 0) and len(set(hi - lo)) == 1
        for a in range(h - 1):
            shared = hi[a] - lo[a + 1]
            # overlap >= o up to the one bin lost to flooring the window starts
            assert (shared + 1) * den >= num * (hi[a] - lo[a])


# ------------------------------------------------------------ exact DOS pins
def test_exact_routes_agree(golden):
    assert X.brute_force("ising", 2, 4) == golden.counts("ising_q2_L4_counts.txt")
    assert X.transfer_matrix("ising", 2, 4) == golden.counts("ising_q2_L4_counts.txt")
    assert X.kaufman_ising(4) == golden.counts("ising_q2_L4_counts.txt")
    assert X.kaufman_ising(6) == X.transfer_matrix("ising", 2, 6)
    assert X.kaufman_ising(8) == golden.counts("ising_q2_L8_counts.txt")
    assert X.brute_force("potts", 3, 3) == golden.counts("potts_q3_L3_counts.txt")
    assert X.transfer_matrix("potts", 3, 3) == golden.counts("potts_q3_L3_counts.txt")


def test_brute_force_small_table():
    """Ising L=4: the enumeration's counts (2^16 states) at a few levels."""
    g = X.brute_force("ising", 2, 4)
    assert g[0] == 2 and g[2] == 32 and g[3] == 64 and g[8] == 20524 and sum(g) == 2**16
    assert g[1] == 0 and g[15] == 0


@pytest.mark.parametrize("L", [16, 24, 32, 48, 64, 128])
def test_ising_exact_invariants(golden, L):
    lg = golden.lng(f"ising_L{L}_lng.txt")
    N = L * L
    assert len(lg) == N + 1
    ok = np.isfinite(lg)
    # sum g = 2^N
    mx = lg[ok].max()
    assert abs(mx + math.log(np.exp(lg[ok] - mx).sum()) - N * math.log(2)) < 1e-9 * N
    # E -> -E symmetry (even L), ground state 2, closed-form low levels 2N, 4N
    assert np.allclose(lg[ok], lg[::-1][ok], rtol=0, atol=1e-9 * N)
    assert lg[0] == pytest.approx(math.log(2))
    assert lg[2] == pytest.approx(math.log(2 * N)) and lg[3] == pytest.approx(math.log(4 * N))
    assert list(np.where(~ok)[0]) == [1, N - 1]


@pytest.mark.parametrize("name,q,L", [("potts_q3_L3_counts.txt", 3, 3), ("potts_q3_L4_counts.txt", 3, 4),
                                      ("potts_q4_L4_counts.txt", 4, 4), ("potts_q3_L5_counts.txt", 3, 5),
                                      ("potts_q10_L3_counts.txt", 10, 3)])
def test_potts_exact_closed_forms(golden, name, q, L):
    g = golden.counts(name)
    N = L * L
    assert sum(g) == q**N and g[0] == q and g[4] == q * (q - 1) * N
    if L >= 4:
        assert g[6] == 2 * N * q * (q - 1)             # aligned dominoes
        assert g[7] == 2 * N * q * (q - 1) * (q - 2)   # two different flipped neighbours


def test_mask_rule_matches_exact_zero_set(golden):
    for name, model, q, L in [("ising_q2_L4_counts.txt", "ising", 2, 4),
                              ("ising_q2_L6_counts.txt", "ising", 2, 6),
                              ("ising_q2_L8_counts.txt", "ising", 2, 8),
                              ("potts_q3_L4_counts.txt", "potts", 3, 4),
                              ("potts_q4_L4_counts.txt", "potts", 4, 4),
                              ("potts_q3_L5_counts.txt", "potts", 3, 5)]:
        g = np.array(golden.counts(name), dtype=object)
        c = O.make_config(model, q=q, L=L)
        assert np.array_equal(O.mask_rule(c), (g > 0).astype(np.uint8)), name
    for L in (16, 32):
        lg = golden.lng(f"ising_L{L}_lng.txt")
        c = O.make_config("ising", L=L)
        assert np.array_equal(O.mask_rule(c), np.isfinite(lg).astype(np.uint8))


def test_energy_function_vs_broken_bond_count():
    """orc_energy against the enumeration's independent broken-bond definition."""
    rng = np.random.default_rng(5)
    for model, q in (("ising", 2), ("potts", 3), ("potts", 10)):
        for L in (3, 4, 7, 8):
            if model == "ising" and L % 2:
                continue
            c = O.make_config(model, q=q, L=L)
            for _ in range(20):
                s = rng.integers(0, q, size=(L, L)).astype(np.uint8)
                broken = int((s != np.roll(s, 1, 0)).sum() + (s != np.roll(s, 1, 1)).sum())
                E = -2 * L * L + (2 * broken if model == "ising" else broken)
                assert O.energy(c, s.ravel()) == E


# ------------------------------------------------------- REWL dynamics pins
def _slots_energy_consistent(sim):
    st = sim.state()
    c = sim.cfg
    N = c.L * c.L
    for sl in range(sim.S):
        E = O.energy(c, st["spins"][sl])
        b = (E + 2 * N) // 4 if c.model == 0 else E + 2 * N
        assert b == st["bins"][sl]
        a = sl // c.walkers_per_window
        assert sim.lo[a] <= b <= sim.hi[a]
    q = 2 if c.model == 0 else c.q
    assert st["spins"].max() < q                      # every spin value is a valid state
    return st


@pytest.mark.parametrize("model,q,L,h,m", [("ising", 2, 8, 4, 2), ("potts", 3, 4, 3, 4),
                                           ("potts", 10, 6, 5, 2), ("potts", 200, 6, 3, 2)])
def test_running_energy_equals_recomputed(model, q, L, h, m):
    c = O.make_config(model, q=q, L=L, n_windows=h, m=m, X=500, kfinal=12, seed=9)
    sim = O.Sim(c)
    _slots_energy_consistent(sim)
    for _ in range(30):
        sim.run(1)
        _slots_energy_consistent(sim)


def test_histogram_count_and_dyadic_exactness():
    m = 4
    c = O.make_config("ising", L=8, n_windows=3, m=m, X=1000, kfinal=14, seed=21)
    sim = O.Sim(c)
    st = sim.state()
    since = np.zeros(3, dtype=np.int64)            # intervals since the window's last merge
    for _ in range(60):
        k_before = st["k"].copy()
        sim.run(1)
        st = sim.state()
        for a in range(3):
            since[a] = 0 if st["k"][a] != k_before[a] else since[a] + 1
            if not st["done"][a]:
                # H counts every attempt since the merge (one entry per attempt)
                assert np.all(st["H"][a * m:(a + 1) * m].sum(axis=1) ==
                              since[a] * c.exchange_interval)
        # ln g values are multiples of 2^-(k + log2 m): the FP64 path is exact
        scale = 2.0 ** (st["k"].max() + 2)
        v = st["lng"] * scale
        assert np.all(v == np.round(v))


def test_thread_count_does_not_change_results():
    c = O.make_config("potts", q=4, L=6, n_windows=4, m=4, X=2000, kfinal=10, seed=5)
    a = O.Sim(c)
    b = O.Sim(c)
    a.run(25, threads=1)
    b.run(25, threads=4)
    sa, sb = a.state(), b.state()
    for k in sa:
        assert np.array_equal(np.asarray(sa[k]), np.asarray(sb[k])), k


def _stationary(lg_exact, lng_walker, lo, hi, mask):
    """Expected energy distribution of a walker with fixed weights 1/g_w(E)."""
    b = np.arange(lo, hi + 1)
    ok = mask[b] > 0
    logp = np.where(ok, lg_exact[b] - lng_walker, -np.inf)
    p = np.exp(logp - logp[ok].max())
    return p / p.sum()


def test_frozen_weights_sample_g_over_gw(golden):
    """Sweep with fixed ln g_w: visits follow g(E)/g_w(E) over the window (A1/A2)."""
    lg = X.ln_g(golden.counts("ising_q2_L4_counts.txt"))
    rng = np.random.default_rng(2)
    mask = O.mask_rule(O.make_config("ising", L=4))
    for seed in (100, 101):
        c = O.make_config("ising", L=4, n_windows=1, m=1, X=1000, k0=39, kfinal=40,
                          flat=(1, 1), seed=seed)
        w = np.round(np.where(mask > 0, lg + rng.normal(0, 0.7, size=17), 0.0) * 2**16) / 2**16
        sim = O.Sim(c, init_lng=w)
        sim.run(12000)
        H = sim.state()["H"][0].astype(float)
        p = _stationary(lg, w, 0, 16, mask)
        obs = H / H.sum()
        big = p > 0.02
        assert np.all(np.abs(obs[big] / p[big] - 1) < 0.05)


def _exchange_marginals(golden):
    """Two windows with different fixed weights, an exchange every 2 attempts; returns
    the exchange counters and, per walker, the largest relative deviation of its visit
    histogram from its single-walker law g/g_w over the levels holding > 2 %."""
    lg = X.ln_g(golden.counts("ising_q2_L4_counts.txt"))
    c = O.make_config("ising", L=4, n_windows=2, overlap=(3, 4), m=2, X=2, k0=39, kfinal=40,
                      flat=(1, 1), seed=31)
    lo, hi = O.layout(c)
    mask = O.mask_rule(c)
    tilt = [0.45 * (np.arange(17) - 8.0), -0.3 * (np.arange(17) - 8.0)]
    sim = O.Sim(c)
    tabs = []
    for a in range(2):
        t = np.where(mask > 0, lg + tilt[a], 0.0)[lo[a]:hi[a] + 1]
        t = np.round(t * 2**16) / 2**16
        sim.set_window_lng(a, t)
        tabs.append(t)
    sim.run(400000)
    st = sim.state()
    dev = []
    for sl in range(4):
        a = sl // 2
        p = _stationary(lg, tabs[a], lo[a], hi[a], mask)
        H = st["H"][sl].astype(float)
        obs = H / H.sum()
        big = p > 0.02
        dev.append(float(np.max(np.abs(obs[big] / p[big] - 1))))
    return sim.stats(), dev


def test_exchange_keeps_stationary_marginals(golden):
    """Under Eq. (1) the joint law is the product of each walker's g/g_w law, so each
    walker's visit histogram keeps its single-walker marginal.  The two windows'
    weights differ inside the overlap, so Eq. (1) is not trivially 1 there."""
    stats, dev = _exchange_marginals(golden)
    assert stats["ex_acc"][0] > 1000 and stats["ex_acc"][0] < stats["ex_prop"][0]
    assert max(dev) < 0.06, dev


# ------------------------------------------------------- concatenation (A16)
def test_concatenation_recovers_exact_dos(golden):
    """Exact ln g cut into overlapping pieces with random offsets is rejoined exactly."""
    lg = golden.lng("ising_L16_lng.txt")
    rng = np.random.default_rng(4)
    for h in (2, 5, 8):
        c = O.make_config("ising", L=16, n_windows=h)
        lo, hi = O.layout(c)
        mask = O.mask_rule(c)
        WB = hi[0] - lo[0] + 1
        pieces = np.zeros((h, WB))
        for a in range(h):
            pieces[a] = np.where(mask[lo[a]:hi[a] + 1] > 0, lg[lo[a]:hi[a] + 1], 0.0) + \
                        rng.uniform(-50, 50)
        out, join = O.concat(c, mask, pieces)
        ok = mask > 0
        assert np.max(np.abs(out[ok] - lg[ok])) < 1e-9
        assert np.all(np.isneginf(out[~ok]))
        assert np.all(np.diff(join) > 0)
        for a in range(h - 1):
            assert lo[a + 1] <= join[a] <= hi[a]


# ------------------------------------------------------------ REWL accuracy
def _concat_error(sim, exact):
    c = sim.cfg
    mask = O.mask_rule(c) if c.L >= 4 else (np.isfinite(exact)).astype(np.uint8)
    out, _ = O.concat(c, mask, sim.pieces())
    ok = mask > 0
    return np.abs(out[ok] - exact[ok])


def test_rewl_converges_to_exact_ising_L8(golden):
    """The Ising L=8 geometry (4 windows, o = 3/4) with m = 16 walkers, ln f -> 2^-20."""
    exact = X.ln_g(golden.counts("ising_q2_L8_counts.txt"))
    c = O.make_config("ising", L=8, n_windows=4, m=16, kfinal=20, seed=1)
    sim = O.Sim(c)
    assert sim.run(100000)
    err = _concat_error(sim, exact)
    assert err.max() < 0.08


def test_error_falls_with_walkers_per_window(golden):
    """Sec. IV.B (`fig:scaling`): averaging the m walkers of a window at every merge
    lowers the error of ln g at least as fast as m^-1/2.  Ising L=8 (4 windows,
    ln f -> 2^-16), six seeds for each of m = 1, 4, 16: the RMS over seeds of the RMS
    error against the exact DOS must shrink by at least 2/1.3 from m to 4 m (measured:
    0.145 -> 0.045 -> 0.0185; a merge that keeps walker 0's table instead of the mean
    gives 0.145 -> 0.090 -> 0.101 and fails)."""
    exact = X.ln_g(golden.counts("ising_q2_L8_counts.txt"))
    ok = np.isfinite(exact)

    def rms(m):
        errs = []
        for seed in range(1, 7):
            c = O.make_config("ising", L=8, n_windows=4, m=m, kfinal=16, seed=seed)
            sim = O.Sim(c)
            assert sim.run(200000)
            out, _ = O.concat(c, O.mask_rule(c), sim.pieces())
            errs.append(np.sqrt(np.mean((out[ok] - exact[ok]) ** 2)))
        return float(np.sqrt(np.mean(np.square(errs))))

    r1, r4, r16 = rms(1), rms(4), rms(16)
    assert r4 <= 1.3 * r1 / 2 and r16 <= 1.3 * r4 / 2, (r1, r4, r16)


def test_rewl_converges_to_exact_potts_q3_L4(golden):
    exact = X.ln_g(golden.counts("potts_q3_L4_counts.txt"))
    c = O.make_config("potts", q=3, L=4, n_windows=3, m=8, kfinal=18, X=5000, seed=2)
    sim = O.Sim(c)
    assert sim.run(100000)
    err = _concat_error(sim, exact)
    assert err.max() < 0.12


def test_potts_q10_L3_six_broken_bonds(golden):
    """10-state Potts L=3: six broken bonds come from a flipped domino (2N q(q-1)) or,
    on the 3 x 3 torus only, from a whole row or column taking one other state
    (2L q(q-1)); the transfer-matrix table must hold both and nothing else."""
    g = golden.counts("potts_q10_L3_counts.txt")
    q, L, N = 10, 3, 9
    assert g[6] == 2 * N * q * (q - 1) + 2 * L * q * (q - 1)
    assert g[1] == g[2] == g[3] == g[5] == 0


def test_rewl_converges_to_exact_potts_q10_L3(golden):
    """The paper's 10-state Potts model on the smallest lattice with an exact DOS
    (transfer matrix): REWL, 2 windows x 8 walkers, ln f -> 2^-18, joined result
    within 0.08 of the exact ln g at every level that occurs."""
    g = golden.counts("potts_q10_L3_counts.txt")
    exact = X.ln_g(g)
    mask = (np.array(g) > 0).astype(np.uint8)
    c = O.make_config("potts", q=10, L=3, n_windows=2, m=8, kfinal=18, X=5000, seed=3)
    sim = O.Sim(c, mask=mask)
    assert sim.run(100000)
    out, _ = O.concat(c, mask, sim.pieces())
    ok = mask > 0
    assert np.abs(out[ok] - exact[ok]).max() < 0.08


def test_rewl_brute_force_potts_q3_L3(golden):
    """L=3 with the mask taken from enumeration (the closed-form rule needs L >= 4)."""
    g = golden.counts("potts_q3_L3_counts.txt")
    exact = X.ln_g(g)
    mask = (np.array(g) > 0).astype(np.uint8)
    c = O.make_config("potts", q=3, L=3, n_windows=2, m=8, kfinal=18, X=5000, seed=3)
    sim = O.Sim(c, mask=mask)
    assert sim.run(100000)
    out, _ = O.concat(c, mask, sim.pieces())
    ok = mask > 0
    assert np.abs(out[ok] - exact[ok]).max() < 0.12


# ------------------------------------------------------------ Eq. (8) flatness
def _visits_flat(H, mask_w, k, num, den):
    """Eq. (8) on one walker's counts, in Python integers: min H >= (num/den) 2^(k/2)."""
    mn = int(min(int(v) for v, ok in zip(H, mask_w) if ok))
    return (mn * den) ** 2 >= num * num * 2 ** k


@pytest.mark.parametrize("num,den,model,q,L", [(1, 1, "ising", 2, 8), (3, 2, "potts", 4, 5), (5, 1, "ising", 2, 6)])
def test_visits_rule_latches_exactly_eq8(num, den, model, q, L):
    """Between merges a walker's counts only grow, so its latched flag must equal
    Eq. (8) evaluated on its current counts; checked interval by interval."""
    cfg = O.make_config(model, q=q, L=L, n_windows=2, m=2, kfinal=14, X=400, seed=3,
                        flat_rule="visits", flat=(num, den))
    sim = O.Sim(cfg)
    mask = O.mask_rule(cfg)
    lo, hi = O.layout(cfg)
    prev_k = sim.state()["k"].copy()
    checked = merged = 0
    for _ in range(400):
        done = sim.run(1)
        st = sim.state()
        for a in range(cfg.n_windows):
            if st["done"][a]:
                continue
            if st["k"][a] != prev_k[a]:
                merged += 1
                assert st["k"][a] == prev_k[a] + 1
                assert not st["flat"][a * 2:(a + 1) * 2].any() and not st["H"][a * 2:(a + 1) * 2].any()
                continue
            mw = mask[lo[a]:hi[a] + 1]
            for r in range(2):
                slot = a * 2 + r
                want = _visits_flat(st["H"][slot][: hi[a] - lo[a] + 1], mw, int(st["k"][a]), num, den)
                assert bool(st["flat"][slot]) == want
                checked += 1
        prev_k = st["k"].copy()
        if done:
            break
    assert merged >= 4 and checked > 50


def test_visits_rule_with_a_zero_merges_every_interval():
    # a = 0: every count satisfies H >= 0, so each window merges at every interval
    cfg = O.make_config("ising", L=8, n_windows=3, m=4, k0=2, kfinal=9, X=50, seed=9,
                        flat_rule="visits", flat=(0, 1))
    sim = O.Sim(cfg)
    for t in range(1, 8):
        done = sim.run(1)
        assert list(sim.state()["k"]) == [2 + t] * 3
        assert done == (t == 7)


# ------------------------------------------------------------ unequal windows
def test_unequal_windows_converge_to_exact_ising_L8(golden):
    """Explicit windows of different widths (narrow at the ends) through the whole
    method: sweep, merge, exchange and the Sec. II.B joins."""
    exact = X.ln_g(golden.counts("ising_q2_L8_counts.txt"))
    c = O.make_config("ising", L=8, n_windows=4, m=16, kfinal=20, seed=3,
                      windows=([0, 12, 26, 44], [20, 38, 52, 64]))
    sim = O.Sim(c)
    assert sim.WB == 27
    assert sim.run(100000)
    err = _concat_error(sim, exact)
    assert err.max() < 0.08


@pytest.mark.parametrize("lo,hi", [([0, 25, 30], [20, 40, 64]),     # gap between windows 0 and 1
                                   ([0, 10, 30], [20, 40, 63]),     # does not reach the top
                                   ([1, 10, 30], [20, 40, 64]),     # does not start at 0
                                   ([0, 10, 10], [20, 40, 64]),     # starts not ascending
                                   ([0, 10, 30], [20, 40, 30])])    # a one-bin window
def test_bad_explicit_windows_rejected(lo, hi):
    with pytest.raises(ValueError):
        O.Sim(O.make_config("ising", L=8, n_windows=3, windows=(lo, hi)))


# ------------------------------------------------------ 80 % flatness (A4)
def _mean_rule(H, mask_w, num, den):
    """Sec. II.A on one walker's counts, in Python integers: min H >= (num/den) mean H."""
    v = [int(x) for x, ok in zip(H, mask_w) if ok]
    return den * min(v) * len(v) >= num * sum(v), den * min(v) * len(v) == num * sum(v)


def test_mean_rule_latches_exactly_80_percent():
    """The latched flag equals 'the 80 % rule held at some interval end since the last
    merge', with the non-strict comparison of "may not be smaller than 80 % of the
    mean" (Sec. II.A).  Windows of three bins and a few attempts per interval make
    exact equality 5 min n = 4 sum occur, which tells >= from >."""
    W = 17                                        # Ising L = 4: bins 0..16
    lo = list(range(0, 16, 2))
    hi = [b + 2 for b in lo]
    cfg = O.make_config("ising", L=4, n_windows=len(lo), m=4, kfinal=30, X=3, seed=5,
                        windows=(lo, hi))
    sim = O.Sim(cfg)
    mask = O.mask_rule(cfg)
    assert mask.size == W
    h, m = len(lo), 4
    latched = np.zeros(h * m, bool)
    prev_k = sim.state()["k"].copy()
    checked = ties = 0
    for _ in range(3000):
        sim.run(1)
        st = sim.state()
        for a in range(h):
            if st["done"][a]:
                continue
            if st["k"][a] != prev_k[a]:           # merged: flags and counts start over
                assert not st["flat"][a * m:(a + 1) * m].any()
                latched[a * m:(a + 1) * m] = False
                continue
            mw = mask[lo[a]:hi[a] + 1]
            for r in range(m):
                sl = a * m + r
                ok, tie = _mean_rule(st["H"][sl][: hi[a] - lo[a] + 1], mw, 4, 5)
                if tie and not latched[sl]:
                    ties += 1                     # only >= latches here
                latched[sl] |= ok
                assert bool(st["flat"][sl]) == latched[sl], (a, r, st["H"][sl])
                checked += 1
        prev_k = st["k"].copy()
    assert checked > 10000 and ties >= 10


# ------------------------------------------------------- exchange, planted mistakes
@pytest.mark.parametrize("mode", [1, 2, 3], ids=["always-accept", "sign-flip", "dropped-term"])
def test_exchange_marginal_check_fails_on_planted_mistakes(golden, mode):
    """The marginal test of Eq. (1) above must fail when the oracle's exchange rule is
    wrong: accepting every proposal, flipping the sign of the log ratio, or dropping
    walker j's factor each bias the walkers' visit histograms well past the 6 %
    tolerance that the correct rule meets."""
    try:
        O.exchange_mutation(mode)
        stats, dev = _exchange_marginals(golden)
    finally:
        O.exchange_mutation(0)
    assert stats["ex_acc"][0] > 1000
    assert max(dev) > 0.15, dev


# ------------------------------------------------------------ round trips (R29)
def _recount_round_trips(windows_by_interval):
    """Round trips of each replica from its window after every interval: a visit to
    window 0, then one to window h-1, then one to window 0 again (Sec. IV.A)."""
    seq = np.asarray(windows_by_interval)        # (intervals + 1, replicas)
    h_top = seq.max()
    out = []
    for r in range(seq.shape[1]):
        trips, seen0, seen_top = 0, False, False
        for w in seq[:, r]:
            if w == 0:
                if seen0 and seen_top:
                    trips += 1
                seen0, seen_top = True, False
            elif w == h_top and seen0:
                seen_top = True
        out.append(trips)
    return np.array(out)


@pytest.mark.parametrize("h,m,exchange", [(4, 2, True), (3, 4, True), (2, 1, True), (4, 2, False)])
def test_round_trips_match_replica_trajectories(h, m, exchange):
    """The oracle's round-trip counter against a recount from the windows each replica
    visited interval by interval.  Each counted trip crosses every window pair once
    upwards and once downwards, and an accepted exchange moves one replica each way,
    so the accepted exchanges of every pair bound the total from above."""
    cfg = O.make_config("ising", L=6, n_windows=h, m=m, k0=12, kfinal=30, X=60, seed=17,
                        exchange=exchange)
    sim = O.Sim(cfg)
    S = h * m
    traj = []

    def windows_of_replicas():
        rid = sim.replicas()["rid"]
        w = np.empty(S, np.int64)
        w[rid] = np.arange(S) // m                # replica rid[s] sits in window s // m
        return w

    traj.append(windows_of_replicas())
    assert np.array_equal(np.sort(sim.replicas()["rid"]), np.arange(S))
    for _ in range(3000):
        sim.run(1)
        traj.append(windows_of_replicas())
    rt = sim.replicas()["round_trips"]
    assert np.array_equal(np.sort(sim.replicas()["rid"]), np.arange(S))   # a permutation
    if h > 1:                                     # the top window index is h - 1
        assert np.array(traj).max() == h - 1
    assert np.array_equal(rt, _recount_round_trips(traj))
    if h > 1:
        assert rt.sum() <= sim.stats()["ex_acc"][: h - 1].min()
    if exchange:
        assert rt.sum() > 20
    else:
        assert rt.sum() == 0
