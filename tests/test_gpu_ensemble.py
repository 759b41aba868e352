"""GPU parity of the n-run error analysis (rewl_ensemble) and of the canonical
averages (rewl_thermo) against the oracle.

Join points are integer decisions taken on bit-identical mean pieces (the sum
in run order and the division by n are single IEEE operations on both sides),
so they must match exactly; the joined ln g differs only in the normalisation's
exp/log (bound 1e-9, as for rewl_concat).  The canonical sums run in another
order and with another exp: relative differences stay near 1e-13, tested at
1e-10 (u, f) and 1e-9 (c, plus 1e-12 of the row's largest c for values that
vanish at low temperature).
"""
import numpy as np
import pytest

import oracle as O
from oracle import ensemble as EN

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    import paper_1407_5140_amd as rw
    return rw


def _assert_thermo(g, o):
    gu, gc, gf = g
    ou, oc, of = o
    assert np.all(np.abs(gu - ou) <= 1e-10 * np.maximum(1.0, np.abs(ou)))
    assert np.all(np.abs(gf - of) <= 1e-10 * np.maximum(1.0, np.abs(of)))
    cmax = np.max(oc, axis=1, keepdims=True)
    assert np.all(np.abs(gc - oc) <= 1e-9 * np.abs(oc) + 1e-12 * cmax)


def _oracle_thermo(model, L, rows, T):
    out = [EN.canonical(model, L, r, T) for r in rows]
    return tuple(np.array([o[k] for o in out]) for k in range(3))


T_GRID = np.concatenate([np.geomspace(0.05, 1e4, 45), np.linspace(2.1, 2.5, 16)])   # 61: ragged tile


@pytest.mark.parametrize("name,L", [("ising_L16_lng.txt", 16), ("ising_L64_lng.txt", 64)])
def test_thermo_parity_ising_exact_and_noisy(rw, golden, name, L):
    lg = golden.lng(name)
    rng = np.random.default_rng(L)
    rows = [lg, np.where(np.isfinite(lg), lg + rng.normal(0, 0.05, lg.size), -np.inf), lg + 1e3]
    g = rw.rewl_thermo("ising", L, np.array(rows), T_GRID)
    _assert_thermo(g, _oracle_thermo("ising", L, rows, T_GRID))


def test_thermo_parity_potts_exact(rw, golden):
    from oracle import exact_dos as X
    lg = X.ln_g(golden.counts("potts_q3_L5_counts.txt"))
    T = np.geomspace(0.05, 100.0, 9)                               # one full tile and one of 1
    g = rw.rewl_thermo("potts", 5, lg[None, :], T)
    _assert_thermo(g, _oracle_thermo("potts", 5, [lg], T))


def test_thermo_rejects_bad_input(rw):
    lg = np.zeros(17)
    with pytest.raises(rw.RewlError):
        rw.rewl_thermo("ising", 4, lg, [0.0])
    with pytest.raises(rw.RewlError):
        rw.rewl_thermo("ising", 4, np.full(17, -np.inf), [1.0])
    bad = lg.copy()
    bad[3] = np.nan
    with pytest.raises(rw.RewlError):
        rw.rewl_thermo("ising", 4, bad, [1.0])
    with pytest.raises(rw.RewlError):
        rw.rewl_thermo(2, 4, lg, [1.0])                     # no such model
    with pytest.raises(ValueError):
        rw.rewl_thermo("ising", 4, np.zeros(16), [1.0])     # rows must span the model's W bins


def _small_kws():
    return [dict(model="ising", L=8, n_windows=4, m=2, kfinal=12, X=1000, seed=s) for s in (1, 2, 3)]


def test_ensemble_of_converged_runs(rw):
    """Three independent runs to convergence (the oracle's own runs supply its
    pieces; lockstep parity makes the GPU's identical), mean + 24 resamples."""
    kws = _small_kws()
    gpu = rw.Rewl([rw.make_config(**kw) for kw in kws])
    for _ in range(400):
        if gpu.run(200):
            break
    runs = []
    for kw in kws:
        sim = O.Sim(O.make_config(**kw))
        assert sim.run(100000)
        runs.append(sim.pieces())
    runs = np.array(runs)
    for i in range(3):
        assert np.array_equal(gpu.pieces(i), runs[i])
    c = O.make_config(**kws[0])
    mask = O.mask_rule(c)
    orows, ojoin = EN.ensemble(c, mask, runs, R=24, seed=77)
    grows, gjoin = gpu.ensemble([0, 1, 2], R=24, seed=77)
    assert np.array_equal(gjoin, ojoin)
    ok = mask > 0
    assert np.array_equal(np.isfinite(grows), np.broadcast_to(ok, grows.shape))
    assert np.max(np.abs(grows[:, ok] - orows[:, ok])) < 1e-9
    # one run: every row is that run's concatenation
    one, _ = gpu.ensemble([2], R=3, seed=5)
    ref, _ = gpu.concat(2)
    for r in range(4):
        assert np.max(np.abs(one[r][ok] - ref[ok])) < 1e-12
    # order of runs is the draw order of resample 0
    rev, _ = gpu.ensemble([2, 1, 0], R=0, seed=1)
    orev, _ = EN.ensemble(c, mask, runs[::-1], R=0, seed=1)
    assert np.max(np.abs(rev[0][ok] - orev[0][ok])) < 1e-9
    with pytest.raises(rw.RewlError):
        gpu.ensemble([0, 5], R=1)
    gpu.close()


def test_ensemble_rejects_mismatched_runs(rw):
    a = dict(model="ising", L=8, n_windows=4, m=1, kfinal=8, X=100, seed=1)
    b = dict(a, L=10)
    gpu = rw.Rewl([rw.make_config(**a), rw.make_config(**b)])
    with pytest.raises(rw.RewlError):
        gpu.ensemble([0, 1], R=1)
    gpu.close()


def test_ensemble_full_size_potts_L100(rw):
    """The paper's smallest Potts lattice (q=10, L=100, 77 windows of 1001 bins,
    overlap 3/4): three runs whose window tables are set from known global tables
    (smooth + per-bin noise + per-run constant), mean + 6 resamples, then the
    canonical averages of every row."""
    from paper_1407_5140_amd import workloads as Wl
    base = dict(Wl.single("potts100"))
    base["m"] = 1
    kws = [dict(base, seed=s) for s in (1, 2, 3)]
    c = O.make_config(**kws[0])
    W = O.n_bins(c)
    lo, hi = O.layout(c)
    WB = int((hi - lo).max()) + 1
    rng = np.random.default_rng(100)
    b = np.arange(W)
    tables = []
    for j in range(3):
        t = 3000.0 * np.sin(np.pi * b / (W - 1)) + rng.normal(0, 0.02, W) + 17.0 * j
        tables.append(np.round(t * 2.0 ** 20) / 2.0 ** 20)
    gpu = rw.Rewl([rw.make_config(**kw) for kw in kws])
    for j in range(3):
        gpu.set_initial_lng(tables[j], j)
    runs = np.zeros((3, len(lo), WB))
    for j in range(3):
        for a in range(len(lo)):
            runs[j, a, : hi[a] - lo[a] + 1] = tables[j][lo[a]: hi[a] + 1]
    mask = O.mask_rule(c)
    orows, ojoin = EN.ensemble(c, mask, runs, R=6, seed=2024)
    grows, gjoin = gpu.ensemble([0, 1, 2], R=6, seed=2024)
    gpu.close()
    assert np.array_equal(gjoin, ojoin)
    ok = mask > 0
    assert np.max(np.abs(grows[:, ok] - orows[:, ok])) < 1e-9
    assert np.all(np.isneginf(grows[:, ~ok]))
    T = np.linspace(0.5, 3.0, 40)
    g = rw.rewl_thermo("potts", 100, orows, T)
    _assert_thermo(g, _oracle_thermo("potts", 100, orows, T))
