"""The density-of-states network's warm start against plain flat-start REWL.

The network is trained on the device on REWL's own results for small lattices
(produced in the test), then supplies the starting ln g of a larger lattice,
which begins its ln f schedule at 2^-k0 instead of 1.  Convergence is counted in
exchange intervals, which the counter-based random numbers make exactly
reproducible, so the comparison carries no timing noise.  The warm-started
result is also judged against the exact DOS (Ising) for accuracy.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TRAIN = [("ising", 2, 8), ("ising", 2, 12), ("ising", 2, 16), ("potts", 4, 8), ("potts", 4, 12),
         ("potts", 8, 8), ("potts", 8, 12), ("potts", 10, 8), ("potts", 10, 12)]


@pytest.fixture(scope="module")
def trained():
    from paper_1407_5140_amd import warm as Wm
    kws = Wm.training_workload(TRAIN, m=8, kfinal=13, X=2000, seed0=500)
    for kw in kws:
        kw["n_windows"] = 4
    g, res = Wm.run_to_convergence(kws, 120.0)
    assert all(r["converged"] for r in res), res
    x, t = Wm.training_rows(g, kws)
    g.close()
    net, info = Wm.train(x, t, steps=1500, batch=1024, lr=1e-3, seed=1)
    print(f"[warm] training rows {len(t)}, network {info}")
    assert info["rms"] < 2e-2
    yield Wm, net
    net.close()


def _intervals(Wm, kw, table):
    g, res = Wm.run_to_convergence([kw], 120.0, warm_tables=[table] if table is not None else None, poll=10)
    r = res[0]
    lng = g.concat(0)[0] if r["converged"] else None
    g.close()
    assert r["converged"], (kw, r)
    return r["intervals"], lng


def test_warm_start_converges_in_fewer_intervals(trained):
    Wm, net = trained
    base = dict(model="potts", q=10, L=16, n_windows=4, m=8, kfinal=13, X=2000)
    table = Wm.warm_table(net, base)
    warm, plain = [], []
    for seed in (1, 2, 3):
        warm.append(_intervals(Wm, dict(base, seed=seed, k0=8), table)[0])
        plain.append(_intervals(Wm, dict(base, seed=seed, k0=0), None)[0])
    print(f"[warm] Potts q=10 L=16 intervals to 2^-13: warm {warm}, plain {plain}")
    assert np.median(warm) < np.median(plain)


def test_warm_start_keeps_accuracy(trained, golden):
    """Warm (k0 = 8) and plain (k0 = 0) runs of Ising L=24 to ln f = 2^-13, three seeds
    each, judged against the exact DOS: the mean relative error of ln g over the
    levels that occur, and the largest absolute error of ln g where ln g > 10 (the
    relative error at the two ground levels, ln g = ln 2, is not a useful scale).
    Bounds: every run within 1e-2 mean and 2.0 absolute (plain runs of this size
    reach 2.4e-3..7.4e-3 and 0.5..1.1), and the warm runs' median mean error within
    1.5x of the plain runs' median."""
    Wm, net = trained
    kw = dict(model="ising", q=2, L=24, n_windows=4, m=8, kfinal=13, X=2000)
    exact = golden.lng("ising_L24_lng.txt")
    ok = np.isfinite(exact)
    big = exact[ok] > 10
    errs = {}
    for mode, k0, table in (("warm", 8, Wm.warm_table(net, kw)), ("plain", 0, None)):
        kws = [dict(kw, k0=k0, seed=s) for s in (1, 2, 3)]
        g, res = Wm.run_to_convergence(kws, 300.0, warm_tables=[table] * 3 if table is not None else None,
                                       poll=10)
        assert all(r["converged"] for r in res), (mode, res)
        errs[mode] = []
        for i in range(3):
            lng = g.concat(i)[0]
            assert np.array_equal(np.isfinite(lng), ok)
            d = np.abs(lng[ok] - exact[ok])
            errs[mode].append((res[i]["intervals"], float(np.mean(d / np.abs(exact[ok]))), float(d[big].max())))
        g.close()
    print(f"[warm] Ising L=24 to 2^-13 (intervals, mean relative error, max |error| where ln g > 10): {errs}")
    for mode in errs:
        for n, mean_eps, dmax in errs[mode]:
            assert mean_eps < 1e-2 and dmax < 2.0, (mode, n, mean_eps, dmax)
    med = {mode: float(np.median([e[1] for e in errs[mode]])) for mode in errs}
    assert med["warm"] < 1.5 * med["plain"], med
