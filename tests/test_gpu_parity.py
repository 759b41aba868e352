"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for bit.

Integer state (lattices, energy bins, histograms, flags, swap decisions, ln f
exponents, interval counter) must be identical; ln g must be identical to the
last bit: every FP64 step on the path is exact (dyadic ln f, m = 2^j), so any
difference is a bug, not rounding.
"""
import math

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    import paper_1407_5140_amd as rw
    return rw


def _cfgs(rw, **kw):
    return rw.make_config(**kw), O.make_config(**kw)


def assert_same(g, o, where=""):
    for key in ("bins", "spins", "H", "flat", "k", "done", "swaps"):
        assert np.array_equal(np.asarray(g[key]), np.asarray(o[key])), f"{where}: {key} differs"
    gl, ol = np.asarray(g["lng"]), np.asarray(o["lng"])
    assert np.array_equal(gl.view(np.uint64), ol.view(np.uint64)), f"{where}: ln g bits differ"
    assert g["t"] == o["t"], f"{where}: t {g['t']} vs {o['t']}"


def _lockstep(rw, kw, steps, tune=None, every=1):
    """Advance GPU and oracle together, comparing after every `every` intervals."""
    gc, oc = _cfgs(rw, **kw)
    gpu = rw.Rewl([gc], tune=tune)
    orc = O.Sim(oc)
    assert_same(gpu.state(), orc.state(), f"{kw} after init")
    done = False
    for s in range(0, steps, every):
        n = min(every, steps - s)
        done_g = gpu.run(n)
        done_o = orc.run(n)
        assert done_g == done_o
        assert_same(gpu.state(), orc.state(), f"{kw} after {orc.t} intervals")
        done = done_o
        if done:
            break
    return gpu, orc, done


# ------------------------------------------------------------ building blocks
def test_device_philox_matches_oracle(rw, golden):
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2**32, size=(4000, 6), dtype=np.uint64).astype(np.uint32)
    a[0] = 0
    a[1] = 0xFFFFFFFF
    out = rw.rewl_probe_philox(a)
    for row, got in zip(a, out):
        assert tuple(int(v) for v in got) == O.philox(row[:4], row[4:])


def test_device_acceptance_predicate_exact(rw):
    """Fast log-domain test + guard band + double-double slow path == exact comparison."""
    import mpmath as mp
    mp.mp.dps = 60
    rng = np.random.default_rng(8)
    d_list, u_list, want = [], [], []
    for _ in range(3000):
        d = -float(rng.uniform(0, 37)) if rng.random() < 0.9 else -float(rng.uniform(0, 1e-6))
        d = math.ldexp(round(math.ldexp(d, 33)), -33)
        y = mp.ldexp(mp.exp(mp.mpf(d)), 53)
        base = int(mp.floor(y))
        for off in (0, 1, -1, 2, 40, -40, 10**6):
            u = base + off
            if 0 <= u < 2**53:
                d_list.append(d)
                u_list.append(u)
                want.append(bool(mp.mpf(u) < y))
    d_list += [0.0, 1.5, -1e5, -1e5, -37.0, -36.0, -1e-300]
    u_list += [2**53 - 1, 2**53 - 1, 0, 1, 1, 1, 2**53 - 1]
    want += [True, True, True, False, False, True, True]   # 2^53-1 < 2^53 e^-1e-300
    out = rw.rewl_probe_accept(np.array(d_list), np.array(u_list, dtype=np.uint64))
    got = (out == 1) | (out == 3)
    bad = np.nonzero(got != np.array(want))[0]
    assert bad.size == 0, [(d_list[i], u_list[i], want[i], int(out[i])) for i in bad[:10]]
    assert np.count_nonzero(out >= 2) > 100          # the slow path really ran
    for d, u, g in zip(d_list[:2000], u_list[:2000], got[:2000]):
        assert O.accept(d, int(u)) == bool(g)


# ----------------------------------------------------------- lockstep runs
SMALL = [
    dict(model="ising", L=8, n_windows=4, m=1, kfinal=20, X=10000, seed=1),       # the Ising L=8 workload
    dict(model="ising", L=16, n_windows=4, m=8, kfinal=12, X=3000, seed=5),
    dict(model="potts", q=10, L=8, n_windows=4, m=4, kfinal=12, X=3000, seed=7),
    dict(model="potts", q=4, L=12, n_windows=6, m=16, overlap=(1, 2), kfinal=12, X=2000, seed=11),
    dict(model="potts", q=3, L=5, n_windows=3, m=2, kfinal=10, X=1500, seed=13),   # odd L
    dict(model="ising", L=100, n_windows=8, m=2, kfinal=8, X=2000, seed=17),     # two words per row
    dict(model="potts", q=10, L=70, n_windows=6, m=2, kfinal=8, X=2000, seed=47),  # N > 4096: shared site map
    dict(model="potts", q=255, L=6, n_windows=2, m=8, kfinal=6, X=1000, seed=19),  # largest q
    dict(model="ising", L=4, n_windows=1, m=4, kfinal=10, X=1, seed=23),         # one window, X = 1
    dict(model="ising", L=12, n_windows=5, m=4, kfinal=10, X=700, seed=29, exchange=False),
    # Eq. (8): every level visited at least a / sqrt(ln f) times by every walker
    dict(model="ising", L=16, n_windows=4, m=8, kfinal=12, X=3000, seed=31, flat_rule="visits", flat=(1, 1)),
    dict(model="potts", q=10, L=8, n_windows=4, m=4, kfinal=12, X=3000, seed=37, flat_rule="visits", flat=(3, 2)),
    # explicit windows of unequal width (narrower tables padded to the widest)
    dict(model="ising", L=16, n_windows=4, m=8, kfinal=12, X=3000, seed=41,
         windows=([0, 30, 70, 110], [50, 100, 140, 256])),
    dict(model="potts", q=10, L=8, n_windows=4, m=4, kfinal=12, X=3000, seed=43,
         windows=([0, 20, 50, 80], [40, 70, 100, 128])),
]


def _tune(rw, kind, wpb=0, graph=0, poll=8):
    return rw.make_tune(kind, wpb, graph, poll)


@pytest.mark.parametrize("kind", ["lane", "wave"])
@pytest.mark.parametrize("kw", SMALL, ids=lambda kw: f"{kw['model']}-L{kw['L']}-h{kw['n_windows']}-m{kw['m']}"
                                                   f"{'-' + kw['flat_rule'] if 'flat_rule' in kw else ''}"
                                                   f"{'-windows' if 'windows' in kw else ''}")
def test_lockstep_small(rw, kw, kind):
    steps = 40 if kw["X"] > 1 else 3000
    gpu, _, _ = _lockstep(rw, kw, steps, tune=_tune(rw, kind), every=1 if kw["X"] > 1 else 500)
    assert gpu.info()["sweep_kind"] == kind          # every lattice here fits either variant


def test_ising_L8_full_run_bitwise(rw):
    """Ising L=8, 4 windows, m=1, ln f 1 -> 2^-20, X=1e4, seed 1: run to convergence."""
    kw = dict(model="ising", L=8, n_windows=4, m=1, kfinal=20, X=10000, seed=1)
    gpu, orc, done = _lockstep(rw, kw, 100000, every=25)
    assert done
    go, gj = gpu.concat()
    oo, oj = O.concat(O.make_config(**kw), O.mask_rule(O.make_config(**kw)), orc.pieces())
    assert np.array_equal(gj, oj)
    ok = np.isfinite(oo)
    assert np.array_equal(np.isfinite(go), ok)
    assert np.max(np.abs(go[ok] - oo[ok])) < 1e-9
    st = gpu.stats()
    ost = orc.stats()
    assert np.array_equal(st["ex_prop"], ost["ex_prop"]) and np.array_equal(st["ex_acc"], ost["ex_acc"])


@pytest.mark.parametrize("kw", [
    dict(model="ising", L=64, n_windows=16, m=64, kfinal=27, X=10000, seed=1),
    dict(model="potts", q=10, L=32, n_windows=32, m=128, kfinal=27, X=10000, seed=1),
], ids=["ising-L64-h16-m64", "potts-q10-L32-h32-m128"])
@pytest.mark.parametrize("kind", ["auto", "lane"])
def test_full_size_workloads_first_intervals(rw, kw, kind):
    _lockstep(rw, kw, 2, tune=_tune(rw, kind))


def test_walkers_per_block_does_not_change_results(rw):
    kw = dict(model="potts", q=8, L=16, n_windows=4, m=32, kfinal=12, X=2000, seed=3)
    gc, oc = _cfgs(rw, **kw)
    orc = O.Sim(oc)
    orc.run(12)
    ref = orc.state()
    for kind, wpb in (("lane", 1), ("lane", 4), ("lane", 16), ("lane", 32), ("wave", 1), ("wave", 2),
                      ("wave", 8)):
        g = rw.Rewl([gc], tune=_tune(rw, kind, wpb, poll=4))
        assert g.info()["walkers_per_block"] == wpb and g.info()["sweep_kind"] == kind
        g.run(12)
        assert_same(g.state(), ref, f"{kind} wpb={wpb}")
        g.close()


def test_graph_replay_matches_oracle(rw):
    """The interval captured once as a HIP graph and replayed, host syncs in between."""
    kw = dict(model="ising", L=16, n_windows=6, m=4, kfinal=10, X=1500, seed=31)
    gc, oc = _cfgs(rw, **kw)
    g = rw.Rewl([gc], tune=_tune(rw, "auto", graph=1, poll=5))
    orc = O.Sim(oc)
    for _ in range(8):
        g.run(10)
        orc.run(10)
        assert_same(g.state(), orc.state(), f"graph t={orc.t}")


def test_batch_of_mixed_instances(rw):
    """Instances of different models and sizes in one handle each follow their own oracle."""
    kws = [dict(model="ising", L=16, n_windows=4, m=8, kfinal=10, X=2000, seed=101),
           dict(model="potts", q=10, L=16, n_windows=8, m=4, kfinal=10, X=2000, seed=102),
           dict(model="potts", q=4, L=12, n_windows=3, m=16, kfinal=10, X=2000, seed=103),
           dict(model="ising", L=24, n_windows=8, m=2, kfinal=10, X=2000, seed=104)]
    for kind in ("lane", "wave"):
        g = rw.Rewl([rw.make_config(**kw) for kw in kws], tune=_tune(rw, kind))
        orcs = [O.Sim(O.make_config(**kw)) for kw in kws]
        for _ in range(3):
            g.run(7)
            for i, o in enumerate(orcs):
                o.run(7)
                assert_same(g.state(i), o.state(), f"{kind} instance {i}")
        g.close()


def test_checkpoint_restore_bitwise(rw):
    kw = dict(model="potts", q=6, L=10, n_windows=4, m=8, kfinal=12, X=1500, seed=41)
    gc, oc = _cfgs(rw, **kw)
    a = rw.Rewl([gc])
    a.run(15)
    blob = rw.rewl_checkpoint(a.h)
    a.run(15)
    b = rw.Rewl([gc])
    rw.rewl_restore(b.h, blob)
    b.run(15)
    assert_same(a.state(), b.state(), "restored run")
    orc = O.Sim(oc)
    orc.run(30)
    assert_same(b.state(), orc.state(), "restored vs oracle")


def test_warm_start_parity(rw):
    from oracle import exact_dos as X
    kw = dict(model="ising", L=8, n_windows=4, m=4, k0=10, kfinal=16, X=3000, seed=43)
    gc, oc = _cfgs(rw, **kw)
    lg = X.ln_g(X.kaufman_ising(8))
    rng = np.random.default_rng(0)
    warm = np.where(np.isfinite(lg), lg + rng.normal(0, 0.3, lg.shape), 0.0)
    warm = np.round(warm * 2**16) / 2**16
    g = rw.Rewl([gc])
    g.set_initial_lng(warm)
    orc = O.Sim(oc, init_lng=warm)
    for _ in range(6):
        g.run(10)
        orc.run(10)
        assert_same(g.state(), orc.state(), f"warm t={orc.t}")
    with pytest.raises(rw.RewlError):
        g.set_initial_lng(warm)                 # only before the first interval


def test_bad_warm_start_rejected(rw):
    g = rw.Rewl([rw.make_config(model="ising", L=8)])
    bad = np.full(65, 0.1)                       # not a multiple of 2^-20
    with pytest.raises(rw.RewlError):
        g.set_initial_lng(bad)


def test_batch64_first_interval_autotuned(rw):
    """The 64-instance uneven batch, autotuned, one interval: every instance bit-exact."""
    from paper_1407_5140_amd import workloads as W
    kws = W.batch()
    g = rw.Rewl([rw.make_config(**kw) for kw in kws], tune=rw.make_tune(autotune=1))
    chosen = g.tune()
    assert chosen["autotune"] == 0 and chosen["sweep_kind"] in (1, 2)
    orcs = [O.Sim(O.make_config(**kw)) for kw in kws]
    for i, o in enumerate(orcs):
        assert_same(g.state(i), o.state(), f"batch instance {i} after init")
    g.run(1)
    for i, o in enumerate(orcs):
        o.run(1)
        assert_same(g.state(i), o.state(), f"batch instance {i} after 1 interval")
