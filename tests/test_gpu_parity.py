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


def _tune(rw, kind, wpb=0, graph=0, poll=8, placement="auto"):
    persistent = map_log2 = 0
    if kind == "wave-device":
        kind, placement = "wave", "device"
    if kind == "wave-map64":
        kind, map_log2 = "wave", 6
    if kind == "lane-persist":
        kind, persistent = "lane", 1
    return rw.make_tune(kind, wpb, graph, poll, table_placement=placement, persistent=persistent,
                        map_log2=map_log2)


@pytest.mark.parametrize("kind", ["lane", "lane-persist", "wave", "wave-device", "wave-map64"])
@pytest.mark.parametrize("kw", SMALL, ids=lambda kw: f"{kw['model']}-L{kw['L']}-h{kw['n_windows']}-m{kw['m']}"
                                                   f"{'-' + kw['flat_rule'] if 'flat_rule' in kw else ''}"
                                                   f"{'-windows' if 'windows' in kw else ''}")
def test_lockstep_small(rw, kw, kind):
    """Lane sweep (one block per tile, or a persistent grid over a tile queue), wave
    sweep with the counts in LDS, with the counts read from device memory, and with
    a site map of 64 entries (sites equal modulo 64 share one: extra re-evaluations
    on every lattice above 8 x 8): each bit-identical to the oracle."""
    steps = 40 if kw["X"] > 1 else 3000
    gpu, _, _ = _lockstep(rw, kw, steps, tune=_tune(rw, kind), every=1 if kw["X"] > 1 else 500)
    info = gpu.info()
    assert info["sweep_kind"] == kind.split("-")[0]          # every lattice here fits either variant
    if kind == "wave-device":
        assert info["table_placement"] == "device"
    if kind == "wave-map64":
        assert info["map_entries"] == min(kw["L"] ** 2, 64)
    elif kind.startswith("wave"):
        assert info["map_entries"] == min(kw["L"] ** 2, 4096)    # small batches: the full map


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
    assert np.array_equal(st["round_trips"], orc.replicas()["round_trips"])
    assert st["round_trips_total"] > 0


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


# ------------------------------------------- the exact slow path under lockstep
WIDE_BAND = [SMALL[1], SMALL[2], SMALL[3], SMALL[5], SMALL[6], SMALL[10], SMALL[12]]


@pytest.mark.parametrize("kind", ["lane", "wave", "wave-device"])
@pytest.mark.parametrize("kw", WIDE_BAND, ids=lambda kw: f"{kw['model']}-L{kw['L']}-m{kw['m']}-seed{kw['seed']}")
def test_lockstep_wide_guard_band(rw, kw, kind):
    """Guard band widened from 2^-40 to 2^-6: hundreds to thousands of decisions per run
    fall inside it and are taken by the double-double slow path (the lane sweep's per-lane branch,
    the wave sweep's in-order re-decision loop, the exchange); every decision is exact,
    so the run must stay bit-identical to the oracle."""
    tune = rw.make_tune(kind.split("-")[0], 0, 0, 8, guard_band_log2=-6,
                        table_placement="device" if kind == "wave-device" else "auto")
    gpu, _, _ = _lockstep(rw, kw, 25, tune=tune, every=5)
    assert gpu.info()["sweep_kind"] == kind.split("-")[0]
    assert gpu.stats()["slow_decisions"] > 500


def test_default_guard_band_rarely_used(rw):
    """At the default 2^-40 band the slow path is ~1e-12 per attempt: none in a short run."""
    kw = SMALL[2]
    g = rw.Rewl([rw.make_config(**kw)])
    g.run(20)
    assert g.stats()["slow_decisions"] == 0


# ------------------------------------- full-size merges, done and frozen windows
@pytest.mark.parametrize("kw", [
    dict(model="ising", L=64, n_windows=16, m=64, kfinal=10, X=10000, seed=1, flat_rule="visits", flat=(0, 1)),
    dict(model="potts", q=10, L=32, n_windows=32, m=128, kfinal=10, X=10000, seed=1, flat_rule="visits",
         flat=(0, 1)),
], ids=["ising-L64-h16-m64", "potts-q10-L32-h32-m128"])
@pytest.mark.parametrize("kind", ["auto", "lane", "wave-device"])
def test_full_size_merges_to_done(rw, kw, kind):
    """The full-size workloads with Eq. (8) at a = 0: every walker passes at every
    interval, so all windows merge (m = 64 / 128 walkers of 864 / 236 bins) at every
    interval until ln f reaches 2^-10 and the run stops, bit-exact throughout."""
    gpu, orc, done = _lockstep(rw, kw, 12, tune=_tune(rw, kind))
    assert done and orc.t == 10
    assert list(gpu.stats()["k"]) == [10] * kw["n_windows"]


def test_lds_counts_that_do_not_fit_go_to_device_memory(rw):
    """10-state Potts L=90 in one window of 16 201 bins: the base table (130 KB) leaves
    no room for an LDS copy of the counts, so counts asked for in LDS are kept in
    device memory, with the largest site map that fits (2 048 entries for 8 100
    sites); bit-exact to the oracle."""
    kw = dict(model="potts", q=10, L=90, n_windows=1, m=2, kfinal=8, X=2000, seed=53)
    gpu, _, _ = _lockstep(rw, kw, 5, tune=_tune(rw, "wave", placement="lds"))
    info = gpu.info()
    assert info["sweep_kind"] == "wave" and info["table_placement"] == "device"
    assert info["map_entries"] == 2048


@pytest.mark.parametrize("name", ["potts64", "ising128"])
def test_resident_site_map_full_size(rw, name):
    """The larger targets (10-state Potts L=64, 32 windows x 128 walkers; Ising
    L=128, 32 x 64) with the library's own choice of placement and site map: a map
    below the 4096-entry cap, so that every walker is resident at once, and with it
    sites sharing map entries.  Three intervals bit-exact to the oracle."""
    from paper_1407_5140_amd import workloads as W
    kw = W.single(name)
    gpu, orc, _ = _lockstep(rw, kw, 3)
    info = gpu.info()
    print(name, info, flush=True)
    assert info["sweep_kind"] == "wave" and info["map_entries"] < 4096


@pytest.mark.parametrize("kw", [
    dict(model="ising", L=16, n_windows=4, m=64, kfinal=7, X=2000, seed=3),
    dict(model="potts", q=4, L=8, n_windows=3, m=128, kfinal=5, X=1000, seed=5),
], ids=["ising-L16-m64", "potts-q4-L8-m128"])
@pytest.mark.parametrize("kind", ["lane", "wave", "wave-device"])
def test_staggered_convergence_with_frozen_windows(rw, kw, kind):
    """m = 64 / 128 walkers per window run to the end under the 80 % rule; windows
    converge hundreds of intervals apart, so converged windows walk frozen and keep
    exchanging while the others merge.  Bit-exact to the oracle, including the
    exchange counters and every replica's round trips."""
    gpu, orc, done = _lockstep(rw, kw, 5000, tune=_tune(rw, kind, poll=50), every=50)
    assert done
    st, ost = gpu.stats(), orc.stats()
    assert np.array_equal(st["ex_prop"], ost["ex_prop"]) and np.array_equal(st["ex_acc"], ost["ex_acc"])
    rt = orc.replicas()["round_trips"]
    assert np.array_equal(st["round_trips"], rt) and rt.sum() > 100
    assert st["round_trips_total"] == rt.sum()


# ----------------------------------------------------------- batch graph replay
@pytest.mark.parametrize("kind", ["lane", "lane-persist", "wave", "wave-device"])
def test_batch_graph_replay_mixed(rw, kind):
    """A mixed batch replays its captured interval graph for 60 intervals, with host
    syncs, state reads and eager oracle work between replays; every replay's result
    is compared with the oracle."""
    kws = [dict(model="ising", L=16, n_windows=4, m=8, kfinal=12, X=2000, seed=111),
           dict(model="potts", q=10, L=16, n_windows=8, m=4, kfinal=12, X=2000, seed=112),
           dict(model="potts", q=4, L=12, n_windows=3, m=16, kfinal=12, X=2000, seed=113),
           dict(model="ising", L=24, n_windows=8, m=2, kfinal=12, X=2000, seed=114),
           dict(model="ising", L=8, n_windows=4, m=4, kfinal=8, X=2000, seed=115)]
    g = rw.Rewl([rw.make_config(**kw) for kw in kws], tune=_tune(rw, kind, graph=1, poll=3))
    orcs = [O.Sim(O.make_config(**kw)) for kw in kws]
    for _ in range(20):
        g.run(3)
        for i, o in enumerate(orcs):
            o.run(3)
            assert_same(g.state(i), o.state(), f"graph {kind} instance {i}")
    for i, o in enumerate(orcs):
        assert np.array_equal(g.stats(i)["round_trips"], o.replicas()["round_trips"])
    g.close()


def test_batch64_graph_replay_autotuned(rw):
    """The 64-instance batch, autotuned, four intervals replayed from its captured graph."""
    from paper_1407_5140_amd import workloads as W
    kws = W.batch()
    g = rw.Rewl([rw.make_config(**kw) for kw in kws], tune=rw.make_tune(autotune=1, use_graph=1, poll_every=2))
    assert g.tune()["use_graph"] == 1
    orcs = [O.Sim(O.make_config(**kw)) for kw in kws]
    for _ in range(2):
        g.run(2)
        for i, o in enumerate(orcs):
            o.run(2)
            assert_same(g.state(i), o.state(), f"batch instance {i} t={o.t}")
    g.close()


# ------------------------------------------------------- counts past 2^32
def _ckpt_H_offset(rw, g, cfg):
    """Byte offset and shape of the first instance's H array inside a checkpoint."""
    W, WB, lo, hi = rw.rewl_layout(cfg)
    S, N = cfg.n_windows * cfg.walkers_per_window, cfg.L * cfg.L
    lat = cfg.L * ((cfg.L + 63) // 64) * S * 8 if cfg.model == 0 else N * S
    return 16 + lat + S * 4, (S, WB)


@pytest.mark.parametrize("kind", ["lane", "wave", "wave-device"])
def test_counts_past_2_32_bitwise(rw, kind):
    """Every walker's counts raised by C = 2^32 + 2^31 + 12345 at every occurring level
    of its window (the oracle's ln g raised by C 2^-k to match), written into a
    checkpoint and restored: the run continues bit-exact with counts above 2^32.
    Eq. (8) with a = 2^20 keeps every window from merging at ln f = 2^-30."""
    kw = dict(model="potts", q=5, L=8, n_windows=3, m=4, k0=30, kfinal=34, X=1500, seed=71,
              flat_rule="visits", flat=(1 << 20, 1))
    gc, oc = _cfgs(rw, **kw)
    g = rw.Rewl([gc], tune=_tune(rw, kind))
    orc = O.Sim(oc)
    g.run(3)
    orc.run(3)
    assert_same(g.state(), orc.state(), "before")
    C = (1 << 32) + (1 << 31) + 12345
    W, WB, lo, hi = rw.rewl_layout(gc)
    mask = rw.rewl_mask(gc)
    occ = np.zeros((kw["n_windows"] * kw["m"], WB), bool)
    for s in range(occ.shape[0]):
        a = s // kw["m"]
        occ[s, : hi[a] - lo[a] + 1] = mask[lo[a]:hi[a] + 1] > 0
    blob = bytearray(rw.rewl_checkpoint(g.h))
    off, shape = _ckpt_H_offset(rw, g, gc)
    H = np.frombuffer(bytes(blob[off:off + 8 * shape[0] * shape[1]]), np.uint64).reshape(shape).copy()
    H[occ] += np.uint64(C)
    blob[off:off + H.nbytes] = H.tobytes()
    rw.rewl_restore(g.h, bytes(blob))
    st = orc.state()
    k = st["k"][np.arange(occ.shape[0]) // kw["m"]]
    orc.set_tables(np.where(occ, st["H"] + C, st["H"]),
                   np.where(occ, st["lng"] + np.ldexp(float(C), -k)[:, None], st["lng"]))
    assert_same(g.state(), orc.state(), "restored")
    for _ in range(4):
        g.run(5)
        orc.run(5)
        assert_same(g.state(), orc.state(), f"t={orc.t}")
    assert g.state()["H"].min(initial=C, where=occ) >= C


def test_count_spread_past_2_32_is_reported(rw):
    """One level of one walker raised by 2^32: the walker's counts now spread over more
    than the 32-bit range that a sweep keeps per level in LDS, and the run stops with
    REWL_E_OVERFLOW instead of continuing on wrapped counts."""
    kw = dict(model="ising", L=8, n_windows=2, m=2, k0=10, kfinal=20, X=500, seed=73)
    gc = rw.make_config(**kw)
    g = rw.Rewl([gc], tune=_tune(rw, "wave", placement="lds"))
    g.run(2)
    blob = bytearray(rw.rewl_checkpoint(g.h))
    off, shape = _ckpt_H_offset(rw, g, gc)
    H = np.frombuffer(bytes(blob[off:off + 8 * shape[0] * shape[1]]), np.uint64).reshape(shape).copy()
    H[0, 0] += np.uint64(1 << 32)
    blob[off:off + H.nbytes] = H.tobytes()
    rw.rewl_restore(g.h, bytes(blob))
    with pytest.raises(rw.RewlError) as e:
        g.run(2)
    assert e.value.status == -5
