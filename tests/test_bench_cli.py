"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message, and the profiled-traffic lookup only answers for the
kernel sources the counters were taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profiled_traffic_requires_matching_sources(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    got = bench.profiled_traffic("ising64", "k_sweep_wave")
    # either the committed summary matches the current kernel sources (two byte
    # counts) or it does not (None); a wrong kernel name never matches
    assert got is None or (len(got) == 2 and all(v > 0 for v in got))
    assert bench.profiled_traffic("ising64", "no_such_kernel") is None
    for k in ("k_sweep_persist", "k_rng"):
        got = bench.profiled_traffic("batch64", k)
        assert got is None or (len(got) == 2 and all(v > 0 for v in got))
    assert bench.profiled_traffic("potts100", "k_sweep_wave") is None     # no summary committed
    # the persistent and the plain lane sweep are different kernels
    info = {"sweep_kind": "lane"}
    assert bench.sweep_kernel(info, {"persistent": 1}) == "k_sweep_persist"
    assert bench.sweep_kernel(info, {"persistent": 0}) == "k_sweep"
    assert bench.sweep_kernel({"sweep_kind": "wave"}, {"persistent": 1}) == "k_sweep_wave"


def test_ground_tilted_windows_are_a_valid_layout():
    """The windows narrowed towards the ground state for the L = 100 Potts runs
    (pure host): accepted by the oracle's layout check, narrowest at the ground
    level, widening up to b ~ 2000 and even above it."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    import oracle as O
    import paper_1407_5140_amd as rw
    kw = dict(model="potts", q=10, L=100, n_windows=90, m=8, kfinal=14, X=10000, seed=1)
    lo, hi = bench.tilted_windows(rw, kw)
    c = O.make_config(**dict(kw, windows=(lo, hi)))
    olo, ohi = O.layout(c)
    assert np.array_equal(olo, lo) and np.array_equal(ohi, hi)
    w = hi - lo + 1
    assert lo[0] == 0 and hi[-1] == 2 * 100 * 100
    assert w[0] < 200 and np.all(np.diff(w[:8]) > 0)
    upper = w[lo > 2000]
    assert upper.max() - upper.min() <= 2 and upper.max() < 1001


def test_suggested_k0_follows_the_table_error():
    sys.path.insert(0, ROOT)
    from paper_1407_5140_amd import warm as Wm
    assert Wm.suggest_k0(1e-5, 1024) == 10          # error ~0.01 in ln g: the full skip
    assert Wm.suggest_k0(9e-4, 1024) == 10          # just below 1
    assert Wm.suggest_k0(1e-2, 1024) == 6           # ~10: the measured better start
    assert Wm.suggest_k0(3.8e-3, 10000) == 4        # the L = 100 network, ~38
    assert Wm.suggest_k0(1.0, 10 ** 6) == 0
