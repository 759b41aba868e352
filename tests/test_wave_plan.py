"""The wave sweep's plan (walkers per block, count placement, site-map size), the
host logic that create() applies with the device's attributes, checked through
its pure-host entry point at MI355X's figures (160 KiB of LDS per block, 256 CUs,
16 waves of the sweep kernel per CU).  No GPU is needed."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def rw():
    import paper_1407_5140_amd as rw
    return rw


def _plan(rw, kw, **tune):
    return rw.rewl_wave_plan(rw.make_config(**kw), rw.make_tune(**tune) if tune else None)


def test_all_walkers_resident_keeps_the_full_map_in_lds(rw):
    """Ising L=64, 16 x 64 walkers: 4 per block with the counts and the one-entry-
    per-site map in LDS already hold all 1 024 walkers at once."""
    from paper_1407_5140_amd import workloads as W
    p = _plan(rw, W.single("ising64"))
    assert p == dict(walkers_per_block=4, table_placement="lds", map_entries=4096, lds_bytes=154048)


@pytest.mark.parametrize("name,placement,entries", [
    ("potts32", "device", 1024),    # 4 blocks per CU instead of 3: all 4 096 resident, one entry per site
    ("ising128", "device", 1024),   # 16 sites per entry: 2 048 resident instead of 2 rounds
    ("potts64", "device", 512),     # 8 sites per entry: 4 096 resident instead of 4 rounds
    ("potts100", "lds", 2048),      # 616 walkers resident instead of 2 rounds
])
def test_resident_walkers_decide_placement_and_map(rw, name, placement, entries):
    from paper_1407_5140_amd import workloads as W
    kw = W.single(name)
    p = _plan(rw, kw)
    assert (p["table_placement"], p["map_entries"], p["walkers_per_block"]) == (placement, entries, 4)
    # every walker resident in one round: blocks per CU x walkers per block x 256 >= walkers
    per_cu = min(163840 // p["lds_bytes"], 16 // p["walkers_per_block"])
    assert per_cu * p["walkers_per_block"] * 256 >= kw["n_windows"] * kw["m"]


def test_forced_choices_are_kept(rw):
    from paper_1407_5140_amd import workloads as W
    p = _plan(rw, W.single("potts64"), table_placement="device", map_log2=12)
    assert (p["table_placement"], p["map_entries"]) == ("device", 4096)
    p = _plan(rw, W.single("ising64"), map_log2=6)
    assert p["map_entries"] == 64
    p = _plan(rw, dict(model="ising", L=16, n_windows=4, m=8, kfinal=12, X=3000, seed=5), map_log2=12)
    assert p["map_entries"] == 256                      # fewer sites than the cap: one entry per site


def test_lds_counts_that_do_not_fit_go_to_device_memory(rw):
    """The case of the GPU parity test: 10-state Potts L=90 in one 16 201-bin window."""
    kw = dict(model="potts", q=10, L=90, n_windows=1, m=2, kfinal=8, X=2000, seed=53)
    p = _plan(rw, kw, kind="wave", table_placement="lds")
    assert p == dict(walkers_per_block=1, table_placement="device", map_entries=2048,
                     lds_bytes=p["lds_bytes"]) and p["lds_bytes"] <= 163840


def test_bad_arguments_are_rejected(rw):
    from paper_1407_5140_amd import workloads as W
    cfg = rw.make_config(**W.single("ising64"))
    with pytest.raises(RuntimeError, match="map_log2"):
        rw.rewl_wave_plan(cfg, rw.make_tune(map_log2=5))
    with pytest.raises(RuntimeError, match="positive"):
        rw.rewl_wave_plan(cfg, None, n_cu=0)
    with pytest.raises(RuntimeError, match="exceed"):
        rw.rewl_wave_plan(cfg, None, lds_per_block=4096)
