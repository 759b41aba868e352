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
    assert bench.profiled_traffic("batch64", "k_sweep") is None
