"""The C-ABI library: it loads, exports every symbol include/*.h declares, and
its pure-host calls (layout, mask, validation) agree with the paper's example and
reject bad input before touching the device.  No GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rw():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "_rewl_build", os.path.join(ROOT, "paper_1407_5140_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.build_library(force=False)
    import paper_1407_5140_amd as rw
    return rw


def _declared():
    names = set()
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hdr.endswith(".h"):
            with open(os.path.join(ROOT, "include", hdr)) as f:
                txt = f.read()
            names |= set(re.findall(r"^\s*(?:rewl_status|void|const char\*)\s+((?:rewl|mlp)_\w+)\s*\(",
                                    txt, re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol(rw):
    names = _declared()
    assert len(names) >= 25 and any(n.startswith("mlp_") for n in names)
    lib = ctypes.CDLL(rw.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(rw.EXPORTED)


def test_layout_matches_paper_example(rw):
    for L, h in ((100, 77), (200, 317), (300, 717), (400, 1277)):
        if L > 255:
            continue                 # Potts lattices above 255 are outside the library's range
        W, WB, lo, hi = rw.rewl_layout(rw.make_config("potts", q=10, L=L, n_windows=h))
        assert WB == 1001 and np.array_equal(lo, 250 * np.arange(h)) and hi[-1] == W - 1


def test_layout_and_mask_match_oracle(rw):
    import oracle as O
    for model, q, L, h, ov in [("ising", 2, 8, 4, (3, 4)), ("ising", 2, 64, 16, (3, 4)),
                               ("potts", 10, 32, 32, (3, 4)), ("potts", 4, 24, 8, (1, 2)),
                               ("ising", 2, 128, 32, (3, 4)), ("potts", 3, 5, 1, (0, 1))]:
        c = rw.make_config(model, q=q, L=L, n_windows=h, overlap=ov)
        oc = O.make_config(model, q=q, L=L, n_windows=h, overlap=ov)
        W, WB, lo, hi = rw.rewl_layout(c)
        olo, ohi = O.layout(oc)
        assert W == O.n_bins(oc) and np.array_equal(lo, olo) and np.array_equal(hi, ohi)
        assert np.array_equal(rw.rewl_mask(c), O.mask_rule(oc))


@pytest.mark.parametrize("kw,status", [
    (dict(model="ising", L=7), -1), (dict(model="ising", L=130), -1), (dict(model="potts", q=2, L=8), -1),
    (dict(m=3), -1), (dict(m=2048), -1), (dict(k0=5, kfinal=5), -1), (dict(kfinal=41), -1),
    (dict(overlap=(4, 4)), -1), (dict(overlap=(1, 0)), -1), (dict(flat=(6, 5)), -1), (dict(X=0), -1),
    (dict(n_windows=0), -1), (dict(model="potts", q=300, L=8), -1)])
def test_invalid_configs_rejected_before_allocation(rw, kw, status):
    c = rw.make_config(**kw)
    with pytest.raises(rw.RewlError) as e:
        rw.rewl_create(c)
    assert e.value.status == status
    with pytest.raises(rw.RewlError):
        rw.rewl_layout(c)


def test_explicit_windows_layout_matches_oracle(rw):
    import oracle as O
    wins = ([0, 12, 26, 44], [20, 38, 52, 64])
    c = rw.make_config("ising", L=8, n_windows=4, windows=wins)
    oc = O.make_config("ising", L=8, n_windows=4, windows=wins)
    W, WB, lo, hi = rw.rewl_layout(c)
    olo, ohi = O.layout(oc)
    assert W == 65 and WB == 27 and np.array_equal(lo, olo) and np.array_equal(hi, ohi)
    for bad in (([0, 25, 30], [20, 40, 64]), ([0, 10, 30], [20, 40, 63]), ([0, 10, 30], [20, 40, 30])):
        with pytest.raises(rw.RewlError):
            rw.rewl_layout(rw.make_config("ising", L=8, n_windows=3, windows=bad))


@pytest.mark.parametrize("model,q,L,h", [("ising", 2, 32, 8), ("potts", 10, 24, 12), ("ising", 2, 64, 16)])
def test_balanced_layout_equalises_difficulty(rw, model, q, L, h):
    c = rw.make_config(model, q=q, L=L, n_windows=h)
    W, WB, lo_eq, hi_eq = rw.rewl_layout(c)
    # uniform difficulty gives back the equal partition up to rounding
    lo, hi = rw.rewl_balanced_layout(c, np.ones(W))
    assert np.abs(lo - lo_eq).max() <= 2 and np.abs(hi - hi_eq).max() <= 2
    # harder ends: narrower end windows, sums of rho about equal, a valid layout
    rho = np.ones(W)
    rho[: W // 5] = 4.0
    rho[-(W // 5):] = 4.0
    lo, hi = rw.rewl_balanced_layout(c, rho)
    c2 = rw.make_config(model, q=q, L=L, n_windows=h, windows=(lo, hi))
    W2, WB2, lo2, hi2 = rw.rewl_layout(c2)
    assert np.array_equal(lo2, lo) and np.array_equal(hi2, hi) and WB2 == (hi - lo + 1).max()
    width = hi - lo + 1
    assert width[0] < width[h // 2] and width[-1] < width[h // 2]
    sums = np.array([rho[l:u + 1].sum() for l, u in zip(lo, hi)])
    assert sums.max() / sums.min() < 1.25
    assert ((hi[:-1] - lo[1:] + 1) >= 8).all()


def test_thermo_and_ensemble_validate_on_the_host(rw):
    """Bad arguments are rejected before any device call (runs without a GPU)."""
    lg = np.zeros(17)
    inf_row = lg.copy()
    inf_row[2] = np.inf
    cases = [("ising", 4, lg, [0.0]), ("ising", 4, lg, [np.nan]), ("ising", 4, lg, [-1.0]),
             (5, 4, lg, [1.0]), ("ising", 4, np.full(17, -np.inf), [1.0]), ("ising", 1, np.zeros(2), [1.0]),
             ("ising", 4, inf_row, [1.0])]
    for args in cases:
        with pytest.raises(rw.RewlError) as e:
            rw.rewl_thermo(*args)
        assert e.value.status == rw.REWL_E_INVALID
    with pytest.raises(rw.RewlError) as e:
        rw.rewl_ensemble(None, [0], 1, 1, 17, 4)
    assert e.value.status == rw.REWL_E_INVALID


def test_import_without_the_library_fails_loudly(tmp_path):
    """No CPU fallback: the binding refuses to import when librewl.so is absent."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_1407_5140_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_1407_5140_amd", "__init__.py"), pkg / "__init__.py")
    r = subprocess.run([sys.executable, "-c", "import paper_1407_5140_amd"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "no CPU fallback" in r.stderr


def test_tilt_density_model(rw):
    """rewl_tilt_density: sqrt of the rejected-move factor near the ground levels
    (Ising both ends, symmetric; Potts the ground end), flat beyond N/5."""
    ci = rw.make_config(model="ising", L=16, n_windows=4)
    r = rw.rewl_tilt_density(ci)
    N = 256
    assert r.size == N + 1 and np.allclose(r, r[::-1])
    assert np.isclose(r[0], np.sqrt(1 + N / 2)) and np.isclose(r[10], np.sqrt(1 + N / 12))
    assert np.allclose(r[52:N - 51], np.sqrt(1 + N / (N / 5 + 2)))
    cp = rw.make_config(model="potts", q=10, L=20, n_windows=6)
    r = rw.rewl_tilt_density(cp)
    N = 400
    assert r.size == 2 * N + 1
    assert np.isclose(r[0], np.sqrt(1 + 18 * N / 4)) and np.isclose(r[36], np.sqrt(1 + 18 * N / 40))
    assert np.all(np.diff(r[:81]) < 0) and np.allclose(r[80:], np.sqrt(1 + 18 * N / 84))
    lo, hi = rw.tilted_layout(cp)
    w = hi - lo + 1
    assert w[0] < w[-1] and lo[0] == 0 and hi[-1] == 2 * N
    with pytest.raises(rw.RewlError):
        rw.rewl_tilt_density(rw.make_config(model="ising", L=16, n_windows=0))
