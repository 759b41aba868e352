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
