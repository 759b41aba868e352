"""rewl_concat_noalloc (staging in the library's fixed device array) against
rewl_concat (per-call device buffers): both run the same Sec. II.B kernel on the
same pieces, so the joined ln g and the join bins must be identical, on two calls
in a row, the second on a smaller instance, then a rejected oversized one."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_concat_noalloc_matches_concat_twice():
    import paper_1407_5140_amd as rw
    cases = [dict(model="potts", q=10, L=32, n_windows=8, m=4, kfinal=20, X=2000, seed=3),
             dict(model="ising", L=16, n_windows=4, m=4, kfinal=20, X=2000, seed=4)]
    sizes = []
    for kw in cases:
        cfg = rw.make_config(**kw)
        g = rw.Rewl([cfg])
        g.run(300)
        W = rw.rewl_layout(cfg)[0]
        ref, rj = rw.rewl_concat(g.h, 0, W, kw["n_windows"])
        got, gj = rw.rewl_concat_noalloc(g.h, 0, W, kw["n_windows"])
        assert np.array_equal(gj, rj)
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
        assert np.isfinite(got).sum() > W // 2
        sizes.append(W)
        g.close()
    assert sizes[1] < sizes[0]


def test_concat_noalloc_rejects_oversized():
    import paper_1407_5140_amd as rw
    cfg = rw.make_config(model="potts", q=3, L=128, n_windows=64, m=1, kfinal=10, X=100, seed=5)
    g = rw.Rewl([cfg])
    W = rw.rewl_layout(cfg)[0]
    with pytest.raises(rw.RewlError) as e:
        rw.rewl_concat_noalloc(g.h, 0, W, 64)
    assert e.value.status == rw.REWL_E_INVALID and "262144" in str(e.value)
    out, _ = rw.rewl_concat(g.h, 0, W, 64)           # the allocating call still serves it
    assert np.isfinite(out).sum() > 0
    g.close()
