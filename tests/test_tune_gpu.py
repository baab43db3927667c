"""xyz_autotune: launch shapes timed once per search shape and reused from the
cache file; the shapes never change a search's result."""
import numpy as np
import pytest

import synthgen
import paper_1610_05108_amd as xyz

pytestmark = pytest.mark.gpu


def _case():
    d = synthgen.small_binary(1500, 60000, seed=51, planted=[(3, 59990), (10, 20)], flip=0.1)
    return d


def test_tune_then_reuse_cache(tmp_path):
    d = _case()
    path = tmp_path / "tune.txt"
    c1 = xyz.Context(0)
    try:
        x = c1.x_create(d.XT)
        before = c1.search(x, d.Y, m=9, L=40, kappa=0.3, seed=2)
        t1 = c1.autotune(x, d.Y, m=9, L=40, kappa=0.3, seed=2, cache_path=str(path))
        assert t1["from_cache"] == 0 and t1["variants"] >= 4 and t1["ms"] > 0
        after = c1.search(x, d.Y, m=9, L=40, kappa=0.3, seed=2)
        assert np.array_equal(before["pairs"], after["pairs"])
        assert np.array_equal(before["reps"], after["reps"])
        lines = [s for s in path.read_text().splitlines() if not s.startswith("#")]
        assert len(lines) == 1 and ":n1500:p60000:m9:" in lines[0]
    finally:
        c1.close()
    # a fresh context reads the record: nothing is timed, the same choice comes back
    c2 = xyz.Context(0)
    try:
        x = c2.x_create(d.XT)
        t2 = c2.autotune(x, d.Y, m=9, L=40, kappa=0.3, seed=2, cache_path=str(path))
        assert t2["from_cache"] == 1 and t2["variants"] == 0
        for f in ("chunk_gib", "verify_wg_per_cu", "big_wg_per_cu"):
            assert t2[f] == t1[f], f
        res = c2.search(x, d.Y, m=9, L=40, kappa=0.3, seed=2)
        assert np.array_equal(before["pairs"], res["pairs"])
        # another m is another shape: timed and added to the file
        t3 = c2.autotune(x, d.Y, m=7, L=20, kappa=0.3, seed=2, cache_path=str(path))
        assert t3["from_cache"] == 0
        lines = [s for s in path.read_text().splitlines() if not s.startswith("#")]
        assert len(lines) == 2
    finally:
        c2.close()


def test_tune_big_tiles_and_checks(tmp_path):
    """Large buckets (m = 3): the big-tile launch shape is tried too; no cache
    path keeps the choice in the context only."""
    d = synthgen.small_binary(800, 6000, seed=52, planted=[(1, 5)], flip=0.2)
    c = xyz.Context(0)
    try:
        x = c.x_create(d.XT)
        ref = c.search(x, d.Y, m=3, L=6, kappa=0.3, seed=4)
        t = c.autotune(x, d.Y, m=3, L=6, kappa=0.3, seed=4)
        assert t["from_cache"] == 0 and t["variants"] >= 7
        res = c.search(x, d.Y, m=3, L=6, kappa=0.3, seed=4)
        assert np.array_equal(ref["pairs"], res["pairs"])
        with pytest.raises(xyz.XyzError):
            c.autotune(x, d.Y, m=3, L=0, kappa=0.3)
    finally:
        c.close()
