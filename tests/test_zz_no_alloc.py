"""The search entry point that allocates nothing (xyz_search_noalloc) against
xyz_search on the same inputs, through the C ABI.

Its workspaces live in the library's static device scratch, which keeps the
previous call's contents, so the checks run calls back to back with the
second input smaller than the first.  Pairs, every pair statistic and every
per-repetition statistic must be identical to xyz_search's, and the context
must hold exactly the bytes of its resident matrices throughout (no
workspace is allocated for these calls).
"""
import sys

import numpy as np
import pytest
import torch

import synthgen
import paper_1610_05108_amd as xyz

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _same(a, b):
    assert len(a["pairs"]) == len(b["pairs"]), (len(a["pairs"]), len(b["pairs"]))
    for f in ("j", "k", "s", "value", "stat", "first_rep", "hits"):
        assert np.array_equal(a["pairs"][f], b["pairs"][f]), f
    assert len(a["reps"]) == len(b["reps"])
    for f in ("candidates", "passed", "fresh", "cmask", "max_bucket"):
        assert np.array_equal(a["reps"][f], b["reps"][f]), f


def test_noalloc_matches_search_on_consecutive_calls():
    dev = torch.device("cuda:0")
    with xyz.Context(0) as ctx:
        big = synthgen.small_binary(600, 6000, seed=41, planted=[(5, 77), (300, 4000)], flip=0.2)
        small = synthgen.small_binary(150, 900, seed=42, planted=[(1, 2)], flip=0.1)
        real = synthgen.small_continuous(300, 1200, seed=43, planted=[(4, 9)])
        xb = ctx.x_create(torch.from_numpy(big.XT).to(dev))
        xs = ctx.x_create(small.XT)                  # host input
        xr = ctx.x_create(real.XT)
        held = xyz.xyz_ctx_bytes(ctx.h)
        Yb = torch.from_numpy(big.Y).to(dev)
        cases = [
            ("big, device Y, m=10", xb, Yb, dict(m=10, L=24, kappa=0.1, seed=3)),
            ("small, host Y, m=6", xs, small.Y, dict(m=6, L=11, kappa=0.05, seed=4, two_sided=True)),
            ("big, sort path m=17", xb, Yb, dict(m=17, L=9, kappa=0.1, seed=5)),
            ("small, m=0 rep_offset", xs, small.Y, dict(m=0, L=2, kappa=0.2, seed=6, rep_offset=7)),
            ("real data, weighted rows", xr, real.Y, dict(m=5, L=12, kappa=0.4, seed=7)),
        ]
        got = []
        for name, x, Y, kw in cases:
            _log(f"no-alloc case: {name} {kw}")
            got.append(xyz.xyz_search_noalloc(ctx.h, x, Y, pairs_cap=1 << 18, **kw))
            torch.cuda.synchronize()
            assert xyz.xyz_ctx_bytes(ctx.h) == held
        # too many pairs for the caller's buffer: XYZ_ENOMEM with the count
        with pytest.raises(xyz.XyzError) as ei:
            xyz.xyz_search_noalloc(ctx.h, xs, small.Y, m=0, L=1, kappa=-2.0, pairs_cap=10)
        assert ei.value.code == xyz.XYZ_ENOMEM and ei.value.npairs == 900 * 899 // 2
        assert xyz.xyz_ctx_bytes(ctx.h) == held
        for (name, x, Y, kw), g in zip(cases, got):
            _log(f"reference search: {name}")
            ref = ctx.search(x, Y, **kw)
            _same(g, ref)
        assert len(got[0]["pairs"]) > 0 and got[0]["reps"]["candidates"].sum() > 10000


def test_noalloc_rejects_what_does_not_fit():
    with xyz.Context(0) as ctx:
        d = synthgen.small_binary(64, 16, seed=44)
        x = ctx.x_create(d.XT)
        # the statistics of 3 * 2^20 repetitions alone (64 B each) exceed half of the scratch
        with pytest.raises(xyz.XyzError) as ei:
            xyz.xyz_search_noalloc(ctx.h, x, d.Y, m=2, L=3 << 20, kappa=0.5)
        assert ei.value.code == xyz.XYZ_ENOMEM
        with pytest.raises(xyz.XyzError) as ei:
            xyz.xyz_search_noalloc(ctx.h, x, d.Y, m=2, L=3, kappa=0.5, pairs_cap=-1)
        assert ei.value.code == xyz.XYZ_EINVAL
        # still usable after the rejections
        r = xyz.xyz_search_noalloc(ctx.h, x, d.Y, m=2, L=3, kappa=-2.0)
        _same(r, ctx.search(x, d.Y, m=2, L=3, kappa=-2.0))
