"""GPU parity of Algorithm 1 with dense projections (xyz_dense_search) against
the oracle (oracle.dense): integer projections make E_l exact, so pairs (j, k,
s, first_rep, hits) and per-repetition candidates, passed, fresh and
max_bucket must be identical.  Sizes are ragged against the 64-column words,
the 256-column workgroups, the 8-repetition projection groups and the
32-bit words of a column.
"""
import numpy as np
import pytest

import synthgen
import paper_1610_05108_amd as xyz
from oracle import theory
from oracle.dense import dense_search, project

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = xyz.Context(0)
    yield c
    c.close()


def assert_same(res, rp, rr):
    gp, gr = res["pairs"], res["reps"]
    assert len(gp) == len(rp), (len(gp), len(rp))
    for f in ("j", "k", "s", "first_rep", "hits"):
        assert np.array_equal(gp[f], rp[f]), f
    assert np.array_equal(gp["value"], rp["value"].astype(np.float64))
    for f in ("candidates", "passed", "fresh", "max_bucket"):
        assert np.array_equal(gr[f], rr[f]), (f, gr[f][:8], rr[f][:8])


@pytest.mark.parametrize("n,p,L,kappa,budget,seed", [
    (700, 1500, 12, 0.1, 1500, 1),        # tau for mean |E_l| = p
    (333, 1037, 9, 0.12, 60, 2),          # tau for a budget of p = 60: windows of about p / 60 columns
    (64, 257, 3, 0.0, 4, 3),              # one word per column, big windows, half the pairs pass
])
def test_dense_gaussian_parity(ctx, n, p, L, kappa, budget, seed):
    d = synthgen.small_binary(n, p, seed=seed, planted=[(0, 5), (17, 200)], flip=0.15)
    R, sd = synthgen.gaussian_projections(n, L, seed=seed)
    tau = int(round(theory.tau_gauss(budget, n, sd)))
    x = ctx.x_create(d.XT)
    res = ctx.dense_search(x, d.Y, R, tau, kappa)
    rp, rr = dense_search(d.XT, d.Y, R, tau, kappa)
    assert rr["candidates"].sum() > 0
    assert_same(res, rp, rr)


def test_dense_tau0_subsampling(ctx):
    """tau = 0 with a subsampling projection: many equal projections (windows of
    whole buckets); equals the oracle and the Algorithm 2 search on the same rows."""
    d = synthgen.small_binary(400, 2000, seed=4, planted=[(3, 9)], flip=0.1)
    L, M = 10, 9
    R, rows, _ = synthgen.subsample_projections(d.n, L, M, seed=5)
    x = ctx.x_create(d.XT)
    res = ctx.dense_search(x, d.Y, R, 0, 0.15)
    rp, rr = dense_search(d.XT, d.Y, R, 0, 0.15)
    assert rr["max_bucket"].max() > 5
    assert_same(res, rp, rr)
    alg2 = ctx.search(x, d.Y, m=M, L=L, kappa=0.15, rows=rows)
    for f in ("j", "k", "s", "first_rep", "hits"):
        assert np.array_equal(res["pairs"][f], alg2["pairs"][f]), f
    assert np.array_equal(res["reps"]["candidates"], alg2["reps"]["candidates"])


def test_dense_all_pairs_and_survivor_growth(ctx):
    """tau beyond every distance: every pair is a candidate; kappa = -1 keeps all of
    them (3 x 44850 survivors, more than the first survivor buffer holds)."""
    d = synthgen.small_binary(97, 300, seed=6)
    R, _ = synthgen.gaussian_projections(d.n, 3, seed=7)
    x = ctx.x_create(d.XT)
    res = ctx.dense_search(x, d.Y, R, 1 << 40, -1.0, rep_offset=5)
    rp, rr = dense_search(d.XT, d.Y, R, 1 << 40, -1.0, rep_offset=5)
    assert (rr["candidates"] == 300 * 299 // 2).all()
    assert_same(res, rp, rr)


def test_dense_edges(ctx):
    # one column: no pairs
    d = synthgen.small_binary(50, 1, seed=8)
    R, _ = synthgen.gaussian_projections(50, 2, seed=1)
    x = ctx.x_create(d.XT)
    res = ctx.dense_search(x, d.Y, R, 1 << 40, -1.0)
    assert len(res["pairs"]) == 0 and (res["reps"]["candidates"] == 0).all()
    assert (res["reps"]["max_bucket"] == 1).all()
    # one row, all-zero projection: every column projects to 0
    d = synthgen.small_binary(1, 70, seed=9)
    x = ctx.x_create(d.XT)
    R0 = np.zeros((2, 1), dtype=np.int32)
    res = ctx.dense_search(x, d.Y, R0, 0, 0.5)
    rp, rr = dense_search(d.XT, d.Y, R0, 0, 0.5)
    assert_same(res, rp, rr)


def test_dense_split_repetitions(ctx):
    d = synthgen.small_binary(300, 900, seed=10, planted=[(1, 2)])
    R, sd = synthgen.gaussian_projections(d.n, 20, seed=11)
    tau = int(round(theory.tau_gauss(30, d.n, sd)))
    x = ctx.x_create(d.XT)
    full = ctx.dense_search(x, d.Y, R, tau, 0.1)
    a = ctx.dense_search(x, d.Y, R[:7], tau, 0.1)
    b = ctx.dense_search(x, d.Y, R[7:], tau, 0.1, rep_offset=7)
    assert np.array_equal(full["reps"]["candidates"],
                          np.concatenate([a["reps"]["candidates"], b["reps"]["candidates"]]))
    assert np.array_equal(full["reps"]["passed"], np.concatenate([a["reps"]["passed"], b["reps"]["passed"]]))


def test_dense_rejects(ctx):
    d = synthgen.small_binary(60, 40, seed=12)
    x = ctx.x_create(d.XT)
    R, _ = synthgen.gaussian_projections(60, 2, seed=1)
    with pytest.raises(xyz.XyzError):
        ctx.dense_search(x, d.Y, R, -1, 0.1)
    big = np.full((1, 60), 1 << 26, dtype=np.int32)           # sum |R| = 60 * 2^26 > 2^31
    with pytest.raises(xyz.XyzError):
        ctx.dense_search(x, d.Y, big, 10, 0.1)
    one = np.zeros((1, 60), dtype=np.int32)
    one[0, 7] = (1 << 31) - (1 << 24) + 1                     # one weight past the digits' range
    with pytest.raises(xyz.XyzError):
        ctx.dense_search(x, d.Y, one, 10, 0.1)
    one[0, 7] = -((1 << 31) - (1 << 24))                      # the largest accepted weight is exact
    res = ctx.dense_search(x, d.Y, one, 0, -1.0)
    rp, rr = dense_search(d.XT, d.Y, one, 0, -1.0)
    assert_same(res, rp, rr)
    with pytest.raises(xyz.XyzError):
        ctx.dense_search(x, d.Y.astype(np.float32), R, 10, 0.1)
    c = synthgen.small_continuous(60, 40, seed=1)
    xf = ctx.x_create(c.XT)
    with pytest.raises(xyz.XyzError):
        ctx.dense_search(xf, d.Y, R, 10, 0.1)
    # a matrix freed through the context is not freed again by close()
    ctx.x_destroy(xf)


def test_dense_large_p_chunks(ctx):
    """p = 2.2e6 columns, n = 100: the repetitions run in chunks of 8 (32 bytes per
    repetition and column under a 1 GiB bound).  Properties that hold at any size:
    the per-repetition counts equal those of single-repetition calls, and every
    reported pair is close in one orientation and has the reported s."""
    n, p, L = 100, 2_200_000, 20
    XT = synthgen.rademacher(n, p, seed=13)
    Y = np.where(np.random.default_rng(14).random(n) < 0.5, 1, -1).astype(np.int8)
    R, sd = synthgen.gaussian_projections(n, L, seed=15)
    tau = int(round(theory.tau_gauss(p, n, sd)))
    x = ctx.x_create(XT)
    kappa = 0.3
    full = ctx.dense_search(x, Y, R, tau, kappa)
    reps = full["reps"]
    assert reps["candidates"].min() > p // 4
    for l in (0, 9, 19):
        one = ctx.dense_search(x, Y, R[l:l + 1], tau, kappa, rep_offset=l)
        for f in ("candidates", "passed", "max_bucket"):
            assert one["reps"][f][0] == reps[f][l], (l, f)
    pairs = full["pairs"]
    assert len(pairs) > 0
    sel = pairs[:: max(1, len(pairs) // 200)]
    cols = np.unique(np.concatenate([sel["j"], sel["k"]]))
    sub = XT[cols]
    xs, zs = project(sub, Y, R)
    pos = {int(c): q for q, c in enumerate(cols)}
    for pr in sel:
        a, b = pos[int(pr["j"])], pos[int(pr["k"])]
        s = int((sub[a].astype(np.int64) * sub[b] * Y).sum())
        assert s == pr["s"] and s / n > kappa
        l = int(pr["first_rep"])
        assert abs(xs[l, a] - zs[l, b]) <= tau or abs(xs[l, b] - zs[l, a]) <= tau


def test_dense_device_y_and_growing_workspaces(ctx):
    """Y handed over in device memory, and calls of growing size on one context (the
    workspaces grow between calls) give the oracle's results."""
    import torch
    for n, p, L, seed in ((90, 300, 3, 21), (400, 2500, 17, 22), (150, 700, 9, 23)):
        d = synthgen.small_binary(n, p, seed=seed, planted=[(4, 8)], flip=0.1)
        R, sd = synthgen.gaussian_projections(n, L, seed=seed)
        tau = int(round(theory.tau_gauss(50, n, sd)))
        x = ctx.x_create(d.XT)
        yd = torch.from_numpy(d.Y).cuda()
        res = ctx.dense_search(x, yd, R, tau, 0.1, rep_offset=3)
        rp, rr = dense_search(d.XT, d.Y, R, tau, 0.1, rep_offset=3)
        assert_same(res, rp, rr)
        ctx.x_destroy(x)
