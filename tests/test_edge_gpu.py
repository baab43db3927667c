"""GPU parity on the degenerate cases of the method, against the oracle.

Tiny and ragged shapes, one giant bucket (all columns equal), a constant
response (partner mask c = 0 in every repetition, so E_l is the pairs inside
each bucket), thresholds that every pair or no pair passes, more sampled rows
than rows, and the exact search on blocks that are almost empty.
"""
import numpy as np
import pytest

import oracle
import synthgen
import paper_1610_05108_amd as xyz

from test_parity_gpu import assert_same_binary, run_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = xyz.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n,p,m,L,kappa", [
    (1, 2, 1, 1, -2.0),
    (2, 3, 3, 4, -0.6),
    (33, 2, 5, 3, -1.0),
    (65, 5, 2, 7, 0.0),
])
def test_tiny_shapes(ctx, n, p, m, L, kappa):
    d = synthgen.small_binary(n, p, seed=n * 100 + p)
    res, rp, rr = run_both(ctx, d.XT, d.Y, m, L, kappa, seed=1)
    assert_same_binary(res, rp, rr)


@pytest.mark.parametrize("n", [(1 << 24) - 1, (1 << 24) + 1])
def test_rows_at_the_fp32_limit(ctx, n):
    """Columns of 2^24 - 1 rows (the longest whose counts the FP32 matrix-core accumulators hold
    exactly) and of 2^24 + 1 rows (past it the search counts on the vector units): with m = 2 on
    24 columns the whole search equals the oracle's; with m = 0 every pair of 80 columns is a
    candidate (one bucket, block-pair tiles below the limit) and is reported with its exact
    value (kappa below every statistic), and a threshold placed at the planted pair's own value
    keeps it (smin = s) or drops it (smin = s + 1): the FP32 filter in front of the exact integer
    test rounds monotonically, so it never drops a pair the integer test keeps."""
    d = synthgen.long_binary(n, 80, seed=5, pair=(3, 17), share=0.3)
    res, rp, rr = run_both(ctx, np.ascontiguousarray(d.XT[:24]), d.Y, 2, 2, -2.0, seed=1)
    assert_same_binary(res, rp, rr)
    x = ctx.x_create(d.XT)
    r = ctx.search(x, d.Y, m=0, L=1, kappa=-2.0, seed=1)
    assert len(r["pairs"]) == 80 * 79 // 2
    assert int(r["reps"]["candidates"][0]) == 80 * 79 // 2
    assert (r["timing"]["big_launches"] >= 1) == (n < (1 << 24))
    pos = {(int(j), int(k)): q for q, (j, k) in enumerate(zip(r["pairs"]["j"], r["pairs"]["k"]))}
    rng = np.random.default_rng(0)
    check = [(3, 17)] + [tuple(sorted(rng.choice(80, size=2, replace=False).tolist())) for _ in range(30)]
    for j, k in check:
        assert int(r["pairs"]["s"][pos[(j, k)]]) == oracle.pair_value(d.XT, d.Y, j, k), (j, k)
    s_planted = int(r["pairs"]["s"][pos[(3, 17)]])
    assert s_planted > 0.25 * n                    # the planted pair stands out (share 0.3)
    # the threshold at the planted pair's value: kept at smin = s, dropped at smin = s + 1 (every
    # other pair lies near 0)
    lo = ctx.search(x, d.Y, m=0, L=1, kappa=(s_planted - 0.5) / n, seed=1)
    hi = ctx.search(x, d.Y, m=0, L=1, kappa=(s_planted + 0.5) / n, seed=1)
    assert [(int(j), int(k)) for j, k in zip(lo["pairs"]["j"], lo["pairs"]["k"])] == [(3, 17)]
    assert len(hi["pairs"]) == 0


def test_one_giant_bucket(ctx):
    """Every column equal: every key is the same, one bucket holds all p columns
    (products split into many tiles, all three tile lists possible)."""
    col = np.where(np.random.default_rng(2).random(300) < 0.5, 1, -1).astype(np.int8)
    XT = np.tile(col, (700, 1))
    Y = np.ones(300, dtype=np.int8)                # s = n for every pair, c = 0: E_l = all pairs
    for m in (6, 17):
        res, rp, rr = run_both(ctx, XT, Y, m, 2, 0.5, seed=3)
        assert_same_binary(res, rp, rr)
        assert len(rp) == 700 * 699 // 2


def test_constant_response(ctx):
    """Y = +1: Z = X, c = 0 in every repetition, E_l = pairs inside each bucket."""
    d = synthgen.small_binary(200, 1500, seed=4)
    Y = np.ones(200, dtype=np.int8)
    for m, two in ((6, False), (6, True), (16, False)):
        res, rp, rr = run_both(ctx, d.XT, Y, m, 5, 0.05, seed=5, two_sided=two)
        assert_same_binary(res, rp, rr)
        assert (rr["cmask"] == 0).all()


def test_every_pair_passes_and_none_passes(ctx):
    d = synthgen.small_binary(100, 400, seed=6)
    res, rp, rr = run_both(ctx, d.XT, d.Y, 4, 3, -1.5, seed=7)     # s/n >= -1 > -1.5 always
    assert_same_binary(res, rp, rr)
    assert int(rr["passed"].sum()) == int(rr["candidates"].sum())
    res, rp, rr = run_both(ctx, d.XT, d.Y, 4, 3, 1.0, seed=7)      # s/n > 1 never
    assert_same_binary(res, rp, rr)
    assert len(rp) == 0


def test_more_sampled_rows_than_rows(ctx):
    d = synthgen.small_binary(5, 300, seed=8)
    res, rp, rr = run_both(ctx, d.XT, d.Y, 12, 6, 0.1, seed=9)
    assert_same_binary(res, rp, rr)


@pytest.mark.parametrize("p", [1, 2, 255, 257, 513])
def test_exact_search_ragged_blocks(ctx, p):
    d = synthgen.small_binary(97, p, seed=p)
    x = ctx.x_create(d.XT)
    got = ctx.bruteforce(x, d.Y, 0.05)
    want = oracle.brute(d.XT, d.Y, 0.05)
    assert np.array_equal(got["pairs"]["j"], want["j"]) and np.array_equal(got["pairs"]["k"], want["k"])
    assert np.array_equal(got["pairs"]["s"], want["s"])


def test_empty_inputs_rejected(ctx):
    with pytest.raises(xyz.XyzError):
        ctx.x_create(np.zeros((0, 10), dtype=np.int8))
    with pytest.raises(xyz.XyzError):
        ctx.x_create(np.zeros((10, 0), dtype=np.int8))


def test_bruteforce_rejects_bad_y_then_recovers(ctx):
    """An invalid response (0 in +-1 data, NaN in float data) is an error of the exact
    search, reported after its kernels ran; the next call on the same context is exact."""
    d = synthgen.small_binary(90, 70, seed=31, planted=[(2, 3)])
    x = ctx.x_create(d.XT)
    bad = d.Y.copy()
    bad[5] = 0
    with pytest.raises(xyz.XyzError):
        ctx.bruteforce(x, bad, 0.1)
    yf = d.Y.astype(np.float32)
    yf[3] = np.nan
    with pytest.raises(xyz.XyzError):
        ctx.bruteforce(x, yf, 0.1)
    got = ctx.bruteforce(x, d.Y, 0.1)
    want = oracle.brute(d.XT, d.Y, 0.1)
    assert len(want) > 0
    for f in ("j", "k", "s"):
        assert np.array_equal(got["pairs"][f], want[f]), f
