"""GPU parity for keys of more than 15 bits (m > 15).

Such keys are bucketed by sorting (repetition, key) pairs instead of counting
them in LDS; the results must be bit-identical to the oracle exactly as on the
LDS path: pair sets, pair statistics and per-repetition statistics.
"""
import numpy as np
import pytest

import oracle
import synthgen
import paper_1610_05108_amd as xyz

from test_parity_gpu import assert_same_binary, assert_same_real, run_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = xyz.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n,p,m,L,kappa,two,seed", [
    (300, 3000, 16, 20, 0.15, False, 1),
    (257, 2500, 18, 12, 0.12, True, 2),
    (200, 4100, 20, 10, 0.1, False, 3),
    (180, 1500, 24, 6, 0.05, False, 4),
    (150, 900, 30, 5, 0.0, True, 5),
])
def test_random_binary_large_m(ctx, n, p, m, L, kappa, two, seed):
    d = synthgen.small_binary(n, p, seed=seed, planted=[(1, 7)], flip=0.03)
    res, rp, rr = run_both(ctx, d.XT, d.Y, m, L, kappa, seed=seed, two_sided=two)
    assert_same_binary(res, rp, rr)
    assert len(rp) > 0


def test_genotype_heavy_buckets_large_m(ctx):
    """Low-frequency genotype columns share keys even with 17 sampled rows, so
    some bucket products are large (matrix-core and multi-tile products)."""
    XT, _ = synthgen.genotype(700, 6000, seed=21)
    r = np.random.default_rng(4)
    Y = np.where(r.random(700) < 0.45, 1, -1).astype(np.int8)
    res, rp, rr = run_both(ctx, XT, Y, 17, 6, 0.12, seed=6)
    assert_same_binary(res, rp, rr)
    assert res["reps"]["max_bucket"].max() > 64


def test_rows_table_large_m(ctx):
    d = synthgen.small_binary(220, 1800, seed=22, planted=[(3, 9)], flip=0.05)
    rows = synthgen.rows_table(220, 7, 19, seed=8)
    res, rp, rr = run_both(ctx, d.XT, d.Y, 19, 7, 0.15, rows=rows)
    assert_same_binary(res, rp, rr)


def test_batch_large_m(ctx):
    XT = synthgen.rademacher(300, 2200, seed=23)
    r = np.random.default_rng(5)
    Ys = [np.where(r.random(300) < 0.5, 1, -1).astype(np.int8) for _ in range(3)]
    x = ctx.x_create(XT)
    params = [dict(m=17, L=8, kappa=0.1 + 0.02 * q, seed=4) for q in range(3)]
    params[2]["two_sided"] = True
    batch = ctx.search_batch(x, Ys, params)
    for q in range(3):
        kw = params[q]
        single = ctx.search(x, Ys[q], **kw)
        assert np.array_equal(batch[q]["pairs"], single["pairs"]), q
        assert np.array_equal(batch[q]["reps"], single["reps"]), q
        rp, rr = oracle.search(XT, Ys[q], kw["m"], kw["L"], kw["kappa"], seed=kw["seed"],
                               two_sided=kw.get("two_sided", False))
        assert_same_binary(batch[q], rp, rr)


def test_split_repetitions_large_m(ctx):
    d = synthgen.small_binary(260, 2000, seed=24, planted=[(4, 5)], flip=0.02)
    x = ctx.x_create(d.XT)
    full = ctx.search(x, d.Y, m=18, L=9, kappa=0.1, seed=3)
    a = ctx.search(x, d.Y, m=18, L=4, kappa=0.1, seed=3, rep_offset=0)
    b = ctx.search(x, d.Y, m=18, L=5, kappa=0.1, seed=3, rep_offset=4)
    for f in ("candidates", "passed", "cmask", "max_bucket"):
        assert np.array_equal(full["reps"][f], np.concatenate([a["reps"][f], b["reps"][f]]))


def test_continuous_large_m(ctx):
    d = synthgen.small_continuous(240, 1600, seed=25, planted=[(2, 11)])
    x = ctx.x_create(d.XT)
    res = ctx.search(x, d.Y, m=16, L=10, kappa=0.3, seed=7)
    rp, rr = oracle.search(d.XT, d.Y, 16, 10, 0.3, seed=7)
    assert_same_real(res, rp, rr, 0.3, 240)
