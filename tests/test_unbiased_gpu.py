"""GPU parity of the unbiased transform (Section 3.2, Proposition 4) against the
oracle: continuous X hashed with per-repetition random signs drawn with
probability (1 + X_ij / nu_i) / 2 from the documented counter-based stream,
rows drawn with probability proportional to |Y_i| nu_i^2.

Both sides take every sign decision in binary64 with the same operations, so
candidate counts, partner masks and bucket maxima per repetition are
bit-identical; pair values follow the real-data rule of the other parity tests.
"""
import numpy as np
import pytest

import oracle
import synthgen
import paper_1610_05108_amd as xyz

from test_parity_gpu import assert_same_real

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = xyz.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n,p,m,L,kappa,two,seed", [
    (300, 400, 6, 8, 0.2, False, 1),
    (513, 700, 9, 5, 0.25, True, 2),
    (200, 1500, 17, 6, 0.1, False, 3),        # m > 15: the sort path
])
def test_unbiased_real_y(ctx, n, p, m, L, kappa, two, seed):
    d = synthgen.small_continuous(n, p, seed=seed, planted=[(0, 1), (7, 40)], noise=0.8)
    x = ctx.x_create(d.XT)
    res = ctx.search(x, d.Y, m=m, L=L, kappa=kappa, seed=seed, two_sided=two, unbiased=True)
    rp, rr = oracle.search(d.XT, d.Y, m, L, kappa, seed=seed, two_sided=two, unbiased=True)
    assert_same_real(res, rp, rr, kappa, n)
    # the transform differs from the sign transform's hashing
    sign = ctx.search(x, d.Y, m=m, L=L, kappa=kappa, seed=seed, two_sided=two)
    assert not np.array_equal(sign["reps"]["candidates"], res["reps"]["candidates"])


def test_unbiased_binary_y_scaled_rows(ctx):
    """+-1 Y: rows drawn with probability proportional to nu_i^2; rows with very
    different maxima and one all-zero row (weight 0, never drawn)."""
    d = synthgen.small_continuous(350, 500, seed=20)
    XT = d.XT.copy()
    XT[:, ::3] *= 4.0
    XT[:, 11] = 0.0
    Y = np.where(np.random.default_rng(2).random(350) < 0.5, 1, -1).astype(np.int8)
    x = ctx.x_create(XT)
    res = ctx.search(x, Y, m=7, L=9, kappa=0.15, seed=4, unbiased=True)
    rp, rr = oracle.search(XT, Y, 7, 9, 0.15, seed=4, unbiased=True)
    assert_same_real(res, rp, rr, 0.15, 350)


def test_unbiased_rows_table_with_zero_row(ctx):
    """A row table may name an all-zero row (nu = 0): its signs are fair coins."""
    d = synthgen.small_continuous(120, 300, seed=21, planted=[(3, 5)])
    XT = d.XT.copy()
    XT[:, 9] = 0.0
    rows = synthgen.rows_table(120, 5, 6, seed=3)
    rows[:, 0] = 9
    x = ctx.x_create(XT)
    res = ctx.search(x, d.Y, m=6, L=5, kappa=0.1, rows=rows, unbiased=True)
    rp, rr = oracle.search(XT, d.Y, 6, 5, 0.1, rows=rows, unbiased=True)
    assert_same_real(res, rp, rr, 0.1, 120)


def test_unbiased_split_repetitions(ctx):
    d = synthgen.small_continuous(260, 600, seed=22, planted=[(2, 9)])
    x = ctx.x_create(d.XT)
    full = ctx.search(x, d.Y, m=8, L=9, kappa=0.2, seed=3, unbiased=True)
    a = ctx.search(x, d.Y, m=8, L=4, kappa=0.2, seed=3, unbiased=True)
    b = ctx.search(x, d.Y, m=8, L=5, kappa=0.2, seed=3, rep_offset=4, unbiased=True)
    assert np.array_equal(full["reps"]["candidates"],
                          np.concatenate([a["reps"]["candidates"], b["reps"]["candidates"]]))


def test_unbiased_needs_float_x(ctx):
    d = synthgen.small_binary(100, 50, seed=1)
    x = ctx.x_create(d.XT)
    with pytest.raises(xyz.XyzError):
        ctx.search(x, d.Y, m=4, L=2, kappa=0.1, unbiased=True)


@pytest.mark.parametrize("cap,two,m", [(1.0, False, 6), (0.37, True, 9), (3.0, False, 17)])
def test_capped_unbiased_matches_oracle(ctx, cap, two, m):
    """Capping before the unbiased transform (Section 3.2's remark): rows with
    outliers of +-6 on every fifth row; the cap (0.37 is not a float32 value,
    so both sides round it alike) reaches the row maxima, the row weights and
    the transform.  m = 17 takes the sort path."""
    d = synthgen.small_continuous(240, 700, seed=30, planted=[(0, 1), (7, 40)], noise=0.8)
    XT = d.XT.copy()
    XT[::5, ::5] = np.where(XT[::5, ::5] < 0, -6.0, 6.0)
    x = ctx.x_create(XT)
    res = ctx.search(x, d.Y, m=m, L=7, kappa=0.2, seed=5, two_sided=two, unbiased=True, cap=cap)
    rp, rr = oracle.search(XT, d.Y, m, 7, 0.2, seed=5, two_sided=two, unbiased=True, cap=cap)
    assert_same_real(res, rp, rr, 0.2, 240)
    plain = ctx.search(x, d.Y, m=m, L=7, kappa=0.2, seed=5, two_sided=two, unbiased=True)
    assert not np.array_equal(plain["reps"]["candidates"], res["reps"]["candidates"])


def test_cap_checks(ctx):
    d = synthgen.small_continuous(60, 50, seed=31)
    x = ctx.x_create(d.XT)
    for kw in ({"cap": 1.0}, {"cap": -1.0, "unbiased": True}, {"cap": float("nan"), "unbiased": True},
               {"cap": 1e-60, "unbiased": True}):
        with pytest.raises(xyz.XyzError):
            ctx.search(x, d.Y, m=4, L=2, kappa=0.1, **kw)
    # a cap above every entry changes nothing
    big = float(np.abs(d.XT).max())
    a = ctx.search(x, d.Y, m=5, L=4, kappa=0.1, seed=2, unbiased=True, cap=big)
    b = ctx.search(x, d.Y, m=5, L=4, kappa=0.1, seed=2, unbiased=True)
    assert np.array_equal(a["reps"]["candidates"], b["reps"]["candidates"])
    assert np.array_equal(a["pairs"], b["pairs"])
