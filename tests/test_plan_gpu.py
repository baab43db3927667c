"""GPU checks of the parameter-choice path (sampled strengths, planner)."""
import numpy as np
import pytest

import oracle
from oracle import theory
import synthgen
import paper_1610_05108_amd as xyz

pytestmark = pytest.mark.gpu
M64 = 2 ** 64


@pytest.fixture(scope="module")
def ctx():
    c = xyz.Context(0)
    yield c
    c.close()


def _pairs(seed, p, count):
    """The pair draws of the strength sampler, recomputed from SplitMix64's definition."""
    out = []
    for q in range(count):
        u = oracle.splitmix64(seed, 2 * q + 1)
        v = oracle.splitmix64(seed, 2 * q + 2)
        j = (u * p) >> 64
        k = (v * (p - 1)) >> 64
        k += 1 if k >= j else 0
        out.append((j, k))
    return out


def test_sampled_strengths_binary(ctx):
    d = synthgen.small_binary(333, 500, seed=3, planted=[(1, 2)], flip=0.1)
    x = ctx.x_create(d.XT)
    g = ctx.sample_strengths(x, d.Y, 400, seed=17)
    for (j, k), gv in zip(_pairs(17, 500, 400), g):
        assert j != k
        s = oracle.pair_value(d.XT, d.Y, j, k)
        assert abs(gv - theory.gamma_from_stat(s / 333)) < 1e-14


def test_sampled_strengths_real_y(ctx):
    d = synthgen.small_continuous(250, 300, seed=4, planted=[(0, 5)])
    x = ctx.x_create(d.XT)
    g = ctx.sample_strengths(x, d.Y, 300, seed=5)
    Xs = np.where(d.XT < 0, -1, 1)
    for (j, k), gv in zip(_pairs(5, 300, 300), g):
        assert abs(gv - theory.gamma_tilde(Xs, d.Y, j, k)) < 1e-12


def test_sampled_strengths_predict_candidates(ctx):
    """sum of gamma^m over all pairs is E|E_l| (proof of Theorem 2): the sampled
    estimate must match the mean candidate count of real repetitions."""
    XT, _ = synthgen.genotype(800, 4000, seed=6)
    Y = np.where(np.random.default_rng(0).random(800) < 0.45, 1, -1).astype(np.int8)
    x = ctx.x_create(XT)
    g = ctx.sample_strengths(x, Y, 1 << 16, seed=1)
    P = 4000 * 3999 / 2
    for m in (6, 9):
        pred = P * np.mean(g ** m)
        r = ctx.search(x, Y, m=m, L=400, kappa=1.0, seed=2)
        got = r["reps"]["candidates"].mean()
        assert abs(got - pred) / pred < 0.1, (m, got, pred)


def test_plan_strong_pair_uses_xyz_and_finds_it(ctx):
    # large p: the exact search grows as p^2, xyz about as p for a strong pair
    XT = synthgen.rademacher(1000, 200_000, seed=7)
    r = np.random.default_rng(1)
    Y = (XT[10].astype(np.int16) * XT[120_000]).astype(np.int8)
    flip = r.random(1000) < 0.05          # strength about 0.95
    Y[flip] = -Y[flip]
    x = ctx.x_create(XT)
    plan = ctx.plan(x, Y, kappa=0.5, gamma_target=0.9, eta_target=0.99)
    assert plan["method"] == xyz.XYZ_PLAN_XYZ, plan
    assert plan["predicted_recall"] >= 0.99 and plan["predicted_ms"] < plan["brute_ms"]
    assert plan["L"] == theory.L_for(0.99, 0.9 ** plan["m"])
    res = ctx.search(x, Y, m=plan["m"], L=plan["L"], kappa=0.5, seed=3)
    assert (10, 120_000) in set(zip(res["pairs"]["j"].tolist(), res["pairs"]["k"].tolist()))


def test_plan_weak_target_prefers_brute_force(ctx):
    XT, _ = synthgen.genotype(2000, 30000, seed=8)
    Y = np.where(np.random.default_rng(2).random(2000) < 0.45, 1, -1).astype(np.int8)
    x = ctx.x_create(XT)
    plan = ctx.plan(x, Y, kappa=0.1, gamma_target=0.56, eta_target=0.95)
    assert plan["method"] == xyz.XYZ_PLAN_BRUTE, plan
    assert plan["mstar"] >= 1
