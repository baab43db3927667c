"""Pins of the dense-projection oracle (Algorithm 1, Section 2.1 class (a);
Section 5.1) to facts other than its own code:

* with tau = 0 and a subsampling projection (eq. (projR): weights D_m on the
  rows i_1..i_M), Algorithm 1 reduces to minimal subsampling, so its
  candidates and reported pairs equal those of the Algorithm 2 oracle on the
  same rows (the remark after the definition of the minimal class in
  Section 2.1: the close pairs are the pairs equal on the subsampled rows);
* with tau larger than any projected distance every pair is a candidate and
  the reported set is the exact search of eq. (1) (the brute-force oracle);
* with Gaussian R the rate at which a pair of known strength lands in E_l
  matches the Section 5.1 closed form eta_gauss (the projected distance of
  +-1 data is exactly normal), checked by simulation;
* eta_gauss puts a pair of strength 1/2 into E_1 with probability 1/p, the
  budget that defines tau in Section 5.1.
"""
import math

import numpy as np
import pytest

import oracle
import synthgen
from oracle import theory
from oracle.dense import dense_search


def test_eta_gauss_budget_and_order():
    for p in (10, 100, 10_000, 1_000_000):
        assert theory.eta_gauss(0.5, p) * p == pytest.approx(1.0, rel=1e-9)
        e = [theory.eta_gauss(g, p) for g in (0.55, 0.7, 0.8, 0.9, 0.99)]
        assert all(a < b for a, b in zip(e, e[1:]))
        # minimal subsampling at the same budget: eq. (9) with M = ceil(log2 p)
        assert theory.M_minimal(p) == math.ceil(math.log2(p) - 1e-9)
        assert theory.eta_minimal(0.5, p) * p <= 1.0 + 1e-12
    # Section 5.1: at p = 10^6 minimal subsampling is orders of magnitude more powerful
    r = theory.eta_minimal(0.9, 10**6) / theory.eta_gauss(0.9, 10**6)
    assert 1e4 < r < 1e5


def test_tau_gauss_is_the_budget_quantile():
    """P(|W| <= tau) = 1/p for W ~ N(0, 2n sd^2), by the normal CDF (scipy.stats)."""
    from scipy.stats import norm
    for p, n, sd in ((50, 400, 1.0), (1000, 1000, 65536.0), (10**5, 2000, 3.0)):
        tau = theory.tau_gauss(p, n, sd)
        sigma = math.sqrt(2.0 * n) * sd
        assert 2.0 * norm.cdf(tau / sigma) - 1.0 == pytest.approx(1.0 / p, rel=1e-7)


def test_tau0_subsampling_equals_algorithm2():
    d = synthgen.small_binary(220, 300, seed=5, planted=[(3, 17), (40, 41)], flip=0.1)
    L, M = 6, 8
    R, rows, _ = synthgen.subsample_projections(d.n, L, M, seed=9, bits=40)
    pd, rd = dense_search(d.XT, d.Y, R, 0, 0.1)
    pa, ra = oracle.search(d.XT, d.Y, M, L, 0.1, rows=rows)
    assert len(pa) > 0 and ra["candidates"].sum() > 0
    for f in ("j", "k", "s", "first_rep", "hits"):
        assert np.array_equal(pd[f], pa[f]), f
    for f in ("candidates", "passed", "fresh"):
        assert np.array_equal(rd[f], ra[f]), f


def test_huge_tau_is_the_exact_search():
    d = synthgen.small_binary(150, 90, seed=6, planted=[(1, 2)])
    R, _ = synthgen.gaussian_projections(d.n, 3, seed=1)
    pd, rd = dense_search(d.XT, d.Y, R, 1 << 40, 0.05, rep_offset=4)
    pb = oracle.brute(d.XT, d.Y, 0.05)
    for f in ("j", "k", "s"):
        assert np.array_equal(pd[f], pb[f]), f
    assert (rd["candidates"] == 90 * 89 // 2).all()
    assert (rd["max_bucket"] == 90).all()
    assert (pd["first_rep"] == 4).all() and (pd["hits"] == 3).all()
    assert rd["fresh"].tolist() == [len(pb), 0, 0]


def test_gaussian_rate_matches_eta_gauss():
    """One pair of strength gamma = 0.8 (n = 400: 80 disagreeing rows, half of
    them with Y = -1, so that the two orientations (j, k) and (k, j) project to
    uncorrelated normals); tau for a budget of p = 50.  A repetition holds the
    pair when either orientation is close: probability 1 - (1 - eta)^2."""
    n, gamma, budget, L = 400, 0.8, 50, 12_000
    rng = np.random.default_rng(3)
    xj = np.where(rng.random(n) < 0.5, 1, -1)
    y = np.where(rng.random(n) < 0.5, 1, -1)
    dis = np.zeros(n, dtype=bool)
    # 40 disagreeing rows with Y = +1 and 40 with Y = -1
    dis[rng.permutation(np.flatnonzero(y == 1))[:40]] = True
    dis[rng.permutation(np.flatnonzero(y == -1))[:40]] = True
    xk = np.where(dis, -y * xj, y * xj)          # agree: X_j = Y X_k
    XT = np.stack([xj, xk]).astype(np.int8)
    Y = y.astype(np.int8)
    assert int((XT[0] == Y * XT[1]).sum()) == int(gamma * n)
    R, sd = synthgen.gaussian_projections(n, L, seed=11, frac_bits=16)
    tau = int(round(theory.tau_gauss(budget, n, sd)))
    pairs, reps = dense_search(XT, Y, R, tau, 0.5)
    hits = int(pairs["hits"][0]) if len(pairs) else 0
    assert hits == int(reps["candidates"].sum())
    eta = theory.eta_gauss(gamma, budget)
    q = 1.0 - (1.0 - eta) ** 2
    mu, sdev = L * q, math.sqrt(L * q * (1.0 - q))
    assert abs(hits - mu) < 4.5 * sdev, (hits, mu, sdev)


def test_gaussian_budget_is_p_candidates():
    """Section 5.1's budget: with tau = tau_gauss(p, n) and random +-1 data (strengths
    near 1/2), a repetition holds about p candidate pairs (each orientation about 1/p
    per ordered pair; p(p-1) ordered pairs, overlaps of order 1)."""
    p, n, L = 300, 200, 40
    XT = synthgen.rademacher(n, p, seed=31)
    Y = np.where(np.random.default_rng(32).random(n) < 0.5, 1, -1).astype(np.int8)
    R, sd = synthgen.gaussian_projections(n, L, seed=33, frac_bits=16)
    tau = int(round(theory.tau_gauss(p, n, sd)))
    _, reps = dense_search(XT, Y, R, tau, 2.0)
    mean = float(reps["candidates"].mean())
    assert abs(mean - p) < 0.08 * p, mean
