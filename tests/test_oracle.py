"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine, an exhaustive enumeration, a closed form of the paper, a value the
paper prints, or a published reference output.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import theory
import synthgen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _pairset(arr):
    return {(int(a), int(b)) for a, b in zip(arr["j"], arr["k"])}


# ----------------------------------------------------------------- sampler --

def test_splitmix64_published_outputs():
    g = _gold("splitmix64_reference.json")
    got = [oracle.splitmix64(g["seed"], k) for k in range(1, 6)]
    assert got == [int(v) for v in g["outputs"]]


def test_uniform_rows_chi2():
    n, m = 13, 8
    counts = np.zeros(n)
    for l in range(3000):
        r = oracle.draw_rows(n, 7, l, m)
        assert r.min() >= 0 and r.max() < n
        np.add.at(counts, r, 1)
    exp = counts.sum() / n
    chi2 = ((counts - exp) ** 2 / exp).sum()
    # 12 degrees of freedom: P(chi2 > 40) < 1e-4
    assert chi2 < 40.0


def test_weighted_rows_follow_abs_y():
    Y = np.array([0.0, 3.0, -1.0, 0.0, 0.5, -2.5, 1.0, 0.0], dtype=np.float64)
    n = len(Y)
    counts = np.zeros(n)
    for l in range(4000):
        np.add.at(counts, oracle.draw_rows(n, 3, l, 5, Y=Y), 1)
    assert counts[Y == 0].sum() == 0, "rows with Y_i = 0 have weight 0 (Section 3.1)"
    w = np.abs(Y) / np.abs(Y).sum()
    nz = w > 0
    exp = counts.sum() * w[nz]
    chi2 = ((counts[nz] - exp) ** 2 / exp).sum()
    assert chi2 < 30.0   # 4 degrees of freedom


def test_weighted_rows_reject_all_zero():
    with pytest.raises(oracle.OracleError):
        oracle.draw_rows(4, 0, 0, 3, Y=np.zeros(4))


# ---------------------------------------------------------- inner products --

def test_inner_products_match_numpy_gemm_and_distance_identity():
    d = synthgen.small_binary(37, 23, seed=5)
    X = d.XT.T.astype(np.int64)                # n x p
    Y = d.Y.astype(np.int64)
    G = X.T @ (Y[:, None] * X)                 # library GEMM: Y^T (X_j o X_k)
    allp = oracle.brute(d.XT, d.Y, kappa=-2.0)  # every pair passes
    assert len(allp) == 23 * 22 // 2
    for rec in allp:
        assert rec["s"] == G[rec["j"], rec["k"]]
        assert rec["stat"] == rec["s"] / 37
    # eq. (4): 2 gamma - 1 = s/n = Z_j^T X_k / n = 1 - ||Z_j - X_k||^2 / (2n)
    Z = Y[:, None] * X
    for rec in allp[:50]:
        j, k = int(rec["j"]), int(rec["k"])
        dist2 = int(((Z[:, j] - X[:, k]) ** 2).sum())
        assert Fraction(int(rec["s"]), 37) == 1 - Fraction(dist2, 2 * 37)
        gamma = Fraction(int((Y == X[:, j] * X[:, k]).sum()), 37)
        assert 2 * gamma - 1 == Fraction(int(rec["s"]), 37)


@pytest.mark.parametrize("kappa", [0.0, 0.11, 0.21, 0.31, -0.16])
def test_threshold_equals_distance_form(kappa):
    """eqs. (1)/(2): s/n > kappa  <=>  ||X_j - Z_k||_2 < kappa' with kappa'^2 = 2n(1-kappa).

    kappa is kept off the grid of attainable s/n values (multiples of 1/20
    here) so that exact rational comparison and the binary64 division agree."""
    d = synthgen.small_binary(40, 30, seed=11)
    X = d.XT.T.astype(np.int64)
    Z = d.Y.astype(np.int64)[:, None] * X
    kq = Fraction(kappa)
    want = set()
    for j in range(30):
        for k in range(j + 1, 30):
            dist2 = int(((X[:, j] - Z[:, k]) ** 2).sum())
            if dist2 < 2 * 40 * (1 - kq):
                want.add((j, k))
    assert _pairset(oracle.brute(d.XT, d.Y, kappa)) == want


def test_ties_at_threshold_are_excluded():
    """eq. (1) keeps s/n strictly above kappa; s/n is the binary64 quotient."""
    d = synthgen.small_binary(40, 30, seed=11)
    allp = oracle.brute(d.XT, d.Y, -2.0)
    for kappa in (0.1, 0.2, 0.3):
        kept = _pairset(oracle.brute(d.XT, d.Y, kappa))
        tied = {(int(r["j"]), int(r["k"])) for r in allp if int(r["s"]) / 40 == kappa}
        above = {(int(r["j"]), int(r["k"])) for r in allp if int(r["s"]) / 40 > kappa}
        assert tied and not (tied & kept)
        assert kept == above


def test_continuous_value_matches_numpy_dot():
    d = synthgen.small_continuous(50, 12, seed=3, planted=[(1, 4)])
    X = d.XT.astype(np.float64)
    Y = d.Y.astype(np.float64)
    for j, k in [(0, 1), (1, 4), (5, 11), (3, 3)]:
        v = oracle.pair_value(d.XT, d.Y, j, k)
        ref = float(np.dot(Y * X[j], X[k]))
        assert abs(v - ref) <= 1e-12 * (1 + np.abs(Y * X[j] * X[k]).sum())


# ------------------------------------------------------------- equal pairs --

def _direct_E(Xs, Zs, rows, two_sided):
    """E_l by direct O(p^2 m) enumeration: ordered (j, k), j != k, with
    X_j and Z_k equal on every sampled row; returned as unordered pairs."""
    p = Xs.shape[1]
    xs = Xs[rows]          # m x p
    zs = Zs[rows]
    out = set()
    for j in range(p):
        for k in range(p):
            if j == k:
                continue
            if np.all(xs[:, j] == zs[:, k]) or (two_sided and np.all(xs[:, j] == -zs[:, k])):
                out.add((min(j, k), max(j, k)))
    return out


@pytest.mark.parametrize("two_sided", [False, True])
@pytest.mark.parametrize("m", [1, 2, 4])
def test_equal_pairs_match_direct_enumeration(m, two_sided):
    d = synthgen.small_binary(24, 35, seed=m + 10 * two_sided)
    X = d.XT.T.astype(np.int64)
    Z = d.Y.astype(np.int64)[:, None] * X
    L = 6
    rows = synthgen.rows_table(24, L, m, seed=99 + m)
    for l in range(L):
        pairs, reps = oracle.search(d.XT, d.Y, m, 1, -2.0, rows=rows[l:l + 1], two_sided=two_sided)
        want = _direct_E(X, Z, rows[l], two_sided)
        assert _pairset(pairs) == want
        assert reps["candidates"][0] == len(want)
        assert reps["passed"][0] == len(want)
        cm = sum(1 << t for t in range(m) if d.Y[rows[l][t]] < 0)
        assert int(reps["cmask"][0]) == cm


def test_sampler_rows_are_used():
    """Without a rows table the oracle uses its own sampler: same E_l as
    passing the sampler's rows explicitly."""
    d = synthgen.small_binary(30, 25, seed=2)
    a, ra = oracle.search(d.XT, d.Y, 3, 5, -2.0, seed=42)
    rows = np.stack([oracle.draw_rows(30, 42, l, 3) for l in range(5)])
    b, rb = oracle.search(d.XT, d.Y, 3, 5, -2.0, rows=rows)
    assert np.array_equal(a, b) and np.array_equal(ra, rb)


def test_m0_reduces_to_brute_force():
    """With no sampled rows every pair collides, so xyz returns T(kappa) exactly."""
    d = synthgen.small_binary(60, 40, seed=4, planted=[(2, 9)], flip=0.2)
    for kappa in (0.1, 0.25):
        pairs, reps = oracle.search(d.XT, d.Y, 0, 3, kappa)
        br = oracle.brute(d.XT, d.Y, kappa)
        assert _pairset(pairs) == _pairset(br)
        assert np.array_equal(pairs["s"], br["s"])
        assert np.all(pairs["hits"] == 3) and np.all(pairs["first_rep"] == 0)
        assert np.all(reps["candidates"] == 40 * 39 // 2)


def test_perfect_pair_found_in_every_repetition():
    """Y = X_a o X_b gives X_a = Z_b exactly, so every projection collides (Section 2.1)."""
    d = synthgen.small_binary(80, 30, seed=6)
    Y = (d.XT[4].astype(np.int16) * d.XT[17].astype(np.int16)).astype(np.int8)
    pairs, reps = oracle.search(d.XT, Y, 10, 25, 0.5, seed=1)
    rec = pairs[(pairs["j"] == 4) & (pairs["k"] == 17)]
    assert len(rec) == 1 and rec["hits"][0] == 25 and rec["s"][0] == 80 and rec["first_rep"][0] == 0


def test_anti_perfect_pair_only_two_sided():
    d = synthgen.small_binary(80, 30, seed=8)
    Y = (-d.XT[3].astype(np.int16) * d.XT[20].astype(np.int16)).astype(np.int8)
    one, _ = oracle.search(d.XT, Y, 8, 30, -2.0, seed=5)
    assert (3, 20) not in _pairset(one)
    two, _ = oracle.search(d.XT, Y, 8, 30, 0.5, seed=5, two_sided=True)
    rec = two[(two["j"] == 3) & (two["k"] == 20)]
    assert len(rec) == 1 and rec["hits"][0] == 30 and rec["s"][0] == -80


def test_collision_probability_is_gamma_pow_m():
    """Section 2.3: a pair of strength gamma is in E_1 with probability gamma^M."""
    n, p, m, L = 40, 7, 3, 6000
    d = synthgen.small_binary(n, p, seed=12, planted=[(0, 1), (2, 5)], flip=0.1)
    pairs, reps = oracle.search(d.XT, d.Y, m, L, -2.0, seed=77)
    X = d.XT.astype(np.int64)
    got = {(int(r["j"]), int(r["k"])): int(r["hits"]) for r in pairs}
    gammas = []
    for j in range(p):
        for k in range(j + 1, p):
            g = float(np.mean(d.Y == X[j] * X[k]))
            gammas.append(g)
            pr = g ** m
            h = got.get((j, k), 0)
            z = (h - L * pr) / math.sqrt(L * pr * (1 - pr)) if 0 < pr < 1 else 0.0
            assert abs(z) < 5.0, (j, k, g, h / L, pr)
    # proof of Theorem 2: E|E_1| = sum_jk gamma_jk^M
    exp = theory.expected_candidates(np.array(gammas), m)
    c = reps["candidates"].astype(np.float64)
    z = (c.mean() - exp) / (c.std(ddof=1) / math.sqrt(L))
    assert abs(z) < 5.0


def test_weighted_collision_probability_is_gamma_tilde_pow_m():
    """Section 3.1: with |Y|-weighted rows the collision probability is gamma~^M."""
    n, p, m, L = 30, 6, 2, 6000
    d = synthgen.small_continuous(n, p, seed=13, planted=[(1, 3)], noise=0.7)
    pairs, _ = oracle.search(d.XT, d.Y, m, L, -1e300, seed=9)
    Xs = np.where(d.XT < 0, -1, 1)
    got = {(int(r["j"]), int(r["k"])): int(r["hits"]) for r in pairs}
    for j in range(p):
        for k in range(j + 1, p):
            g = theory.gamma_tilde(Xs, d.Y, j, k)
            pr = g ** m
            h = got.get((j, k), 0)
            z = (h - L * pr) / math.sqrt(L * pr * (1 - pr)) if 0 < pr < 1 else 0.0
            assert abs(z) < 5.0, (j, k, g, h / L, pr)


def test_paper_worked_example_miss_rate():
    """Section 5.3: strength 0.85, M = 21, L = 100 -> missed with probability about 0.03."""
    g = _gold("paper_numbers.json")["worked_example_miss"]
    gamma, M, L = g["gamma"], g["M"], g["L"]
    exact = 1.0 - theory.eta(gamma, M, L)
    assert abs(exact - g["printed"]) < 0.01       # printed as "approximately 0.03"
    n = 200
    agree = int(round(gamma * n))      # exactly 85% of the rows agree
    d = synthgen.small_binary(n, 4, seed=21)
    X = d.XT
    Y = (X[0].astype(np.int16) * X[1].astype(np.int16)).astype(np.int8)
    Y[agree:] = -Y[agree:]
    assert np.mean(Y == X[0] * X[1]) == gamma
    runs, missed = 1500, 0
    for seed in range(runs):
        pairs, _ = oracle.search(X, Y, M, L, 0.5, seed=seed)
        if (0, 1) not in _pairset(pairs):
            missed += 1
    sd = math.sqrt(exact * (1 - exact) / runs)
    assert abs(missed / runs - exact) < 5 * sd


def test_split_repetitions_union_equals_full_run():
    d = synthgen.small_binary(50, 40, seed=14, planted=[(1, 2), (5, 30)], flip=0.15)
    full, rf = oracle.search(d.XT, d.Y, 4, 12, 0.2, seed=3)
    a, ra = oracle.search(d.XT, d.Y, 4, 5, 0.2, seed=3, rep_offset=0)
    b, rb = oracle.search(d.XT, d.Y, 4, 7, 0.2, seed=3, rep_offset=5)
    assert np.array_equal(rf["candidates"], np.concatenate([ra["candidates"], rb["candidates"]]))
    merged = {}
    for arr in (a, b):
        for r in arr:
            key = (int(r["j"]), int(r["k"]))
            h, f = merged.get(key, (0, 10 ** 9))
            merged[key] = (h + int(r["hits"]), min(f, int(r["first_rep"])))
    assert merged == {(int(r["j"]), int(r["k"])): (int(r["hits"]), int(r["first_rep"])) for r in full}


def test_sign_transform_maps_zero_to_plus_one():
    d = synthgen.small_continuous(30, 10, seed=15, planted=[(0, 2)])
    XT = d.XT.copy()
    XT[:, ::4] = 0.0
    XT[1, 1] = -0.0
    a, _ = oracle.search(XT, d.Y, 3, 8, -1e300, seed=2)
    XT2 = XT.copy()
    XT2[XT2 == 0] = 1e-30     # same signs, same hashing
    b, _ = oracle.search(XT2, d.Y, 3, 8, -1e300, seed=2)
    assert _pairset(a) == _pairset(b)
    assert np.array_equal(a["hits"], b["hits"])


def test_invalid_inputs_rejected():
    d = synthgen.small_binary(10, 5, seed=0)
    Y = d.Y.copy()
    Y[3] = 0
    with pytest.raises(oracle.OracleError):
        oracle.search(d.XT, Y, 2, 2, 0.1)
    with pytest.raises(oracle.OracleError):
        oracle.search(d.XT, d.Y, 2, 2, float("nan"))
    Xf = d.XT.astype(np.float32)
    Xf[0, 0] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.search(Xf, d.Y.astype(np.float32), 2, 2, 0.1)


# ------------------------------------------------------------ closed forms --

def test_printed_exponents_and_break_even():
    g = _gold("paper_numbers.json")
    for gamma, g0, printed in g["exponents"]["cases"]:
        # printed as "around" two digits (1.1762 appears as 1.17): within 0.01
        assert abs(theory.exponent(gamma, g0) - printed) < 0.01
    mm = g["matrix_multiplication_break_even"]
    gam = mm["gamma0"] ** (mm["exponent"] - 1.0)   # solves 1 + log(g)/log(g0) = exponent
    assert abs(theory.exponent(gam, mm["gamma0"]) - mm["exponent"]) < 1e-12
    assert abs(gam - mm["printed_gamma"]) <= 0.01


def test_printed_naive_miss():
    g = _gold("paper_numbers.json")["naive_miss"]
    # printed as "about 0.999" for the value 0.99971
    assert abs(theory.naive_miss(g["p"], g["L"]) - g["printed"]) < 10 ** -g["printed_digits"]


def test_sigma2_table_is_the_unweighted_strength():
    """Section 3.1's table equals 1/2 (1 + P(|eps| < 1)) to the printed digits
    (the unweighted agreement probability; see the readings of the paper)."""
    g = _gold("paper_numbers.json")["sigma2_table"]
    for s2, printed in zip(g["sigma2"], g["gamma"]):
        assert abs(theory.gamma_example_unweighted(s2) - printed) <= 0.011


def test_L_for_is_minimal():
    for eta_t in (0.5, 0.9, 0.95, 0.99):
        for beta in (0.5, 0.1, 0.01, 1e-4):
            L = theory.L_for(eta_t, beta)
            assert 1 - (1 - beta) ** L >= eta_t - 1e-12
            assert L == 1 or 1 - (1 - beta) ** (L - 1) < eta_t


def test_M_star_is_pareto_optimal():
    """Proposition 2: no (M', L') with at least M*'s power costs less."""
    r = np.random.default_rng(0)
    n, p = 1000, 20000
    sample = np.clip(r.normal(0.5, 0.02, size=20000), 0, 1)
    total = p * (p - 1) / 2
    for gamma in (0.6, 0.7, 0.85):
        Ms = theory.M_star(gamma, n, p, sample, total)
        for L in (1, 5, 30):
            e_star = theory.eta(gamma, Ms, L)
            c_star = theory.cost(Ms, L, n, p, theory.sum_gamma_pow(sample, total, Ms))
            for M2 in range(1, 40):
                L2 = theory.L_for(e_star, gamma ** M2) if gamma ** M2 < 1 else 1
                if theory.eta(gamma, M2, L2) < e_star - 1e-12:
                    L2 += 1
                c2 = theory.cost(M2, L2, n, p, theory.sum_gamma_pow(sample, total, M2))
                assert c2 >= c_star * (1 - 1e-9) or M2 == Ms


# ------------------------------------------------- unbiased transform (Section 3.2)

@pytest.mark.parametrize("m", [1, 2])
def test_unbiased_transform_collision_rate_is_proposition_4(m):
    """Two continuous columns plus one column that only sets the row maxima: the
    oracle's collision frequency of the pair over many repetitions equals
    Proposition 4's strength (with row scaling) to the power m.  A transform
    drawn as (1 - x)/2 or row weights without nu_i^2 move the rate by more than
    ten times the tolerance."""
    r = np.random.default_rng(11)
    n = 40
    XT = r.uniform(-1, 1, size=(3, n)).astype(np.float32)
    XT[2] *= 2.5                                     # the row maxima come from column 2 on most rows
    XT[1] = (0.8 * XT[0] + 0.2 * r.uniform(-1, 1, size=n)).astype(np.float32)
    Y = (XT[0].astype(np.float64) * XT[1] + 0.1 * r.standard_normal(n)).astype(np.float32)
    L = 40_000
    _, reps = oracle.search(XT, Y, m, L, 10.0, seed=5, unbiased=True)
    # unordered candidates: (0,1) collides with prob g01^m, (0,2), (1,2) with theirs
    want = sum(theory.gamma_unbiased(XT, Y, a, b) ** m for a, b in ((0, 1), (0, 2), (1, 2)))
    got = float(reps["candidates"].mean())
    se = math.sqrt(3 * 0.25 / L)
    assert abs(got - want) < 5 * se, (got, want)
    # the scaled strength differs clearly from the unscaled one on this data
    assert abs(theory.gamma_unbiased(XT, Y, 0, 1) - theory.gamma_unbiased(XT, Y, 0, 1, scale=False)) > 0.05


@pytest.mark.parametrize("m", [1, 2])
def test_capped_unbiased_collision_rate_is_proposition_4_of_capped_x(m):
    """Capping before the unbiased transform (Section 3.2): the pair's collision
    frequency equals Proposition 4's strength of the capped matrix to the power
    m.  Capping that reached only the transform, only the row maxima or only
    the row weights, or no capping at all, moves the rate by more than ten times
    the tolerance on this data (column 2 holds outliers of +-8 on eight rows,
    capped at 1)."""
    r = np.random.default_rng(21)
    n = 40
    XT = r.uniform(-1, 1, size=(3, n)).astype(np.float32)
    XT[2, :8] = np.where(r.random(8) < 0.5, -8.0, 8.0)    # outliers set the maxima of rows 0..7
    XT[1] = (0.8 * XT[0] + 0.2 * r.uniform(-1, 1, size=n)).astype(np.float32)
    Y = (XT[0].astype(np.float64) * XT[1] + 0.1 * r.standard_normal(n)).astype(np.float32)
    L = 40_000
    cap = 1.0
    _, reps = oracle.search(XT, Y, m, L, 10.0, seed=6, unbiased=True, cap=cap)
    pairs = ((0, 1), (0, 2), (1, 2))
    want = sum(theory.gamma_unbiased(XT, Y, a, b, cap=cap) ** m for a, b in pairs)
    got = float(reps["candidates"].mean())
    se = math.sqrt(3 * 0.25 / L)
    assert abs(got - want) < 5 * se, (got, want)
    uncapped = sum(theory.gamma_unbiased(XT, Y, a, b) ** m for a, b in pairs)
    assert abs(uncapped - want) > 10 * se, (uncapped, want)
    # capping that reaches only the transform or only the row weights: the per-row collision
    # probability 1/2 + sgn(Y_i) x_a x_b / (2 nu_i^2) under row weights |Y_i| nu_i^2
    Xr = XT.astype(np.float64)
    Xc = np.clip(Xr, -cap, cap)
    nu_raw, nu_cap = np.abs(Xr).max(axis=0), np.abs(Xc).max(axis=0)

    def rate(X, nu_draw, nu_scale):
        w = np.abs(Y) * nu_draw ** 2
        w = w / w.sum()
        return sum(float(np.sum(w * (0.5 + np.sign(Y) * X[a] * X[b] / (2 * nu_scale ** 2)))) ** m
                   for a, b in pairs)

    assert abs(rate(Xc, nu_cap, nu_cap) - want) < 1e-9
    for wrong in (rate(Xr, nu_raw, nu_raw), rate(Xc, nu_raw, nu_cap), rate(Xc, nu_cap, nu_raw)):
        assert abs(wrong - want) > 10 * se, (wrong, want)


def test_capped_unbiased_below_every_entry_is_the_sign_transform():
    """A cap below every |X_ij| leaves X~_ij = sgn(X_ij) with probability one and
    row weights |Y_i| c^2: with c a power of two the capped unbiased search is
    the sign-transform search exactly (Section 3.2 relates capping at small c to
    the sign transform)."""
    d = synthgen.small_continuous(60, 40, seed=22, planted=[(2, 9), (4, 31)])
    XT = d.XT.astype(np.float32)
    assert np.abs(XT).min() > 2.0 ** -20
    for two in (False, True):
        a = oracle.search(XT, d.Y, 6, 12, 0.15, seed=8, two_sided=two, unbiased=True, cap=2.0 ** -20)
        b = oracle.search(XT, d.Y, 6, 12, 0.15, seed=8, two_sided=two)
        assert np.array_equal(a[0], b[0])
        for f in ("candidates", "passed", "cmask", "max_bucket", "fresh"):
            assert np.array_equal(a[1][f], b[1][f]), f
        assert a[1]["candidates"].sum() > 0


def test_capped_unbiased_above_every_entry_changes_nothing():
    d = synthgen.small_continuous(50, 30, seed=23, planted=[(1, 4)])
    XT = d.XT.astype(np.float32)
    big = float(np.abs(XT).max())
    a = oracle.search(XT, d.Y, 5, 8, 0.2, seed=3, unbiased=True, cap=big)
    b = oracle.search(XT, d.Y, 5, 8, 0.2, seed=3, unbiased=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # a cap just below the largest entry changes the draws
    c = oracle.search(XT, d.Y, 5, 8, 0.2, seed=3, unbiased=True, cap=0.5 * big)
    assert not np.array_equal(a[1]["candidates"], c[1]["candidates"])


def test_cap_rejected_without_unbiased_or_negative():
    d = synthgen.small_continuous(20, 10, seed=24)
    with pytest.raises(oracle.OracleError):
        oracle.search(d.XT, d.Y, 3, 2, 0.2, cap=1.0)
    with pytest.raises(oracle.OracleError):
        oracle.search(d.XT, d.Y, 3, 2, 0.2, unbiased=True, cap=-1.0)


def test_unbiased_strength_uniform_example_is_13_18():
    """Section 3.2 prints 13/18 as the limit of the true pair's strength under the
    unbiased transform for X ~ Uniform(-1, 1) and Y = X_j X_k without noise."""
    r = np.random.default_rng(12)
    n = 400_000
    XT = r.uniform(-1, 1, size=(2, n))
    Y = XT[0] * XT[1]
    g = theory.gamma_unbiased(XT, Y, 0, 1, scale=False)
    assert abs(g - 13 / 18) < 3e-3, g


def test_unbiased_search_deterministic_and_rows_table():
    """The transform's draws are counter based: the same seed gives the same
    candidates, and a row table with an all-zero row (nu = 0, drawn only
    through the table) is accepted."""
    d = synthgen.small_continuous(50, 30, seed=13, planted=[(1, 4)])
    XT = d.XT.copy()
    XT[:, 7] = 0.0                                  # row 7 all zero
    a = oracle.search(XT, d.Y, 5, 6, 0.2, seed=3, unbiased=True)
    b = oracle.search(XT, d.Y, 5, 6, 0.2, seed=3, unbiased=True)
    assert np.array_equal(a[1]["candidates"], b[1]["candidates"]) and np.array_equal(a[0], b[0])
    rows = np.full((4, 5), 7, dtype=np.int32)
    rows[:, 0] = [0, 1, 2, 3]
    oracle.search(XT, d.Y, 5, 4, 0.2, rows=rows, unbiased=True)


# ------------------------------------------ bucket sizes and first repetitions
#
# Section 2.2 groups the columns by their projected value (Figure 2); the
# statistic max_bucket is the size of the largest group of X columns.  Algorithm
# 2 adds the pairs of each repetition to I; fresh_l counts the pairs of I whose
# first repetition is l.  Both are checked against counts made here directly
# from the data, not from the oracle's records.

def _x_groups(XT, rows):
    """Sizes of the groups of X columns with equal entries on the sampled rows."""
    sub = np.ascontiguousarray(XT[:, rows])            # p x m
    if sub.shape[1] == 0:
        return np.array([XT.shape[0]])
    _, counts = np.unique(sub, axis=0, return_counts=True)
    return counts


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_max_bucket_all_columns_equal_is_p(m):
    """Every column the same: one group of p X columns, whatever Y is.  Counting
    the Z side into the group as well would give 2p whenever Y is +1 on every
    sampled row (m = 0 always)."""
    n, p, L = 16, 9, 60
    col = synthgen.rademacher(n, 1, seed=3)[0]
    XT = np.repeat(col[None, :], p, axis=0)
    Y = synthgen.small_binary(n, 2, seed=4).Y
    assert (Y == 1).any() and (Y == -1).any()
    _, reps = oracle.search(XT, Y, m, L, 0.0, seed=8)
    assert np.all(reps["max_bucket"] == p)
    if m > 0:
        assert np.any(reps["cmask"] == 0), "some repetition samples only rows with Y = +1"


def test_max_bucket_hand_built_groups():
    """Columns built with chosen patterns on the sampled rows (0, 1): group sizes
    5, 3, 2, 1.  Y = -1 on row 0 makes each X group meet the Z side of the
    group with bit 0 flipped, so X + Z counts (5 + 3, ...) differ from 5."""
    n = 8
    patterns = {(1, 1): 5, (-1, 1): 3, (1, -1): 2, (-1, -1): 1}
    cols = []
    r = np.random.default_rng(1)
    for (a, b), cnt in patterns.items():
        for _ in range(cnt):
            c = (2 * r.integers(0, 2, size=n) - 1).astype(np.int8)
            c[0], c[1] = a, b
            cols.append(c)
    XT = np.stack(cols).astype(np.int8)
    Y = np.ones(n, dtype=np.int8)
    Y[0] = -1
    rows = np.array([[0, 1], [1, 0], [0, 0], [1, 1]], dtype=np.int32)
    _, reps = oracle.search(XT, Y, 2, 4, 0.0, rows=rows)
    want = [int(_x_groups(XT, rows[l]).max()) for l in range(4)]
    assert want == [5, 5, 7, 8]          # rows (0,0): row 0 alone -> 5+2 | 3+1; rows (1,1): 5+3 | 2+1
    assert reps["max_bucket"].tolist() == want


def test_max_bucket_random_matches_group_count():
    d = synthgen.small_binary(30, 200, seed=17, planted=[(3, 9)], flip=0.2)
    for m in (1, 3, 5):
        rows = synthgen.rows_table(30, 6, m, seed=m)
        for two in (False, True):
            _, reps = oracle.search(d.XT, d.Y, m, 6, 0.1, rows=rows, two_sided=two)
            assert reps["max_bucket"].tolist() == [int(_x_groups(d.XT, rows[l]).max()) for l in range(6)]


def _first_reps_direct(XT, Y, rows, rep_offset, kappa, two_sided=False):
    """first repetition of every pair of I by direct enumeration: the smallest
    l = rep_offset + l' with (j, k) in E_l (O(p^2 m)) and s/n > kappa."""
    X = XT.T.astype(np.int64)
    Z = Y.astype(np.int64)[:, None] * X
    n = X.shape[0]
    S = X.T @ (Y.astype(np.int64)[:, None] * X)         # s_jk for every pair (textbook GEMM)
    first = {}
    for li, rw in enumerate(rows):
        for (j, k) in _direct_E(X, Z, rw, two_sided):
            st = int(S[j, k]) / n
            if (abs(st) if two_sided else st) > kappa and (j, k) not in first:
                first[(j, k)] = rep_offset + li
    return first


@pytest.mark.parametrize("rep_offset", [0, 5])
@pytest.mark.parametrize("two_sided", [False, True])
def test_fresh_counts_first_repetitions(rep_offset, two_sided):
    d = synthgen.small_binary(28, 40, seed=23, planted=[(2, 7), (11, 30)], flip=0.15)
    m, L, kappa = 2, 9, 0.1
    rows = synthgen.rows_table(28, L, m, seed=31)
    pairs, reps = oracle.search(d.XT, d.Y, m, L, kappa, rows=rows, rep_offset=rep_offset, two_sided=two_sided)
    first = _first_reps_direct(d.XT, d.Y, rows, rep_offset, kappa, two_sided)
    assert {(int(a), int(b)): int(f) for a, b, f in zip(pairs["j"], pairs["k"], pairs["first_rep"])} == first
    want = np.bincount(np.array(list(first.values()), dtype=np.int64) - rep_offset, minlength=L)
    assert reps["fresh"].tolist() == want.tolist()
    assert int(reps["fresh"].sum()) == len(pairs)
    assert int(reps["fresh"].sum()) < int(reps["passed"].sum()), "some pairs pass in several repetitions"


def test_fresh_of_split_runs():
    """Each part's fresh counts sum to its own unique pairs; the full run's fresh
    is the histogram of the first repetitions merged over the parts."""
    d = synthgen.small_binary(50, 40, seed=14, planted=[(1, 2), (5, 30)], flip=0.15)
    full, rf = oracle.search(d.XT, d.Y, 4, 12, 0.2, seed=3)
    a, ra = oracle.search(d.XT, d.Y, 4, 5, 0.2, seed=3, rep_offset=0)
    b, rb = oracle.search(d.XT, d.Y, 4, 7, 0.2, seed=3, rep_offset=5)
    assert int(ra["fresh"].sum()) == len(a) and int(rb["fresh"].sum()) == len(b)
    assert int(rf["fresh"].sum()) == len(full)
    first = {}
    for arr in (a, b):
        for r in arr:
            key = (int(r["j"]), int(r["k"]))
            first[key] = min(first.get(key, 10 ** 9), int(r["first_rep"]))
    assert rf["fresh"].tolist() == np.bincount(list(first.values()), minlength=12).tolist()
