"""The two factors of Theorem 2's running time, measured on the GPU search
for the scaling experiment of Section 5.2 (Rademacher X, one strong pair).

Theorem 2 bounds the work to discovery by (repetitions to discovery) x (work
per repetition).  With M sampled rows and i.i.d. row draws:

* the strong pair collides in a repetition with probability gamma^M, so the
  first repetition that finds it is geometric with mean 1 / gamma^M (eq. (9)
  with L = 1);
* a repetition's candidate set E_l has expected size sum_{j<k} gamma_jk^M
  (each pair collides with probability gamma_jk^M), which the test computes
  from every pair's strength (eq. (4): the fraction of rows with
  Y_i X_ij X_ik = +1) with a plain matrix product.

Both are checked against the search's own output: the first repetition of
the pair over many seeds, and the per-repetition candidate counts.
"""
import math

import numpy as np
import pytest

import synthgen
import paper_1610_05108_amd as xyz

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = xyz.Context(0)
    yield c
    c.close()


def _strength_sum(bits, Y, n, M):
    """sum over j < k of gamma_jk^M, gamma_jk = #{i : Y_i X_ij X_ik = +1} / n."""
    X = np.stack([synthgen.unpack_column(b, n) for b in bits]).astype(np.float64)   # (p, n)
    S = (X * Y.astype(np.float64)) @ X.T                                            # s_jk, exact integers
    g = 0.5 * (1.0 + S / n)
    iu = np.triu_indices(len(bits), 1)
    return float((g[iu] ** M).sum())


@pytest.mark.parametrize("p", [2000, 6000])
def test_discovery_and_candidates_follow_theorem_2(ctx, p):
    n, gamma, sims = 1000, 0.8, 160
    M = int(round(math.log(p) / math.log(1 / 0.55)))
    bits = synthgen.scaling_x(n, p, seed=p)
    agree = int(round(gamma * n))
    Y = synthgen.scaling_y(bits, n, agree, seed=1)
    q = (agree / n) ** M
    x = ctx.x_create(bits, n=n)
    chunk = max(4, math.ceil(0.5 / q))
    kappa = (2 * agree / n - 1) / 2
    first, cands = [], []
    for sim in range(sims):
        off = 0
        while True:
            r = ctx.search(x, Y, m=M, L=chunk, kappa=kappa, seed=500 + sim, rep_offset=off)
            cands.extend(r["reps"]["candidates"].tolist())
            pr = r["pairs"]
            hit = (pr["j"] == 0) & (pr["k"] == 1)
            if hit.any():
                first.append(int(pr["first_rep"][hit][0]) + 1)
                break
            off += chunk
            assert off < 400 / q, "strong pair never found"
    # repetitions to discovery: geometric, mean 1/q, sd sqrt(1-q)/q
    se = math.sqrt(1 - q) / q / math.sqrt(sims)
    assert abs(np.mean(first) - 1 / q) < 4.5 * se, (np.mean(first), 1 / q, se)
    # candidates per repetition: mean sum_{j<k} gamma_jk^M
    want = _strength_sum(bits, Y, n, M)
    got = float(np.mean(cands))
    assert abs(got - want) < 0.05 * want, (got, want, len(cands))
