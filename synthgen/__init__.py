"""Seeded synthetic inputs for the xyz interaction search.

This module only *draws data*: predictor matrices X, responses Y and the list
of planted column pairs.  It holds none of the search's arithmetic (no keys,
no strengths, no thresholds), so that the CPU oracle and the GPU library can
both consume the same inputs without sharing any of the method's code.

Conventions
-----------
* ``XT`` is the transpose of X, shape ``(p, n)`` and C-contiguous, i.e. X in
  column-major order: column j of X is ``XT[j]``.  Binary data is int8 in
  {-1, +1}; continuous data is float32.
* ``bits`` (large binary inputs only) is X already bit-packed column-major:
  ``(p, ceil(n/64))`` uint64, bit ``i % 64`` of word ``i // 64`` of row j is
  1 exactly when ``X[i, j] == -1``; bits past row n are 0.
* Every generator takes an integer ``seed`` and uses ``numpy.random.PCG64``.

The shapes and distributions follow the workloads the paper measures on:
Rademacher designs (Section 5.2), genotype-like binary SNP data (Section 5.3,
where the real data set is not available and a minor-allele-frequency model
stands in for it) and Gaussian continuous designs (Section 5.4).
"""
from __future__ import annotations

import dataclasses
import math
import numpy as np

__all__ = [
    "Dataset", "rademacher", "genotype", "gaussian",
    "config1", "config2", "config3", "config4", "config5_shared", "config5_requests",
    "config5_fresh", "small_binary", "small_continuous", "rows_table", "pack_bits_colmajor",
    "scaling_x", "scaling_y", "lasso_setting", "gaussian_projections", "subsample_projections",
    "strength_pairs",
]


@dataclasses.dataclass
class Dataset:
    """One synthetic search problem."""
    n: int
    p: int
    XT: np.ndarray | None          # (p, n) int8 or float32, or None when only bits are held
    Y: np.ndarray                  # (n,) int8 (+-1) or float32
    planted: list                  # list of (j, k) with j < k (0-based)
    params: dict                   # search parameters of the workload (L, m, kappa, seed, ...)
    bits: np.ndarray | None = None  # (p, ceil(n/64)) uint64 column-major bits, large inputs only
    meta: dict = dataclasses.field(default_factory=dict)


def _rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(stream), 0x5eed]))


def rademacher(n: int, p: int, seed: int) -> np.ndarray:
    """(p, n) int8 matrix of i.i.d. uniform {-1, +1} entries (X in column-major order)."""
    r = _rng(seed, 1)
    b = r.integers(0, 2, size=(p, n), dtype=np.int8)
    return (2 * b - 1).astype(np.int8)


def genotype(n: int, p: int, seed: int, f_lo: float = 0.05, f_hi: float = 0.5):
    """(p, n) int8 genotype-shaped matrix and its minor-allele frequencies.

    Column j has frequency f_j ~ U[f_lo, f_hi]; X_ij = +1 when a Binomial(2, f_j)
    draw is positive (at least one minor allele), else -1.
    """
    r = _rng(seed, 2)
    f = r.uniform(f_lo, f_hi, size=p)
    XT = np.empty((p, n), dtype=np.int8)
    chunk = max(1, (1 << 24) // max(n, 1))
    for j0 in range(0, p, chunk):
        j1 = min(p, j0 + chunk)
        g = r.binomial(2, f[j0:j1, None], size=(j1 - j0, n))
        XT[j0:j1] = np.where(g > 0, 1, -1).astype(np.int8)
    return XT, f


def gaussian(n: int, p: int, seed: int) -> np.ndarray:
    """(p, n) float32 matrix of i.i.d. N(0, 1) entries."""
    r = _rng(seed, 3)
    XT = np.empty((p, n), dtype=np.float32)
    chunk = max(1, (1 << 24) // max(n, 1))
    for j0 in range(0, p, chunk):
        j1 = min(p, j0 + chunk)
        XT[j0:j1] = r.standard_normal(size=(j1 - j0, n), dtype=np.float32)
    return XT


def pack_bits_colmajor(XT: np.ndarray) -> np.ndarray:
    """Pack a (p, n) +-1 int8 matrix into (p, ceil(n/64)) uint64 words, bit = [x == -1].

    This is an input-format conversion (the same information in another
    layout), used to hand large binary inputs over in packed form.
    """
    p, n = XT.shape
    w = (n + 63) // 64
    b = (XT == -1)
    pad = w * 64 - n
    if pad:
        b = np.concatenate([b, np.zeros((p, pad), dtype=bool)], axis=1)
    packed8 = np.packbits(b.reshape(p, w * 8, 8), axis=2, bitorder="little").reshape(p, w * 8)
    return packed8.view(np.uint64).reshape(p, w).copy()


def _distinct_columns(r: np.random.Generator, p: int, count: int) -> np.ndarray:
    return r.choice(p, size=count, replace=False)


def config1(seed: int = 0) -> Dataset:
    """Plain single-instance workload: n=200, p=2000, Rademacher X.

    Each row's response is driven by one of three planted pairs chosen
    uniformly at random, (3,7), (50,900) and (1200,1999), as Y_i = X_ia X_ib,
    then flipped with probability 0.1 for the first pair and 0.25 for the
    other two.  Search parameters: L=20, m=10, kappa=0.3, sampler seed 0.
    """
    n, p = 200, 2000
    XT = rademacher(n, p, seed)
    r = _rng(seed, 11)
    pairs = [(3, 7), (50, 900), (1200, 1999)]
    flips = [0.1, 0.25, 0.25]
    drv = r.integers(0, 3, size=n)
    u = r.random(n)
    Y = np.empty(n, dtype=np.int8)
    for i in range(n):
        a, b = pairs[drv[i]]
        y = int(XT[a, i]) * int(XT[b, i])
        if u[i] < flips[drv[i]]:
            y = -y
        Y[i] = y
    return Dataset(n, p, XT, Y, pairs, dict(L=20, m=10, kappa=0.3, seed=0, two_sided=False))


def config2(seed: int = 0, n: int = 2000, p: int = 100_000) -> Dataset:
    """Genotype-shaped binary workload (stands in for the SNP data of Section 5.3).

    X from the minor-allele-frequency model; Y = +-1 drawn from a logistic model
    with 20 main effects of 0.3 and 10 planted pairs with coefficients
    theta ~ U[0.2, 0.6], on 40 distinct random columns; intercept 0.
    Search parameters: L=200, m=12; kappa is set by the caller so that about
    1e4 pairs exceed it.
    """
    XT, f = genotype(n, p, seed)
    r = _rng(seed, 12)
    cols = _distinct_columns(r, p, 40)
    mains = cols[:20]
    pc = cols[20:]
    pairs = [tuple(sorted((int(pc[2 * q]), int(pc[2 * q + 1])))) for q in range(10)]
    theta = r.uniform(0.2, 0.6, size=10)
    eta = np.zeros(n, dtype=np.float64)
    for j in mains:
        eta += 0.3 * XT[j].astype(np.float64)
    for q, (a, b) in enumerate(pairs):
        eta += theta[q] * (XT[a].astype(np.float64) * XT[b].astype(np.float64))
    prob = 1.0 / (1.0 + np.exp(-eta))
    Y = np.where(r.random(n) < prob, 1, -1).astype(np.int8)
    return Dataset(n, p, XT, Y, pairs, dict(L=200, m=12, kappa=None, seed=seed, two_sided=False),
                   meta=dict(maf=f, mains=[int(j) for j in mains], theta=theta.tolist()))


def config3(seed: int = 0, n: int = 5000, p: int = 1_000_000, npairs: int = 20,
            s_lo: float = 0.15, s_hi: float = 0.5, signed: bool = False) -> Dataset:
    """Large Rademacher workload handed over bit-packed (about 625 MB at full size).

    Y is Rademacher.  Each of ``npairs`` planted pairs (j, k) on distinct
    columns gets a target strength s ~ U[s_lo, s_hi]: column k is rewritten as
    Y o X_j and then exactly round(n (1 - s) / 2) of its rows, chosen at
    random, are negated.  With ``signed`` each planted pair's sign is random
    (column k is negated as a whole with probability 1/2).
    Search parameters: L=500, m=14, kappa=0.12.
    """
    r = _rng(seed, 13)
    w = (n + 63) // 64
    bits = r.integers(0, np.iinfo(np.uint64).max, size=(p, w), dtype=np.uint64, endpoint=True)
    tail = n - (w - 1) * 64
    if tail < 64:
        bits[:, w - 1] &= np.uint64((1 << tail) - 1)
    yb = r.integers(0, 2, size=n, dtype=np.int8)
    Y = (1 - 2 * yb).astype(np.int8)
    ybits = pack_bits_colmajor(Y[None, :])[0]
    cols = _distinct_columns(r, p, 2 * npairs)
    pairs, targets, signs = [], [], []
    for q in range(npairs):
        j, k = int(cols[2 * q]), int(cols[2 * q + 1])
        s = float(r.uniform(s_lo, s_hi))
        nflip = int(round(n * (1.0 - s) / 2.0))
        col = bits[j] ^ ybits
        flip = r.choice(n, size=nflip, replace=False)
        fb = np.zeros(w * 64, dtype=bool)
        fb[flip] = True
        fw = np.packbits(fb.reshape(w * 8, 8), axis=1, bitorder="little").reshape(w * 8).view(np.uint64)
        col = col ^ fw
        sg = 1
        if signed and r.random() < 0.5:
            col = ~col
            if tail < 64:
                col[w - 1] &= np.uint64((1 << tail) - 1)
            sg = -1
        bits[k] = col
        pairs.append((min(j, k), max(j, k)))
        targets.append(s)
        signs.append(sg)
    return Dataset(n, p, None, Y, pairs, dict(L=500, m=14, kappa=0.12, seed=seed, two_sided=signed),
                   bits=bits, meta=dict(target_s=targets, signs=signs))


def scaling_x(n: int, p: int, seed: int) -> np.ndarray:
    """Rademacher X of the scaling experiment (Section 5.2), bit-packed as
    ``(p, ceil(n/64))`` uint64 (same layout as ``Dataset.bits``)."""
    r = _rng(seed, 17)
    w = (n + 63) // 64
    bits = r.integers(0, np.iinfo(np.uint64).max, size=(p, w), dtype=np.uint64, endpoint=True)
    tail = n - (w - 1) * 64
    if tail < 64:
        bits[:, w - 1] &= np.uint64((1 << tail) - 1)
    return bits


def scaling_y(bits: np.ndarray, n: int, agree: int, seed: int) -> np.ndarray:
    """Response of the scaling experiment: Y_i = X_i0 X_i1 on ``agree`` rows chosen
    at random and -X_i0 X_i1 on the others, so that columns 0 and 1 form the one
    strong pair, with Y_i X_i0 X_i1 = +1 on exactly ``agree`` rows.  int8 +-1."""
    r = _rng(seed, 19)
    x0, x1 = unpack_column(bits[0], n), unpack_column(bits[1], n)
    sign = np.full(n, -1, dtype=np.int8)
    sign[r.choice(n, size=agree, replace=False)] = 1
    return (x0 * x1 * sign).astype(np.int8)


def dag_gaussian(n: int, p: int, r, mean_parents: float = 10.0):
    """Rows i.i.d. N(0, Sigma) with Sigma from a random DAG (Section 5.4, setting 3).

    Nodes come in a random order; node t takes Poisson(mean_parents) parents
    (at most t) drawn uniformly among the earlier nodes, and is their linear
    combination with weights U[0, 1] plus independent centred Gaussian noise of
    variance 0.1 times the variance of that combination; a node without
    parents is N(0, 1).  Every column is then divided by its population
    standard deviation, so Sigma is a correlation matrix.  Returns (X float32
    (n, p), Sigma float64 (p, p))."""
    order = r.permutation(p)
    S = np.zeros((p, p))                        # covariance in generation order
    Z = np.empty((n, p))
    for t in range(p):
        k = min(t, int(r.poisson(mean_parents))) if t else 0
        if k == 0:
            S[t, t] = 1.0
            Z[:, t] = r.standard_normal(n)
            continue
        pa = r.choice(t, size=k, replace=False)
        w = r.uniform(0.0, 1.0, size=k)
        v = float(w @ S[np.ix_(pa, pa)] @ w)     # variance from the direct parents
        c = S[:t][:, pa] @ w
        S[:t, t] = c
        S[t, :t] = c
        S[t, t] = 1.1 * v
        Z[:, t] = Z[:, pa] @ w + math.sqrt(0.1 * v) * r.standard_normal(n)
    sd = np.sqrt(np.diag(S))
    X = np.empty((n, p), dtype=np.float32)
    X[:, order] = (Z / sd).astype(np.float32)
    C = S / sd[:, None] / sd[None, :]
    Sigma = np.empty((p, p))
    Sigma[np.ix_(order, order)] = C
    return X, Sigma


def lasso_setting(n: int, p: int, setting: int, seed: int = 0):
    """Regression data of Section 5.4: X float32 (n, p) with rows N(0, Sigma);
    20 main effects and 10 interactions with magnitudes U[2, 6] and random
    signs, mu = 0, eps ~ N(0, 1).  Setting 1 (Sigma = I) is hierarchical
    (interactions drawn among pairs of main effects), setting 2 (Sigma = I)
    strictly non-hierarchical (interactions among the other columns), setting
    3 is setting 2 on the correlated design of dag_gaussian.
    Returns (X, Y, mains {j: beta}, inters {(j, k): theta})."""
    if setting not in (1, 2, 3):
        raise ValueError(f"setting {setting}: Section 5.4 has settings 1, 2 and 3")
    r = _rng(seed, 23 + setting)
    if setting == 3:
        X, _ = dag_gaussian(n, p, r)
    else:
        X = r.standard_normal((n, p)).astype(np.float32)
    cols = r.permutation(p)
    main = [int(j) for j in cols[:20]]
    pool = main if setting == 1 else [int(j) for j in cols[20:]]
    pairs = set()
    while len(pairs) < 10:
        j, k = r.choice(len(pool), size=2, replace=False)
        pairs.add((min(pool[j], pool[k]), max(pool[j], pool[k])))
    mains = {j: float(r.uniform(2, 6) * r.choice([-1, 1])) for j in main}
    inters = {pq: float(r.uniform(2, 6) * r.choice([-1, 1])) for pq in sorted(pairs)}
    Xd = X.astype(np.float64)
    y = r.standard_normal(n)
    for j, b in mains.items():
        y += b * Xd[:, j]
    for (j, k), t in inters.items():
        y += t * Xd[:, j] * Xd[:, k]
    return X, y, mains, inters


def config4(seed: int = 0, n: int = 1000, p: int = 200_000) -> Dataset:
    """Continuous workload: X ~ N(0,1) float32, real-valued Y.

    Y = sum over 5 planted pairs of X_j X_k + 0.5 * sum over 10 main effects
    of X_j + N(0,1), on 20 distinct random columns.  Hashing uses the signs of
    X and |Y|-weighted row sampling.  Search parameters: L=300, m=12, kappa=0.5.
    """
    XT = gaussian(n, p, seed)
    r = _rng(seed, 14)
    cols = _distinct_columns(r, p, 20)
    pc, mains = cols[:10], cols[10:]
    pairs = [tuple(sorted((int(pc[2 * q]), int(pc[2 * q + 1])))) for q in range(5)]
    y = r.standard_normal(n)
    for a, b in pairs:
        y += XT[a].astype(np.float64) * XT[b].astype(np.float64)
    for j in mains:
        y += 0.5 * XT[j].astype(np.float64)
    Y = y.astype(np.float32)
    return Dataset(n, p, XT, Y, pairs, dict(L=300, m=12, kappa=0.5, seed=seed, two_sided=False),
                   meta=dict(mains=[int(j) for j in mains]))


def config5_shared(seed: int = 0, n: int = 2000, p: int = 200_000):
    """Shared resident X of the serving workload (genotype model as in config 2)."""
    XT, f = genotype(n, p, seed + 1000)
    return XT, f


def _mixture_response(r: np.random.Generator, XT: np.ndarray, pairs, strengths) -> np.ndarray:
    """Row mixture: row i copies X_ia X_ib of planted pair q with probability s_q,
    otherwise it is a fair coin.  sum(s_q) must be at most 1."""
    n = XT.shape[1]
    u = r.random(n)
    Y = np.where(r.random(n) < 0.5, 1, -1).astype(np.int8)
    acc = 0.0
    for (a, b), s in zip(pairs, strengths):
        sel = (u >= acc) & (u < acc + s)
        Y[sel] = (XT[a, sel].astype(np.int16) * XT[b, sel].astype(np.int16)).astype(np.int8)
        acc += s
    return Y


def config5_requests(XT: np.ndarray, count: int = 256, seed: int = 0, rate: float = 50.0):
    """Response vectors arriving for the shared X: Poisson arrivals at ``rate`` per s.

    Each request plants 1-3 pairs with strengths U[0.2, 0.5] (total at most 0.9)
    through a row mixture; its repetition count is drawn from {50, 200, 500};
    kappa = 0.15.  Returns a list of dicts (arrival time, Y, planted, L, kappa).
    """
    r = _rng(seed, 15)
    p = XT.shape[0]
    t = 0.0
    out = []
    for q in range(count):
        t += r.exponential(1.0 / rate)
        k = int(r.integers(1, 4))
        while True:
            s = r.uniform(0.2, 0.5, size=k)
            if s.sum() <= 0.9:
                break
        cols = _distinct_columns(r, p, 2 * k)
        pairs = [tuple(sorted((int(cols[2 * i]), int(cols[2 * i + 1])))) for i in range(k)]
        Y = _mixture_response(r, XT, pairs, s)
        L = int(r.choice([50, 200, 500]))
        out.append(dict(t=t, Y=Y, planted=pairs, strengths=s.tolist(), L=L, kappa=0.15))
    return out


def config5_fresh(count: int = 32, seed: int = 0, n: int = 1000, sizes=(10_000, 100_000, 500_000),
                  rate: float = 50.0 / 8.0):
    """Requests on fresh data sets (Rademacher X, n=1000, p from ``sizes``)."""
    r = _rng(seed, 16)
    t = 0.0
    out = []
    for q in range(count):
        t += r.exponential(1.0 / rate)
        p = int(r.choice(sizes))
        XT = rademacher(n, p, seed * 1000 + q + 7)
        k = int(r.integers(1, 4))
        s = r.uniform(0.2, 0.3, size=k)
        cols = _distinct_columns(r, p, 2 * k)
        pairs = [tuple(sorted((int(cols[2 * i]), int(cols[2 * i + 1])))) for i in range(k)]
        Y = _mixture_response(r, XT, pairs, s)
        L = int(r.choice([50, 200, 500]))
        out.append(dict(t=t, XT=XT, Y=Y, planted=pairs, strengths=s.tolist(), L=L, kappa=0.15))
    return out


def unpack_column(bits: np.ndarray, n: int) -> np.ndarray:
    """One packed column (ceil(n/64) uint64 words, bit = [x == -1]) back to +-1 int8."""
    b = np.unpackbits(bits.view(np.uint8), bitorder="little")[:n]
    return (1 - 2 * b.astype(np.int8)).astype(np.int8)


def config5_fresh_bits(count: int = 32, seed: int = 0, n: int = 1000, sizes=(10_000, 100_000, 500_000),
                       rate: float = 50.0 / 8.0):
    """The fresh-data requests of the serving workload, with X handed over bit-packed.

    Same model as ``config5_fresh`` (Rademacher X, n=1000, p from ``sizes``,
    1-3 pairs of strength U[0.2, 0.3] planted by a row mixture, L from
    {50, 200, 500}, kappa = 0.15); X is drawn directly as random words, which
    is the same distribution and avoids building the int8 matrix.  Each entry
    holds ``bits`` of shape (p, ceil(n/64)) instead of ``XT``.
    """
    r = _rng(seed, 17)
    w = (n + 63) // 64
    t = 0.0
    out = []
    for q in range(count):
        t += r.exponential(1.0 / rate)
        p = int(r.choice(sizes))
        bits = _rng(seed * 1000 + q, 18).integers(0, np.iinfo(np.uint64).max, size=(p, w), dtype=np.uint64,
                                                    endpoint=True)
        tail = n - (w - 1) * 64
        if tail < 64:
            bits[:, w - 1] &= np.uint64((1 << tail) - 1)
        k = int(r.integers(1, 4))
        s = r.uniform(0.2, 0.3, size=k)
        cols = _distinct_columns(r, p, 2 * k)
        pairs = [tuple(sorted((int(cols[2 * i]), int(cols[2 * i + 1])))) for i in range(k)]
        sub = {j: unpack_column(bits[j], n) for pq in pairs for j in pq}
        u = r.random(n)
        Y = np.where(r.random(n) < 0.5, 1, -1).astype(np.int8)
        acc = 0.0
        for (a, b), sq in zip(pairs, s):
            sel = (u >= acc) & (u < acc + sq)
            Y[sel] = (sub[a][sel].astype(np.int16) * sub[b][sel]).astype(np.int8)
            acc += sq
        L = int(r.choice([50, 200, 500]))
        out.append(dict(t=t, bits=bits, n=n, Y=Y, planted=pairs, strengths=s.tolist(), L=L, kappa=0.15))
    return out


def small_binary(n: int, p: int, seed: int, planted=(), flip: float = 0.0, y_bias: float = 0.5) -> Dataset:
    """Small Rademacher problem for parity tests.

    Without planted pairs Y is Bernoulli(y_bias) on {+1, -1}.  Each planted
    pair (a, b) drives an equal share of the rows as Y_i = X_ia X_ib, flipped
    with probability ``flip``.
    """
    XT = rademacher(n, p, seed)
    r = _rng(seed, 21)
    Y = np.where(r.random(n) < y_bias, 1, -1).astype(np.int8)
    if planted:
        drv = r.integers(0, len(planted), size=n)
        u = r.random(n)
        for i in range(n):
            a, b = planted[drv[i]]
            y = int(XT[a, i]) * int(XT[b, i])
            Y[i] = -y if u[i] < flip else y
    return Dataset(n, p, XT, Y, [tuple(sorted(pq)) for pq in planted], {})


def long_binary(n: int, p: int, seed: int, pair=(0, 1), share: float = 0.3) -> Dataset:
    """Rademacher problem with long columns (vectorised, for n in the millions).

    Y_i = X_ia X_ib for the planted pair (a, b) on a random ``share`` of the
    rows, uniform on {+1, -1} elsewhere.
    """
    XT = rademacher(n, p, seed)
    r = _rng(seed, 23)
    Y = np.where(r.random(n) < 0.5, 1, -1).astype(np.int8)
    on = r.random(n) < share
    a, b = pair
    Y[on] = XT[a, on] * XT[b, on]
    return Dataset(n, p, XT, Y, [tuple(sorted(pair))], {})


def small_continuous(n: int, p: int, seed: int, planted=(), noise: float = 1.0) -> Dataset:
    """Small Gaussian problem: Y = sum of planted X_a X_b + noise * N(0,1)."""
    XT = gaussian(n, p, seed)
    r = _rng(seed, 22)
    y = noise * r.standard_normal(n)
    for a, b in planted:
        y += XT[a].astype(np.float64) * XT[b].astype(np.float64)
    return Dataset(n, p, XT, y.astype(np.float32), [tuple(sorted(pq)) for pq in planted], {})


def rows_table(n: int, L: int, m: int, seed: int) -> np.ndarray:
    """An explicit (L, m) int32 table of i.i.d. uniform row indices.

    Used to hand the same row draws to both sides directly, independently of
    any sampler either side implements.
    """
    r = _rng(seed, 31)
    return r.integers(0, n, size=(L, m), dtype=np.int32)


def gaussian_projections(n: int, L: int, seed: int, frac_bits: int | None = None):
    """L dense Gaussian projection vectors on a fixed-point grid: R[l, i] =
    round(2^frac_bits G), G ~ N(0, 1) clipped to [-8, 8], as int32 (L, n).

    The default grid 2^frac_bits <= 2^30 / n keeps sum_i |R[l, i]| below 2^31
    (the bound under which integer projections of +-1 data cannot overflow
    32 bits).  Returns (R, sd) with sd = 2^frac_bits, the scale of one unit
    normal on the grid.
    """
    if frac_bits is None:
        frac_bits = max(0, int(np.floor(np.log2((1 << 30) / max(n, 1)))))
    r = _rng(seed, 41)
    g = np.clip(r.standard_normal(size=(L, n)), -8.0, 8.0)
    R = np.rint(g * float(1 << frac_bits)).astype(np.int32)
    return R, float(1 << frac_bits)


def subsample_projections(n: int, L: int, M: int, seed: int, bits: int = 20):
    """L sparse projection vectors built from subsampled rows: M row indices per
    vector drawn uniformly with replacement, each given a weight D of random
    sign and magnitude uniform in [2^bits, 2^(bits+1)); weights of a repeated
    row add up.  Returns (R (L, n), rows int32 (L, M), D (L, M)), int32 for
    bits <= 20 (then M <= 512 keeps sum_i |R[l, i]| below 2^31), else int64."""
    if bits <= 20 and M > 512:
        raise ValueError("M <= 512")
    r = _rng(seed, 42)
    rows = r.integers(0, n, size=(L, M), dtype=np.int32)
    D = r.integers(1 << bits, 1 << (bits + 1), size=(L, M), dtype=np.int64) * np.where(r.random((L, M)) < 0.5, -1, 1)
    R = np.zeros((L, n), dtype=np.int64)
    for l in range(L):
        np.add.at(R[l], rows[l], D[l])
    dt = np.int32 if bits <= 20 else np.int64
    return R.astype(dt), rows, D.astype(dt)


def strength_pairs(n: int, p: int, gammas, per: int, seed: int):
    """+-1 data with `per` disjoint planted pairs of each strength gamma in
    `gammas` against one Y: columns 2q and 2q + 1 form pair q; X_{2q+1} equals
    Y o X_{2q} on round(gamma n) rows and its negation on the others (half of
    those rows with Y = +1 and half with Y = -1, as far as possible).  The
    remaining columns are Rademacher.  Returns (XT (p, n) int8, Y (n,) int8,
    pairs [(j, k, gamma)])."""
    r = _rng(seed, 43)
    XT = rademacher(n, p, seed)
    Y = np.where(r.random(n) < 0.5, 1, -1).astype(np.int8)
    pos, neg = np.flatnonzero(Y == 1), np.flatnonzero(Y == -1)
    pairs = []
    q = 0
    for g in gammas:
        dis_n = n - int(round(g * n))
        for _ in range(per):
            j, k = 2 * q, 2 * q + 1
            if k >= p:
                raise ValueError("p too small for the planted pairs")
            a = min(dis_n // 2, len(pos))
            b = min(dis_n - a, len(neg))
            dis = np.zeros(n, dtype=bool)
            dis[r.choice(pos, a, replace=False)] = True
            dis[r.choice(neg, b, replace=False)] = True
            dis[r.choice(np.flatnonzero(~dis), dis_n - a - b, replace=False)] = True
            XT[k] = np.where(dis, -Y * XT[j], Y * XT[j]).astype(np.int8)
            pairs.append((j, k, float(g)))
            q += 1
    return XT, Y, pairs
