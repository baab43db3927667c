"""Algorithm 1 with dense projections, run by the oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module; the GPU library shares no code with it.

Section 2.1 gives the general form of the search (Algorithm 1): for each
repetition l a random vector R_l projects the columns of X and of Z = Y o X
onto one dimension, x = X^T R_l and z = Z^T R_l; E_l collects the pairs (j, k)
whose projections are within tau of each other, |x_j - z_k| <= tau; and the
pairs of E_l that are strong are added to I.  Class (a) of Section 2.1 (dense
projections) draws every component of R_l independently; Section 5.1 compares
dense Gaussian R with minimal subsampling.

This is the plain definition, with no sorting: the projections are exact
int64 sums of integer weights R (a fixed-point grid for the continuous
distribution F, chosen by the caller), E_l is found by comparing every x_j with
every z_k, and the strength check is eq. (1) on the binary64 quotient s/n
(strict).  Pairs are reported unordered: {j, k} is a candidate of repetition l
when (j, k) or (k, j) lies in E_l with j != k.
"""
from __future__ import annotations

import numpy as np

from . import PAIR_DTYPE, REP_DTYPE


def project(XT, Y, R):
    """Algorithm 1, projection step: x = X^T R_l and z = Z^T R_l with Z = Y o X
    (Algorithm 1, first step).  XT: (p, n) int8 +-1; Y: (n,) int8 +-1; R: (L, n)
    integers.  Returns int64 arrays x, z of shape (L, p)."""
    X = np.asarray(XT, dtype=np.int64)
    Yv = np.asarray(Y, dtype=np.int64)
    Rv = np.asarray(R, dtype=np.int64)
    return Rv @ X.T, Rv @ (X * Yv).T


def dense_search(XT, Y, R, tau: int, kappa: float, rep_offset: int = 0):
    """Algorithm 1 with the projections R (one row per repetition) and close-pairs
    threshold tau.  Returns (pairs, reps) structured arrays laid out like the
    Algorithm 2 oracle's: pairs sorted by (j, k) with s = Y^T(X_j o X_k),
    first_rep (rep_offset + l of the first repetition whose candidates hold the
    pair) and hits (repetitions whose candidates hold it); per repetition the
    number of unordered candidates, how many of them pass, how many reported
    pairs were first found there, and max_bucket = the largest close-pairs
    window max_j |{k : |x_j - z_k| <= tau}| (k = j included)."""
    XT = np.asarray(XT)
    if XT.dtype != np.int8:
        raise TypeError("dense_search takes +-1 data as int8")
    p, n = XT.shape
    Rv = np.asarray(R, dtype=np.int64).reshape(-1, n)
    L = Rv.shape[0]
    xs, zs = project(XT, Y, Rv)
    X = XT.astype(np.int64)
    Yv = np.asarray(Y, dtype=np.int64)
    reps = np.zeros(L, dtype=REP_DTYPE)
    first, hits, sval = {}, {}, {}
    for l in range(L):
        close = np.abs(xs[l][:, None] - zs[l][None, :]) <= tau      # close[j, k]: (j, k) in E_l
        reps[l]["max_bucket"] = int(close.sum(axis=1).max()) if p else 0
        np.fill_diagonal(close, False)
        jj, kk = np.nonzero(np.triu(close | close.T, 1))
        reps[l]["candidates"] = len(jj)
        if len(jj) == 0:
            continue
        s = (X[jj] * X[kk] * Yv).sum(axis=1)                          # Y^T(X_j o X_k), exact
        keep = (s.astype(np.float64) / float(n)) > kappa               # eq. (1), strict
        reps[l]["passed"] = int(keep.sum())
        for j, k, v in zip(jj[keep].tolist(), kk[keep].tolist(), s[keep].tolist()):
            if (j, k) not in first:
                first[(j, k)] = rep_offset + l
                sval[(j, k)] = v
                reps[l]["fresh"] += 1
            hits[(j, k)] = hits.get((j, k), 0) + 1
    keys = sorted(first)
    pairs = np.zeros(len(keys), dtype=PAIR_DTYPE)
    for q, (j, k) in enumerate(keys):
        v = sval[(j, k)]
        pairs[q] = (j, k, v, float(v), float(v) / float(n), first[(j, k)], hits[(j, k)])
    return pairs, reps
