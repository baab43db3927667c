"""Lasso with all main effects and pairwise interactions, with the KKT check of
the interactions done by the xyz search (Section 4, Algorithm 3, eq. (16)).

The objective is eq. (17): with Y and the columns of X centred and W~ the
column-centred matrix of all products X_j o X_k (j <= k),

    minimise 1/(2n) ||Y - X beta - W~ theta||^2 + lambda (||beta||_1 + ||theta||_1).

Algorithm 3 (the active-set strategy): for each lambda of a decreasing grid,
solve the problem restricted to the active main effects A and interactions B
(warm-started from the previous lambda), then collect the coordinates that
violate the KKT conditions at the restricted solution,

    U = {k : |X_k^T r| / n > lambda},   V = {(j,k) : |W~_jk^T r| / n > lambda},

with r the residual, add them to A and B, and repeat until none is left.  The
restricted problems are small and solved here by cyclic coordinate descent on
the host; the bottleneck, V over all p(p-1)/2 products with j < k, is the
interaction search of eq. (16) on the residual (r is centred, so the products
need no centring), run by the library's GPU search with Y = r two-sided
(+r and -r in turn); the p squares X_j o X_j are checked directly.

This layer sits above the C ABI: it calls ``xyz_search`` and does its own
small dense algebra; it has no other route to the interaction search.
"""
from __future__ import annotations

import numpy as np

__all__ = ["LassoPath", "lasso_interactions", "xyz_screen"]


class LassoPath:
    """Solutions along the lambda grid: ``main[l]`` maps main-effect j to beta_j,
    ``inter[l]`` maps (j, k), j <= k, to theta_jk (non-zero coefficients only),
    ``rounds[l]`` counts the KKT rounds (restricted solves) at lambda l."""

    def __init__(self, lambdas):
        self.lambdas = list(lambdas)
        self.main, self.inter, self.rounds = [], [], []


def _soft(z, t):
    return np.sign(z) * max(abs(z) - t, 0.0)


def _cd(M, y, lam, coef, tol, max_sweeps):
    """Cyclic coordinate descent for 1/(2n)||y - M c||^2 + lam ||c||_1 from coef."""
    n = M.shape[0]
    sq = (M * M).sum(axis=0) / n
    r = y - M @ coef
    for _ in range(max_sweeps):
        delta = 0.0
        for q in range(M.shape[1]):
            if sq[q] == 0.0:
                continue
            old = coef[q]
            z = old * sq[q] + M[:, q] @ r / n
            new = _soft(z, lam) / sq[q]
            if new != old:
                r -= M[:, q] * (new - old)
                coef[q] = new
                delta = max(delta, abs(new - old) * np.sqrt(sq[q]))
        if delta < tol:
            break
    return coef, r


def xyz_screen(ctx, x, m: int, L: int, seed: int = 0):
    """Interaction KKT check by the GPU search: returns screen(r, lam), the pairs
    (j, k), j < k, with |r^T (X_j o X_k)| / n > lam that the two-sided search
    with Y = r (real-valued, |r|-weighted rows, Section 3.1) finds in L
    repetitions of m sampled rows.  x is the library's resident X."""
    state = {"calls": 0}

    def screen(r, lam):
        state["calls"] += 1
        res = ctx.search(x, np.ascontiguousarray(r, dtype=np.float64), m=m, L=L, kappa=float(lam),
                         seed=seed + 7919 * state["calls"], two_sided=True)
        pr = res["pairs"]
        return {(int(j), int(k)) for j, k in zip(pr["j"], pr["k"])}

    return screen


def lasso_interactions(X, Y, lambdas, screen, tol: float = 1e-10, max_sweeps: int = 10_000,
                       max_rounds: int = 100) -> LassoPath:
    """Algorithm 3 on a decreasing grid ``lambdas``.  X: (n, p) array (int8 +-1
    or real), Y: (n,).  ``screen(r, lam)`` returns the interactions (j, k), j < k,
    violating the KKT condition at residual r (``xyz_screen`` for the GPU search).
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    n, p = X.shape
    Xc = X - X.mean(axis=0)
    Yc = Y - Y.mean()
    Xsq = X * X
    Xsq_c = Xsq - Xsq.mean(axis=0)           # centred squares (zero columns for +-1 data)

    def wcol(j, k):
        w = X[:, j] * X[:, k]
        return w - w.mean()

    A, B = [], []                              # active main effects, active interactions (ordered)
    coefA, coefB = {}, {}
    path = LassoPath(lambdas)
    for lam in lambdas:
        rounds = 0
        while True:
            rounds += 1
            M = np.column_stack([Xc[:, j] for j in A] + [wcol(j, k) for j, k in B]) if (A or B) \
                else np.zeros((n, 0))
            c0 = np.array([coefA.get(j, 0.0) for j in A] + [coefB.get(b, 0.0) for b in B], dtype=np.float64)
            c, r = _cd(M, Yc, lam, c0, tol, max_sweeps) if M.shape[1] else (c0, Yc.copy())
            coefA = {j: c[q] for q, j in enumerate(A)}
            coefB = {b: c[len(A) + q] for q, b in enumerate(B)}
            # KKT violators outside the active sets
            inA, inB = set(A), set(B)
            gmain = np.abs(Xc.T @ r) / n
            U = [j for j in np.flatnonzero(gmain > lam).tolist() if j not in inA]
            gsq = np.abs(Xsq_c.T @ r) / n
            V = [(j, j) for j in np.flatnonzero(gsq > lam).tolist() if (j, j) not in inB]
            V += sorted(pq for pq in screen(r, lam) if pq not in inB)
            if not U and not V or rounds >= max_rounds:
                break
            A += U
            B += V
        path.main.append({j: v for j, v in coefA.items() if v != 0.0})
        path.inter.append({b: v for b, v in coefB.items() if v != 0.0})
        path.rounds.append(rounds)
    return path
