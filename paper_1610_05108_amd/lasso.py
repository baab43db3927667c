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


def _cd(M, y, lam, coef, tol, max_sweeps, polish_every: int = 25, gram_max: int = 2048):
    """Coordinate descent for 1/(2n)||y - M c||^2 + lam ||c||_1 from coef.

    Cyclic sweeps run over the coordinates that can move: the non-zero ones and
    the zero ones whose gradient |M_q^T r| / n exceeds lam (a zero coordinate
    with a smaller gradient stays zero under a coordinate step), with the
    gradient of those coordinates kept up to date through their Gram matrix
    (covariance updates).  Every `polish_every` sweeps the optimality
    conditions are solved on the current support S with its signs s,
    (M_S^T M_S / n) c_S = M_S^T y / n - lam s; the result is accepted when its
    signs are s and every other coordinate has |M_q^T r| / n <= lam, i.e. when
    it is the minimiser.  Otherwise the sweeps go on until no coordinate moves
    by more than tol, and the gradient of every coordinate is then checked at
    once.  While more than `gram_max` coordinates can move, sweeps run on the
    residual instead.  On strongly correlated designs (Section 5.4, setting 3) plain sweeps
    need 10^5 passes to settle; the support is usually right after a few dozen."""
    n, k = M.shape
    sq = np.einsum("ij,ij->j", M, M) / n
    r = y - M @ coef
    sweeps = 0
    while sweeps < max_sweeps:
        g_all = M.T @ r / n
        idx = np.flatnonzero((sq > 0.0) & ((coef != 0.0) | (np.abs(g_all) > lam)))
        if idx.size == 0:
            break
        if idx.size > gram_max:
            # too many movable coordinates for a Gram matrix (thousands of fresh violators):
            # one sweep on the residual, which leaves most of them at zero
            sweeps += 1
            moved = False
            for q in idx:
                old = coef[q]
                z = old * sq[q] + M[:, q] @ r / n
                a = abs(z) - lam
                new = (a if z > 0 else -a) / sq[q] if a > 0.0 else 0.0
                if new != old:
                    r -= M[:, q] * (new - old)
                    coef[q] = new
                    moved = True
            if not moved:
                break
            continue
        MI = np.asfortranarray(M[:, idx])
        G = np.asfortranarray(MI.T @ MI / n)
        g = g_all[idx].copy()
        c = coef[idx].copy()
        d = np.diag(G).copy()
        rd = np.sqrt(d)
        moved = False
        settled = False
        while sweeps < max_sweeps and not settled:
            for _ in range(min(polish_every, max_sweeps - sweeps)):
                sweeps += 1
                delta = 0.0
                for t in range(idx.size):
                    old = c[t]
                    z = old * d[t] + g[t]
                    a = abs(z) - lam
                    new = (a if z > 0 else -a) / d[t] if a > 0.0 else 0.0
                    if new != old:
                        g -= G[:, t] * (new - old)
                        c[t] = new
                        delta = max(delta, abs(new - old) * rd[t])
                        moved = True
                if delta < tol:
                    settled = True
                    break
            S = np.flatnonzero(c != 0.0)
            if S.size:
                MS = MI[:, S]
                sgn = np.sign(c[S])
                try:
                    cS = np.linalg.solve(G[np.ix_(S, S)], MS.T @ y / n - lam * sgn)
                except np.linalg.LinAlgError:
                    cS = None
                if cS is not None and np.all(np.sign(cS) == sgn):
                    r2 = y - MS @ cS
                    g2 = np.abs(M.T @ r2 / n)
                    g2[idx[S]] = 0.0
                    if g2.max(initial=0.0) <= lam:
                        coef[:] = 0.0
                        coef[idx[S]] = cS
                        return coef, r2
        coef[idx] = c
        r = y - M @ coef
        if not moved:
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

    # columns of the active coordinates, in the order they joined (main effects and
    # interactions interleaved), kept across rounds and lambdas; column-major so that
    # each column is contiguous for the coordinate steps
    store = np.empty((n, 64), order="F")
    keys = []                                  # ("m", j) or ("i", (j, k)) per stored column

    def append(block, names):
        nonlocal store
        need = len(keys) + block.shape[1]
        if need > store.shape[1]:
            grown = np.empty((n, max(need, 2 * store.shape[1])), order="F")
            grown[:, :len(keys)] = store[:, :len(keys)]
            store = grown
        store[:, len(keys):need] = block
        keys.extend(names)

    A, B = [], []                              # active main effects, active interactions (ordered)
    coef = np.zeros(0)
    path = LassoPath(lambdas)
    for lam in lambdas:
        rounds = 0
        while True:
            rounds += 1
            M = store[:, :len(keys)]
            c0 = np.concatenate([coef, np.zeros(len(keys) - coef.size)])
            coef, r = _cd(M, Yc, lam, c0, tol, max_sweeps) if M.shape[1] else (c0, Yc.copy())
            coefA = {name: coef[q] for q, (kind, name) in enumerate(keys) if kind == "m"}
            coefB = {name: coef[q] for q, (kind, name) in enumerate(keys) if kind == "i"}
            # KKT violators outside the active sets
            inA, inB = set(A), set(B)
            gmain = np.abs(Xc.T @ r) / n
            U = [j for j in np.flatnonzero(gmain > lam).tolist() if j not in inA]
            gsq = np.abs(Xsq_c.T @ r) / n
            V = [(j, j) for j in np.flatnonzero(gsq > lam).tolist() if (j, j) not in inB]
            V += sorted(pq for pq in screen(r, lam) if pq not in inB)
            if not U and not V or rounds >= max_rounds:
                break
            if U:
                append(Xc[:, U], [("m", j) for j in U])
            if V:
                js = np.array([j for j, _ in V])
                ks = np.array([k for _, k in V])
                W = X[:, js] * X[:, ks]
                append(W - W.mean(axis=0), [("i", pq) for pq in V])
            A += U
            B += V
        path.main.append({j: v for j, v in coefA.items() if v != 0.0})
        path.inter.append({b: v for b, v in coefB.items() if v != 0.0})
        path.rounds.append(rounds)
    return path
