"""Algorithm 3 (Section 4): the active-set Lasso over all main effects and
pairwise interactions, with an exact interaction screen, against scikit-learn's
coordinate-descent Lasso on the explicit design of eq. (17) (centred X, all
centred products X_j o X_k with j <= k), at every lambda of the grid."""
import itertools

import numpy as np
from sklearn.linear_model import Lasso

from paper_1610_05108_amd.lasso import lasso_interactions


def _exact_screen(X):
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    pairs = list(itertools.combinations(range(p), 2))
    W = np.column_stack([X[:, j] * X[:, k] for j, k in pairs])

    def screen(r, lam):
        g = np.abs(W.T @ r) / n
        return {pairs[q] for q in np.flatnonzero(g > lam)}
    return screen


def _full_design(X):
    n, p = X.shape
    Xc = X - X.mean(axis=0)
    names, cols = [], []
    for j in range(p):
        names.append(("m", j))
        cols.append(Xc[:, j])
    for j in range(p):
        for k in range(j, p):
            w = X[:, j] * X[:, k]
            names.append(("i", (j, k)))
            cols.append(w - w.mean())
    return names, np.column_stack(cols)


def _compare(X, Y, lambdas):
    path = lasso_interactions(X, Y, lambdas, _exact_screen(X))
    names, D = _full_design(np.asarray(X, dtype=np.float64))
    Yc = Y - Y.mean()
    for l, lam in enumerate(lambdas):
        sk = Lasso(alpha=lam, fit_intercept=False, tol=1e-13, max_iter=1_000_000).fit(D, Yc)
        ours = np.zeros(len(names))
        for q, (kind, key) in enumerate(names):
            ours[q] = (path.main[l] if kind == "m" else path.inter[l]).get(key, 0.0)
        assert np.max(np.abs(ours - sk.coef_)) < 1e-6, (lam, np.max(np.abs(ours - sk.coef_)))
    return path


def test_continuous_design_matches_full_lasso():
    r = np.random.default_rng(3)
    n, p = 200, 12
    X = r.standard_normal((n, p))
    Y = 1.5 * X[:, 0] * X[:, 1] - X[:, 2] + 0.8 * X[:, 3] * X[:, 5] + 0.5 * X[:, 4] ** 2 + 0.3 * r.standard_normal(n)
    Xc, Yc = X - X.mean(0), Y - Y.mean()
    lam_max = max(np.abs(Xc.T @ Yc).max(), np.abs(((X[:, :, None] * X[:, None, :]).reshape(n, -1)
                                                     - (X[:, :, None] * X[:, None, :]).reshape(n, -1).mean(0)).T
                                                    @ Yc).max()) / n
    path = _compare(X, Y, lam_max * np.array([0.6, 0.3, 0.15, 0.08, 0.04]))
    assert (0, 1) in path.inter[-1] and (3, 5) in path.inter[-1] and 2 in path.main[-1]


def test_binary_design_matches_full_lasso():
    r = np.random.default_rng(4)
    n, p = 300, 15
    X = np.where(r.random((n, p)) < 0.5, 1, -1).astype(np.int8)
    Xf = X.astype(np.float64)
    Y = 2.0 * Xf[:, 3] * Xf[:, 7] - Xf[:, 1] + 0.5 * r.standard_normal(n)
    path = _compare(X, Y, np.array([0.9, 0.5, 0.2, 0.1]))
    assert (3, 7) in path.inter[-1]
    # squares of +-1 columns are constant: never selected
    assert all(j != k for j, k in path.inter[-1])
