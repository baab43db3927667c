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


def test_dag_design_setting_3():
    """Section 5.4, setting 3: rows N(0, Sigma) with Sigma from a random DAG whose
    nodes are linear in their parents plus noise of 10 % of the parents'
    variance.  Sigma is a correlation matrix, the sample correlation of many
    rows converges to it, and the design is strongly correlated (most columns
    have another column with correlation above 0.9)."""
    import synthgen
    r = np.random.default_rng(3)
    X, S = synthgen.dag_gaussian(100_000, 80, r)
    assert np.allclose(np.diag(S), 1.0) and np.allclose(S, S.T)
    assert np.linalg.eigvalsh(S).min() > 0
    E = np.corrcoef(X.T.astype(np.float64))
    assert np.abs(E - S).max() < 0.02
    strong = (np.abs(S) > 0.9).sum(1) - 1
    assert np.mean(strong > 0) > 0.7 and np.median(strong) >= 2
    # a node with parents explains 1/1.1 of its variance by them: some column's
    # best linear fit from all the others has R^2 of at least 0.909
    Sinv = np.linalg.inv(S)
    r2 = 1.0 - 1.0 / np.diag(Sinv)
    assert r2.max() > 1 / 1.1 - 1e-9
    Xs, Ys, mains, inters = synthgen.lasso_setting(300, 60, 3, seed=4)
    assert Xs.shape == (300, 60) and Xs.dtype == np.float32 and len(mains) == 20 and len(inters) == 10
    assert all(j not in mains and k not in mains for j, k in inters)
