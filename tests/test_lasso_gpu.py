"""Algorithm 3 with the interaction KKT check of eq. (16) done by the GPU search
(two-sided, Y = residual): with m = 2 sampled rows a pair of strength >= 1/2
collides with probability >= 1/4 per repetition, so L = 200 repetitions miss a
violator with probability below 1e-24 and the path must equal the one computed
with an exact screen; the KKT conditions must hold on the full design."""
import itertools

import numpy as np
import pytest

import paper_1610_05108_amd as xyz
from paper_1610_05108_amd.lasso import lasso_interactions, xyz_screen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = xyz.Context(0)
    yield c
    c.close()


def _exact_screen(X):
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    pairs = list(itertools.combinations(range(p), 2))
    W = np.column_stack([X[:, j] * X[:, k] for j, k in pairs])

    def screen(r, lam):
        return {pairs[q] for q in np.flatnonzero(np.abs(W.T @ r) / n > lam)}
    return screen


def _same_path(a, b):
    for l in range(len(a.lambdas)):
        assert set(a.main[l]) == set(b.main[l]) and set(a.inter[l]) == set(b.inter[l]), l
        for j in a.main[l]:
            assert abs(a.main[l][j] - b.main[l][j]) < 1e-9
        for q in a.inter[l]:
            assert abs(a.inter[l][q] - b.inter[l][q]) < 1e-9


def _kkt_full(X, Y, path, slack=1e-7):
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    Xc, Yc = X - X.mean(0), Y - Y.mean()
    for l, lam in enumerate(path.lambdas):
        fit = np.zeros(n)
        for j, v in path.main[l].items():
            fit += v * Xc[:, j]
        for (j, k), v in path.inter[l].items():
            w = X[:, j] * X[:, k]
            fit += v * (w - w.mean())
        r = Yc - fit
        assert np.abs(Xc.T @ r).max() / n <= lam + slack
        for j in range(p):
            for k in range(j, p):
                w = X[:, j] * X[:, k]
                assert abs((w - w.mean()) @ r) / n <= lam + slack, (l, j, k)


@pytest.mark.parametrize("binary", [True, False])
def test_gpu_screen_path_equals_exact(ctx, binary):
    r = np.random.default_rng(5)
    n, p = 400, 40 if not binary else 60
    if binary:
        X = np.where(r.random((n, p)) < 0.5, 1, -1).astype(np.int8)
        Xf = X.astype(np.float64)
        Y = 2.0 * Xf[:, 3] * Xf[:, 7] - Xf[:, 1] + 0.7 * Xf[:, 10] * Xf[:, 22] + 0.5 * r.standard_normal(n)
        x = ctx.x_create(np.ascontiguousarray(X.T))
        lambdas = [0.9, 0.5, 0.25, 0.12]
    else:
        X = r.standard_normal((n, p)).astype(np.float32)
        Xf = X.astype(np.float64)
        Y = 1.5 * Xf[:, 0] * Xf[:, 1] - Xf[:, 2] + 0.8 * Xf[:, 3] * Xf[:, 5] + 0.3 * r.standard_normal(n)
        x = ctx.x_create(np.ascontiguousarray(X.T))
        lambdas = [1.0, 0.5, 0.25, 0.12]
    gpu = lasso_interactions(X, Y, lambdas, xyz_screen(ctx, x, m=2, L=200, seed=1))
    ref = lasso_interactions(X, Y, lambdas, _exact_screen(X))
    _same_path(gpu, ref)
    _kkt_full(X, Y, gpu)


def test_gpu_screen_path_equals_exact_correlated_design(ctx):
    """Section 5.4's setting 3: the non-hierarchical model on the strongly
    correlated DAG design, where products of columns correlated with the true
    pairs also predict Y; the screened path must still equal the exact one."""
    import synthgen
    X, Y, mains, inters = synthgen.lasso_setting(400, 40, 3, seed=7)
    Xc = X.astype(np.float64) - X.mean(0)
    lam_max = float(np.abs(Xc.T @ (Y - Y.mean())).max() / 400)
    lambdas = list(lam_max * np.array([1.0, 0.5, 0.25, 0.12]))
    x = ctx.x_create(np.ascontiguousarray(X.T))
    gpu = lasso_interactions(X, Y, lambdas, xyz_screen(ctx, x, m=2, L=200, seed=1))
    ref = lasso_interactions(X, Y, lambdas, _exact_screen(X))
    _same_path(gpu, ref)
    _kkt_full(X, Y, gpu)
    assert len(gpu.inter[-1]) > 0
