"""Closed forms of the paper used as test oracles -- TEST INFRASTRUCTURE ONLY.

Each function states the passage it follows.  Strength gamma in (0, 1) is
the fraction of rows with Y_i = X_ij X_ik (eq. (3)), related to the
inner-product scale by 2 gamma - 1 = Y^T(X_j o X_k)/n (eq. (4)).
"""
from __future__ import annotations

import math
import numpy as np


def gamma_from_stat(stat: float) -> float:
    """eq. (4): gamma = (1 + s/n) / 2."""
    return 0.5 * (1.0 + stat)


def eta(gamma: float, M: int, L: int) -> float:
    """eq. (9): probability that a pair of strength gamma is found in L repetitions."""
    return 1.0 - (1.0 - gamma ** M) ** L


def L_for(eta_target: float, beta: float) -> int:
    """eq. (15): the smallest L with 1 - (1 - beta)^L >= eta_target (beta = gamma^M)."""
    if beta >= 1.0:
        return 1
    if beta <= 0.0:
        raise ValueError("beta must be positive")
    return int(math.ceil(math.log(1.0 - eta_target) / math.log(1.0 - beta)))


def exponent(gamma: float, gamma0: float) -> float:
    """Theorem 2 / eq. (10): the run time grows like p^(1 + log(gamma)/log(gamma0))."""
    return 1.0 + math.log(gamma) / math.log(gamma0)


def gamma0(p: int, M: int) -> float:
    """Theorem 2: gamma_0 = p^(-1/M)."""
    return p ** (-1.0 / M)


def naive_miss(p: int, L: int) -> float:
    """Section 5.3: chance that p*L uniformly drawn pairs all miss one given pair."""
    return (1.0 - 2.0 / (p * (p - 1.0))) ** (L * p)


def cost(M: int, L: int, n: int, p: int, sum_gamma_M: float) -> float:
    """eq. (8): C(M, L) = np + L {M p + p log p + n E|E_1|}, E|E_1| = sum_jk gamma_jk^M."""
    return n * p + L * (M * p + p * math.log(p) + n * sum_gamma_M)


def sum_gamma_pow(gammas_sample: np.ndarray, total_pairs: float, M: int) -> float:
    """Plug-in estimate of sum over all pairs of gamma_jk^M from uniformly sampled
    strengths (Section 2.3: 'estimated by sampling from {gamma_jk}')."""
    g = np.asarray(gammas_sample, dtype=np.float64)
    return float(total_pairs * np.mean(g ** M))


def objective(M: int, gamma: float, n: int, p: int, sum_gamma_M: float) -> float:
    """The quantity minimised in eq. (11)."""
    b = gamma ** M
    if b >= 1.0:
        return M * p + p * math.log(p) + n * sum_gamma_M
    return -(M * p + p * math.log(p) + n * sum_gamma_M) / math.log(1.0 - b)


def M_star(gamma: float, n: int, p: int, gammas_sample: np.ndarray, total_pairs: float,
           M_max: int = 64) -> int:
    """eq. (11): the subsample size minimising cost per unit of -log(miss probability)."""
    best, best_v = 1, math.inf
    for M in range(1, M_max + 1):
        v = objective(M, gamma, n, p, sum_gamma_pow(gammas_sample, total_pairs, M))
        if v < best_v:
            best, best_v = M, v
    return best


def expected_candidates(gammas: np.ndarray, M: int) -> float:
    """Proof of Theorem 2: E|E_1| = sum over pairs of gamma_jk^M."""
    return float(np.sum(np.asarray(gammas, dtype=np.float64) ** M))


def gamma_tilde(XsT: np.ndarray, Y: np.ndarray, j: int, k: int) -> float:
    """Section 3.1: |Y|-weighted strength, the sum of |Y_i| over rows with
    sgn(Y_i) = X_ij X_ik, divided by ||Y||_1.  XsT: (p, n) +-1 signs."""
    Y = np.asarray(Y, dtype=np.float64)
    sg = np.where(Y < 0, -1, 1)
    agree = sg == (XsT[j].astype(np.int64) * XsT[k].astype(np.int64))
    return float(np.abs(Y)[agree].sum() / np.abs(Y).sum())


def gamma_example_unweighted(sigma2: float) -> float:
    """Section 3.1 example, Y = X_1 X_2 + eps with eps ~ N(0, sigma^2):
    1/2 (1 + P(|eps| < 1)), the quantity the paper's sigma^2 table lists."""
    return 0.5 * (1.0 + math.erf(1.0 / math.sqrt(2.0 * sigma2)))


def gamma_unbiased(XT: np.ndarray, Y: np.ndarray, j: int, k: int, scale: bool = True, cap=None) -> float:
    """Proposition 4 (Section 3.2): strength under the unbiased transform,
    1/2 + sum_i Y_i X_ij X_ik / (2 ||Y||_1).  With ``scale`` the rows are first
    divided by nu_i = max_j |X_ij| and Y_i multiplied by nu_i^2 (the remark after
    Proposition 4), which leaves the numerator unchanged and turns the
    denominator into 2 sum_i |Y_i| nu_i^2.  With ``cap`` the entries are first
    capped at +-cap (Section 3.2's remark on capping), cap rounded to float32:
    the proposition then holds for the capped matrix."""
    X = np.asarray(XT, dtype=np.float64)
    if cap is not None:
        c = float(np.float32(cap))
        X = np.minimum(np.maximum(X, -c), c)
    Y = np.asarray(Y, dtype=np.float64)
    num = float(np.sum(Y * X[j] * X[k]))
    w = np.abs(Y)
    if scale:
        w = w * np.max(np.abs(X), axis=0) ** 2
    return 0.5 + num / (2.0 * float(w.sum()))


# ------------------------------------------------------------------
# Section 5.1: dense Gaussian projections against minimal subsampling at an
# equal budget (the mean size of E_1 is p when every pair has strength 1/2),
# one repetition.

def M_minimal(p: int) -> int:
    """Section 5.1: subsample size M = ceil(log(1/p) / log(1/2)) of minimal subsampling."""
    return int(math.ceil(math.log(1.0 / p) / math.log(0.5) - 1e-12))


def eta_minimal(gamma: float, p: int) -> float:
    """Section 5.1 with eq. (9), L = 1: minimal subsampling finds a pair of strength gamma with
    probability gamma^M, M = M_minimal(p)."""
    return gamma ** M_minimal(p)


def tau_gauss(p: int, n: int, sd: float = 1.0) -> float:
    """Section 5.1: the close-pairs threshold of dense Gaussian projections, the (1/p)-quantile of
    |W| for the projected distance W = x_j - z_k of a pair of strength 1/2.  For +-1 data
    X_j - Z_k is 0 on agreeing rows and +-2 elsewhere, so with R ~ N(0, sd^2 I) the distance is
    exactly N(0, 4 n (1 - gamma) sd^2); the paper writes the variance as n (1 - gamma), a
    different unit that cancels from eta_gauss.  P(|W| <= tau) = erf(tau / (sigma sqrt 2))."""
    from scipy.special import erfinv
    sigma = math.sqrt(4.0 * n * 0.5) * sd
    return sigma * math.sqrt(2.0) * float(erfinv(1.0 / p))


def eta_gauss(gamma: float, p: int) -> float:
    """Section 5.1: probability that dense Gaussian projections with tau = tau_gauss(p, n) put a
    pair of strength gamma into E_1, P(|W| <= tau) for W ~ N(0, 4 n (1 - gamma)); the sd ratio
    sqrt((1 - gamma) / (1/2)) leaves erf(erfinv(1/p) sqrt(0.5 / (1 - gamma))), free of n."""
    from scipy.special import erfinv
    if gamma >= 1.0:
        return 1.0
    return math.erf(float(erfinv(1.0 / p)) * math.sqrt(0.5 / (1.0 - gamma)))
