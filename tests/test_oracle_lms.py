"""Pins of the CPU oracle's least-median-of-squares residuals (Section 6).

- Each residual equals the value obtained by exact rational arithmetic with
  one correct rounding per step (products, then the left-to-right sum over j,
  the difference, the square), computed with Python fractions: a different
  route that any fused multiply-add, reordering or dropped term would break.
- Exact fit: with the true parameters and noise-free rows whose y was formed
  in the same order, clean rows have residual 0, so the lower median is 0
  whenever fewer than half of the rows are contaminated.
- Because squaring is monotone in |d|, Med(d^2) = fl(Med(|d|)^2).
"""
from fractions import Fraction

import numpy as np

import workloads


def _fl(q: Fraction) -> float:
    return float(q)  # correctly rounded, ties to even


def _residual_exact(row, yi, b):
    s = _fl(Fraction(row[0]) * Fraction(b[0]))
    for j in range(1, len(b)):
        prod = _fl(Fraction(row[j]) * Fraction(b[j]))
        s = _fl(Fraction(s) + Fraction(prod))
    d = _fl(Fraction(yi) - Fraction(s))
    return _fl(Fraction(d) * Fraction(d)), d


def test_residuals_match_stepwise_rounding(oracle_mod):
    X, y, beta, betas = workloads.lms_problem(300, 8, 4, seed=1)
    for b in list(betas) + [beta]:
        r = oracle_mod.lms_residuals(X, y, b)
        for i in range(X.shape[0]):
            ref, _ = _residual_exact(X[i], y[i], b)
            assert r[i] == ref


def test_exact_fit_gives_zero_median(oracle_mod):
    rng = np.random.default_rng(4)
    n, p = 2001, 8
    X = rng.standard_normal((n, p))
    beta = rng.standard_normal(p)
    # noise-free y in the same left-to-right order
    s = X[:, 0] * beta[0]
    for j in range(1, p):
        s = s + X[:, j] * beta[j]
    y = s.copy()
    bad = rng.choice(n, size=int(0.3 * n), replace=False)
    y[bad] += 10.0
    r = oracle_mod.lms_residuals(X, y, beta)
    clean = np.ones(n, bool)
    clean[bad] = False
    assert np.all(r[clean] == 0.0)
    assert np.all(r[~clean] > 0.0)
    res = oracle_mod.lms_median_sq(X, y, beta[None, :])[0]
    assert res["value"] == 0.0 and res["less"] == 0 and res["equal"] == clean.sum()


def test_median_of_squares_is_square_of_median_abs(oracle_mod):
    X, y, beta, betas = workloads.lms_problem(1501, 8, 3, seed=2)
    n = X.shape[0]
    k = (n + 1) // 2
    out = oracle_mod.lms_median_sq(X, y, betas)
    for b, res in zip(betas, out):
        d = np.array([_residual_exact(X[i], y[i], b)[1] for i in range(n)])
        med_abs = np.sort(np.abs(d))[k - 1]
        assert res["value"] == med_abs * med_abs
        r = oracle_mod.lms_residuals(X, y, b)
        assert res["less"] < k <= res["less"] + res["equal"]
        assert res["less"] == int(np.sum(r < res["value"]))
