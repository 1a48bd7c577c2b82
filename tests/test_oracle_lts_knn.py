"""Pins of the oracle's least-trimmed-squares and k-nearest-neighbour functions (Section 6).

Least trimmed squares: the objective is the sum of the h smallest squared residuals; Section 6
rewrites it through the h-th order statistic m as  sum_{r < m} r + a m  with a = h - #(r < m)
(the weight rho: 1 below m, a/b at m, 0 above).  The pins: brute force over every short
integer array and every h in exact integer arithmetic (both the sorted-prefix definition and
Section 6's form), the correctly rounded sum of a sorted prefix (math.fsum) on random data,
the special cases h = 1 (the minimum) and h = n (the whole sum), constant arrays, permutation
invariance, and the agreement of m and its counts with the least-median-of-squares oracle at
h = floor((n+1)/2).

k nearest neighbours: squared Euclidean distances on integer grids (exact in float), the
k-th smallest distance against a library sort, and the mean ordinate with the a/b weight on
ties against the average over every choice of the tied points (brute force, exact rationals).
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads


# ------------------------------------------------------------------ least trimmed squares

def test_trimmed_sum_brute_force_small_integers(oracle_mod):
    alphabet = [0.0, 1.0, 2.0, 4.0]
    for n in range(1, 6):
        for r in itertools.product(alphabet, repeat=n):
            r = np.array(r)
            srt = sorted(int(v) for v in r)
            for h in range(1, n + 1):
                got = oracle_mod.trimmed_sum(r, h)
                m = srt[h - 1]
                below = sum(1 for v in srt if v < m)
                eq = sum(1 for v in srt if v == m)
                assert got["F"] == sum(srt[:h]), (r, h)
                assert (got["m"], got["below"], got["b"], got["a"]) == (m, below, eq, h - below)
                # Section 6's form through the order statistic
                assert sum(v for v in srt if v < m) + (h - below) * m == got["F"]
                assert 1 <= got["a"] <= got["b"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_trimmed_sum_matches_correctly_rounded_prefix(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    r = rng.standard_normal(10_001) ** 2 * 10.0 ** rng.uniform(-3, 3, 10_001)
    for h in (1, 2, 17, 5000, 5001, 10_000, 10_001):
        got = oracle_mod.trimmed_sum(r, h)
        exact = math.fsum(np.sort(r)[:h])
        assert abs(got["F"] - exact) <= 2 * np.finfo(np.float64).eps * exact, (h, got["F"], exact)
        assert got["m"] == np.sort(r)[h - 1]
    assert oracle_mod.trimmed_sum(r, 1)["F"] == r.min()
    assert oracle_mod.trimmed_sum(r, r.size)["F"] == pytest.approx(math.fsum(r), rel=1e-15)


def test_trimmed_sum_constant_and_permutation(oracle_mod):
    c = np.full(1001, 0.375)
    got = oracle_mod.trimmed_sum(c, 400)
    assert (got["F"], got["m"], got["below"], got["a"], got["b"]) == (150.0, 0.375, 0, 400, 1001)
    rng = np.random.default_rng(5)
    r = np.round(rng.standard_normal(2000) ** 2, 2)  # many ties
    base = oracle_mod.trimmed_sum(r, 777)
    for _ in range(3):
        assert oracle_mod.trimmed_sum(rng.permutation(r), 777) == base


def test_lts_integer_regression_exact(oracle_mod):
    """Integer design, parameters and responses: every residual is an exact integer, so the
    objective is the exact sum of the h smallest squares."""
    rng = np.random.default_rng(7)
    n, p = 301, 4
    X = rng.integers(-5, 6, size=(n, p)).astype(np.float64)
    y = rng.integers(-20, 21, size=n).astype(np.float64)
    betas = rng.integers(-3, 4, size=(6, p)).astype(np.float64)
    for h in (1, 100, (n + 1) // 2, n):
        got = oracle_mod.lts_objective(X, y, betas, h)
        for c in range(betas.shape[0]):
            res = [int(y[i]) - sum(int(X[i, j]) * int(betas[c, j]) for j in range(p)) for i in range(n)]
            sq = sorted(v * v for v in res)
            assert got[c]["F"] == sum(sq[:h]) and got[c]["m"] == sq[h - 1], (h, c)


def test_lts_median_agrees_with_lms(oracle_mod):
    X, y, _, betas = workloads.lms_problem(4097, 8, 5, seed=3)
    lts = oracle_mod.lts_objective(X, y, betas)
    lms = oracle_mod.lms_median_sq(X, y, betas)
    for c in range(5):
        assert lts[c]["m"] == lms[c]["value"]
        assert (lts[c]["below"], lts[c]["b"]) == (lms[c]["less"], lms[c]["equal"])
        assert lts[c]["a"] == (4097 + 1) // 2 - lms[c]["less"]


# ------------------------------------------------------------------ k nearest neighbours

def test_knn_distances_integer_grid(oracle_mod):
    rng = np.random.default_rng(0)
    P = rng.integers(-50, 51, size=(500, 5)).astype(np.float32)
    q = rng.integers(-50, 51, size=5).astype(np.float32)
    d = oracle_mod.knn_distances(P, q)
    want = [sum((int(P[i, j]) - int(q[j])) ** 2 for j in range(5)) for i in range(500)]
    assert d.tolist() == want
    # translation by an integer vector leaves every distance unchanged
    t = rng.integers(-100, 101, size=5).astype(np.float32)
    assert np.array_equal(oracle_mod.knn_distances(P + t, q + t), d)
    # the point itself is at distance 0
    assert oracle_mod.knn_distances(P, P[17])[17] == 0.0


def _knn_all_tie_choices(d, f, k):
    """Average over every choice of k nearest (all subsets of the tied points that complete
    the points strictly below the k-th distance) of the mean ordinate, in exact rationals."""
    order = sorted(range(len(d)), key=lambda i: d[i])
    dk = d[order[k - 1]]
    below = [i for i in range(len(d)) if d[i] < dk]
    tied = [i for i in range(len(d)) if d[i] == dk]
    a = k - len(below)
    means = []
    for pick in itertools.combinations(tied, a):
        means.append(Fraction(sum(Fraction(float(f[i])) for i in below + list(pick)), k))
    return dk, sum(means) / len(means), len(below), len(tied)


def test_knn_mean_brute_force_with_ties(oracle_mod):
    rng = np.random.default_rng(1)
    for trial in range(40):
        n, dim = int(rng.integers(1, 9)), int(rng.integers(1, 4))
        P = rng.integers(0, 3, size=(n, dim)).astype(np.float32)  # many equal distances
        f = rng.integers(-8, 9, size=n).astype(np.float32)
        Q = rng.integers(0, 3, size=(2, dim)).astype(np.float32)
        for k in range(1, n + 1):
            got = oracle_mod.knn_mean(P, f, Q, k)
            for c in range(2):
                d = [float(sum((float(P[i, j]) - float(Q[c, j])) ** 2 for j in range(dim)))
                     for i in range(n)]
                dk, mean, below, eq = _knn_all_tie_choices(d, f, k)
                assert got[c]["dk"] == dk and (got[c]["below"], got[c]["equal"]) == (below, eq)
                assert abs(Fraction(got[c]["mean"]) - mean) <= Fraction(1, 10 ** 12), (trial, k, c)


def test_knn_mean_special_cases(oracle_mod):
    rng = np.random.default_rng(2)
    P = rng.standard_normal((1000, 8)).astype(np.float32)
    f = rng.standard_normal(1000).astype(np.float32)
    Q = P[[3, 500]] + np.float32(0.0)
    one = oracle_mod.knn_mean(P, f, Q, 1)  # a query on a data point: that point
    assert one[0]["mean"] == float(f[3]) and one[1]["mean"] == float(f[500])
    assert one[0]["dk"] == 0.0
    allk = oracle_mod.knn_mean(P, f, Q, 1000)  # every point
    assert allk[0]["mean"] == pytest.approx(math.fsum(f.astype(np.float64)) / 1000, rel=1e-14)
    # no ties: the plain mean of the k nearest by a library sort of the distances
    q = rng.standard_normal((1, 8)).astype(np.float32)
    d = oracle_mod.knn_distances(P, q[0])
    idx = np.argsort(d, kind="stable")[:25]
    assert len(np.unique(d)) == d.size
    got = oracle_mod.knn_mean(P, f, q, 25)[0]
    assert got["mean"] == pytest.approx(math.fsum(f[idx].astype(np.float64)) / 25, rel=1e-14)
    assert got["dk"] == np.sort(d)[24]
