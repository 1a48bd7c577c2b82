"""Pins of the CPU oracle's selection against facts fixed outside the oracle.

Brute force (a library sort), closed forms (permutations, constants, min/max),
the hand-worked golden example, permutation invariance (Section 5.3) and the
defining invariant #(x<m) < k <= #(x<=m) with m in x (Section 1).
"""
import itertools
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "median9.txt")


def _bits(v, dtype):
    return int(np.array([v], dtype=dtype).view(np.uint32 if dtype == np.float32 else np.uint64)[0])


def _brute(x, k):
    s = np.sort(x.astype(np.float64), kind="stable")
    m = s[k - 1] + 0.0
    return m, int(np.sum(x < m)), int(np.sum(x == m))


def test_golden_select(oracle_mod):
    x = None
    rows = []
    for line in open(GOLDEN):
        if line.startswith("x:"):
            x = np.array([float(t) for t in line[2:].split()])
        elif line.startswith("select:"):
            rows.append([float(t) for t in line.split()[1:]])
    assert x is not None and len(rows) == 9
    for dt in (np.float32, np.float64):
        xx = x.astype(dt)
        for k, v, less, eq, gt in rows:
            r = oracle_mod.select_kth(xx, int(k))
            assert r["value"] == v and r["less"] == less and r["equal"] == eq and r["greater"] == gt


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_exhaustive_small_alphabet(oracle_mod, dtype):
    # every array of length <= 6 over an alphabet with duplicates and both zeros
    alphabet = [-1.5, -0.0, 0.0, 2.0]
    for n in range(1, 7):
        for combo in itertools.product(alphabet, repeat=n):
            x = np.array(combo, dtype=dtype)
            for k in range(1, n + 1):
                r = oracle_mod.select_kth(x, k)
                m, less, eq = _brute(x, k)
                assert r["value"] == m
                assert r["value_bits"] == _bits(m, dtype)  # canonical +0.0
                assert (r["less"], r["equal"], r["greater"]) == (less, eq, n - less - eq)


@pytest.mark.parametrize("dist", ["uniform", "normal", "cauchy", "quantized_normal", "lognormal",
                                  "mix2", "mix3", "smallint", "outliers"])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_random_vs_sort(oracle_mod, dist, dtype):
    rng = np.random.default_rng(5)
    for trial in range(4):
        n = int(rng.integers(1, 10_000))
        x = workloads.single_array(dist, n, dtype, seed=trial, tag="oracle-pin")
        for k in {1, n, (n + 1) // 2, int(rng.integers(1, n + 1))}:
            r = oracle_mod.select_kth(x, k)
            m, less, eq = _brute(x, k)
            assert r["value"] == m and r["less"] == less and r["equal"] == eq
            # the defining invariant: m is an element and #(x<m) < k <= #(x<=m)
            assert np.any(x == r["value"])
            assert r["less"] < k <= r["less"] + r["equal"]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_closed_forms(oracle_mod, dtype):
    n = 50_001
    perm = workloads.single_array("permutation", n, dtype, seed=3)
    for k in (1, 2, 17, n // 2, n - 1, n):
        r = oracle_mod.select_kth(perm, k)
        assert r["value"] == k - 1 and r["less"] == k - 1 and r["equal"] == 1
    const = workloads.single_array("constant", 1000, dtype, seed=4)
    for k in (1, 500, 1000):
        r = oracle_mod.select_kth(const, k)
        assert r["value"] == float(const[0]) and r["equal"] == 1000 and r["less"] == 0
    x = workloads.single_array("normal", 12_345, dtype, seed=9)
    assert oracle_mod.select_kth(x, 1)["value"] == float(np.min(x))
    assert oracle_mod.select_kth(x, x.size)["value"] == float(np.max(x))


def test_permutation_invariance(oracle_mod):
    # Section 5.3: the result does not depend on the order of the data
    x = workloads.single_array("mix1", 20_000, np.float64, seed=1)
    rng = np.random.default_rng(0)
    for k in (1, 333, 10_000, 19_999):
        ref = oracle_mod.select_kth(x, k)
        for y in (np.sort(x), np.sort(x)[::-1].copy(), rng.permutation(x)):
            assert oracle_mod.select_kth(y, k) == ref


def test_errors(oracle_mod):
    x = np.array([1.0, np.nan, 2.0])
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.select_kth(x, 1)
    y = np.array([1.0, 2.0])
    for k in (0, 3, -1):
        with pytest.raises(oracle_mod.OracleError):
            oracle_mod.select_kth(y, k)


def test_infinities(oracle_mod):
    x = np.array([np.inf, -np.inf, 1.0, -np.inf, 0.5, np.inf, np.inf], dtype=np.float32)
    s = np.sort(x)
    for k in range(1, x.size + 1):
        r = oracle_mod.select_kth(x, k)
        assert r["value"] == s[k - 1]
