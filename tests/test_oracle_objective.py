"""Pins of the CPU oracle's objective f(y) against facts fixed outside it.

- Eq. 1 (Section 3): for odd n and the median rank the weights are equal,
  so f(y) = (n/2) * sum |x_i - y| exactly as a different formula.
- The minimiser over the data of f is x_(k) (Eq. 2 with the orientation that
  selects the k-th smallest), checked by brute force for every k.
- Step 0 of the cutting plane (Section 4): f and g at the data extremes in
  closed form from min, max and sum(x).
- Integer data x_i = i: A, B, counts, pred and succ are integer polynomials.
- Convexity / supporting lines: f(z) >= f(y) + g (z - y) for g in {g-, g+}.
- The hand-worked golden example.
"""
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "median9.txt")


def test_golden_objective(oracle_mod):
    x = None
    rows = []
    gmin = gmax = None
    for line in open(GOLDEN):
        if line.startswith("x:"):
            x = np.array([float(t) for t in line[2:].split()])
        elif line.startswith("objective:"):
            rows.append([float(t) for t in line.split()[1:]])
        elif line.startswith("gplus_at_min:"):
            gmin = float(line.split()[1])
        elif line.startswith("gminus_at_max:"):
            gmax = float(line.split()[1])
    k = 5
    out = oracle_mod.objective(x, k, [r[0] for r in rows])
    for o, (y, sabs, f, L, E, G) in zip(out, rows):
        assert o["f"] == f and (o["L"], o["E"], o["G"]) == (L, E, G)
        assert o["A"] + o["B"] == sabs
    ext = oracle_mod.objective(x, k, [x.min(), x.max()])
    assert ext[0]["gplus"] == gmin and ext[1]["gminus"] == gmax


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_eq1_median_weights(oracle_mod, dtype):
    n = 4001  # odd: alpha = beta = n/2 at the median
    x = workloads.single_array("normal", n, dtype, seed=2)
    k = (n + 1) // 2
    ys = np.concatenate([np.linspace(-4, 4, 37), x[:20].astype(np.float64)])
    out = oracle_mod.objective(x, k, ys)
    xd = x.astype(np.float64)
    for o, y in zip(out, ys):
        ref = (n / 2.0) * np.sum(np.abs(xd - y))
        assert abs(o["f"] - ref) <= 1e-12 * ref


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_argmin_over_data_is_kth(oracle_mod, dtype):
    rng = np.random.default_rng(11)
    for trial in range(30):
        n = int(rng.integers(1, 40))
        x = rng.integers(-5, 6, n).astype(dtype) * 0.75  # duplicates on purpose
        s = np.sort(x)
        for k in range(1, n + 1):
            out = oracle_mod.objective(x, k, x.astype(np.float64))
            j = int(np.argmin(out["f"]))
            assert x[j] == s[k - 1]
            # the minimiser is unique over the data: every other value is strictly worse
            worse = out["f"][x != s[k - 1]]
            assert np.all(worse > out["f"][j])
            # 0 in the subdifferential exactly there
            o = out[j]
            assert o["gminus"] < 0 < o["gplus"]


def test_step0_closed_forms(oracle_mod):
    # integer-valued data so that sum(x) and the products are exact
    rng = np.random.default_rng(3)
    for trial in range(10):
        n = int(rng.integers(2, 3000))
        x = rng.integers(-1000, 1000, n).astype(np.float64)
        k = int(rng.integers(1, n + 1))
        alpha, beta = k - 0.5, n - k + 0.5
        lo, hi, S = x.min(), x.max(), x.sum()
        out = oracle_mod.objective(x, k, [lo, hi])
        assert out[0]["f"] == alpha * (S - n * lo)
        assert out[1]["f"] == beta * (n * hi - S)
        nmin, nmax = int(np.sum(x == lo)), int(np.sum(x == hi))
        assert out[0]["gplus"] == n * (nmin - k + 0.5)
        assert out[1]["gminus"] == n * (n - nmax - k + 0.5)
        assert out[0]["pred"] == -np.inf and out[1]["succ"] == np.inf


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_integer_data_polynomials(oracle_mod, dtype):
    n = 1000
    x = workloads.single_array("permutation", n, dtype, seed=8)  # a shuffle of 0..n-1
    k = 300
    ys = np.array([0, 1, 17, 499, 998, 999, 0.5, 17.5, 998.5, -3.0, 1003.0])
    out = oracle_mod.objective(x, k, ys)
    for o, y in zip(out, ys):
        if float(y).is_integer() and 0 <= y <= n - 1:
            j = int(y)
            B = j * (j + 1) / 2
            A = (n - 1 - j) * (n - j) / 2
            L, E = j, 1
            pred = j - 1 if j > 0 else -np.inf
            succ = j + 1 if j < n - 1 else np.inf
        elif 0 <= y <= n - 1:
            j = int(np.floor(y))
            B = (j + 1) ** 2 / 2
            A = (n - 1 - j) ** 2 / 2
            L, E = j + 1, 0
            pred, succ = j, j + 1
        elif y < 0:
            B, A, L, E = 0.0, n * (n - 1) / 2 - n * y, 0, 0
            pred, succ = -np.inf, 0
        else:
            B, A, L, E = n * y - n * (n - 1) / 2, 0.0, n, 0
            pred, succ = n - 1, np.inf
        assert o["A"] == A and o["B"] == B
        assert (o["L"], o["E"], o["G"]) == (L, E, n - L - E)
        assert o["pred"] == pred and o["succ"] == succ
        assert o["f"] == (k - 0.5) * A + (n - k + 0.5) * B


def test_supporting_lines(oracle_mod):
    x = workloads.single_array("lognormal", 3000, np.float64, seed=6)
    k = 1234
    rng = np.random.default_rng(1)
    ys = np.concatenate([rng.uniform(0, 5, 20), x[:10]])
    zs = rng.uniform(-1, 8, 50)
    oy = oracle_mod.objective(x, k, ys)
    oz = oracle_mod.objective(x, k, zs)
    for o, y in zip(oy, ys):
        for g in (o["gminus"], o["gplus"]):
            lower = o["f"] + g * (zs - y)
            assert np.all(oz["f"] >= lower - 1e-9 * np.abs(oz["f"]))
        # one-sided difference quotients approach g+ and g- when no data point is crossed
        h = 1e-7
        fr = oracle_mod.objective(x, k, [y + h, y - h])
        if not np.any((x > y) & (x <= y + h)):
            assert abs((fr[0]["f"] - o["f"]) / h - o["gplus"]) <= 1e-6 * abs(o["gplus"]) + 1.0
        if not np.any((x < y) & (x >= y - h)):
            assert abs((o["f"] - fr[1]["f"]) / h - o["gminus"]) <= 1e-6 * abs(o["gminus"]) + 1.0


def test_f32_widening_matches_f64(oracle_mod):
    x = workloads.single_array("cauchy", 5000, np.float32, seed=7)
    ys = [-3.0, 0.1, 0.25, 7.5]
    a = oracle_mod.objective(x, 77, ys)
    b = oracle_mod.objective(x.astype(np.float64), 77, ys)
    assert np.array_equal(a, b)


def test_nan_rejected(oracle_mod):
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.objective(np.array([1.0, np.nan]), 1, [0.0])
