"""The cutting-plane state machine (csrc/cp_state.h) driven on the CPU.

tests/cpp/cp_state_sim.cpp runs the kernel's sequence of passes with plain
loops around the same header the GPU uses; its results are compared with the
oracle bit for bit, for every option that changes the path: final thresholds,
splitting on/off, bisection only (maxit 0), proposed brackets that hold or miss
x_(k), infinities, duplicates and outliers (Section 5.3's ~1e9 values).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


class SimResult(ctypes.Structure):
    _fields_ = [("value", ctypes.c_double), ("less", ctypes.c_int64), ("equal", ctypes.c_int64),
                ("status", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("work_passes", ctypes.c_int32), ("kelley", ctypes.c_int32),
                ("bisect", ctypes.c_int32), ("bracket_used", ctypes.c_int32),
                ("elements_read", ctypes.c_int64), ("elements_written", ctypes.c_int64)]


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    out = tmp_path_factory.mktemp("sim") / "libcpsim.so"
    src = os.path.join(HERE, "cpp", "cp_state_sim.cpp")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", str(out), src], check=True)
    L = ctypes.CDLL(str(out))
    for name in ("sim_select_f32", "sim_select_f64"):
        fn = getattr(L, name)
        fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int64,
                       ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                       ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                       ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(SimResult)]
        fn.restype = ctypes.c_int

    def run(x, k, maxit=64, final_threshold=64, theta=0.5, bracket=None, p0_split=False,
            p0_cap=None, hist_bits=0, count_first=0, hist_compact=1, p0_sums=1, spec_mode=0,
            transform=0):
        r = SimResult()
        fn = L.sim_select_f32 if x.dtype == np.float32 else L.sim_select_f64
        ub = 1 if bracket is not None else 0
        blo, bhi = bracket if bracket is not None else (0.0, 0.0)
        cap = x.size if p0_cap is None else p0_cap
        rc = fn(x.ctypes.data, x.size, k, maxit, final_threshold, theta, ub, blo, bhi,
                1 if p0_split else 0, cap, hist_bits, count_first, hist_compact, p0_sums,
                spec_mode, transform, ctypes.byref(r))
        assert rc == 0, rc
        return r
    return run


def _check(r, ref, ctx):
    assert r.status == 0, ctx
    assert r.value == ref["value"], (ctx, r.value, ref["value"])
    assert (r.less, r.equal) == (ref["less"], ref["equal"]), ctx


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("dist", ["uniform", "normal", "cauchy", "quantized_normal", "lognormal",
                                  "mix2", "mix3", "smallint", "outliers", "outliers20", "constant",
                                  "permutation"])
def test_state_machine_matches_oracle(sim, oracle_mod, dist, dtype):
    for n in (1, 2, 3, 10, 333, 4096, 50_001):
        x = workloads.single_array(dist, n, dtype, seed=n, tag="sim")
        for k in sorted({1, 2, n // 100 or 1, n // 3 or 1, (n + 1) // 2, n - 1 or 1, n}):
            if k > n:
                continue
            ref = oracle_mod.select_kth(x, k)
            for opts in (dict(), dict(final_threshold=1), dict(final_threshold=4, theta=0.0),
                         dict(maxit=0, final_threshold=8), dict(maxit=2, final_threshold=2, theta=1.0),
                         dict(hist_bits=12), dict(hist_bits=2, final_threshold=1),
                         dict(hist_bits=1, final_threshold=1, theta=1.0),
                         dict(hist_bits=12, theta=1.0, count_first=1),
                         dict(hist_bits=1, final_threshold=1, theta=1.0, count_first=1),
                         dict(hist_bits=3, final_threshold=2, theta=0.5, count_first=1),
                         dict(hist_bits=11, theta=1.0, count_first=1, hist_compact=0),
                         dict(hist_bits=2, final_threshold=1, theta=0.5, count_first=1,
                              hist_compact=0),
                         dict(hist_bits=12, theta=1.0, count_first=1, spec_mode=1),
                         dict(hist_bits=3, final_threshold=2, theta=1.0, count_first=1,
                              spec_mode=1),
                         dict(hist_bits=12, final_threshold=4, theta=1.0, count_first=1,
                              spec_mode=2),
                         dict(transform=1, theta=0.0, final_threshold=4),
                         dict(transform=1, maxit=3, theta=0.0, final_threshold=1),
                         dict(transform=1, hist_bits=12, theta=1.0, count_first=1)):
                _check(sim(x, k, **opts), ref, (dist, n, k, opts))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_infinities_and_zeros(sim, oracle_mod, dtype):
    rng = np.random.default_rng(2)
    base = [np.inf, -np.inf, 0.0, -0.0, 1.0, -1.0, 2.5, np.inf, -np.inf, 3.0, -0.0]
    for trial in range(40):
        x = np.array(rng.choice(base, size=int(rng.integers(1, 60))), dtype=dtype)
        for k in range(1, x.size + 1):
            ref = oracle_mod.select_kth(x, k)
            for opts in (dict(final_threshold=1), dict(maxit=0, final_threshold=1),
                         dict(final_threshold=1, theta=1.0, hist_bits=1),
                         dict(final_threshold=1, theta=1.0, hist_bits=3),
                         dict(final_threshold=1, theta=1.0, hist_bits=2, count_first=1)):
                _check(sim(x, k, **opts), ref, (x, k, opts))


def _expected_ends(x, k, a, b):
    """Which proposed ends the counts prove (bit 0: a, bit 1: b), or 0 when pass 0 already
    answers (x_(k) is the minimum or the maximum)."""
    lo, hi = x.min(), x.max()
    if k <= np.sum(x == lo) or k > x.size - np.sum(x == hi):
        return 0
    a, b = np.array(a, x.dtype), np.array(b, x.dtype)
    left = np.sum(x <= a) < k and a > lo
    right = k <= np.sum(x < b) and b < hi
    return int(left) | (int(right) << 1)


@pytest.mark.parametrize("p0_split", [False, True])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_proposed_brackets(sim, oracle_mod, dtype, p0_split):
    x = workloads.single_array("normal", 100_000, dtype, seed=4)
    s = np.sort(x)
    for k in (1, 2, 10, 5000, 50_000, 99_999, 100_000):
        ref = oracle_mod.select_kth(x, k)
        v = s[k - 1]
        for (a, b) in [(v - 0.01, v + 0.01), (v - 1e-7, v + 1e-7), (v, v + 1.0), (v - 1.0, v),
                       (-10.0, 10.0), (v + 0.5, v + 1.0), (v - 1.0, v - 0.5), (3.0, -3.0),
                       (v - 0.3, v + 1e-9), (-np.inf, v + 0.2), (v - 0.2, np.inf),
                       (np.nan, v + 0.1), (v - 0.1, np.nan)]:
            for cap, hb, sums in ((None, 0, 1), (10, 0, 1), (None, 12, 1), (None, 3, 1),
                                  (None, 12, 0), (10, 3, 0)):
                r = sim(x, k, final_threshold=16, bracket=(float(a), float(b)),
                        p0_split=p0_split, p0_cap=cap, hist_bits=hb, count_first=int(hb == 3),
                        p0_sums=sums)
                _check(r, ref, (k, a, b, cap, hb))
                assert r.bracket_used == _expected_ends(x, k, a, b), (k, a, b)
                xa, xb = np.array(a, dtype), np.array(b, dtype)
                inside = int(np.sum((x > xa) & (x < xb)))
                fits = cap is None or inside <= cap
                beyond = (r.bracket_used & 1 or xa <= x.min()) and (r.bracket_used & 2 or xb >= x.max())
                adopted = p0_split and fits and (r.bracket_used == 3 or
                                                 (hb > 0 and r.bracket_used and beyond and xa < xb))
                # an adopted pass-0 split spares the evaluation passes over x
                if adopted:
                    assert r.passes == 1, (k, a, b, hb, r.passes)


def test_passes_halve_on_smooth_data(sim):
    # The cutting plane behaves like bisection near x_(k) (end of Section 4): the number of
    # passes grows like log2(n / final_threshold), far below the bisection safeguard's bound.
    n = 1 << 20
    x = workloads.single_array("uniform", n, np.float32, seed=0)
    r = sim(x, (n + 1) // 2, final_threshold=4096)
    assert r.work_passes <= 14
    assert r.passes <= 4  # pass 0, two evaluations of the whole input and the split pass
    assert r.elements_read <= 6 * n


def test_bisection_bound(sim, oracle_mod):
    # maxit = 0: only bit-pattern bisection; at most 32 halvings of the key range for float32
    x = workloads.single_array("cauchy", 20_000, np.float32, seed=1)
    ref = oracle_mod.select_kth(x, 777)
    r = sim(x, 777, maxit=0, final_threshold=1)
    _check(r, ref, "bisect")
    assert r.kelley == 0 and r.bisect <= 34


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_histogram_select_edges(sim, oracle_mod, dtype):
    """The key-histogram finish around signed zeros, denormals and one-key bins."""
    tiny = np.finfo(dtype).smallest_subnormal
    vals = np.array([-0.0, 0.0, tiny, -tiny, 2 * tiny, -2 * tiny, 1.0, -1.0, 1e-30, -1e-30],
                    dtype=dtype)
    rng = np.random.default_rng(9)
    for trial in range(30):
        x = rng.choice(vals, size=int(rng.integers(50, 400))).astype(dtype)
        for k in (1, 2, x.size // 3, x.size // 2, x.size - 1, x.size):
            ref = oracle_mod.select_kth(x, k)
            for hb in (1, 2, 4, 12):
                for cf in (0, 1):
                    _check(sim(x, k, final_threshold=1, theta=1.0, hist_bits=hb, count_first=cf),
                           ref, (trial, k, hb, cf))


def test_histogram_finish_cuts_passes(sim):
    n = 1 << 20
    x = workloads.single_array("normal", n, np.float32, seed=3)
    plain = sim(x, (n + 1) // 2, final_threshold=4096)
    hist = sim(x, (n + 1) // 2, final_threshold=4096, hist_bits=12)
    assert hist.work_passes < plain.work_passes and hist.work_passes <= 7


@pytest.mark.parametrize("dist", ["normal", "uniform", "cauchy", "quantized_normal"])
def test_counted_split_and_compaction(sim, oracle_mod, dist):
    """Splitting from the first trial point with the histogram finish: the split counts
    both parts in key bins, so the part holding x_(k) narrows without a pass of its own,
    and a narrowed bracket far smaller than its part is compacted by the histogram pass
    that follows.  Values stay exact; the passes read at most three inputs' worth (pass 0,
    the split, and one pass over the part that holds x_(k))."""
    n = 1 << 20
    x = workloads.single_array(dist, n, np.float32, seed=11)
    for k in (n // 100, (n + 1) // 2, n - n // 100):
        r = sim(x, k, final_threshold=8192, theta=1.0, hist_bits=12)
        _check(r, oracle_mod.select_kth(x, k), (dist, k))
        assert r.elements_read <= 3 * n, (dist, k, r.elements_read / n)
        assert r.work_passes <= 5, (dist, k, r.work_passes)


@pytest.mark.parametrize("dist", ["normal", "uniform", "cauchy", "quantized_normal", "spike",
                                  "smallint"])
def test_count_first_then_compact(sim, oracle_mod, dist):
    """The first evaluation counts both sides of its trial point in key bins and writes
    nothing; the bracket narrows to the bin of the rank, and the next pass over the input
    counts that bin's elements and copies them (they are far fewer than n).  Values stay
    exact; the input is read at most three times and little is written (with a spike of
    equal values the bin is too full to copy: one more pass over the input finds the key)."""
    n = 1 << 20
    if dist == "spike":  # 90 % of the elements equal
        rng = np.random.default_rng(12)
        x = np.where(rng.random(n) < 0.9, 1.0, rng.standard_normal(n)).astype(np.float32)
    else:
        x = workloads.single_array(dist, n, np.float32, seed=12)
    for k in (n // 100, (n + 1) // 2, n - n // 100):
        ref = oracle_mod.select_kth(x, k)
        r = sim(x, k, final_threshold=8192, theta=1.0, hist_bits=12, count_first=1)
        _check(r, ref, (dist, k))
        most = 4 if dist == "spike" else 3
        assert r.passes <= most, (dist, k, r.passes)
        assert r.elements_read <= most * n + n // 4, (dist, k, r.elements_read / n)
        assert r.elements_written <= n // 4 + 8192, (dist, k, r.elements_written)


@pytest.mark.parametrize("dist", ["normal", "uniform", "cauchy", "quantized_normal", "lognormal"])
def test_count_first_with_likely_interval(sim, oracle_mod, dist):
    """The counting evaluation also copies the elements of a likely interval (quantiles of a
    strided sample around the rank); when the narrowed bracket lies inside it the copy is
    the working set and the input is read twice in all.  An interval away from the rank
    (spec_mode 2) is not adopted: the result is the same and a third read of x follows."""
    n = 1 << 20
    x = workloads.single_array(dist, n, np.float32, seed=13)
    for k in (n // 100, (n + 1) // 2, n - n // 100):
        ref = oracle_mod.select_kth(x, k)
        r = sim(x, k, final_threshold=8192, theta=1.0, hist_bits=12, count_first=1, spec_mode=1)
        _check(r, ref, (dist, k, "spec"))
        assert r.passes == 2, (dist, k, r.passes)
        assert r.elements_written <= n // 8, (dist, k, r.elements_written)
        miss = sim(x, k, final_threshold=8192, theta=1.0, hist_bits=12, count_first=1,
                   spec_mode=2)
        _check(miss, ref, (dist, k, "miss"))
        assert miss.passes == 3, (dist, k, miss.passes)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_transform_with_huge_outliers(sim, oracle_mod, dtype):
    """Section 5.3: a few elements near 1e20 make the sums over x lose every other term, and
    the cutting plane on x degrades towards bisection; on F(x) = log(1 + x - min x) its steps
    stay informative.  Exact either way; the transform takes fewer passes in total."""
    tot_plain = tot_log = 0
    for seed in range(4):
        x = workloads.single_array("outliers20", 50_001, dtype, seed=seed, tag="sim-outliers")
        for k in (5_000, 25_001, 45_000):
            ref = oracle_mod.select_kth(x, k)
            plain = sim(x, k, theta=0.0, final_threshold=64)
            logt = sim(x, k, theta=0.0, final_threshold=64, transform=1)
            _check(plain, ref, ("plain", seed, k))
            _check(logt, ref, ("log", seed, k))
            tot_plain += plain.work_passes
            tot_log += logt.work_passes
    assert tot_log < tot_plain, (tot_log, tot_plain)
