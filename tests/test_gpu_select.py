"""GPU parity of select_kth / select_kth_ex against the CPU oracle.

Element by element on the same seeded inputs: the selected value is compared
bit for bit and its counts exactly (Section 1's definition of x_(k)).  Options
force every branch of the cutting-plane path: tiny final thresholds (many
passes and splits), no splitting, bisection only (maxit = 0), one workgroup,
ragged grids, unaligned starts, duplicates, infinities, signed zeros,
denormals, NaN.
"""
import numpy as np
import pytest

import workloads
from tests.gpu_util import assert_same_result, invariant_holds

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sel():
    import paper_1104_2732_amd as cps
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = cps.Selector(0)
    yield s
    s.close()


def _dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _run(sel, x, k, ctx, **opt):
    import paper_1104_2732_amd as cps
    o = cps.default_options(**opt) if opt else None
    print(f"case {ctx} n={x.size} k={k} dtype={x.dtype} opt={opt}", flush=True)
    return sel.select_kth(_dev(x), k, options=o)


SMALL_DISTS = ["uniform", "normal", "cauchy", "quantized_normal", "lognormal", "mix1", "mix2",
               "mix3", "mix5", "smallint", "outliers", "outliers20", "beta25", "halfnormal"]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("dist", SMALL_DISTS)
def test_parity_default_options(sel, oracle_mod, dist, dtype):
    for n in (1, 2, 3, 5, 31, 1000, 4099, 70_001, 300_007):
        x = workloads.single_array(dist, n, dtype, seed=n, tag="gpu-parity")
        for k in sorted({1, 2, n // 100 or 1, (n + 1) // 2, max(1, n - 1), n}):
            if k > n:
                continue
            res = _run(sel, x, k, f"{dist}")
            assert_same_result(res, oracle_mod.select_kth(x, k), f"{dist} n={n} k={k}")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("opt", [
    dict(final_threshold=16),
    dict(final_threshold=16, partition_fraction=0.0),
    dict(final_threshold=1, partition_fraction=1.0),
    dict(final_threshold=64, maxit=0),
    dict(final_threshold=64, maxit=1),
    dict(final_threshold=32, grid_blocks=1),
    dict(final_threshold=32, grid_blocks=7),
    dict(final_threshold=100, grid_blocks=3, partition_fraction=0.25),
    dict(final_threshold=16, hist_bits=0),
    dict(final_threshold=1, partition_fraction=1.0, hist_bits=1),
    dict(final_threshold=1, partition_fraction=1.0, hist_bits=3, grid_blocks=5),
    dict(final_threshold=64, partition_fraction=1.0, hist_bits=12),
])
def test_parity_forced_paths(sel, oracle_mod, dtype, opt):
    for dist in ("uniform", "quantized_normal", "cauchy", "mix2", "smallint"):
        for n in (2, 9, 257, 5003, 131_073):
            x = workloads.single_array(dist, n, dtype, seed=7 * n + 1, tag="gpu-forced")
            for k in sorted({1, (n + 1) // 2, max(1, n // 3), n - 1 or 1, n}):
                res = _run(sel, x, k, dist, **opt)
                assert_same_result(res, oracle_mod.select_kth(x, k), f"{dist} n={n} k={k} {opt}")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_unaligned_and_ragged(sel, oracle_mod, dtype):
    import paper_1104_2732_amd as cps
    base = workloads.single_array("normal", 100_003, dtype, seed=3)
    xt = _dev(base)
    for off in (1, 2, 3):
        for n in (5, 1021, 99_000):
            view = xt[off:off + n]
            assert view.is_contiguous()
            x = base[off:off + n]
            for k in (1, (n + 1) // 2, n):
                print(f"case unaligned off={off} n={n} k={k}", flush=True)
                res = sel.select_kth(view, k, options=cps.default_options(final_threshold=8))
                assert_same_result(res, oracle_mod.select_kth(x, k), f"off={off} n={n} k={k}")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_special_values(sel, oracle_mod, dtype):
    info = np.finfo(dtype)
    tiny = info.smallest_subnormal
    cases = {
        "signed_zeros": np.array([0.0, -0.0, -0.0, 0.0, 1.0, -1.0, -0.0] * 50, dtype=dtype),
        "denormals": np.array([tiny, -tiny, 2 * tiny, 0.0, -0.0, 3 * tiny, -2 * tiny] * 40, dtype=dtype),
        "infinities": np.array([np.inf, -np.inf, 1.0, 2.0, -np.inf, 0.5, np.inf, 3.0, np.inf] * 30,
                               dtype=dtype),
        "only_inf": np.array([np.inf, -np.inf, np.inf, -np.inf, -np.inf], dtype=dtype),
        "huge": np.array([info.max, -info.max, 1.0, info.max, 0.0, -info.max, 2.0] * 20, dtype=dtype),
        "constant": np.full(10_000, 2.5, dtype=dtype),
        "two_values": np.array([1.0, 2.0] * 5000, dtype=dtype),
        "sorted": np.sort(workloads.single_array("normal", 20_000, dtype, seed=1)),
        "reversed": np.sort(workloads.single_array("normal", 20_000, dtype, seed=1))[::-1].copy(),
    }
    rng = np.random.default_rng(0)
    for name, x in cases.items():
        x = x.copy()
        if name not in ("sorted", "reversed"):
            rng.shuffle(x)
        n = x.size
        for k in sorted({1, 2, n // 3 or 1, (n + 1) // 2, n - 1 or 1, n}):
            for opt in ({}, {"final_threshold": 2}):
                res = _run(sel, x, k, name, **opt)
                assert_same_result(res, oracle_mod.select_kth(x, k), f"{name} k={k} {opt}")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_cooperative_launch(sel, oracle_mod, dtype):
    """The same selections under the cooperative launch (residency guaranteed by the runtime)
    as under the default ordinary launch, on a ragged multi-tile input."""
    n = (1 << 21) + 333
    x = workloads.single_array("normal", n, dtype, seed=12, tag="gpu-coop")
    for k in (1, n // 100, (n + 1) // 2, n):
        res = _run(sel, x, k, "cooperative", cooperative=1)
        assert_same_result(res, oracle_mod.select_kth(x, k), f"cooperative k={k}")


def test_nan_status(sel):
    import paper_1104_2732_amd as cps
    x = np.array([1.0, np.nan, 3.0, 4.0], dtype=np.float32)
    res = _run(sel, x, 2, "nan")
    assert res["status"] == cps.STATUS_NAN


def test_argument_errors(sel):
    import paper_1104_2732_amd as cps
    x = _dev(np.arange(10, dtype=np.float32))
    for k in (0, 11, -5):
        with pytest.raises(cps.CpsError):
            sel.select_kth(x, k)
    with pytest.raises(cps.CpsError):
        sel.select_kth(x, 1, options=cps.default_options(final_threshold=0))
    with pytest.raises(TypeError):
        sel.select_kth(_dev(np.arange(10, dtype=np.int32)), 1)


def test_permutation_invariance(sel):
    x = workloads.single_array("mix4", 200_000, np.float32, seed=5)
    ref = None
    for y in (x, np.sort(x), np.sort(x)[::-1].copy()):
        r = _run(sel, y, 123_456, "perm")
        v = (r["value_bits"], r["less"], r["equal"])
        ref = ref or v
        assert v == ref


def test_stats_and_invariants(sel):
    import paper_1104_2732_amd as cps
    n = 1 << 20
    x = workloads.single_array("uniform", n, np.float32, seed=0)
    k = (n + 1) // 2
    print("case stats uniform 2^20", flush=True)
    res, st = sel.select_kth(_dev(x), k, stats=True)
    invariant_holds(x, k, res)
    assert res["passes"] == st["passes"] >= 2
    wp = st["work_passes"]
    assert 2 <= wp <= 4 * 96
    pops = st["population"][: min(wp, cps.STATS_MAX_PASSES)]
    # the bracket population never grows (Section 4: the bracket only shrinks)
    nz = pops[pops > 0]
    assert np.all(np.diff(nz) <= 0)
    # bisection-like halving on smooth data (end of Section 4): far fewer passes than log2(n) + 8
    assert wp <= 24


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_histogram_finish_signed_zeros_and_denormals(sel, oracle_mod, dtype):
    """Key-histogram narrowing around -0/+0 and subnormals, with one-key bins."""
    tiny = np.finfo(dtype).smallest_subnormal
    vals = np.array([-0.0, 0.0, tiny, -tiny, 2 * tiny, -2 * tiny, 1.0, -1.0, 1e-30, -1e-30],
                    dtype=dtype)
    rng = np.random.default_rng(9)
    for trial in range(6):
        x = rng.choice(vals, size=int(rng.integers(5000, 90_000))).astype(dtype)
        for k in (1, 2, x.size // 3, x.size // 2, x.size - 1, x.size):
            ref = oracle_mod.select_kth(x, k)
            for hb in (1, 2, 12):
                res = _run(sel, x, k, f"zeros trial {trial}", final_threshold=1,
                           partition_fraction=1.0, hist_bits=hb)
                assert_same_result(res, ref, (trial, k, hb))


@pytest.mark.parametrize("count_first", [1, 0])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_default_path_counted_split_and_compaction(sel, oracle_mod, dtype, count_first):
    """The default path at a few million elements.  count_first 1 (the default): the first
    evaluation counts both sides of the trial point in key bins, the bracket narrows to the
    bin of the rank and the next pass over x compacts that bin's elements.  count_first 0:
    the split at the first trial point writes both parts and counts them, the part that
    holds x_(k) narrows at once and a histogram pass compacts a narrowed bracket.  The
    gather and the final select end both.  Includes a spike (90 % of the elements equal)
    and integer data, so narrowed brackets hold many equal keys."""
    import paper_1104_2732_amd as cps
    n = (1 << 22) + 17
    rng = np.random.default_rng(21)
    spike = np.where(rng.random(n) < 0.9, 1.0, rng.standard_normal(n)).astype(dtype)
    cases = [(d, workloads.single_array(d, n, dtype, seed=5, tag="gpu-default"))
             for d in ("normal", "lognormal", "quantized_normal", "smallint")]
    cases.append(("spike", spike))
    for dist, x in cases:
        xt = _dev(x)
        for k in (1 + n // 100, n // 3, (n + 1) // 2, n - n // 100):
            print(f"case default-path {dist} n={n} k={k} dtype={x.dtype} cf={count_first}",
                  flush=True)
            res, st = sel.select_kth(xt, k, options=cps.default_options(count_first=count_first),
                                     stats=True)
            assert_same_result(res, oracle_mod.select_kth(x, k), f"{dist} k={k}")
            # a spike's bin is too full to copy, so with count_first the histogram passes
            # read x itself: each cuts the key range 2^12-fold (up to 5 for float64 keys)
            most = 7 if (count_first and dist == "spike") else 4
            assert st["passes"] <= most, (dist, k, st["passes"])
            if count_first and dist != "spike":
                # the counting evaluation writes nothing; the compaction copies one bin
                assert st["elements_written"] <= n // 4 + 8192, (dist, k, st["elements_written"])


@pytest.mark.parametrize("dist", ["normal", "quantized_normal", "periodic"])
def test_large_input_counting_with_interval_copy(sel, oracle_mod, dist):
    """From 256 MiB of input the counting evaluation also copies a likely interval (sample
    quantiles around the rank) and the copy becomes the working set when the narrowed
    bracket lies inside it: x is then read twice in all.  The periodic input has pass 0's
    tile (1024 threads x four 16-byte vectors = 16384 float elements) as its period, so the
    sample (each tile's first vector) holds only 0..3 and the interval misses: the copy is
    not adopted and a third pass over x finds the same exact result."""
    n = (1 << 27) + 17
    if dist == "periodic":
        x = (np.arange(n, dtype=np.int64) % 16384).astype(np.float32)
    else:
        x = workloads.single_array(dist, n, np.float32, seed=8, tag="gpu-large")
    xt = _dev(x)
    for k in (1 + n // 100, (n + 1) // 2):
        print(f"case large-interval {dist} n={n} k={k}", flush=True)
        res, st = sel.select_kth(xt, k, stats=True)
        assert_same_result(res, oracle_mod.select_kth(x, k), f"{dist} k={k}")
        assert st["passes"] <= 3, (dist, k, st["passes"])
        if dist == "periodic":
            assert st["passes"] == 3, (k, st["passes"])  # the copy was not adopted
    del xt
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dist", ["normal", "cauchy", "quantized_normal"])
def test_float64_counting_with_interval_copy(sel, oracle_mod, dist):
    """float64 from 256 MiB of input (2^25 elements): the counting evaluation copies the
    likely interval as 8-byte elements (two per 16-byte vector) and the copy becomes the
    working set when the narrowed bracket lies inside it."""
    n = (1 << 25) + 17
    x = workloads.single_array(dist, n, np.float64, seed=9, tag="gpu-large64")
    xt = _dev(x)
    for k in (n // 100, (n + 1) // 2):
        print(f"case large-interval-f64 {dist} n={n} k={k}", flush=True)
        res, st = sel.select_kth(xt, k, stats=True)
        assert_same_result(res, oracle_mod.select_kth(x, k), f"{dist} k={k}")
        assert st["passes"] <= 3, (dist, k, st["passes"])
    del xt
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dist", ["uniform", "cauchy"])
def test_float32_counting_with_interval_copy_more_distributions(sel, oracle_mod, dist):
    n = (1 << 26) + 17
    x = workloads.single_array(dist, n, np.float32, seed=10, tag="gpu-large32")
    xt = _dev(x)
    for k in (1 + n // 100, (n + 1) // 2, n - n // 100):
        print(f"case large-interval-f32 {dist} n={n} k={k}", flush=True)
        res, st = sel.select_kth(xt, k, stats=True)
        assert_same_result(res, oracle_mod.select_kth(x, k), f"{dist} k={k}")
        assert st["passes"] <= 3, (dist, k, st["passes"])
    del xt
    torch.cuda.empty_cache()


def test_timeout_leaves_the_handle_usable(sel, oracle_mod):
    """A call whose waits give up at once (spin limit 1: the waiting workgroups leave with
    status TIMEOUT, the one that went on alone leaves at its next wait) must not leave the
    grid's arrival counters part-way counted for the next call on the same handle."""
    import paper_1104_2732_amd as cps
    n = (1 << 22) + 5
    x = workloads.single_array("normal", n, np.float32, seed=4, tag="gpu-timeout")
    xt = _dev(x)
    k = (n + 1) // 2
    ref = oracle_mod.select_kth(x, k)
    for rep in range(2):
        print(f"case timeout rep={rep} n={n}", flush=True)
        res = sel.select_kth(xt, k, options=cps.default_options(spin_limit=1))
        assert res["status"] in (cps.STATUS_OK, cps.STATUS_TIMEOUT), res
        if res["status"] == cps.STATUS_OK:
            assert_same_result(res, ref)
        for kk in (1 + n // 100, k):
            assert_same_result(sel.select_kth(xt, kk), oracle_mod.select_kth(x, kk), f"after {rep}")
    del xt


def test_counts_past_32_bits(sel):
    """2^32 + 17 float32 elements (16 GiB, drawn on the device; uniform [0, 1) on a 2^-24 grid,
    so every value repeats ~256 times): counts, bins and positions past 32 bits.  The value
    is pinned by its counts (Section 1's x_(k): less < k <= less + equal, equal >= 1), taken
    on the device with plain comparisons, and the reported counts must equal them."""
    n = (1 << 32) + 17
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    xt = torch.rand(n, device="cuda", generator=g, dtype=torch.float32)
    for k in (1 + n // 100, (n + 1) // 2):
        print(f"case counts past 32 bits n={n} k={k}", flush=True)
        res = sel.select_kth(xt, k)
        assert res["status"] == 0, res
        v = torch.tensor(res["value"], dtype=torch.float32, device="cuda")
        less = int((xt < v).sum().item())
        equal = int((xt == v).sum().item())
        assert (res["less"], res["equal"]) == (less, equal)
        assert less < k <= less + equal and equal >= 1
    del xt
    torch.cuda.empty_cache()
