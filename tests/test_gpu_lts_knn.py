"""GPU parity of the sum of the k smallest elements (select_kth_batched_ksum), the least
trimmed squares objective (lts_trimmed_sq) and the k nearest neighbours' mean (knn_mean)
against the CPU oracle (Section 6).

Selected values and counts bit for bit; the sums in double precision within 1e-12 of the
sum of absolute values of the terms (both sides add exact widenings of the same elements,
in different orders: the error of either is below n * 2^-53 of that sum, and 1e-12 covers
n up to 2^20 with room); kNN distances bit for bit (the same float operations in the same
order, no fused multiply-add on either side).
"""
import math

import numpy as np
import pytest

import workloads

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


def _abs_scale(x, k):
    return math.fsum(np.abs(np.sort(x.astype(np.float64))[:k]))


def _batch(dtype, seed):
    rng = np.random.default_rng(seed)
    dists = ["normal", "uniform", "quantized_normal", "cauchy", "lognormal", "smallint"]
    arrays, ks = [], []
    sizes = [1, 7, 1000, 4099, 40_000, 70_001, 131_073, 300_007, 1_000_003]
    for i, n in enumerate(sizes):
        x = workloads.single_array(dists[i % len(dists)], n, dtype, seed=seed * 10 + i, tag="gpu-ksum")
        arrays.append(x)
        ks.append([1, n, (n + 1) // 2, int(rng.integers(1, n + 1)), max(1, n // 100)][i % 5])
    return arrays, ks


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("opt", [dict(), dict(proposal=0),
                                 dict(elements_per_block=1 << 15, blocks_per_array=16),
                                 dict(elements_per_block=1 << 16, blocks_per_array=4,
                                      team_capacity=2048),
                                 dict(block_threads=256)])
def test_batched_ksum(sel, oracle_mod, dtype, opt):
    import paper_1104_2732_amd as cps
    arrays, ks = _batch(dtype, seed=len(opt) + (3 if dtype == np.float64 else 0))
    dev = [torch.from_numpy(a).cuda() for a in arrays]
    print(f"case ksum {np.dtype(dtype).name} {opt}", flush=True)
    res, ksum = sel.select_kth_batched_ksum(dev, ks, cps.default_batch_options(**opt))
    for i, (x, k) in enumerate(zip(arrays, ks)):
        ref = oracle_mod.select_kth(x, k)
        assert int(res[i]["value_bits"]) == ref["value_bits"] and int(res[i]["less"]) == ref["less"]
        t = oracle_mod.trimmed_sum(x.astype(np.float64), k)
        assert abs(ksum[i] - t["F"]) <= 1e-12 * max(_abs_scale(x, k), 1e-300), (i, ksum[i], t["F"])


@pytest.mark.parametrize("form", [0, 1, 2])  # automatic, materialised, filtered
@pytest.mark.parametrize("n,p,m", [(1001, 8, 40), ((1 << 17) + 3, 8, 64), (50_000, 3, 17),
                                   ((1 << 18) + 2, 8, 70)])
def test_lts_parity(sel, oracle_mod, n, p, m, form):
    import paper_1104_2732_amd as cps
    if form == 2 and n < (1 << 15):
        return  # (the filtered form needs 2^15 rows; the argument check is in the LMS tests)
    X, y, _, betas = workloads.lms_problem(n, p, m, seed=n % 97)
    Xd, yd, bd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (X, y, betas))
    for h in sorted({(n + 1) // 2, (n + p) // 2, 1, n, n // 3 + 1}):
        print(f"case lts n={n} p={p} m={m} h={h} form={form}", flush=True)
        got = sel.lts_trimmed_sq(Xd, yd, bd, h, form=form)
        ref = oracle_mod.lts_objective(X, y, betas, h)
        for c in range(m):
            assert got[c]["status"] == 0
            assert got[c]["m"] == ref[c]["m"], (h, c)
            assert (got[c]["below"], got[c]["a"], got[c]["b"]) == (ref[c]["below"], ref[c]["a"],
                                                                   ref[c]["b"]), (h, c)
            assert abs(got[c]["F"] - ref[c]["F"]) <= 1e-12 * ref[c]["F"], (h, c)


def test_lts_full_size_sampled(sel, oracle_mod):
    """The least-median-of-squares workload's shape (2^20 rows, p = 8, 1024 candidates) with
    h = floor((n+1)/2): eight candidates against the oracle, and the median of every candidate
    against lms_median_sq_residuals."""
    n, p, m = 1 << 20, 8, 1024
    X, y, _, betas = workloads.lms_problem(n, p, m, seed=0)
    Xd, yd, bd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (X, y, betas))
    print("case lts full size", flush=True)
    got = sel.lts_trimmed_sq(Xd, yd, bd)
    lms = sel.lms_median_sq_residuals(Xd, yd, bd)
    assert np.array_equal(got["m"], lms["value"]) and np.array_equal(got["below"], lms["less"])
    mat = sel.lts_trimmed_sq(Xd, yd, bd, form=1)  # the materialised form: same records
    for f in ("m", "below", "a", "b", "status"):
        assert np.array_equal(got[f], mat[f]), f
    assert np.all(np.abs(got["F"] - mat["F"]) <= 1e-12 * mat["F"])
    pick = np.random.default_rng(1).choice(m, size=8, replace=False)
    ref = oracle_mod.lts_objective(X, y, betas[pick])
    for j, c in enumerate(pick):
        assert got[c]["m"] == ref[j]["m"] and got[c]["a"] == ref[j]["a"]
        assert abs(got[c]["F"] - ref[j]["F"]) <= 1e-12 * ref[j]["F"], c


def _knn_inputs(n, dim, nq, seed, grid=False):
    rng = np.random.default_rng(seed)
    if grid:  # integer coordinates: many equal distances
        P = rng.integers(0, 4, size=(n, dim)).astype(np.float32)
        Q = rng.integers(0, 4, size=(nq, dim)).astype(np.float32)
    else:
        P = rng.standard_normal((n, dim)).astype(np.float32)
        Q = rng.standard_normal((nq, dim)).astype(np.float32)
    f = (np.sin(P.sum(axis=1)) + 0.1 * rng.standard_normal(n)).astype(np.float32)
    return P, f, Q


@pytest.mark.parametrize("form", [0, 1, 2])  # automatic, materialised, filtered
@pytest.mark.parametrize("n,dim,nq,grid", [(5, 2, 3, False), (4099, 8, 33, False),
                                           ((1 << 16) + 5, 8, 64, False), (30_000, 3, 20, True),
                                           (70_001, 5, 17, False), (40_000, 8, 300, True)])
def test_knn_parity(sel, oracle_mod, n, dim, nq, grid, form):
    if form == 2 and n < (1 << 15):
        return  # (the filtered form needs 2^15 points)
    P, f, Q = _knn_inputs(n, dim, nq, seed=n + dim, grid=grid)
    Pd, fd, Qd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (P, f, Q))
    for k in sorted({1, min(n, 16), min(n, 100), n, max(1, n // 3)}):
        print(f"case knn n={n} dim={dim} nq={nq} k={k} grid={grid} form={form}", flush=True)
        got = sel.knn_mean(Pd, fd, Qd, k, form=form)
        ref = oracle_mod.knn_mean(P, f, Q, k)
        for c in range(nq):
            assert got[c]["status"] == 0, (k, c)
            assert got[c]["dk"] == ref[c]["dk"], (k, c)
            assert (got[c]["below"], got[c]["equal"]) == (ref[c]["below"], ref[c]["equal"]), (k, c)
            scale = float(np.sum(np.abs(f.astype(np.float64)))) / k
            assert abs(got[c]["mean"] - ref[c]["mean"]) <= 1e-12 * scale, (k, c)


def test_knn_full_size_sampled(sel, oracle_mod):
    """2^20 points in 8 dimensions, 1024 queries, k = 64: eight queries against the oracle."""
    n, dim, nq, k = 1 << 20, 8, 1024, 64
    P, f, Q = _knn_inputs(n, dim, nq, seed=0)
    Pd, fd, Qd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (P, f, Q))
    print("case knn full size", flush=True)
    got = sel.knn_mean(Pd, fd, Qd, k)
    assert np.all(got["status"] == 0)
    mat = sel.knn_mean(Pd, fd, Qd, k, form=1)  # the materialised form: the same records
    for fld in ("dk", "below", "equal", "status"):
        assert np.array_equal(got[fld], mat[fld]), fld
    assert np.all(np.abs(got["mean"] - mat["mean"]) <= 1e-12 * float(np.sum(np.abs(f))) / k)
    pick = np.random.default_rng(2).choice(nq, size=8, replace=False)
    ref = oracle_mod.knn_mean(P, f, Q[pick], k)
    for j, c in enumerate(pick):
        assert got[c]["dk"] == ref[j]["dk"] and got[c]["below"] == ref[j]["below"]
        assert abs(got[c]["mean"] - ref[j]["mean"]) <= 1e-12 * float(np.sum(np.abs(f))) / k


def test_knn_filtered_misleading_sample(sel, oracle_mod):
    """Points that the sample sees near every query and the rest far away: the sampled bracket
    is far too narrow or too wide for some k, and those queries are selected over their
    recomputed distances; every result matches the oracle's."""
    n, dim, nq = 1 << 16, 4, 6
    rng = np.random.default_rng(8)
    P = (50.0 + rng.standard_normal((n, dim))).astype(np.float32)
    S = 4096
    stride = n // (S // 16)
    i = np.arange(S)
    rows = (i // 16) * stride + i % 16
    P[rows] = rng.standard_normal((rows.size, dim)).astype(np.float32)  # the sampled points
    Q = rng.standard_normal((nq, dim)).astype(np.float32)
    f = rng.standard_normal(n).astype(np.float32)
    Pd, fd, Qd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (P, f, Q))
    for k in (1, 64, 5000, 30_000):
        print(f"case knn misleading sample k={k}", flush=True)
        got = sel.knn_mean(Pd, fd, Qd, k, form=2)
        ref = oracle_mod.knn_mean(P, f, Q, k)
        for c in range(nq):
            assert got[c]["status"] == 0 and got[c]["dk"] == ref[c]["dk"], (k, c)
            assert (got[c]["below"], got[c]["equal"]) == (ref[c]["below"], ref[c]["equal"]), (k, c)
            assert abs(got[c]["mean"] - ref[c]["mean"]) <= 1e-12 * float(np.sum(np.abs(f))) / k


def test_knn_filtered_shapes(sel, oracle_mod):
    """The filtered form with one query over 2^21 + 7 points (one query group, many
    segments) and with 257 queries (two groups, the second with one live query)."""
    for n, nq, k in (((1 << 21) + 7, 1, 1000), ((1 << 16) + 1, 257, 64)):
        P, f, Q = _knn_inputs(n, 8, nq, seed=nq)
        Pd, fd, Qd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (P, f, Q))
        print(f"case knn filtered shape n={n} nq={nq} k={k}", flush=True)
        got = sel.knn_mean(Pd, fd, Qd, k, form=2)
        ref = oracle_mod.knn_mean(P, f, Q, k)
        for c in range(nq):
            assert got[c]["status"] == 0 and got[c]["dk"] == ref[c]["dk"], c
            assert (got[c]["below"], got[c]["equal"]) == (ref[c]["below"], ref[c]["equal"]), c
            assert abs(got[c]["mean"] - ref[c]["mean"]) <= 1e-12 * float(np.sum(np.abs(f))) / k
