"""GPU parity of lms_median_sq_residuals against the CPU oracle (Section 6).

The residuals are formed left to right without fused multiply-add on both
sides, so the medians must agree bit for bit and the counts exactly.  Small
problems are compared candidate by candidate in every form (materialised, and
filtered where n allows it); the full-size problem (2^20 rows, p = 8, 1024
candidates, 30 % of rows shifted) on a seeded sample of candidates against
residuals recomputed by the oracle, and the two forms against each other on
every candidate.  Inputs whose sampled rows mislead the filter's bracket check
the fallback to the materialised form.
"""
import numpy as np
import pytest

import workloads
from tests.gpu_util import assert_same_result

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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


FORMS = {"auto": 0, "materialised": 1, "filtered": 2}


@pytest.mark.parametrize("form", ["auto", "materialised", "filtered"])
@pytest.mark.parametrize("n,p,m", [(1, 1, 1), (7, 3, 5), (1001, 8, 40), (50_000, 8, 33),
                                   (20_001, 5, 17), (4096, 16, 3), (40_001, 5, 70),
                                   (1 << 15, 16, 3), (300_000, 8, 65), (262_147, 3, 2)])
def test_lms_small(sel, oracle_mod, n, p, m, form):
    import paper_1104_2732_amd as cps
    if form == "filtered" and n < (1 << 15):
        with pytest.raises(cps.CpsError):
            sel.lms_median_sq_residuals(_dev(np.zeros((n, p))), _dev(np.zeros(n)),
                                        _dev(np.zeros((m, p))), form=FORMS[form])
        return
    X, y, beta, betas = workloads.lms_problem(n, p, m, seed=n + p, contamination=0.3) if n >= p \
        else (np.random.default_rng(0).standard_normal((n, p)), np.zeros(n), None,
              np.random.default_rng(1).standard_normal((m, p)))
    print(f"case lms n={n} p={p} m={m} form={form}", flush=True)
    res = sel.lms_median_sq_residuals(_dev(X), _dev(y), _dev(betas), form=FORMS[form])
    ref = oracle_mod.lms_median_sq(X, y, betas)
    for c in range(m):
        r = {f: res[c][f].item() for f in res.dtype.names}
        assert_same_result(r, ref[c], f"candidate {c}")


@pytest.mark.parametrize("n", [30_001, 70_000])
def test_lms_exact_fit_zero_median(sel, n):
    """Residuals exactly 0 on 70 % of the rows (a median of 0 with 70 % ties; at 70 000 rows
    the filtered form's bracket cannot hold it, and the candidate is selected whole)."""
    rng = np.random.default_rng(5)
    p = 8
    X = rng.standard_normal((n, p))
    beta = rng.standard_normal(p)
    s = X[:, 0] * beta[0]
    for j in range(1, p):
        s = s + X[:, j] * beta[j]
    y = s.copy()
    bad = rng.choice(n, size=int(0.3 * n), replace=False)
    y[bad] += 10.0
    res = sel.lms_median_sq_residuals(_dev(X), _dev(y), _dev(beta[None, :]))
    assert res[0]["status"] == 0 and res[0]["value"] == 0.0
    assert res[0]["less"] == 0 and res[0]["equal"] == n - bad.size


def test_lms_full_size_sampled(sel, oracle_mod):
    n, p, m = 1 << 20, 8, 1024
    X, y, beta, betas = workloads.lms_problem(n, p, m, seed=0)
    print("case lms full size", flush=True)
    res = sel.lms_median_sq_residuals(_dev(X), _dev(y), _dev(betas))
    assert np.all(res["status"] == 0)
    mat = sel.lms_median_sq_residuals(_dev(X), _dev(y), _dev(betas), form=FORMS["materialised"])
    for f in ("value_bits", "less", "equal", "greater", "status"):
        assert np.array_equal(res[f], mat[f]), f
    k = (n + 1) // 2
    rng = np.random.default_rng(1)
    sample = rng.choice(m, size=12, replace=False)
    for c in sample:
        r = oracle_mod.lms_residuals(X, y, betas[c])
        v = res[c]["value"]
        less = int(np.count_nonzero(r < v))
        eq = int(np.count_nonzero(r == v))
        assert less < k <= less + eq and (less, eq) == (res[c]["less"], res[c]["equal"])
    for c in sample[:3]:
        ref = oracle_mod.lms_median_sq(X, y, betas[c:c + 1])[0]
        assert_same_result({f: res[c][f].item() for f in res.dtype.names}, ref, f"candidate {c}")
    # the estimate: the candidate with the least median of squares fits the clean rows
    best = int(np.argmin(res["value"]))
    assert np.max(np.abs(betas[best] - beta)) < 0.5


def test_lms_nonfinite_residuals(sel, oracle_mod):
    """Step 0 taken inside the residual kernel classifies +inf (rows whose residual
    overflows) and NaN (a NaN in y) as the selection's own pass 0 does."""
    import oracle
    import paper_1104_2732_amd as cps
    rng = np.random.default_rng(17)
    n, p, m = 2001, 4, 11
    X = rng.standard_normal((n, p))
    y = rng.standard_normal(n)
    betas = rng.standard_normal((m, p))
    X[rng.choice(n, size=40, replace=False)] *= 1e200  # residuals overflow to +inf
    print("case lms +inf residuals", flush=True)
    res = sel.lms_median_sq_residuals(_dev(X), _dev(y), _dev(betas))
    ref = oracle_mod.lms_median_sq(X, y, betas)
    for c in range(m):
        assert_same_result({f: res[c][f].item() for f in res.dtype.names}, ref[c], f"candidate {c}")
    y[5] = np.nan
    print("case lms NaN residuals", flush=True)
    res = sel.lms_median_sq_residuals(_dev(X), _dev(y), _dev(betas))
    assert np.all(res["status"] == cps.STATUS_NAN)
    with pytest.raises(oracle.OracleError):
        oracle_mod.lms_median_sq(X, y, betas)


def _sampled_rows(n):
    """The rows whose residuals the filtered form samples for its bracket (runs of 16
    neighbours at n / (S / 16) apart, S = 4096 below 2^18 rows, else 16384)."""
    S = 4096 if n < (1 << 18) else 16384
    stride = n // (S // 16)
    i = np.arange(S)
    return (i // 16) * stride + i % 16


@pytest.mark.parametrize("n", [1 << 16, (1 << 18) + 6])
def test_lms_filtered_misleading_sample(sel, oracle_mod, n):
    """Candidates whose sampled rows fit well and the rest badly (the bracket then misses
    the median, and the candidate's whole array is selected), beside ordinary candidates,
    in one call: every result matches the oracle's."""
    rng = np.random.default_rng(41)
    p, m = 8, 9
    X = rng.standard_normal((n, p))
    betas = rng.standard_normal((m, p))
    s = X[:, 0] * betas[0, 0]
    for j in range(1, p):
        s = s + X[:, j] * betas[0, j]
    y = s + 10.0 + rng.uniform(0.0, 1.0, n)       # candidate 0: residuals in (100, 121)
    rows = _sampled_rows(n)
    y[rows] = s[rows] + rng.uniform(0.0, 1.0, rows.size)  # ... but below 1 on the sample
    print(f"case lms misleading sample n={n}", flush=True)
    for form in ("filtered", "auto", "materialised"):
        res = sel.lms_median_sq_residuals(_dev(X), _dev(y), _dev(betas), form=FORMS[form])
        ref = oracle_mod.lms_median_sq(X, y, betas)
        for c in range(m):
            assert_same_result({f: res[c][f].item() for f in res.dtype.names}, ref[c],
                               f"candidate {c} form {form}")


def test_lms_filtered_nonfinite(sel, oracle_mod):
    """The filtered form with residuals that overflow to +inf (outside every bracket) and
    with NaN (kept by the filter, so the packed selection reports it)."""
    import oracle
    import paper_1104_2732_amd as cps
    rng = np.random.default_rng(23)
    n, p, m = 40_001, 4, 11
    X = rng.standard_normal((n, p))
    y = rng.standard_normal(n)
    betas = rng.standard_normal((m, p))
    X[rng.choice(n, size=400, replace=False)] *= 1e200
    print("case lms filtered +inf residuals", flush=True)
    res = sel.lms_median_sq_residuals(_dev(X), _dev(y), _dev(betas), form=FORMS["filtered"])
    ref = oracle_mod.lms_median_sq(X, y, betas)
    for c in range(m):
        assert_same_result({f: res[c][f].item() for f in res.dtype.names}, ref[c], f"candidate {c}")
    y[7] = np.nan
    print("case lms filtered NaN residuals", flush=True)
    res = sel.lms_median_sq_residuals(_dev(X), _dev(y), _dev(betas), form=FORMS["filtered"])
    assert np.all(res["status"] == cps.STATUS_NAN)
    with pytest.raises(oracle.OracleError):
        oracle_mod.lms_median_sq(X, y, betas)


@pytest.mark.parametrize("n,m", [((1 << 22) + 3, 1), ((1 << 15), 513)])
def test_lms_filtered_shapes(sel, oracle_mod, n, m):
    """The filtered form at the edges of its launch shapes: one candidate over 2^22 + 3 rows
    (one candidate group, the most segments, an odd row count), and 513 candidates over the
    smallest n it takes (two candidate groups, the second with one live candidate)."""
    p = 8
    X, y, _, betas = workloads.lms_problem(n, p, m, seed=n % 101)
    print(f"case lms filtered shape n={n} m={m}", flush=True)
    got = sel.lms_median_sq_residuals(_dev(X), _dev(y), _dev(betas), form=FORMS["filtered"])
    mat = sel.lms_median_sq_residuals(_dev(X), _dev(y), _dev(betas), form=FORMS["materialised"])
    for f in ("value_bits", "less", "equal", "greater", "status"):
        assert np.array_equal(got[f], mat[f]), f
    for c in sorted({0, m - 1}):
        ref = oracle_mod.lms_median_sq(X, y, betas[c:c + 1])[0]
        assert_same_result({f: got[c][f].item() for f in got.dtype.names}, ref, f"candidate {c}")
