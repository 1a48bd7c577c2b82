"""GPU parity of cps_objective against the CPU oracle (Section 3, Eq. 2).

f within the stated relative tolerance (1e-12 for float64 inputs, 1e-6 for
float32 inputs), counts, neighbours and subgradient end points exactly.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {np.float32: 1e-6, np.float64: 1e-12}


@pytest.fixture(scope="module")
def sel():
    import paper_1104_2732_amd as cps
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = cps.Selector(0)
    yield s
    s.close()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("dist", ["uniform", "normal", "cauchy", "quantized_normal", "mix1"])
def test_objective_parity(sel, oracle_mod, dist, dtype):
    for n in (1, 7, 1000, 65_537, 400_001):
        x = workloads.single_array(dist, n, dtype, seed=n + 11, tag="gpu-obj")
        rng = np.random.default_rng(n)
        ys = np.concatenate([x[rng.integers(0, n, 8)].astype(np.float64),
                             rng.normal(size=6), [x.min(), x.max(), -1e30, 1e30]])
        for k in sorted({1, (n + 1) // 2, n}):
            print(f"case objective {dist} n={n} k={k} dtype={dtype}", flush=True)
            got = sel.objective(torch.from_numpy(x).cuda(), k, ys)
            ref = oracle_mod.objective(x, k, ys)
            for g, r in zip(got, ref):
                assert (g["L"], g["E"], g["G"]) == (r["L"], r["E"], r["G"])
                assert g["pred"] == r["pred"] and g["succ"] == r["succ"]
                assert g["gminus"] == r["gminus"] and g["gplus"] == r["gplus"]
                for f in ("f", "A", "B"):
                    if r[f] == 0:
                        assert g[f] == 0
                    else:
                        assert abs(g[f] - r[f]) <= TOL[dtype] * abs(r[f]), (f, g[f], r[f])


ALPHA_BETA = lambda n, k: (k - 0.5, n - k + 0.5)  # noqa: E731  (Section 3, Eq. 2)

SCHEDULES = {
    # every pass an evaluation of A, B, the counts and the neighbours over the whole array,
    # then the gather and the exact select (Algorithm 1 iterated)
    "cutting_plane": dict(partition_fraction=0.0, hist_bits=0, final_threshold=4096),
    # the split at the first trial point: later evaluations read the compacted bracket and
    # rebuild A and B of the whole array from the bracket's sums
    "split": dict(count_first=0, hist_bits=0, final_threshold=4096),
    # the default: pass 0, the counting evaluation, histogram passes
    "default": dict(),
}


def _close(g, r, tol):
    return g == r if r == 0 else abs(g - r) <= tol * abs(r)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("schedule", list(SCHEDULES))
def test_hot_path_pass_trace(sel, oracle_mod, dtype, schedule):
    """What the selection's own passes computed (the per-pass trace of cps_stats) against the
    float64 objective of the oracle at the same points: pass 0's f at the extremes from the
    sum (Section 4, step 0) and the extremes' multiplicities; every evaluation's A, B and
    f = alpha A + beta B within the tolerance, its counts and neighbours exactly; a counting
    evaluation's counts exactly."""
    import paper_1104_2732_amd as cps
    n = (1 << 22) + 17
    dists = ["normal", "uniform", "cauchy", "quantized_normal"]
    if schedule != "cutting_plane":
        dists = dists[:2]
    tol = TOL[dtype]
    for dist in dists:
        x = workloads.single_array(dist, n, dtype, seed=31, tag="gpu-trace")
        xt = torch.from_numpy(x).cuda()
        for k in (n // 100, (n + 1) // 2):
            print(f"case pass-trace {schedule} {dist} n={n} k={k} dtype={x.dtype}", flush=True)
            res, st = sel.select_kth(xt, k, options=cps.default_options(**SCHEDULES[schedule]),
                                     stats=True)
            ref = oracle_mod.select_kth(x, k)
            assert res["status"] == 0 and res["value_bits"] == ref["value_bits"]
            npass = min(int(st["work_passes"]), cps.STATS_MAX_PASSES)
            kinds = st["kind"][:npass]
            assert kinds[0] == cps.PASS_ZERO
            ys = np.array([st["trial"][i] for i in range(npass)
                           if kinds[i] in (cps.PASS_EVAL, cps.PASS_COUNT)]
                          + [float(x.min()), float(x.max())], dtype=np.float64)
            ev = oracle_mod.objective(x, k, ys)
            by_y = {float(y): e for y, e in zip(ys, ev)}
            alpha, beta = ALPHA_BETA(n, k)
            lo, hi = by_y[float(x.min())], by_y[float(x.max())]
            # pass 0: A at the minimum, B at the maximum, the extremes and multiplicities
            assert st["pred"][0] == x.min() and st["succ"][0] == x.max()
            assert (st["L"][0], st["G"][0]) == (lo["E"], hi["E"])
            assert _close(st["A"][0], lo["A"], tol), (st["A"][0], lo["A"])
            assert _close(st["B"][0], hi["B"], tol), (st["B"][0], hi["B"])
            assert _close(alpha * st["A"][0], lo["f"], tol) and _close(beta * st["B"][0], hi["f"], tol)
            n_eval = 0
            for i in range(1, npass):
                if kinds[i] not in (cps.PASS_EVAL, cps.PASS_COUNT):
                    continue
                r = by_y[float(st["trial"][i])]
                ctx = (schedule, dist, k, i, int(kinds[i]))
                assert (st["L"][i], st["G"][i]) == (r["L"], r["G"]), ctx
                if kinds[i] == cps.PASS_COUNT:
                    continue
                n_eval += 1
                assert _close(st["A"][i], r["A"], tol), (ctx, st["A"][i], r["A"])
                assert _close(st["B"][i], r["B"], tol), (ctx, st["B"][i], r["B"])
                f = alpha * st["A"][i] + beta * st["B"][i]
                assert _close(f, r["f"], tol), (ctx, f, r["f"])
                # neighbours of the working set: those of the whole array when it is read,
                # else the same wherever the working set holds one (the bracket's elements
                # below / above t include the array's nearest ones)
                if st["working"][i] == n or np.isfinite(st["pred"][i]):
                    assert st["pred"][i] == r["pred"], ctx
                if st["working"][i] == n or np.isfinite(st["succ"][i]):
                    assert st["succ"][i] == r["succ"], ctx
            if schedule == "cutting_plane":
                assert n_eval >= 3, (dist, k, n_eval)
        del xt


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("dist", ["outliers20", "normal"])
def test_transform_pass_trace(sel, oracle_mod, dtype, dist):
    """The log transform of Section 5.3 (cps_options.transform): every evaluation's A and B are
    those of F(x) = log(1 + x - min x) at F(t) within 1e-6 (the oracle's objective of the
    transformed array, formed in float64 from the exact widening of x; the kernel forms F to
    float precision, ~1e-7 relative per term, and every term of a sum has one sign), its
    counts those of x; the selected value and counts are exact."""
    import paper_1104_2732_amd as cps
    n = (1 << 22) + 17
    x = workloads.single_array(dist, n, dtype, seed=5, tag="gpu-transform")
    xt = torch.from_numpy(x).cuda()
    F = np.log1p(x.astype(np.float64) - float(x.min()))
    cp = dict(partition_fraction=0.0, hist_bits=0, final_threshold=4096)
    for k in (n // 100, (n + 1) // 2):
        print(f"case transform {dist} n={n} k={k} dtype={x.dtype}", flush=True)
        ref = oracle_mod.select_kth(x, k)
        res, st = sel.select_kth(xt, k, options=cps.default_options(transform=1, **cp), stats=True)
        assert res["status"] == 0 and res["value_bits"] == ref["value_bits"]
        assert (res["less"], res["equal"]) == (ref["less"], ref["equal"])
        npass = min(int(st["work_passes"]), cps.STATS_MAX_PASSES)
        evals = [i for i in range(npass) if st["kind"][i] == cps.PASS_EVAL]
        assert evals and st["trial"][evals[0]] == x.min()  # F's objective at the ends first
        ts = np.array([float(st["trial"][i]) for i in evals])
        us = np.log1p(ts - float(x.min()))
        ev = oracle_mod.objective(F, k, us)   # sums on F's scale
        evx = oracle_mod.objective(x, k, ts)  # counts on x
        for j, i in enumerate(evals):
            r = ev[j]
            assert (st["L"][i], st["G"][i]) == (evx[j]["L"], evx[j]["G"]), i
            assert _close(st["A"][i], r["A"], 1e-6), (i, st["A"][i], r["A"])
            assert _close(st["B"][i], r["B"], 1e-6), (i, st["B"][i], r["B"])
        # exact with the default schedule too (the transform only places the trial point)
        res2 = sel.select_kth(xt, k, options=cps.default_options(transform=1))
        assert res2["value_bits"] == ref["value_bits"] and res2["less"] == ref["less"]
        if dist == "outliers20":
            # (the trajectory is not pinned: the passes are reported, not compared)
            _, st0 = sel.select_kth(xt, k, options=cps.default_options(**cp), stats=True)
            print(f"passes with the transform {int(st['work_passes'])}, on x "
                  f"{int(st0['work_passes'])}", flush=True)
    del xt
