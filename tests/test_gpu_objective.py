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
