"""select_kth_noalloc (the selection for callers that cannot allocate, with its scratch in a
static device array) against select_kth on the same inputs, through the C ABI: the selected
value bit for bit, its counts and status exactly, on consecutive calls whose inputs shrink
(the array keeps the previous call's contents), for both element types."""
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


FIELDS = ("value_bits", "less", "equal", "greater", "status")


def _both(sel, x, k):
    import paper_1104_2732_amd as cps
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    out_a, out_b = sel.new_results(1), sel.new_results(1)
    sel.select_kth_async(xt, k, out_a)
    sel.select_kth_noalloc_async(xt, k, out_b)
    torch.cuda.synchronize()
    a = out_a.cpu().numpy().view(cps.RESULT_DTYPE)[0]
    b = out_b.cpu().numpy().view(cps.RESULT_DTYPE)[0]
    return a, b


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("dist", ["normal", "quantized_normal", "cauchy", "uniform"])
def test_noalloc_matches_select_kth(sel, oracle_mod, dist, dtype):
    # consecutive calls, each input smaller than the one before: several tiles with a ragged
    # tail, then one read directly by the final select, then a single element
    for n in ((1 << 22) + 17, 70_001, 1000, 1):
        x = workloads.single_array(dist, n, dtype, seed=n, tag="gpu-noalloc")
        for k in sorted({1, max(1, n // 100), (n + 1) // 2, n}):
            print(f"case noalloc {dist} n={n} k={k} dtype={x.dtype}", flush=True)
            a, b = _both(sel, x, k)
            for f in FIELDS:
                assert a[f] == b[f], (dist, n, k, f, a[f], b[f])
            ref = oracle_mod.select_kth(x, k)
            assert int(b["value_bits"]) == ref["value_bits"] and int(b["less"]) == ref["less"]
            assert b["status"] == 0


def test_noalloc_argument_errors(sel):
    import ctypes

    import paper_1104_2732_amd as cps
    L = cps.lib()
    x = torch.zeros(10, device="cuda")
    out = sel.new_results(1)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n, k in ((0, 1), (10, 0), (10, 11)):
        assert L.select_kth_noalloc(sel._h, ctypes.c_void_p(x.data_ptr()), n, k, cps.CPS_F32,
                                    ctypes.c_void_p(out.data_ptr()), s) == -1
    assert L.select_kth_noalloc(sel._h, ctypes.c_void_p(x.data_ptr()), 10, 1, 7,
                                ctypes.c_void_p(out.data_ptr()), s) == -1
    assert L.select_kth_noalloc(sel._h, ctypes.c_void_p(x.data_ptr()), 10, 1, cps.CPS_F32,
                                None, s) == -1
