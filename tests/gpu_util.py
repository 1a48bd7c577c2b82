"""Helpers shared by the GPU tests (host-side bookkeeping only)."""
import numpy as np


def bits_of(value: float, dtype) -> int:
    a = np.array([value], dtype=dtype)
    return int(a.view(np.uint32 if np.dtype(dtype) == np.float32 else np.uint64)[0])


def assert_same_result(gpu: dict, ref: dict, ctx=""):
    assert gpu["status"] == 0, f"status {gpu['status']} {ctx}"
    assert gpu["value_bits"] == ref["value_bits"], f"value {gpu['value']} vs {ref['value']} {ctx}"
    assert (gpu["less"], gpu["equal"], gpu["greater"]) == (ref["less"], ref["equal"], ref["greater"]), \
        f"counts {gpu} vs {ref} {ctx}"


def invariant_holds(x: np.ndarray, k: int, res: dict) -> None:
    """The defining property of x_(k) (Section 1): #(x<m) < k <= #(x<=m), m in x."""
    v = np.array([res["value"]], dtype=x.dtype)[0]
    less = int(np.count_nonzero(x < v))
    eq = int(np.count_nonzero(x == v))
    assert eq >= 1
    assert less < k <= less + eq
    assert (res["less"], res["equal"], res["greater"]) == (less, eq, x.size - less - eq)
