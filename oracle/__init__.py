"""CPU oracle: plain, slow, obviously correct selection and objective evaluation.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library never
does, and shares no code with it.  The heavy lifting lives in ``oracle.c``
(built by ``oracle/build.py`` with gcc); the learned-proposal network's
double-precision reference is ``oracle/mlp.py``.

What each function computes, with the passage it follows:

- ``select_kth``: x_(k), the k-th smallest element (1-based k, IEEE order) and
  its counts #(x<m), #(x=m), #(x>m) (Section 1; median k = floor((n+1)/2)).
- ``objective``: f(y) = sum_i max(alpha (x_i - y), beta (y - x_i)) with
  alpha = k - 1/2, beta = n - k + 1/2 (Section 3, Eqs. 1-2, weights oriented so
  that the minimiser is x_(k)), its parts A(y), B(y), the counts and the
  Clarke subdifferential end points (Section 3).
- ``lms_residuals`` / ``lms_median_sq``: squared regression residuals summed
  in fixed order without fused multiply-add, and their lower median for each
  candidate parameter vector (Section 6, least median of squares).
- ``trimmed_sum`` / ``lts_objective``: the sum of the h smallest values (sorted
  copy, compensated sum of its first h entries), with the h-th smallest m,
  #(r < m), a = h - #(r < m) and #(r = m) (Section 6, least trimmed squares).
- ``knn_distances`` / ``knn_mean``: squared Euclidean distances in float, left
  to right over the coordinates without fused multiply-add; the k-th smallest
  distance and the mean ordinate of the k nearest points with the weight a / b
  on ties at the k-th distance (Section 6, k nearest neighbours).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ORC_OK, ORC_EINVAL, ORC_ENAN, ORC_ENOMEM = 0, -1, -2, -3


class _Result(ctypes.Structure):
    _fields_ = [("value_bits", ctypes.c_uint64), ("value", ctypes.c_double),
                ("less", ctypes.c_int64), ("equal", ctypes.c_int64), ("greater", ctypes.c_int64)]


class _Eval(ctypes.Structure):
    _fields_ = [("f", ctypes.c_double), ("A", ctypes.c_double), ("B", ctypes.c_double),
                ("L", ctypes.c_int64), ("E", ctypes.c_int64), ("G", ctypes.c_int64),
                ("pred", ctypes.c_double), ("succ", ctypes.c_double),
                ("gminus", ctypes.c_double), ("gplus", ctypes.c_double)]


EVAL_DTYPE = np.dtype([("f", "f8"), ("A", "f8"), ("B", "f8"), ("L", "i8"), ("E", "i8"),
                       ("G", "i8"), ("pred", "f8"), ("succ", "f8"), ("gminus", "f8"),
                       ("gplus", "f8")])
assert EVAL_DTYPE.itemsize == ctypes.sizeof(_Eval)


class OracleError(RuntimeError):
    pass


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        for name in ("orc_select_f32", "orc_select_f64"):
            getattr(L, name).argtypes = [vp, i64, i64, ctypes.POINTER(_Result)]
            getattr(L, name).restype = ctypes.c_int
        for name in ("orc_objective_f32", "orc_objective_f64"):
            getattr(L, name).argtypes = [vp, i64, i64, vp, i64, vp]
            getattr(L, name).restype = ctypes.c_int
        L.orc_quickselect_inplace.argtypes = [vp, i64, i64, ctypes.POINTER(ctypes.c_double)]
        L.orc_quickselect_inplace.restype = ctypes.c_int
        L.orc_lms_residuals.argtypes = [vp, vp, vp, i64, i32, vp]
        L.orc_lms_residuals.restype = ctypes.c_int
        L.orc_lms_median_sq.argtypes = [vp, vp, vp, i64, i32, i64, ctypes.POINTER(_Result)]
        L.orc_lms_median_sq.restype = ctypes.c_int
        L.orc_trimmed_sum_f64.argtypes = [vp, i64, i64, vp]
        L.orc_lts_objective.argtypes = [vp, vp, vp, i64, i32, i64, i64, vp]
        L.orc_knn_distances.argtypes = [vp, vp, i64, i32, vp]
        L.orc_knn_mean.argtypes = [vp, vp, vp, i64, i32, i64, i64, vp]
        for name in ("orc_trimmed_sum_f64", "orc_lts_objective", "orc_knn_distances",
                     "orc_knn_mean"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str) -> None:
    if rc == ORC_ENAN:
        raise OracleError(f"{what}: NaN in input")
    if rc != ORC_OK:
        raise OracleError(f"{what}: error {rc}")


def _as_float_array(x) -> np.ndarray:
    x = np.ascontiguousarray(x)
    if x.dtype not in (np.float32, np.float64):
        raise TypeError("x must be float32 or float64")
    return x


def _res_dict(r: _Result) -> dict:
    return {"value_bits": int(r.value_bits), "value": float(r.value), "less": int(r.less),
            "equal": int(r.equal), "greater": int(r.greater)}


def select_kth(x, k: int) -> dict:
    """The k-th smallest element of x (1-based) and its counts; raises on NaN or bad k."""
    x = _as_float_array(x)
    r = _Result()
    fn = lib().orc_select_f32 if x.dtype == np.float32 else lib().orc_select_f64
    _check(fn(x.ctypes.data, x.size, int(k), ctypes.byref(r)), "select_kth")
    return _res_dict(r)


def select_kth_batched(arrays, ks) -> list[dict]:
    """select_kth on each array in turn."""
    return [select_kth(a, int(k)) for a, k in zip(arrays, ks)]


def objective(x, k: int, ys) -> np.ndarray:
    """f, A, B, L, E, G, pred, succ, g-, g+ at each y (structured array, dtype EVAL_DTYPE)."""
    x = _as_float_array(x)
    ys = np.ascontiguousarray(ys, dtype=np.float64).ravel()
    out = np.zeros(ys.size, dtype=EVAL_DTYPE)
    fn = lib().orc_objective_f32 if x.dtype == np.float32 else lib().orc_objective_f64
    _check(fn(x.ctypes.data, x.size, int(k), ys.ctypes.data, ys.size, out.ctypes.data), "objective")
    return out


def quickselect_inplace(work: np.ndarray, k: int) -> float:
    """Quickselect on a float64 working copy that the caller owns (it is permuted)."""
    if work.dtype != np.float64 or not work.flags.c_contiguous:
        raise TypeError("work must be a contiguous float64 array")
    v = ctypes.c_double()
    _check(lib().orc_quickselect_inplace(work.ctypes.data, work.size, int(k), ctypes.byref(v)),
           "quickselect")
    return v.value


def lms_residuals(X, y, b) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n, p = X.shape
    r = np.empty(n)
    _check(lib().orc_lms_residuals(X.ctypes.data, y.ctypes.data, b.ctypes.data, n, p, r.ctypes.data),
           "lms_residuals")
    return r


def lms_median_sq(X, y, betas) -> list[dict]:
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    n, p = X.shape
    m = betas.shape[0]
    out = (_Result * max(m, 1))()
    _check(lib().orc_lms_median_sq(X.ctypes.data, y.ctypes.data, betas.ctypes.data, n, p, m, out),
           "lms_median_sq")
    return [_res_dict(out[i]) for i in range(m)]


TRIM_DTYPE = np.dtype([("F", "f8"), ("m", "f8"), ("below", "i8"), ("a", "i8"), ("b", "i8")])
KNN_DTYPE = np.dtype([("mean", "f8"), ("dk", "f4"), ("pad", "i4"), ("below", "i8"),
                      ("equal", "i8")])


def trimmed_sum(r, h: int) -> dict:
    """The sum of the h smallest values of r (float64) and its h-th smallest value m, with
    #(r < m), a = h - #(r < m) and #(r = m)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.zeros(1, dtype=TRIM_DTYPE)
    _check(lib().orc_trimmed_sum_f64(r.ctypes.data, r.size, int(h), out.ctypes.data),
           "trimmed_sum")
    return {k: out[0][k].item() for k in TRIM_DTYPE.names}


def lts_objective(X, y, betas, h: int | None = None) -> np.ndarray:
    """Least trimmed squares per candidate: the sum of the h smallest squared residuals
    (h = floor((n+1)/2) by default, the rank of the median); TRIM_DTYPE records."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    n, p = X.shape
    m = betas.shape[0]
    h = (n + 1) // 2 if h is None else int(h)
    out = np.zeros(max(m, 1), dtype=TRIM_DTYPE)
    _check(lib().orc_lts_objective(X.ctypes.data, y.ctypes.data, betas.ctypes.data, n, p, m, h,
                                   out.ctypes.data), "lts_objective")
    return out[:m]


def knn_distances(P, q) -> np.ndarray:
    P = np.ascontiguousarray(P, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.float32)
    n, dim = P.shape
    d = np.empty(n, dtype=np.float32)
    _check(lib().orc_knn_distances(P.ctypes.data, q.ctypes.data, n, dim, d.ctypes.data),
           "knn_distances")
    return d


def knn_mean(P, f, Q, k: int) -> np.ndarray:
    """Per query (rows of Q): the k-th smallest squared distance to the rows of P and the mean
    ordinate f of the k nearest points (ties at the k-th distance weighted a / b); KNN_DTYPE."""
    P = np.ascontiguousarray(P, dtype=np.float32)
    f = np.ascontiguousarray(f, dtype=np.float32)
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    n, dim = P.shape
    nq = Q.shape[0]
    out = np.zeros(max(nq, 1), dtype=KNN_DTYPE)
    _check(lib().orc_knn_mean(P.ctypes.data, f.ctypes.data, Q.ctypes.data, n, dim, nq, int(k),
                              out.ctypes.data), "knn_mean")
    return out[:nq]
