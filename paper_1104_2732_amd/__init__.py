"""Exact k-th order statistic selection on MI355X by Kelley's cutting plane.

A thin ctypes binding of ``libcpselect.so`` (built from ``csrc/`` by
``build.py``).  The binding only marshals arguments: every step of the method
runs in the library's HIP kernels.  PyTorch supplies device memory (tensors)
and the current HIP stream.  There is no fallback: if the library is not
built, importing the binding's entry points raises.

Entry points (same names as the C ABI in ``include/cpselect.h``):

- ``Selector.select_kth(x, k)``: the k-th smallest element of a float32 or
  float64 CUDA tensor (1-based k) with its counts.
- ``Selector.objective(x, k, ys)``: the cutting plane's objective, its parts,
  counts and subgradient end points at given trial points.
- ``Selector.select_kth_batched`` / ``lms_median_sq_residuals``: many
  selections in one persistent launch; least median of squares.
- ``Selector.select_kth_learned`` and the ``cps_mlp_*`` / ``cps_features`` /
  ``cps_mixture_generate`` wrappers: the learned bracket proposal, its
  network's forward, gradient, Adam and training driver.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpselect.so")

CPS_F32, CPS_F64 = 0, 1
CPS_OK = 0
CPS_EIO, CPS_EFORMAT, CPS_ESCRATCH = -7, -8, -9
STATUS_OK, STATUS_NAN, STATUS_TIMEOUT, STATUS_INTERNAL = 0, 1, 2, 3
STATS_MAX_PASSES = 96

RESULT_DTYPE = np.dtype([("value_bits", "<u8"), ("value", "<f8"), ("less", "<i8"),
                         ("equal", "<i8"), ("greater", "<i8"), ("passes", "<i4"),
                         ("status", "<i4")])
EVAL_DTYPE = np.dtype([("f", "<f8"), ("A", "<f8"), ("B", "<f8"), ("L", "<i8"), ("E", "<i8"),
                       ("G", "<i8"), ("pred", "<f8"), ("succ", "<f8"), ("gminus", "<f8"),
                       ("gplus", "<f8")])
STATS_DTYPE = np.dtype([("passes", "<i4"), ("work_passes", "<i4"), ("kelley_steps", "<i4"),
                        ("bisect_steps", "<i4"), ("final_select_size", "<i4"),
                        ("bracket_used", "<i4"), ("elements_read", "<i8"),
                        ("elements_written", "<i8"),
                        ("population", "<i8", (STATS_MAX_PASSES,)),
                        ("working", "<i8", (STATS_MAX_PASSES,)),
                        ("t_start", "<u8"),
                        ("t_arrive", "<u8", (STATS_MAX_PASSES,)),
                        ("t_publish", "<u8", (STATS_MAX_PASSES,)),
                        ("kind", "<i4", (STATS_MAX_PASSES,)),
                        ("trial", "<f8", (STATS_MAX_PASSES,)),
                        ("A", "<f8", (STATS_MAX_PASSES,)),
                        ("B", "<f8", (STATS_MAX_PASSES,)),
                        ("L", "<i8", (STATS_MAX_PASSES,)),
                        ("G", "<i8", (STATS_MAX_PASSES,)),
                        ("pred", "<f8", (STATS_MAX_PASSES,)),
                        ("succ", "<f8", (STATS_MAX_PASSES,))])
PASS_ZERO, PASS_EVAL, PASS_COUNT, PASS_HIST, PASS_GATHER, PASS_FINAL = range(6)
TRIM_DTYPE = np.dtype([("F", "<f8"), ("m", "<f8"), ("below", "<i8"), ("a", "<i8"), ("b", "<i8"),
                       ("status", "<i4"), ("pad", "<i4")])
KNN_DTYPE = np.dtype([("mean", "<f8"), ("dk", "<f4"), ("status", "<i4"), ("below", "<i8"),
                      ("equal", "<i8")])
assert RESULT_DTYPE.itemsize == 48 and EVAL_DTYPE.itemsize == 80


class Options(ctypes.Structure):
    """Mirror of cps_options (see include/cpselect.h)."""
    _fields_ = [("maxit", ctypes.c_int32), ("final_threshold", ctypes.c_int32),
                ("partition_fraction", ctypes.c_double), ("grid_blocks", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("spin_limit", ctypes.c_int64),
                ("use_bracket", ctypes.c_int32), ("compact_proposal", ctypes.c_int32),
                ("bracket_lo", ctypes.c_double), ("bracket_hi", ctypes.c_double),
                ("hist_bits", ctypes.c_int32), ("count_first", ctypes.c_int32),
                ("transform", ctypes.c_int32), ("cooperative", ctypes.c_int32)]


class BatchOptions(ctypes.Structure):
    """Mirror of cps_batch_options (see include/cpselect.h)."""
    _fields_ = [("block_threads", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("split_capacity", ctypes.c_int64), ("final_threshold", ctypes.c_int32),
                ("maxit", ctypes.c_int32), ("partition_fraction", ctypes.c_double),
                ("hist_bits", ctypes.c_int32), ("count_first", ctypes.c_int32),
                ("proposal", ctypes.c_int32), ("blocks_per_array", ctypes.c_int32),
                ("elements_per_block", ctypes.c_int64), ("team_capacity", ctypes.c_int64)]


class TrainOptions(ctypes.Structure):
    """Mirror of cps_train_options (see include/cpselect.h)."""
    _fields_ = [("seed", ctypes.c_uint64), ("n_arrays", ctypes.c_int64),
                ("array_size", ctypes.c_int64), ("epochs", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("lr", ctypes.c_float), ("init", ctypes.c_int32),
                ("holdout", ctypes.c_int64), ("holdout_seed", ctypes.c_uint64)]


class TrainReport(ctypes.Structure):
    """Mirror of cps_train_report."""
    _fields_ = [("first_loss", ctypes.c_double), ("final_loss", ctypes.c_double),
                ("holdout_coverage", ctypes.c_double), ("holdout_width", ctypes.c_double),
                ("steps", ctypes.c_int64), ("examples", ctypes.c_int64)]


MLP_INPUTS, MLP_HIDDEN, MLP_OUTPUTS, MLP_PARAMS = 67, 64, 2, 8642


class CpsError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = lib().cps_status_string(code).decode() if _lib is not None else str(code)
        extra = ""
        if _lib is not None and code == -3:
            extra = f" (hip error {_lib.cps_last_hip_error()})"
        super().__init__(f"{what}: {msg}{extra} [{code}]")
        self.code = code


_lib = None

EXPORTS = ("cps_create", "cps_destroy", "cps_status_string", "cps_last_hip_error",
           "cps_default_options", "cps_reserve", "select_kth", "select_kth_ex", "cps_objective",
           "cps_default_batch_options", "select_kth_batched", "select_kth_batched_ex",
           "cps_reserve_batched", "cps_autotune_batched", "lms_median_sq_residuals",
           "lms_median_sq_residuals_ex",
           "cps_mixture_generate", "cps_features", "cps_mlp_forward", "cps_mlp_loss_grad",
           "cps_mlp_adam", "cps_mlp_init", "cps_learned_bracket", "select_kth_learned",
           "cps_mlp_train", "select_kth_sampled", "cps_sample_bracket", "cps_model_save",
           "cps_model_load", "select_kth_noalloc", "select_kth_batched_ksum", "lts_trimmed_sq", "lts_trimmed_sq_ex",
           "knn_mean", "knn_mean_ex")
STATUS_BADARG = 4
LMS_AUTO, LMS_MATERIALISED, LMS_FILTERED = 0, 1, 2  # cps_lms_form


def lib() -> ctypes.CDLL:
    """Load libcpselect.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    L.cps_create.argtypes = [c_int, ctypes.POINTER(vp)]
    L.cps_create.restype = c_int
    L.cps_destroy.argtypes = [vp]
    L.cps_destroy.restype = c_int
    L.cps_status_string.argtypes = [c_int]
    L.cps_status_string.restype = ctypes.c_char_p
    L.cps_last_hip_error.argtypes = []
    L.cps_last_hip_error.restype = c_int
    L.cps_default_options.argtypes = [ctypes.POINTER(Options)]
    L.cps_default_options.restype = None
    L.cps_reserve.argtypes = [vp, i64, c_int]
    L.cps_reserve.restype = c_int
    L.select_kth.argtypes = [vp, vp, i64, i64, c_int, vp, vp]
    L.select_kth.restype = c_int
    L.select_kth_ex.argtypes = [vp, vp, i64, i64, c_int, ctypes.POINTER(Options), vp, vp, vp]
    L.select_kth_ex.restype = c_int
    L.select_kth_noalloc.argtypes = [vp, vp, i64, i64, c_int, vp, vp]
    L.select_kth_noalloc.restype = c_int
    L.select_kth_batched_ksum.argtypes = [vp, vp, vp, vp, i64, c_int, ctypes.POINTER(BatchOptions),
                                          vp, vp, vp]
    L.select_kth_batched_ksum.restype = c_int
    L.lts_trimmed_sq.argtypes = [vp, vp, vp, vp, i64, i32, i64, i64, vp, vp]
    L.lts_trimmed_sq.restype = c_int
    L.lts_trimmed_sq_ex.argtypes = [vp, vp, vp, vp, i64, i32, i64, i64, i32, vp, vp]
    L.lts_trimmed_sq_ex.restype = c_int
    L.knn_mean.argtypes = [vp, vp, vp, vp, i64, i32, i64, i64, vp, vp]
    L.knn_mean.restype = c_int
    L.knn_mean_ex.argtypes = [vp, vp, vp, vp, i64, i32, i64, i64, i32, vp, vp]
    L.knn_mean_ex.restype = c_int
    L.cps_objective.argtypes = [vp, vp, i64, i64, c_int, vp, i64, vp, vp]
    L.cps_objective.restype = c_int
    L.cps_default_batch_options.argtypes = [ctypes.POINTER(BatchOptions)]
    L.cps_default_batch_options.restype = None
    L.select_kth_batched.argtypes = [vp, vp, vp, vp, i64, c_int, vp, vp]
    L.select_kth_batched.restype = c_int
    L.select_kth_batched_ex.argtypes = [vp, vp, vp, vp, i64, c_int, ctypes.POINTER(BatchOptions),
                                        vp, vp]
    L.select_kth_batched_ex.restype = c_int
    L.cps_reserve_batched.argtypes = [vp, c_int, ctypes.POINTER(BatchOptions)]
    L.cps_reserve_batched.restype = c_int
    L.cps_autotune_batched.argtypes = [vp, vp, vp, vp, i64, c_int, vp, vp,
                                       ctypes.POINTER(BatchOptions), ctypes.POINTER(ctypes.c_double)]
    L.cps_autotune_batched.restype = c_int
    L.lms_median_sq_residuals.argtypes = [vp, vp, vp, vp, i64, i32, i64, vp, vp]
    L.lms_median_sq_residuals.restype = c_int
    L.lms_median_sq_residuals_ex.argtypes = [vp, vp, vp, vp, i64, i32, i64, i32, vp, vp]
    L.lms_median_sq_residuals_ex.restype = c_int
    u64, f32 = ctypes.c_uint64, ctypes.c_float
    L.cps_mixture_generate.argtypes = [vp, u64, i64, i64, i64, vp, vp, vp]
    L.cps_features.argtypes = [vp, vp, vp, vp, i64, c_int, vp, vp, vp, vp]
    L.cps_mlp_forward.argtypes = [vp, vp, vp, i64, vp, vp]
    L.cps_mlp_loss_grad.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp]
    L.cps_mlp_adam.argtypes = [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, vp]
    L.cps_mlp_init.argtypes = [vp, u64, vp, vp]
    L.cps_learned_bracket.argtypes = [vp, vp, i64, i64, c_int, vp, vp, vp]
    L.select_kth_learned.argtypes = [vp, vp, i64, i64, c_int, vp, ctypes.POINTER(Options), vp,
                                     vp, vp]
    L.cps_mlp_train.argtypes = [vp, ctypes.POINTER(TrainOptions), vp, ctypes.POINTER(TrainReport),
                                vp]
    L.select_kth_sampled.argtypes = [vp, vp, i64, i64, c_int, ctypes.c_double,
                                     ctypes.POINTER(Options), vp, vp, vp]
    L.cps_sample_bracket.argtypes = [vp, vp, i64, i64, c_int, ctypes.c_double, vp, vp]
    L.cps_model_save.argtypes = [vp, ctypes.c_char_p]
    L.cps_model_load.argtypes = [ctypes.c_char_p, vp]
    for name in ("cps_mixture_generate", "cps_features", "cps_mlp_forward", "cps_mlp_loss_grad",
                 "cps_mlp_adam", "cps_mlp_init", "cps_learned_bracket", "select_kth_learned",
                 "cps_mlp_train", "select_kth_sampled", "cps_sample_bracket", "cps_model_save",
                 "cps_model_load"):
        getattr(L, name).restype = c_int
    _lib = L
    return L


def default_options(**kw) -> Options:
    o = Options()
    lib().cps_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def default_batch_options(**kw) -> BatchOptions:
    o = BatchOptions()
    lib().cps_default_batch_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return CPS_F32
    if t.dtype == torch.float64:
        return CPS_F64
    raise TypeError(f"unsupported dtype {t.dtype}; expected float32 or float64")


def _stream_ptr(device) -> int:
    import torch
    return torch.cuda.current_stream(device).cuda_stream


def _check(rc: int, what: str) -> None:
    if rc != CPS_OK:
        raise CpsError(rc, what)


def _as_records(buf, dtype: np.dtype) -> np.ndarray:
    return buf.cpu().numpy().view(dtype)


class Selector:
    """A library handle bound to one GPU (owns the workspace)."""

    def __init__(self, device: int = 0):
        import torch
        self.device = torch.device("cuda", device)
        self._h = ctypes.c_void_p()
        _check(lib().cps_create(device, ctypes.byref(self._h)), "cps_create")

    def close(self) -> None:
        if self._h:
            import torch
            torch.cuda.synchronize(self.device)
            lib().cps_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._h and _lib is not None:
                _lib.cps_destroy(self._h)
        except Exception:
            pass

    # -- raw, asynchronous entry points (no host synchronisation) --------------------

    def new_results(self, count: int = 1):
        import torch
        return torch.empty(count * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=self.device)

    def new_stats(self):
        import torch
        return torch.zeros(STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)

    def select_kth_async(self, x, k: int, out, stats=None, options: Options | None = None) -> None:
        """Enqueue select_kth_ex on the current stream; results land in `out` (device bytes)."""
        if not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous CUDA tensor")
        code = _dtype_code(x)
        rc = lib().select_kth_ex(self._h, ctypes.c_void_p(x.data_ptr()), x.numel(), int(k), code,
                                 ctypes.byref(options) if options is not None else None,
                                 ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(stats.data_ptr()) if stats is not None else None,
                                 ctypes.c_void_p(_stream_ptr(self.device)))
        _check(rc, "select_kth_ex")

    def select_kth_noalloc_async(self, x, k: int, out) -> None:
        """Enqueue select_kth_noalloc on the current stream (no allocation, static scratch)."""
        if not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous CUDA tensor")
        rc = lib().select_kth_noalloc(self._h, ctypes.c_void_p(x.data_ptr()), x.numel(), int(k),
                                      _dtype_code(x), ctypes.c_void_p(out.data_ptr()),
                                      ctypes.c_void_p(_stream_ptr(self.device)))
        _check(rc, "select_kth_noalloc")

    def reserve(self, n: int, dtype_code: int) -> None:
        _check(lib().cps_reserve(self._h, int(n), int(dtype_code)), "cps_reserve")

    # -- convenience (synchronising) wrappers ------------------------------------------

    def select_kth(self, x, k: int, options: Options | None = None, stats: bool = False):
        """Synchronous select_kth: returns a dict (and the stats record when asked)."""
        import torch
        out = self.new_results(1)
        st = self.new_stats() if stats else None
        self.select_kth_async(x, k, out, st, options)
        torch.cuda.synchronize(self.device)
        r = _as_records(out, RESULT_DTYPE)[0]
        res = {name: r[name].item() for name in RESULT_DTYPE.names}
        if stats:
            return res, _as_records(st, STATS_DTYPE)[0]
        return res

    # -- batched ---------------------------------------------------------------------

    def batch_descriptors(self, arrays, ks):
        """Device descriptor arrays (pointers, sizes, ranks) for a list of CUDA tensors."""
        import torch
        if not arrays:
            raise ValueError("empty batch")
        dt = arrays[0].dtype
        for a in arrays:
            if not a.is_cuda or not a.is_contiguous() or a.dtype != dt:
                raise ValueError("batch arrays must be contiguous CUDA tensors of one dtype")
        ptrs = torch.tensor([a.data_ptr() for a in arrays], dtype=torch.int64, device=self.device)
        sizes = torch.tensor([a.numel() for a in arrays], dtype=torch.int64, device=self.device)
        kk = torch.tensor([int(k) for k in ks], dtype=torch.int64, device=self.device)
        return ptrs, sizes, kk, _dtype_code(arrays[0])

    def select_kth_batched_async(self, ptrs, sizes, ks, count: int, dtype_code: int, out,
                                 options: BatchOptions | None = None) -> None:
        """Enqueue select_kth_batched(_ex) on the current stream (device descriptors)."""
        rc = lib().select_kth_batched_ex(self._h, ctypes.c_void_p(ptrs.data_ptr()),
                                         ctypes.c_void_p(sizes.data_ptr()),
                                         ctypes.c_void_p(ks.data_ptr()), int(count), int(dtype_code),
                                         ctypes.byref(options) if options is not None else None,
                                         ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(_stream_ptr(self.device)))
        _check(rc, "select_kth_batched")

    def reserve_batched(self, dtype_code: int, options: BatchOptions | None = None) -> None:
        _check(lib().cps_reserve_batched(self._h, int(dtype_code),
                                         ctypes.byref(options) if options is not None else None),
               "cps_reserve_batched")

    def autotune_batched(self, ptrs, sizes, ks, count: int, dtype_code: int, out):
        """Run the library's autotuner on this batch; returns (options, ms)."""
        best = BatchOptions()
        ms = ctypes.c_double()
        rc = lib().cps_autotune_batched(self._h, ctypes.c_void_p(ptrs.data_ptr()),
                                        ctypes.c_void_p(sizes.data_ptr()),
                                        ctypes.c_void_p(ks.data_ptr()), int(count), int(dtype_code),
                                        ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(_stream_ptr(self.device)),
                                        ctypes.byref(best), ctypes.byref(ms))
        _check(rc, "cps_autotune_batched")
        return best, ms.value

    def select_kth_batched_ksum_async(self, ptrs, sizes, ks, count: int, dtype_code: int, out,
                                      ksum, options: BatchOptions | None = None) -> None:
        """Enqueue select_kth_batched_ksum: results in `out`, sums of the k smallest in `ksum`."""
        rc = lib().select_kth_batched_ksum(self._h, ctypes.c_void_p(ptrs.data_ptr()),
                                           ctypes.c_void_p(sizes.data_ptr()),
                                           ctypes.c_void_p(ks.data_ptr()), int(count),
                                           int(dtype_code),
                                           ctypes.byref(options) if options is not None else None,
                                           ctypes.c_void_p(out.data_ptr()), self._ptr(ksum),
                                           ctypes.c_void_p(_stream_ptr(self.device)))
        _check(rc, "select_kth_batched_ksum")

    def select_kth_batched_ksum(self, arrays, ks, options: BatchOptions | None = None):
        """(RESULT_DTYPE records, float64 sums of each array's k smallest) for CUDA tensors."""
        import torch
        ptrs, sizes, kk, code = self.batch_descriptors(arrays, ks)
        out = self.new_results(len(arrays))
        ksum = torch.empty(len(arrays), dtype=torch.float64, device=self.device)
        self.select_kth_batched_ksum_async(ptrs, sizes, kk, len(arrays), code, out, ksum, options)
        torch.cuda.synchronize(self.device)
        return _as_records(out, RESULT_DTYPE).copy(), ksum.cpu().numpy()

    def select_kth_batched(self, arrays, ks, options: BatchOptions | None = None) -> np.ndarray:
        """Synchronous batched selection over a list of CUDA tensors; returns RESULT_DTYPE records."""
        import torch
        ptrs, sizes, kk, code = self.batch_descriptors(arrays, ks)
        out = self.new_results(len(arrays))
        self.select_kth_batched_async(ptrs, sizes, kk, len(arrays), code, out, options)
        torch.cuda.synchronize(self.device)
        return _as_records(out, RESULT_DTYPE).copy()

    # -- least median of squares -------------------------------------------------------

    def lms_median_sq_residuals_async(self, X, y, betas, out, form: int = 0) -> None:
        """Enqueue lms_median_sq_residuals_ex: X (n x p), y (n), betas (m x p), float64 CUDA
        tensors; form LMS_AUTO, LMS_MATERIALISED or LMS_FILTERED."""
        import torch
        for t in (X, y, betas):
            if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float64:
                raise ValueError("X, y and betas must be contiguous float64 CUDA tensors")
        n, p = X.shape
        m = betas.shape[0]
        if y.numel() != n or betas.shape[1] != p:
            raise ValueError("shape mismatch between X, y and betas")
        rc = lib().lms_median_sq_residuals_ex(self._h, ctypes.c_void_p(X.data_ptr()),
                                              ctypes.c_void_p(y.data_ptr()),
                                              ctypes.c_void_p(betas.data_ptr()), n, p, m, form,
                                              ctypes.c_void_p(out.data_ptr()),
                                              ctypes.c_void_p(_stream_ptr(self.device)))
        _check(rc, "lms_median_sq_residuals_ex")

    def lms_median_sq_residuals(self, X, y, betas, form: int = 0) -> np.ndarray:
        import torch
        out = self.new_results(betas.shape[0])
        self.lms_median_sq_residuals_async(X, y, betas, out, form)
        torch.cuda.synchronize(self.device)
        return _as_records(out, RESULT_DTYPE).copy()

    def lts_trimmed_sq_async(self, X, y, betas, h: int, out, form: int = 0) -> None:
        """Enqueue lts_trimmed_sq_ex: X (n x p), y (n), betas (m x p) float64 CUDA tensors;
        form LMS_AUTO, LMS_MATERIALISED or LMS_FILTERED."""
        import torch
        for t in (X, y, betas):
            if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float64:
                raise ValueError("X, y and betas must be contiguous float64 CUDA tensors")
        n, p = X.shape
        m = betas.shape[0]
        if y.numel() != n or betas.shape[1] != p:
            raise ValueError("shape mismatch between X, y and betas")
        _check(lib().lts_trimmed_sq_ex(self._h, self._ptr(X), self._ptr(y), self._ptr(betas), n, p,
                                       m, int(h), int(form), self._ptr(out),
                                       ctypes.c_void_p(_stream_ptr(self.device))), "lts_trimmed_sq_ex")

    def lts_trimmed_sq(self, X, y, betas, h: int | None = None, form: int = 0) -> np.ndarray:
        """Least trimmed squares per candidate (h defaults to floor((n+1)/2)); TRIM_DTYPE."""
        import torch
        m = betas.shape[0]
        h = (X.shape[0] + 1) // 2 if h is None else int(h)
        out = torch.empty(m * TRIM_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        self.lts_trimmed_sq_async(X, y, betas, h, out, form)
        torch.cuda.synchronize(self.device)
        return _as_records(out, TRIM_DTYPE).copy()

    def knn_mean_async(self, P, f, Q, k: int, out, form: int = 0) -> None:
        """Enqueue knn_mean_ex: P (n x dim), f (n), Q (nq x dim) float32 CUDA tensors; form
        LMS_AUTO, LMS_MATERIALISED or LMS_FILTERED."""
        import torch
        for t in (P, f, Q):
            if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float32:
                raise ValueError("P, f and Q must be contiguous float32 CUDA tensors")
        n, dim = P.shape
        nq = Q.shape[0]
        if f.numel() != n or Q.shape[1] != dim:
            raise ValueError("shape mismatch between P, f and Q")
        _check(lib().knn_mean_ex(self._h, self._ptr(P), self._ptr(f), self._ptr(Q), n, dim, nq,
                                 int(k), int(form), self._ptr(out),
                                 ctypes.c_void_p(_stream_ptr(self.device))), "knn_mean_ex")

    def knn_mean(self, P, f, Q, k: int, form: int = 0) -> np.ndarray:
        """The mean ordinate of each query's k nearest points; KNN_DTYPE records."""
        import torch
        out = torch.empty(Q.shape[0] * KNN_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        self.knn_mean_async(P, f, Q, k, out, form)
        torch.cuda.synchronize(self.device)
        return _as_records(out, KNN_DTYPE).copy()

    def objective(self, x, k: int, ys) -> np.ndarray:
        """cps_objective at every y in `ys` (array-like of float64); returns EVAL_DTYPE records."""
        import torch
        if not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous CUDA tensor")
        ys_t = torch.as_tensor(np.ascontiguousarray(ys, dtype=np.float64), device=self.device)
        out = torch.empty(ys_t.numel() * EVAL_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        rc = lib().cps_objective(self._h, ctypes.c_void_p(x.data_ptr()), x.numel(), int(k),
                                 _dtype_code(x), ctypes.c_void_p(ys_t.data_ptr()), ys_t.numel(),
                                 ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(_stream_ptr(self.device)))
        _check(rc, "cps_objective")
        torch.cuda.synchronize(self.device)
        return _as_records(out, EVAL_DTYPE).copy()

    # -- learned bracket proposal ------------------------------------------------------

    def _ptr(self, t) -> ctypes.c_void_p:
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("expected a contiguous CUDA tensor")
        return ctypes.c_void_p(t.data_ptr())

    def _float_params(self, params):
        import torch
        if params.dtype != torch.float32 or params.numel() != MLP_PARAMS:
            raise ValueError(f"params must be {MLP_PARAMS} float32 values")
        return self._ptr(params)

    def new_params(self):
        import torch
        return torch.zeros(MLP_PARAMS, dtype=torch.float32, device=self.device)

    def mixture_generate(self, seed: int, first_id: int, count: int, n: int):
        """(arrays count x n float32, ranks) of the synthetic mixture family."""
        import torch
        x = torch.empty((count, n), dtype=torch.float32, device=self.device)
        ks = torch.empty(count, dtype=torch.int64, device=self.device)
        _check(lib().cps_mixture_generate(self._h, int(seed), int(first_id), int(count), int(n),
                                          self._ptr(x), self._ptr(ks),
                                          ctypes.c_void_p(_stream_ptr(self.device))),
               "cps_mixture_generate")
        return x, ks

    def features(self, ptrs, sizes, ks, count: int, dtype_code: int):
        """(features count x 67 float32, ranges count x 2 float64, valid int32) tensors."""
        import torch
        feat = torch.empty((count, MLP_INPUTS), dtype=torch.float32, device=self.device)
        rng = torch.empty((count, 2), dtype=torch.float64, device=self.device)
        valid = torch.empty(count, dtype=torch.int32, device=self.device)
        _check(lib().cps_features(self._h, self._ptr(ptrs), self._ptr(sizes), self._ptr(ks),
                                  int(count), int(dtype_code), self._ptr(feat), self._ptr(rng),
                                  self._ptr(valid), ctypes.c_void_p(_stream_ptr(self.device))),
               "cps_features")
        return feat, rng, valid

    def mlp_forward(self, params, feat):
        import torch
        out = torch.empty((feat.shape[0], MLP_OUTPUTS), dtype=torch.float32, device=self.device)
        _check(lib().cps_mlp_forward(self._h, self._float_params(params), self._ptr(feat),
                                     int(feat.shape[0]), self._ptr(out),
                                     ctypes.c_void_p(_stream_ptr(self.device))), "cps_mlp_forward")
        return out

    def mlp_loss_grad(self, params, feat, ustar):
        """(loss tensor of 1, gradient tensor of MLP_PARAMS) for one batch."""
        import torch
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(lib().cps_mlp_loss_grad(self._h, self._float_params(params), self._ptr(feat),
                                       self._ptr(ustar), int(feat.shape[0]), self._ptr(grad),
                                       self._ptr(loss), ctypes.c_void_p(_stream_ptr(self.device))),
               "cps_mlp_loss_grad")
        return loss, grad

    def mlp_adam(self, params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999,
                 eps=1e-8) -> None:
        _check(lib().cps_mlp_adam(self._h, self._float_params(params), self._ptr(grad),
                                  self._ptr(m), self._ptr(v), int(step), float(lr), float(beta1),
                                  float(beta2), float(eps),
                                  ctypes.c_void_p(_stream_ptr(self.device))), "cps_mlp_adam")

    def mlp_init(self, seed: int, params=None):
        params = self.new_params() if params is None else params
        _check(lib().cps_mlp_init(self._h, int(seed), self._float_params(params),
                                  ctypes.c_void_p(_stream_ptr(self.device))), "cps_mlp_init")
        return params

    def sample_bracket(self, x, k: int, z: float = 4.0):
        """(a, b, use) of the non-learned sample-quantile baseline for x and rank k."""
        import torch
        br = torch.empty(3, dtype=torch.float64, device=self.device)
        _check(lib().cps_sample_bracket(self._h, self._ptr(x), x.numel(), int(k), _dtype_code(x),
                                        float(z), self._ptr(br),
                                        ctypes.c_void_p(_stream_ptr(self.device))),
               "cps_sample_bracket")
        torch.cuda.synchronize(self.device)
        a, b, use = br.cpu().tolist()
        return a, b, int(use)

    def learned_bracket(self, x, k: int, params):
        """(a, b, use) the network proposes for x and rank k."""
        import torch
        br = torch.empty(3, dtype=torch.float64, device=self.device)
        _check(lib().cps_learned_bracket(self._h, self._ptr(x), x.numel(), int(k), _dtype_code(x),
                                         self._float_params(params), self._ptr(br),
                                         ctypes.c_void_p(_stream_ptr(self.device))),
               "cps_learned_bracket")
        torch.cuda.synchronize(self.device)
        a, b, use = br.cpu().tolist()
        return a, b, int(use)

    def select_kth_learned_async(self, x, k: int, params, out, stats=None,
                                 options: Options | None = None) -> None:
        rc = lib().select_kth_learned(self._h, self._ptr(x), x.numel(), int(k), _dtype_code(x),
                                      self._float_params(params),
                                      ctypes.byref(options) if options is not None else None,
                                      self._ptr(out),
                                      self._ptr(stats) if stats is not None else None,
                                      ctypes.c_void_p(_stream_ptr(self.device)))
        _check(rc, "select_kth_learned")

    def select_kth_learned(self, x, k: int, params, options: Options | None = None,
                           stats: bool = False):
        import torch
        out = self.new_results(1)
        st = self.new_stats() if stats else None
        self.select_kth_learned_async(x, k, params, out, st, options)
        torch.cuda.synchronize(self.device)
        r = _as_records(out, RESULT_DTYPE)[0]
        res = {name: r[name].item() for name in RESULT_DTYPE.names}
        if stats:
            return res, _as_records(st, STATS_DTYPE)[0]
        return res

    def select_kth_sampled_async(self, x, k: int, out, z: float = 4.0, stats=None,
                                 options: Options | None = None) -> None:
        rc = lib().select_kth_sampled(self._h, self._ptr(x), x.numel(), int(k), _dtype_code(x),
                                      float(z),
                                      ctypes.byref(options) if options is not None else None,
                                      self._ptr(out),
                                      self._ptr(stats) if stats is not None else None,
                                      ctypes.c_void_p(_stream_ptr(self.device)))
        _check(rc, "select_kth_sampled")

    def select_kth_sampled(self, x, k: int, z: float = 4.0, options: Options | None = None,
                           stats: bool = False):
        import torch
        out = self.new_results(1)
        st = self.new_stats() if stats else None
        self.select_kth_sampled_async(x, k, out, z, st, options)
        torch.cuda.synchronize(self.device)
        r = _as_records(out, RESULT_DTYPE)[0]
        res = {name: r[name].item() for name in RESULT_DTYPE.names}
        if stats:
            return res, _as_records(st, STATS_DTYPE)[0]
        return res

    def model_save(self, params, path: str) -> None:
        """Write the network's parameters to a versioned, hashed file (cps_model_save)."""
        _check(lib().cps_model_save(self._float_params(params), os.fsencode(path)),
               "cps_model_save")

    def model_load(self, path: str, params=None):
        """Read a network file into `params` (a new device tensor when None)."""
        params = self.new_params() if params is None else params
        _check(lib().cps_model_load(os.fsencode(path), self._float_params(params)),
               "cps_model_load")
        return params

    def mlp_train(self, params, seed: int, n_arrays: int, array_size: int, epochs: int,
                  batch: int = 256, lr: float = 1e-3, init: bool = True, holdout: int = 0,
                  holdout_seed: int = 1) -> dict:
        """Run the library's training driver (synchronises); returns the report as a dict."""
        o = TrainOptions(seed=int(seed), n_arrays=int(n_arrays), array_size=int(array_size),
                         epochs=int(epochs), batch=int(batch), lr=float(lr), init=1 if init else 0,
                         holdout=int(holdout), holdout_seed=int(holdout_seed))
        rep = TrainReport()
        _check(lib().cps_mlp_train(self._h, ctypes.byref(o), self._float_params(params),
                                   ctypes.byref(rep), ctypes.c_void_p(_stream_ptr(self.device))),
               "cps_mlp_train")
        return {name: getattr(rep, name) for name, _ in TrainReport._fields_}
