"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws data.  It holds none of the selection method's
arithmetic (no objective, no counts, no cutting plane, no residual of a
regression candidate), so that the CPU oracle and the HIP library can both
consume its arrays without sharing any code with each other.

Every array is a pure function of (tag, seed, array id, size, dtype): the
bits come from numpy's Philox-4x64 counter-based generator (Salmon, Moraes,
Dror and Shaw, SC'11).  Large arrays are generated in fixed chunks of
``CHUNK`` elements; chunk ``c`` uses the key's stream advanced by ``c`` jumps,
so the result does not depend on the number of worker threads.

Distributions follow the paper's empirical study (Section 5.1: uniform,
normal, half-normal, beta(2,5) and five two-component mixtures, plus arrays
with a few ~1e9 outliers) and the workloads the benchmark is quoted on
(Cauchy, normal quantised to 1024 levels, lognormal, seeded permutations).
"""
from __future__ import annotations

import hashlib
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 1 << 20

DISTRIBUTIONS = (
    "uniform", "normal", "cauchy", "quantized_normal", "lognormal",
    "halfnormal", "beta25", "mix1", "mix2", "mix3", "mix4", "mix5",
    "outliers", "permutation", "constant", "smallint",
)


def _key(tag: str, seed: int, array_id: int) -> int:
    h = hashlib.sha256(f"{tag}|{seed}|{array_id}".encode()).digest()
    return int.from_bytes(h[:16], "little")


def generator(tag: str, seed: int, array_id: int = 0, chunk: int = 0) -> np.random.Generator:
    """A numpy Generator on the Philox stream for (tag, seed, array_id), advanced by `chunk` jumps."""
    bg = np.random.Philox(key=_key(tag, seed, array_id))
    if chunk:
        bg = bg.jumped(chunk)
    return np.random.Generator(bg)


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunk_values(dist: str, rng: np.random.Generator, m: int, dtype) -> np.ndarray:
    f32 = np.dtype(dtype) == np.float32
    if dist == "uniform":
        # f32: 24 random bits scaled by 2^-24; f64: 53 bits by 2^-53 (never rounds up to 1.0)
        return rng.random(m, dtype=np.float32 if f32 else np.float64)
    if dist == "normal":
        return rng.standard_normal(m).astype(dtype)
    if dist == "cauchy":
        return rng.standard_cauchy(m).astype(dtype)
    if dist == "quantized_normal":
        z = rng.standard_normal(m)
        level = np.clip(np.floor((z + 4.0) * 128.0), 0, 1023)
        return (-4.0 + (level + 0.5) / 128.0).astype(dtype)
    if dist == "lognormal":
        return np.exp(rng.standard_normal(m)).astype(dtype)
    if dist == "halfnormal":
        return np.abs(rng.standard_normal(m)).astype(dtype)
    if dist == "beta25":
        return rng.beta(2.0, 5.0, m).astype(dtype)
    if dist in ("mix1", "mix2", "mix4", "mix5"):
        # first component N(0,1) (mix1, mix2) or half-normal (mix4, mix5); second N(100,1)
        frac = 2.0 / 3.0 if dist in ("mix1", "mix4") else 0.5
        first = rng.random(m) < frac
        a = rng.standard_normal(m)
        if dist in ("mix4", "mix5"):
            a = np.abs(a)
        b = 100.0 + rng.standard_normal(m)
        return np.where(first, a, b).astype(dtype)
    if dist == "mix3":
        a = np.abs(rng.standard_normal(m))
        ten = rng.random(m) < 0.1
        return np.where(ten, 10.0, a).astype(dtype)
    if dist in ("outliers", "outliers20"):
        # N(0,1) with about 1e-5 of the elements replaced by huge values (Section 5.3: ~1e9,
        # and ~1e20 where the sums lose precision), at least three of them
        x = rng.standard_normal(m)
        hit = rng.random(m) < 1e-5
        hit[:3] = True
        rng.shuffle(hit)
        scale = 1e9 if dist == "outliers" else 1e20
        return np.where(hit, scale * (1.0 + rng.random(m)), x).astype(dtype)
    if dist == "smallint":
        return rng.integers(0, 16, m).astype(dtype)
    raise ValueError(f"unknown distribution {dist!r}")


def single_array(dist: str, n: int, dtype=np.float32, seed: int = 0, array_id: int = 0,
                 tag: str = "single") -> np.ndarray:
    """One seeded array of n values of `dtype` drawn from `dist`."""
    dtype = np.dtype(dtype)
    if n < 0:
        raise ValueError("n must be >= 0")
    if dist == "permutation":
        # a seeded permutation of 0..n-1: the k-th smallest is exactly k-1
        rng = generator(tag + ":perm", seed, array_id)
        return rng.permutation(n).astype(dtype)
    if dist == "constant":
        rng = generator(tag + ":const", seed, array_id)
        v = float(rng.standard_normal())
        return np.full(n, v, dtype=dtype)
    if dist == "mix2" or dist == "mix5":
        # "50% of the elements plus one" from the first component, the rest from N(100,1):
        # exact proportions, then a seeded shuffle.
        rng = generator(tag + ":" + dist, seed, array_id)
        n1 = n // 2 + 1 if n else 0
        a = rng.standard_normal(n1)
        if dist == "mix5":
            a = np.abs(a)
        b = 100.0 + rng.standard_normal(n - n1)
        x = np.concatenate([a, b])
        rng.shuffle(x)
        return x.astype(dtype)
    out = np.empty(n, dtype=dtype)
    nchunks = (n + CHUNK - 1) // CHUNK

    def fill(c: int) -> None:
        lo, hi = c * CHUNK, min(n, (c + 1) * CHUNK)
        rng = generator(tag + ":" + dist, seed, array_id, chunk=c)
        out[lo:hi] = _chunk_values(dist, rng, hi - lo, dtype)

    if nchunks <= 1:
        for c in range(nchunks):
            fill(c)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fill, range(nchunks)))
    return out


def ks_for(n: int) -> list[int]:
    """The four ranks the single-array workloads use: 1, n/100, the lower median, n-1 (1-based)."""
    ks = [1, max(1, n // 100), (n + 1) // 2, max(1, n - 1)]
    return ks


def batched_sizes(count: int, seed: int = 0, lo_exp: float = 3.0, hi_exp: float = 6.0) -> np.ndarray:
    """Sizes floor(10^(lo_exp + (hi_exp-lo_exp)*u)), u ~ U[0,1) seeded (log-uniform)."""
    rng = generator("batched:sizes", seed)
    u = rng.random(count)
    return np.floor(10.0 ** (lo_exp + (hi_exp - lo_exp) * u)).astype(np.int64)


def batched_arrays(count: int, seed: int = 0, dtype=np.float32, lo_exp: float = 3.0,
                   hi_exp: float = 6.0, dist: str = "lognormal"):
    """`count` arrays with log-uniform sizes, values from `dist`; returns (list of arrays, sizes, median ks)."""
    sizes = batched_sizes(count, seed, lo_exp, hi_exp)
    arrays = [None] * count

    def one(i: int) -> None:
        rng = generator("batched:" + dist, seed, i)
        arrays[i] = _chunk_values(dist, rng, int(sizes[i]), dtype)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(one, range(count)))
    ks = (sizes + 1) // 2
    return arrays, sizes, ks


def _fixed_order_dot(X: np.ndarray, b: np.ndarray) -> np.ndarray:
    # sum_j X[:, j] * b[j] accumulated left to right; numpy elementwise ops are
    # IEEE round-to-nearest with no fused multiply-add.
    s = X[:, 0] * b[0]
    for j in range(1, X.shape[1]):
        s = s + X[:, j] * b[j]
    return s


def lms_problem(n: int, p: int = 8, m: int = 1024, seed: int = 0, contamination: float = 0.3,
                shift: float = 10.0, noise: float = 0.1):
    """Robust-regression inputs: X (n x p, row-major f64), y, the true beta, and m candidate betas.

    y = X beta* + N(0, noise^2), with exactly floor(contamination*n) seeded rows shifted
    by +shift.  Each candidate solves the p x p system of a seeded p-row elemental subset
    (LU with partial pivoting from LAPACK; subsets with a tiny pivot are redrawn).
    """
    rng = generator("lms", seed)
    X = rng.standard_normal((n, p))
    beta_true = rng.standard_normal(p)
    y = _fixed_order_dot(X, beta_true) + noise * rng.standard_normal(n)
    bad = rng.choice(n, size=int(np.floor(contamination * n)), replace=False)
    y[bad] += shift
    betas = np.empty((m, p))
    j = 0
    while j < m:
        rows = rng.choice(n, size=p, replace=False)
        A = X[rows]
        try:
            sol = np.linalg.solve(A, y[rows])
        except np.linalg.LinAlgError:
            continue
        if not np.all(np.isfinite(sol)) or np.min(np.abs(np.linalg.svd(A, compute_uv=False))) < 1e-12:
            continue
        betas[j] = sol
        j += 1
    return np.ascontiguousarray(X), y, beta_true, betas


# ---------------------------------------------------------------------------
# Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
# 1, 2, 3", SC'11) and the mixture arrays of the learned-proposal workload.
#
# The library's training generator draws the same arrays on the GPU from its own
# implementation of the same published definition; both use only integer
# arithmetic and correctly rounded double-precision +, -, *, /, floor and scaling by
# powers of two, so the two sides agree bit for bit.

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32 with 10 rounds; arguments are uint32 arrays (or scalars)."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & _MASK32 for v in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK32
    for _ in range(10):
        p0 = np.uint64(PHILOX_M0) * c0
        p1 = np.uint64(PHILOX_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & _MASK32, lo1, (hi0 ^ c3 ^ k1) & _MASK32, lo0
        k0 = (k0 + np.uint64(PHILOX_W0)) & _MASK32
        k1 = (k1 + np.uint64(PHILOX_W1)) & _MASK32
    return tuple(v.astype(np.uint32) for v in (c0, c1, c2, c3))


_LOG2E = 1.4426950408889634
_LN2 = 0.6931471805599453
_INV_FACT = [1.0]
for _j in range(1, 15):
    _INV_FACT.append(_INV_FACT[-1] / _j)


def exp_basic(z: np.ndarray) -> np.ndarray:
    """exp from IEEE basic operations only: 2^floor(t) * e^(f ln 2), t = z log2(e), f = t - floor(t),
    with e^(f ln 2) as its Taylor polynomial of degree 14 in Horner form."""
    z = np.asarray(z, dtype=np.float64)
    t = z * _LOG2E
    kf = np.floor(t)
    g = (t - kf) * _LN2
    p = np.full_like(g, _INV_FACT[14])
    for j in range(13, -1, -1):
        p = p * g + _INV_FACT[j]
    return np.ldexp(p, kf.astype(np.int64))


MIX_GAUSS, MIX_LOGNORMAL, MIX_UNIFORM = 0, 1, 2
_LN10 = 2.302585092994046


def mixture_params(seed: int, array_id: int, n: int):
    """Random mixture of 1-4 components (Gaussian, lognormal, uniform) and a uniform rank k,
    for array (seed, array_id) of size n.

    Twenty words w[0..19] come from the Philox4x32-10 blocks at counters (0, 0, array_id, j),
    j = 4..8 (disjoint from the element counters), key (seed mod 2^32, seed div 2^32):
      ncomp = 1 + (w0 >> 30); type_c = (3 w[1+c]) >> 32;
      ua = w[5+c] 2^-32, ub = w[9+c] 2^-32, integer weight q_c = 1 + (w[13+c] >> 8);
      cumulative weight cum_c = (q_0 + ... + q_c) / (q_0 + ... + q_(ncomp-1)) (one rounding);
      Gaussian: mean -100 + 200 ua, sd exp((-2 + 3 ub) ln 10);
      lognormal: log-mean -2 + 4 ua, log-sd 0.25 + 1.25 ub;
      uniform on [p1, p1 + p2]: p1 = -100 + 200 ua, p2 = exp((-2 + 4 ub) ln 10);
      k = 1 + floor(((w17 << 32) | w18) n / 2^64).
    Every step is an integer operation or one correctly rounded double operation (exp is
    exp_basic), so a device implementation reproduces it bit for bit.
    """
    k0 = np.uint32(seed & 0xFFFFFFFF)
    k1 = np.uint32((seed >> 32) & 0xFFFFFFFF)
    w = []
    for j in range(4, 9):
        w.extend(int(v) for v in philox4x32_10(0, 0, array_id, j, k0, k1))
    c = 1 + (w[0] >> 30)
    types = np.zeros(4, dtype=np.int32)
    p1 = np.zeros(4)
    p2 = np.zeros(4)
    q = [1 + (w[13 + j] >> 8) for j in range(4)]
    tot = float(sum(q[:c]))
    cum = np.ones(4)
    acc = 0
    for j in range(c):
        acc += q[j]
        cum[j] = float(acc) / tot
        types[j] = (3 * w[1 + j]) >> 32
        ua = float(w[5 + j]) * (2.0 ** -32)
        ub = float(w[9 + j]) * (2.0 ** -32)
        if types[j] == MIX_GAUSS:
            p1[j] = -100.0 + 200.0 * ua
            p2[j] = float(exp_basic((-2.0 + 3.0 * ub) * _LN10))
        elif types[j] == MIX_LOGNORMAL:
            p1[j] = -2.0 + 4.0 * ua
            p2[j] = 0.25 + 1.25 * ub
        else:
            p1[j] = -100.0 + 200.0 * ua
            p2[j] = float(exp_basic((-2.0 + 4.0 * ub) * _LN10))
    k = 1 + ((((w[17] << 32) | w[18]) * n) >> 64)
    return {"ncomp": c, "cum": cum, "types": types, "p1": p1, "p2": p2, "k": int(k)}


def mixture_array(params: dict, n: int, seed: int, array_id: int = 0) -> np.ndarray:
    """Element i of array (seed, array_id): four Philox4x32-10 blocks at counters
    (i mod 2^32, i div 2^32, array_id, j), j = 0..3, key (seed mod 2^32, seed div 2^32).
    Blocks 0-2 give twelve 24-bit uniforms u = (r >> 8) 2^-24, summed minus 6 into an
    approximately normal g (exact in double precision); block 3's first word picks the
    component (r 2^-32 against the cumulative weights) and its second word is the uniform
    of a uniform component.  Values are formed in double precision and rounded to float32.
    """
    i = np.arange(n, dtype=np.uint64)
    lo = (i & _MASK32).astype(np.uint32)
    hi = (i >> np.uint64(32)).astype(np.uint32)
    k0 = np.uint32(seed & 0xFFFFFFFF)
    k1 = np.uint32((seed >> 32) & 0xFFFFFFFF)
    a = np.uint32(array_id)
    g = np.zeros(n)
    for j in range(3):
        r = philox4x32_10(lo, hi, np.full(n, a, np.uint32), np.full(n, j, np.uint32), k0, k1)
        for word in r:
            g = g + (word >> np.uint32(8)).astype(np.float64) * (2.0 ** -24)
    g = g - 6.0
    r3 = philox4x32_10(lo, hi, np.full(n, a, np.uint32), np.full(n, 3, np.uint32), k0, k1)
    uc = r3[0].astype(np.float64) * (2.0 ** -32)
    uu = r3[1].astype(np.float64) * (2.0 ** -32)
    comp = np.zeros(n, dtype=np.int64)
    for j in range(3):
        comp += (uc >= params["cum"][j]).astype(np.int64)
    comp = np.minimum(comp, params["ncomp"] - 1)
    t = params["types"][comp]
    p1 = params["p1"][comp]
    p2 = params["p2"][comp]
    gauss = p1 + p2 * g
    logn = exp_basic(p1 + p2 * g)
    unif = p1 + p2 * uu
    v = np.where(t == MIX_GAUSS, gauss, np.where(t == MIX_LOGNORMAL, logn, unif))
    return v.astype(np.float32)
