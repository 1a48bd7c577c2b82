"""Double-precision reference of the learned bracket proposal.

TEST INFRASTRUCTURE ONLY: imported by the test-suite (and nothing in the GPU
library).  It computes, plainly and in float64, what the device kernels of the
learned proposal compute in float32:

- ``sample_features``: a fixed-stride sample of S = min(n, 4096) elements,
  x[i * floor(n / S)] for i < S; its minimum lo and maximum hi; its histogram
  in 64 equal bins over [lo, hi], bin = min(63, floor(64 (v - lo) / (hi - lo)))
  in double precision (bin 0 when hi == lo), given as cumulative fractions
  (the fraction of the sample in bins 0..b, for b = 0..63); plus lo / (1 + |lo|),
  hi / (1 + |hi|) and k / n.  Each of the 67 features is formed in double
  precision and rounded once to float32, so the device's features agree bit
  for bit (lo and hi are taken as values: a zero extreme is +0).  A sample
  holding NaN or an infinity gives no proposal (None).
- ``forward``: the network 67 -> 64 -> 64 -> 2 with ReLU on both hidden layers.
- ``loss_and_grad``: the training loss and its gradient by back-propagation.
  With u = o_0, omega = exp(clamp(o_1, -20, 4)) and d = u - u*, one example's
  loss is C_SQ d^2 + C_COV max(0, |d| - omega) + C_W omega; the batch loss is
  the mean.  ReLU'(0) = 0, sign(0) = 0, and the clamp passes gradient only
  strictly inside (-20, 4).
- ``hist_position``: the histogram's own estimate of the rank's position,
  (b + (p - F_{b-1}) / (F_b - F_{b-1})) / 64 with F the cumulative features,
  p the k/n feature and b the first bin with F_b >= p (F_{-1} = 0), in double
  precision from the float features; the network predicts the offset from it.
- ``bracket``: the proposed bracket y0 -+ w with y0 = lo + (hi - lo)(h + u),
  h the histogram position, and w = (hi - lo) omega.
- ``target``: the label u* = (x_(k) - lo) / (hi - lo) - h (0 when hi == lo).
- ``adam_step``: one Adam update (Kingma and Ba, 2015) with bias correction.

The method's exactness never rests on the network: the proposed ends are
only used where the counts of the same pass prove them (Section 4's bracket
invariant #(x <= yL) < k <= #(x < yR)).  The pieces above have no passage of
the paper to follow; they are pinned by finite differences, closed forms and
brute force in tests/test_oracle_mlp.py.

Parameter vector layout (8642 values): W1 (64 x 67, row-major, row = hidden
unit), b1 (64), W2 (64 x 64), b2 (64), W3 (2 x 64), b3 (2).
"""
from __future__ import annotations

import math

import numpy as np

SAMPLE = 4096
BINS = 64
N_IN = BINS + 3
N_HID = 64
N_OUT = 2
SIZES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)  # 8642

C_SQ = 100.0
C_COV = 1.0
C_W = 0.02
LOGW_MIN = -20.0
LOGW_MAX = 4.0


def unpack(theta: np.ndarray) -> dict:
    """Views of the six parameter blocks of a flat parameter vector."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, off = {}, 0
    for name, shape in SIZES:
        m = int(np.prod(shape))
        out[name] = theta[off:off + m].reshape(shape)
        off += m
    return out


def sample_features(x: np.ndarray, k: int):
    """(features float32[67], lo, hi) for array x and 1-based rank k, or None when the sample
    holds a non-finite value."""
    n = int(x.size)
    assert n >= 1 and 1 <= k <= n
    s = min(n, SAMPLE)
    stride = n // s
    v = [float(x[i * stride]) for i in range(s)]
    if not all(math.isfinite(t) for t in v):
        return None
    lo, hi = min(v) + 0.0, max(v) + 0.0  # -0 becomes +0: the extremes are values, not bits
    counts = [0] * BINS
    for t in v:
        if hi > lo:
            b = math.floor((64.0 * (t - lo)) / (hi - lo))
            b = min(BINS - 1, b)
        else:
            b = 0
        counts[b] += 1
    f = np.empty(N_IN, dtype=np.float32)
    cum = 0
    for b in range(BINS):
        cum += counts[b]
        f[b] = np.float32(cum / s)
    f[BINS] = np.float32(lo / (1.0 + abs(lo)))
    f[BINS + 1] = np.float32(hi / (1.0 + abs(hi)))
    f[BINS + 2] = np.float32(k / n)
    return f, lo, hi


def _clamp_logw(o1):
    return np.minimum(np.maximum(o1, LOGW_MIN), LOGW_MAX)


def forward(theta: np.ndarray, F: np.ndarray):
    """Outputs o (B x 2) and the activations needed by the backward pass."""
    p = unpack(theta)
    F = np.asarray(F, dtype=np.float64).reshape(-1, N_IN)
    z1 = F @ p["W1"].T + p["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = np.maximum(z2, 0.0)
    o = a2 @ p["W3"].T + p["b3"]
    return o, (F, z1, a1, z2, a2)


def example_losses(o: np.ndarray, ustar: np.ndarray) -> np.ndarray:
    d = o[:, 0] - np.asarray(ustar, dtype=np.float64)
    w = np.exp(_clamp_logw(o[:, 1]))
    return C_SQ * d * d + C_COV * np.maximum(np.abs(d) - w, 0.0) + C_W * w


def loss(theta: np.ndarray, F: np.ndarray, ustar: np.ndarray) -> float:
    o, _ = forward(theta, F)
    return float(np.mean(example_losses(o, ustar)))


def loss_and_grad(theta: np.ndarray, F: np.ndarray, ustar: np.ndarray):
    """Mean loss over the batch and its gradient with respect to the flat parameters."""
    p = unpack(theta)
    o, (F64, z1, a1, z2, a2) = forward(theta, F)
    B = o.shape[0]
    ustar = np.asarray(ustar, dtype=np.float64)
    d = o[:, 0] - ustar
    inside = (o[:, 1] > LOGW_MIN) & (o[:, 1] < LOGW_MAX)
    w = np.exp(_clamp_logw(o[:, 1]))
    out_cov = np.abs(d) > w
    L = float(np.mean(C_SQ * d * d + C_COV * np.maximum(np.abs(d) - w, 0.0) + C_W * w))
    # d loss / d o, per example (already divided by B for the mean)
    do = np.zeros_like(o)
    do[:, 0] = (2.0 * C_SQ * d + C_COV * np.sign(d) * out_cov) / B
    do[:, 1] = ((-C_COV * out_cov + C_W) * w * inside) / B
    g = {}
    g["W3"] = do.T @ a2
    g["b3"] = do.sum(axis=0)
    da2 = do @ p["W3"]
    dz2 = da2 * (z2 > 0.0)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(axis=0)
    da1 = dz2 @ p["W2"]
    dz1 = da1 * (z1 > 0.0)
    g["W1"] = dz1.T @ F64
    g["b1"] = dz1.sum(axis=0)
    grad = np.concatenate([g[name].reshape(-1) for name, _ in SIZES])
    return L, grad


def hist_position(f: np.ndarray) -> float:
    """Where the cumulative histogram features cross the k/n feature, as a fraction of the
    sample range (linear inside the crossing bin)."""
    F = [float(v) for v in np.asarray(f, dtype=np.float32)[:BINS]]
    p = float(np.float32(f[BINS + 2]))
    b = 0
    while b < BINS - 1 and F[b] < p:
        b += 1
    prev = F[b - 1] if b > 0 else 0.0
    if not F[b] > prev:
        return (b + 0.5) / BINS
    return (b + (p - prev) / (F[b] - prev)) / BINS


def bracket(o: np.ndarray, lo: float, hi: float, h: float):
    """The proposed bracket (a, b) for one example's outputs o = (o_0, o_1) and histogram
    position h."""
    span = hi - lo
    y0 = lo + span * (h + float(o[0]))
    w = span * math.exp(float(_clamp_logw(np.float64(o[1]))))
    return y0 - w, y0 + w


def target(value: float, lo: float, hi: float, h: float) -> float:
    """The label of an array whose k-th element is `value`, on the sample range [lo, hi],
    relative to the histogram position h (0 when the sample is constant: the bracket then
    has zero width whatever the output)."""
    if not hi > lo:
        return 0.0
    return (value - lo) / (hi - lo) - h


def adam_step(theta, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """Step t (1-based) of Adam; returns the new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
