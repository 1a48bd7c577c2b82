"""Pins of the learned proposal's double-precision reference (oracle/mlp.py).

Nothing here compares the reference with itself: gradients against central
finite differences of the loss, a network reduced by hand to closed forms,
histograms against numpy.histogram on inputs whose bin edges fall between
sample values, Adam's first step against its closed form, and the generator
that feeds the trainer against Philox's published known-answer vectors.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import mlp


def _random_case(seed, B=16, scale=0.3):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(mlp.N_PARAMS) * scale
    F = rng.uniform(0.0, 0.2, size=(B, mlp.N_IN))
    ustar = rng.uniform(0.0, 1.0, size=B)
    return theta, F, ustar


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    theta, F, ustar = _random_case(seed)
    # put the width output on both sides of the coverage kink across the batch
    L, g = mlp.loss_and_grad(theta, F, ustar)
    rng = np.random.default_rng(100 + seed)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 300, replace=False),
                          np.arange(mlp.N_PARAMS - 2 - 128, mlp.N_PARAMS)])
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd = (mlp.loss(tp, F, ustar) - mlp.loss(tm, F, ustar)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-7, (i, fd, g[i])
    assert L == pytest.approx(mlp.loss(theta, F, ustar), rel=0, abs=0)


def test_zero_network_closed_form():
    """All weights zero, b3 = (u0, s0): every output is (u0, s0) and only b3 gets gradient."""
    theta = np.zeros(mlp.N_PARAMS)
    u0, s0 = 0.3, math.log(0.05)
    theta[-2:] = (u0, s0)
    F = np.random.default_rng(0).uniform(size=(4, mlp.N_IN))
    ustar = np.array([0.3, 0.32, 0.2, 0.5])
    L, g = mlp.loss_and_grad(theta, F, ustar)
    w = 0.05
    d = u0 - ustar
    per = 100.0 * d * d + np.maximum(np.abs(d) - w, 0.0) + 0.02 * w
    assert L == pytest.approx(per.mean(), rel=1e-15)
    # d/du0 = mean(200 d + sign(d) [|d| > w]); d/ds0 = mean((0.02 - [|d| > w]) w)
    outside = np.abs(d) > w
    assert g[-2] == pytest.approx(np.mean(200.0 * d + np.sign(d) * outside), rel=1e-14)
    assert g[-1] == pytest.approx(np.mean((0.02 - outside) * w), rel=1e-14)
    assert np.all(g[:-2] == 0.0)


def test_single_path_forward():
    """One path k/n -> hidden unit 0 -> hidden unit 0 -> u: u = k/n, omega = e^0."""
    p = np.zeros(mlp.N_PARAMS)
    blocks = mlp.unpack(p)
    blocks["W1"][0, mlp.N_IN - 1] = 1.0
    blocks["W2"][0, 0] = 1.0
    blocks["W3"][0, 0] = 1.0
    F = np.zeros((3, mlp.N_IN))
    F[:, -1] = [0.25, 0.5, 0.75]
    o, _ = mlp.forward(p, F)
    assert np.array_equal(o[:, 0], [0.25, 0.5, 0.75]) and np.all(o[:, 1] == 0.0)
    # a negative input is cut by the first ReLU
    F[0, -1] = -1.0
    o, _ = mlp.forward(p, F)
    assert o[0, 0] == 0.0


def test_width_clamp_stops_gradient():
    theta = np.zeros(mlp.N_PARAMS)
    theta[-1] = 10.0  # log-width above the clamp
    F = np.zeros((2, mlp.N_IN))
    _, g = mlp.loss_and_grad(theta, F, np.array([0.0, 0.1]))
    assert g[-1] == 0.0
    a, b = mlp.bracket(np.array([0.0, 10.0]), 0.0, 1.0, 0.0)
    assert (a, b) == (-math.exp(4.0), math.exp(4.0))


def test_bracket_and_target_closed_form():
    a, b = mlp.bracket(np.array([0.5, math.log(0.1)]), 2.0, 4.0, 0.0)
    assert a == pytest.approx(2.8, rel=1e-15) and b == pytest.approx(3.2, rel=1e-15)
    a, b = mlp.bracket(np.array([0.25, math.log(0.1)]), 2.0, 4.0, 0.25)
    assert a == pytest.approx(2.8, rel=1e-15) and b == pytest.approx(3.2, rel=1e-15)
    assert mlp.target(3.0, 2.0, 4.0, 0.0) == 0.5 and mlp.target(3.0, 2.0, 4.0, 0.5) == 0.0
    assert mlp.target(2.0, 2.0, 4.0, 0.0) == 0.0 and mlp.target(4.0, 2.0, 4.0, 0.0) == 1.0
    assert mlp.target(7.0, 2.0, 2.0, 0.3) == 0.0


def test_hist_position_closed_form():
    """Uniform sample: F_b = (b+1)/64, so the crossing of p sits at p itself; a two-bin
    sample interpolates inside its crossing bin."""
    f = np.zeros(mlp.N_IN, np.float32)
    f[:64] = (np.arange(64) + 1) / 64.0
    for p in (0.25, 0.5, 0.75, 1.0):
        f[66] = p
        assert mlp.hist_position(f) == pytest.approx(p, abs=1e-15)
    f[:64] = 0.0
    f[10:] = 0.4     # 40 % of the sample in bin 10
    f[40:] = 1.0     # the rest in bin 40
    f[66] = 0.2      # half-way through bin 10's mass
    assert mlp.hist_position(f) == pytest.approx(10.5 / 64, abs=1e-7)
    f[66] = 0.7
    assert mlp.hist_position(f) == pytest.approx(40.5 / 64, abs=1e-7)
    # against the exact sample quantile of a smooth sample: within about one bin
    x = np.random.default_rng(3).standard_normal(1 << 16).astype(np.float32)
    for k in (100, 30_000, 60_000):
        f, lo, hi = mlp.sample_features(x, k)
        q = np.sort(x[:: 16])[int(k / x.size * 4096)]
        assert abs(mlp.hist_position(f) - (q - lo) / (hi - lo)) < 1.5 / 64


def test_histogram_against_numpy_histogram():
    """Integer samples 0..4095 on [0, 4095]: no value lies on a bin edge 4095 j / 64."""
    rng = np.random.default_rng(3)
    n = 4096 * 5 + 3
    x = rng.permutation(np.arange(n) % 4096).astype(np.float32)
    x[0] = 0.0
    stride = n // 4096
    x[4095 * stride] = 4095.0
    f, lo, hi = mlp.sample_features(x, 17)
    samp = x[np.arange(4096) * stride].astype(np.float64)
    assert (lo, hi) == (samp.min(), samp.max()) == (0.0, 4095.0)
    ref, _ = np.histogram(samp, bins=64, range=(0.0, 4095.0))
    assert np.array_equal(f[:64], (np.cumsum(ref) / 4096).astype(np.float32))
    assert f[64] == np.float32(0.0) and f[65] == np.float32(4095.0 / 4096.0)
    assert f[66] == np.float32(17 / n)


def test_features_degenerate_and_small():
    x = np.full(1000, 2.5, dtype=np.float64)
    f, lo, hi = mlp.sample_features(x, 1000)
    assert lo == hi == 2.5 and np.all(f[:64] == 1.0)
    assert f[64] == f[65] == np.float32(2.5 / 3.5) and f[66] == 1.0
    # n < 4096: the whole array is the sample; brute-force bins by the definition's formula
    x = np.random.default_rng(1).standard_normal(777).astype(np.float32)
    f, lo, hi = mlp.sample_features(x, 5)
    v = x.astype(np.float64)
    bins = np.minimum(63, np.floor(64.0 * (v - lo) / (hi - lo))).astype(int)
    want = np.cumsum(np.bincount(bins, minlength=64)) / 777
    assert np.array_equal(f[:64], want.astype(np.float32))
    # the smallest sample value lands in the first bin, every value in some bin
    assert f[0] > 0 and f[63] == 1.0 and np.all(np.diff(f[:64]) >= 0)


def test_signed_zero_extremes_are_values():
    x = np.array([-0.0, 1.0, 0.0, 2.0] * 2000, dtype=np.float32)
    f, lo, hi = mlp.sample_features(x, 1)
    assert lo == 0.0 and math.copysign(1.0, lo) == 1.0
    assert np.signbit(f[64]) == False  # noqa: E712


def test_nonfinite_sample_gives_no_proposal():
    x = np.ones(10000, dtype=np.float32)
    x[2] = np.inf  # stride 2: element 2 is sampled
    assert mlp.sample_features(x, 3) is None
    x[2] = 1.0
    x[3] = np.nan  # not sampled
    assert mlp.sample_features(x, 3) is not None


def test_forward_weight_orientation():
    """A single path through distinct units, feature 10 -> hidden unit 3 -> hidden unit 7 ->
    output 0, pins each weight matrix as (output unit, input unit): any transposed block
    routes the signal through a unit that carries nothing and the output is 0."""
    p = np.zeros(mlp.N_PARAMS)
    blocks = mlp.unpack(p)
    blocks["W1"][3, 10] = 1.0
    blocks["W2"][7, 3] = 2.0
    blocks["W3"][0, 7] = 0.5
    blocks["b3"][1] = -0.25
    F = np.zeros((3, mlp.N_IN))
    F[:, 10] = [0.1, 0.4, 0.9]
    o, _ = mlp.forward(p, F)
    assert np.array_equal(o[:, 0], [0.1, 0.4, 0.9]) and np.all(o[:, 1] == -0.25)
    # each block with its one weight transposed (W3: on the other output's row)
    for name, idx in (("W1", (10, 3)), ("W2", (3, 7)), ("W3", (1, 7))):
        q = np.zeros(mlp.N_PARAMS)
        qb = mlp.unpack(q)
        qb["W1"][3, 10], qb["W2"][7, 3], qb["W3"][0, 7] = 1.0, 2.0, 0.5
        w = qb[name][np.nonzero(qb[name])][0]
        qb[name][:] = 0.0
        qb[name][idx] = w
        o2, _ = mlp.forward(q, F)
        assert np.all(o2[:, 0] == 0.0), name


def test_adam_constant_gradient_closed_form():
    """With the same gradient g at every step the moments are m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, their bias-corrected values g and g^2 at every t, so each step moves
    by lr g / (|g| + eps): a bias correction frozen at any step fails from t = 2 on."""
    rng = np.random.default_rng(3)
    theta0 = rng.standard_normal(40)
    g = rng.standard_normal(40)
    theta, m, v = theta0.copy(), np.zeros(40), np.zeros(40)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    for t in range(1, 8):
        theta, m, v = mlp.adam_step(theta, g, m, v, t, lr=lr, beta1=b1, beta2=b2, eps=eps)
        assert np.allclose(m, (1 - b1 ** t) * g, rtol=1e-14, atol=0)
        assert np.allclose(v, (1 - b2 ** t) * g * g, rtol=1e-12, atol=0)
        assert np.allclose(theta, theta0 - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    th1, m, v = mlp.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    # bias-corrected first moments are g and g^2, so the step is lr g / (|g| + eps)
    assert np.allclose(th1, theta - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    """A few hundred Adam steps of the reference on a learnable synthetic task."""
    rng = np.random.default_rng(4)
    F = rng.uniform(0, 0.1, size=(256, mlp.N_IN))
    F[:, -1] = rng.uniform(0, 1, 256)
    ustar = F[:, -1] * 0.8 + 0.1
    theta = rng.standard_normal(mlp.N_PARAMS) * 0.05
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    L0, _ = mlp.loss_and_grad(theta, F, ustar)
    for t in range(1, 301):
        L, g = mlp.loss_and_grad(theta, F, ustar)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, lr=3e-3)
    assert L < 0.05 * L0


# ---- the generator the trainer draws its arrays from (counter-based, published definition)

def test_philox_known_answers():
    """Known-answer vectors of Philox4x32-10 (Salmon et al., SC'11, Random123 distribution)."""
    f = workloads.philox4x32_10
    assert [int(v) for v in f(0, 0, 0, 0, 0, 0)] == [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    m = 0xFFFFFFFF
    assert [int(v) for v in f(m, m, m, m, m, m)] == [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]
    assert [int(v) for v in f(0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344, 0xa4093822,
                              0x299f31d0)] == [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]


def test_exp_basic_accuracy():
    z = np.concatenate([np.linspace(-700, 700, 20001), np.linspace(-1, 1, 2001), [0.0]])
    e = workloads.exp_basic(z)
    # a few ulps from the degree-14 Horner sum on [0, ln 2), plus the argument reduction
    # t = z log2(e), whose absolute error of about |t| 2^-53 grows with |z|
    assert np.all(np.abs(e / np.exp(z) - 1.0) < 4e-15 + 2e-16 * np.abs(z))
    assert workloads.exp_basic(np.array([0.0]))[0] == 1.0


def test_mixture_params_ranges():
    n = 1 << 20
    seen = set()
    for a in range(400):
        p = workloads.mixture_params(11, a, n)
        c = p["ncomp"]
        assert 1 <= c <= 4 and 1 <= p["k"] <= n
        assert p["cum"][c - 1] == 1.0 and np.all(np.diff(p["cum"]) >= 0)
        for j in range(c):
            t = int(p["types"][j])
            seen.add((c, t))
            if t == workloads.MIX_GAUSS:
                assert -100 <= p["p1"][j] < 100 and 0.01 <= p["p2"][j] <= 10.0 * (1 + 1e-14)
            elif t == workloads.MIX_LOGNORMAL:
                assert -2 <= p["p1"][j] < 2 and 0.25 <= p["p2"][j] < 1.5
            else:
                assert -100 <= p["p1"][j] < 100 and 0.01 <= p["p2"][j] <= 100.0 * (1 + 1e-14)
    assert {c for c, _ in seen} == {1, 2, 3, 4} and {t for _, t in seen} == {0, 1, 2}


def test_mixture_array_single_component_moments():
    """One Gaussian component: the sum of twelve uniforms minus 6 has mean 0 and variance 1."""
    p = {"ncomp": 1, "cum": np.ones(4), "types": np.zeros(4, np.int32),
         "p1": np.array([5.0, 0, 0, 0]), "p2": np.array([2.0, 0, 0, 0]), "k": 1}
    x = workloads.mixture_array(p, 1 << 16, seed=9, array_id=3).astype(np.float64)
    assert abs(x.mean() - 5.0) < 0.05 and abs(x.std() - 2.0) < 0.05
    assert x.min() >= 5.0 - 12.0 and x.max() <= 5.0 + 12.0
    p["types"][0] = workloads.MIX_UNIFORM
    x = workloads.mixture_array(p, 1 << 16, seed=9, array_id=3).astype(np.float64)
    assert x.min() >= 5.0 and x.max() <= 7.0 and abs(x.mean() - 6.0) < 0.02
