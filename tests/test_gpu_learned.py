"""GPU parity of the learned bracket proposal against the CPU references.

- the mixture generator: bit for bit against workloads' Philox4x32-10 definition;
- the features: bit for bit against oracle/mlp.py (integer counts, one rounding each);
- the network's forward pass, loss, gradient and Adam step in float against the
  float64 reference on the same float inputs: outputs within 1e-5 relative, the
  gradient within 1e-4 of its largest entry, element by element;
- selections with any proposal (a good one, one that misses on either side, a
  degenerate or overflowing one, a trained network's) bit-identical to the
  oracle, with the proposal ends the counts proved reported in the stats;
- a trained network reads the input fewer times than the plain method.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import mlp
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


@pytest.mark.parametrize("n", [1, 1000, 4097, 1 << 16])
def test_generator_bit_exact(sel, n):
    seed = 12345 + n
    count = 6 if n > 1 else 40
    print(f"case generator n={n}", flush=True)
    x, ks = sel.mixture_generate(seed, 7, count, n)
    x = x.cpu().numpy()
    ks = ks.cpu().numpy()
    for a in range(count):
        p = workloads.mixture_params(seed, 7 + a, n)
        ref = workloads.mixture_array(p, n, seed, 7 + a)
        assert ks[a] == p["k"], a
        assert np.array_equal(x[a].view(np.uint32), ref.view(np.uint32)), (a, p)


def _feature_cases():
    rng = np.random.default_rng(0)
    cases = []
    for n in (1, 7, 4095, 4096, 4097, 100_003):
        cases.append(rng.standard_normal(n).astype(np.float32))
        cases.append(rng.standard_normal(n) * 1e3)
    cases.append(np.full(5000, 3.25, dtype=np.float32))
    cases.append(np.array([-0.0, 0.0, 1.0, 2.0] * 3000, dtype=np.float32))
    x = rng.uniform(size=9000).astype(np.float32)
    x[4] = np.inf  # sampled (stride 2)
    cases.append(x)
    x = rng.uniform(size=9000)
    x[5] = np.nan  # not sampled
    cases.append(x)
    p = workloads.mixture_params(3, 0, 1 << 18)
    cases.append(workloads.mixture_array(p, 1 << 18, 3, 0))
    return cases


def test_features_bit_exact(sel):
    import paper_1104_2732_amd as cps
    for dt in (np.float32, np.float64):
        arrays = [a for a in _feature_cases() if a.dtype == dt]
        dev = [_dev(a) for a in arrays]
        ks = [1 + (i * 7919) % a.size for i, a in enumerate(arrays)]
        ptrs, sizes, kk, code = sel.batch_descriptors(dev, ks)
        print(f"case features {np.dtype(dt).name} count={len(arrays)}", flush=True)
        feat, rng_, valid = sel.features(ptrs, sizes, kk, len(arrays), code)
        feat, rng_, valid = feat.cpu().numpy(), rng_.cpu().numpy(), valid.cpu().numpy()
        for i, (a, k) in enumerate(zip(arrays, ks)):
            ref = mlp.sample_features(a, k)
            if ref is None:
                assert valid[i] == 0 and np.all(feat[i] == 0), i
                continue
            f, lo, hi = ref
            assert valid[i] == 1, i
            assert np.array_equal(feat[i].view(np.uint32), f.view(np.uint32)), (i, feat[i], f)
            assert (rng_[i, 0], rng_[i, 1]) == (lo, hi), i
            assert math.copysign(1.0, rng_[i, 0]) == math.copysign(1.0, lo)
    assert cps.MLP_INPUTS == mlp.N_IN and cps.MLP_PARAMS == mlp.N_PARAMS


def _random_net(seed, B, scale=0.3):
    rng = np.random.default_rng(seed)
    theta = (rng.standard_normal(mlp.N_PARAMS) * scale).astype(np.float32)
    F = rng.uniform(0.0, 0.2, size=(B, mlp.N_IN)).astype(np.float32)
    ustar = rng.uniform(0.0, 1.0, size=B).astype(np.float32)
    return theta, F, ustar


@pytest.mark.parametrize("B", [1, 31, 32, 33, 100, 1000])
def test_forward_matches_reference(sel, B):
    theta, F, _ = _random_net(B, B)
    print(f"case mlp forward B={B}", flush=True)
    out = sel.mlp_forward(_dev(theta), _dev(F)).cpu().numpy().astype(np.float64)
    ref, _ = mlp.forward(theta.astype(np.float64), F.astype(np.float64))
    scale = np.max(np.abs(ref))
    assert np.all(np.abs(out - ref) <= 1e-5 * (np.abs(ref) + scale)), np.max(np.abs(out - ref))


@pytest.mark.parametrize("B", [1, 33, 100, 256, 1000])
def test_gradient_matches_reference(sel, B):
    theta, F, ustar = _random_net(100 + B, B)
    # put some examples outside the coverage width and some inside
    theta = theta.copy()
    theta[-1] = np.float32(math.log(0.3))
    print(f"case mlp grad B={B}", flush=True)
    loss, grad = sel.mlp_loss_grad(_dev(theta), _dev(F), _dev(ustar))
    loss = float(loss.cpu().numpy()[0])
    grad = grad.cpu().numpy().astype(np.float64)
    L, g = mlp.loss_and_grad(theta.astype(np.float64), F.astype(np.float64),
                             ustar.astype(np.float64))
    assert abs(loss - L) <= 1e-5 * abs(L)
    gmax = np.max(np.abs(g))
    assert np.all(np.abs(grad - g) <= 1e-4 * gmax + 1e-4 * np.abs(g)), np.max(np.abs(grad - g)) / gmax
    # deterministic: the same call gives the same bits
    _, grad2 = sel.mlp_loss_grad(_dev(theta), _dev(F), _dev(ustar))
    assert np.array_equal(grad2.cpu().numpy().astype(np.float64), grad)


def test_adam_matches_reference(sel):
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(mlp.N_PARAMS).astype(np.float32)
    m = np.zeros(mlp.N_PARAMS, np.float32)
    v = np.zeros(mlp.N_PARAMS, np.float32)
    P, M, V = _dev(theta.copy()), _dev(m.copy()), _dev(v.copy())
    th64, m64, v64 = theta.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for t in range(1, 4):
        g = rng.standard_normal(mlp.N_PARAMS).astype(np.float32)
        sel.mlp_adam(P, _dev(g), M, V, t, 1e-3)
        th64, m64, v64 = mlp.adam_step(th64, g.astype(np.float64), m64, v64, t, lr=1e-3)
    got = P.cpu().numpy().astype(np.float64)
    # float state against the double-precision recursion: a few float roundings per step
    assert np.all(np.abs(got - th64) <= 2e-6 * np.abs(th64) + 1e-8)


def test_init_is_deterministic_and_bounded(sel):
    a = sel.mlp_init(9).cpu().numpy()
    b = sel.mlp_init(9).cpu().numpy()
    c = sel.mlp_init(10).cpu().numpy()
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    blocks = mlp.unpack(a.astype(np.float64))
    assert np.max(np.abs(blocks["W1"])) <= math.sqrt(6 / 67) and np.all(blocks["b1"] == 0)
    assert np.max(np.abs(blocks["W2"])) <= math.sqrt(6 / 64) and np.all(blocks["b2"] == 0)
    assert np.max(np.abs(blocks["W3"])) <= 0.01 * math.sqrt(6 / 64) + 1e-9
    assert blocks["b3"][0] == 0.0 and blocks["b3"][1] == pytest.approx(math.log(0.05), rel=1e-6)


def _proposal_params(u, logw):
    """A network whose output is the constant (u, logw): all weights zero."""
    theta = np.zeros(mlp.N_PARAMS, np.float32)
    theta[-2] = u
    theta[-1] = logw
    return theta


def test_bracket_matches_reference(sel):
    rng = np.random.default_rng(7)
    theta = (rng.standard_normal(mlp.N_PARAMS) * 0.1).astype(np.float32)
    P = _dev(theta)
    for seed, n in ((1, 5000), (2, 1 << 18)):
        p = workloads.mixture_params(seed, 0, n)
        x = workloads.mixture_array(p, n, seed, 0)
        k = p["k"]
        a, b, use = sel.learned_bracket(_dev(x), k, P)
        f, lo, hi = mlp.sample_features(x, k)
        o, _ = mlp.forward(theta.astype(np.float64), f.astype(np.float64)[None, :])
        ra, rb = mlp.bracket(o[0], lo, hi, mlp.hist_position(f))
        assert use == 1
        assert abs(a - ra) <= 1e-5 * (hi - lo) and abs(b - rb) <= 1e-5 * (hi - lo), (a, ra, b, rb)
    # a sample with an infinity gives no proposal
    x = np.ones(10000, np.float32)
    x[2] = np.inf
    assert sel.learned_bracket(_dev(x), 5, P)[2] == 0


def _check_select(sel, x, k, theta, ctx, options=None):
    import paper_1104_2732_amd as cps
    ref = __import__("oracle").select_kth(x, k)
    res, st = sel.select_kth_learned(_dev(x), k, _dev(theta), options=options, stats=True)
    assert_same_result(res, ref, ctx)
    return res, st, ref


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_learned_select_parity_with_any_proposal(sel, dtype):
    """Results never depend on the proposal; the proven ends are reported."""
    import paper_1104_2732_amd as cps
    rng = np.random.default_rng(11)
    for n in (1, 2, 100, 4096, 70_001, 1 << 20):
        x = (rng.standard_normal(n) * 3).astype(dtype)
        xs = np.sort(x)
        for k in sorted({1, n, (n + 1) // 2, int(rng.integers(1, n + 1))}):
            f = mlp.sample_features(x, k)
            lo, hi = f[1], f[2]
            span = hi - lo if hi > lo else 1.0
            # the network's first output is the offset from the histogram position
            ustar = (float(xs[k - 1]) - lo) / span - mlp.hist_position(f[0])
            h = mlp.hist_position(f[0])
            cases = {
                "tight": (ustar, math.log(0.02)),       # both ends hold
                "high": (ustar + 0.3, math.log(0.05)),  # misses above: only the lower end holds
                "low": (ustar - 0.3, math.log(0.05)),   # misses below
                "wide": (0.5 - h, math.log(2.0)),       # covers everything: no end inside data
                "overflow": (ustar, math.log(0.4)),     # holds but too many elements to compact
                "tiny": (ustar, -30.0),                 # width e^-20 of the range after the clamp
            }
            for name, (u, lw) in cases.items():
                th = _proposal_params(u, lw)
                ctx = f"n={n} k={k} {name} {np.dtype(dtype).name}"
                print("case learned", ctx, flush=True)
                res, st, ref = _check_select(sel, x, k, th, ctx)
                a, b, use = sel.learned_bracket(_dev(x), k, _dev(th))
                if use and res["less"] < k <= res["less"] + res["equal"]:
                    xa, xb = np.array(a, dtype), np.array(b, dtype)
                    early = k <= np.sum(x == xs[0]) or k > n - np.sum(x == xs[-1])
                    left = np.sum(x <= xa) < k and xa > xs[0]
                    right = k <= np.sum(x < xb) and xb < xs[-1]
                    want = 0 if early else int(left) | (int(right) << 1)
                    assert st["bracket_used"] == want, (ctx, a, b)
            # the same with pass-0 compaction switched off
            th = _proposal_params(ustar, math.log(0.02))
            _check_select(sel, x, k, th, f"n={n} k={k} no-compact",
                          options=cps.default_options(compact_proposal=0))


def test_host_bracket_with_and_without_compaction(sel, oracle_mod):
    import paper_1104_2732_amd as cps
    x = workloads.single_array("normal", 1 << 22, np.float32, seed=21)
    xs = np.sort(x)
    for k in (1000, (x.size + 1) // 2, x.size - 5):
        v = float(xs[k - 1])
        ref = oracle_mod.select_kth(x, k)
        for (a, b) in [(v - 0.01, v + 0.01), (v - 1.0, v - 0.5), (v + 0.5, v + 1.0), (-9.0, 9.0)]:
            for compact in (0, 1):
                o = cps.default_options(use_bracket=1, bracket_lo=a, bracket_hi=b,
                                        compact_proposal=compact)
                print(f"case host bracket k={k} ({a:.3f},{b:.3f}) compact={compact}", flush=True)
                res, st = sel.select_kth(_dev(x), k, options=o, stats=True)
                assert_same_result(res, ref, (k, a, b, compact))
                if compact and st["bracket_used"] == 3 and (a, b) == (v - 0.01, v + 0.01):
                    assert res["passes"] == 1  # the input was read once


def test_training_reduces_passes(sel, oracle_mod):
    """Train on generated arrays, then compare with the plain method on held-out seeds."""
    P = sel.new_params()
    print("case train", flush=True)
    rep = sel.mlp_train(P, seed=1, n_arrays=8192, array_size=1 << 16, epochs=30, batch=256,
                        lr=2e-3, holdout=1024, holdout_seed=2)
    print("train report", rep, flush=True)
    assert rep["final_loss"] < rep["first_loss"]
    assert rep["holdout_coverage"] > 0.5
    n = 1 << 20
    x, ks = sel.mixture_generate(3, 0, 12, n)
    ks = ks.cpu().numpy()
    plain_passes, learned_passes = [], []
    for a in range(12):
        xa = x[a].contiguous()
        r_plain, s_plain = sel.select_kth(xa, int(ks[a]), stats=True)
        r_learn, s_learn = sel.select_kth_learned(xa, int(ks[a]), P, stats=True)
        ref = oracle_mod.select_kth(xa.cpu().numpy(), int(ks[a]))
        assert_same_result(r_plain, ref, f"plain {a}")
        assert_same_result(r_learn, ref, f"learned {a}")
        plain_passes.append(r_plain["passes"])
        learned_passes.append(r_learn["passes"])
    print("passes plain", plain_passes, "learned", learned_passes, flush=True)
    assert np.mean(learned_passes) < np.mean(plain_passes)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_sampled_proposal_parity(sel, oracle_mod, dtype):
    """The sample-quantile baseline: identical results for any width, fewer full reads."""
    rng = np.random.default_rng(13)
    for n in (1, 3, 4095, 4096, 100_001, 1 << 21):
        for dist in ("normal", "quantized_normal", "cauchy"):
            x = workloads.single_array(dist, n, dtype, seed=n, tag="gpu-sampled")
            for k in sorted({1, n, (n + 1) // 2, int(rng.integers(1, n + 1))}):
                ref = oracle_mod.select_kth(x, k)
                for z in (0.0, 1.0, 4.0, 1e3):
                    print(f"case sampled {dist} n={n} k={k} z={z}", flush=True)
                    res = sel.select_kth_sampled(_dev(x), k, z=z)
                    assert_same_result(res, ref, (dist, n, k, z))
    x = workloads.single_array("normal", 1 << 22, dtype, seed=5, tag="gpu-sampled")
    k = (x.size + 1) // 2
    r_plain = sel.select_kth(_dev(x), k)
    r_s = sel.select_kth_sampled(_dev(x), k, z=4.0)
    assert r_s["passes"] < r_plain["passes"]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_sample_bracket_order_statistics(sel, dtype):
    """The baseline's bracket is the fixed-stride sample's order statistics of ranks
    floor(c - z sd) - 1 and ceil(c + z sd) (0-based), against a library sort of that sample;
    heavy ties (two values, a constant) included."""
    rng = np.random.default_rng(17)
    cases = [("normal", 1 << 20), ("quantized_normal", 100_001), ("cauchy", 4095), ("normal", 5)]
    for dist, n in cases:
        x = workloads.single_array(dist, n, dtype, seed=n, tag="gpu-sample-bracket")
        for extra in ("", "two", "const"):
            xx = x.copy()
            if extra == "two":
                xx = np.where(xx > 0, 1.0, -1.0).astype(dtype)
            elif extra == "const":
                xx = np.full(n, 2.5, dtype=dtype)
            S = min(n, 4096)
            sv = np.sort(xx[:: n // S][:S].astype(np.float64))
            for k in sorted({1, n, (n + 1) // 2, int(rng.integers(1, n + 1))}):
                for z in (0.0, 4.0):
                    p = k / n
                    c = p * S
                    sd = np.sqrt(S * p * (1 - p)) + 1.0
                    lo, hi = int(np.floor(c - z * sd)) - 1, int(np.ceil(c + z * sd))
                    want_a = sv[lo] if lo >= 0 else -np.inf
                    want_b = sv[hi] if hi <= S - 1 else np.inf
                    print(f"case sample-bracket {dist}{extra} n={n} k={k} z={z}", flush=True)
                    a, b, use = sel.sample_bracket(_dev(xx), k, z)
                    assert use == 1 and a == want_a and b == want_b, (dist, extra, n, k, z, a, b)


def _fnv1a64(data: bytes) -> int:
    h = 14695981039346656037
    for b in data:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def test_model_file_round_trip(sel, tmp_path):
    """cps_model_save writes the documented layout (magic, version, shape, feature
    specification, count, FNV-1a hash, parameters); cps_model_load gives back the same bits
    and rejects a file with any field, the hash or the length wrong, leaving the target as it
    was."""
    import struct

    import paper_1104_2732_amd as cps
    print("case model file round trip", flush=True)
    P = sel.mlp_init(11)
    path = str(tmp_path / "net.cpsmlp")
    sel.model_save(P, path)
    raw = open(path, "rb").read()
    assert len(raw) == 40 + 4 * cps.MLP_PARAMS
    assert raw[:8] == b"CPSMLP01"
    assert struct.unpack("<6I", raw[8:32]) == (1, 67, 64, 2, 1, cps.MLP_PARAMS)
    params = np.frombuffer(raw[40:], dtype="<f4")
    assert np.array_equal(params.view(np.uint32), P.cpu().numpy().view(np.uint32))
    assert struct.unpack("<Q", raw[32:40])[0] == _fnv1a64(raw[40:])
    Q = sel.model_load(path)
    assert torch.equal(Q.view(torch.int32), P.view(torch.int32))
    # damaged files: a flipped parameter bit, a wrong version, a truncated or longer file
    sentinel = torch.full_like(P, 7.0)
    for name, blob in (("bit", raw[:100] + bytes([raw[100] ^ 1]) + raw[101:]),
                       ("version", raw[:8] + struct.pack("<I", 2) + raw[12:]),
                       ("shape", raw[:16] + struct.pack("<I", 32) + raw[20:]),
                       ("short", raw[:-4]), ("long", raw + b"\0")):
        bad = tmp_path / f"bad_{name}"
        bad.write_bytes(blob)
        with pytest.raises(cps.CpsError) as ei:
            sel.model_load(str(bad), sentinel)
        assert ei.value.code == cps.CPS_EFORMAT, name
        assert torch.all(sentinel == 7.0), name
    with pytest.raises(cps.CpsError) as ei:
        sel.model_load(str(tmp_path / "missing"), sentinel)
    assert ei.value.code == cps.CPS_EIO
    # a loaded network proposes exactly what the saved one did
    x = workloads.single_array("normal", 1 << 16, np.float32, seed=2, tag="model-io")
    xt = _dev(x)
    assert sel.learned_bracket(xt, 1000, P) == sel.learned_bracket(xt, 1000, Q)
