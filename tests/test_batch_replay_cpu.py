"""Host replay of the batched kernel's work queue (no GPU).

The batched kernel's descriptor checks and largest-first order (csrc/batch_queue.h, the
kernel's own code) and the cutting-plane state machine (csrc/cp_state.h) run on the CPU in
tests/cpp, built with the address and undefined-behaviour sanitizers, on the descriptors of
the GPU test of invalid descriptors: 20 float32 arrays (seed 3) with a zero rank, a rank
beyond the size, a null pointer, a zero size and a pointer not aligned to the element.
Every invalid array must be rejected without being read, every valid one must end with the
oracle's value and counts within the pass bound, and the queue must take every array once,
largest first.
"""
import os
import struct
import subprocess

import numpy as np
import pytest

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    exe = tmp_path_factory.mktemp("replay") / "batch_replay"
    src = os.path.join(HERE, "cpp", "batch_replay_main.cpp")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-o", str(exe), src], check=True)
    return exe


def _mixed_batch(count, seed, max_size=60_000):
    # the batch of the GPU test (tests/test_gpu_batched.py::_mixed_batch), float32
    rng = np.random.default_rng(seed)
    dists = ["uniform", "normal", "cauchy", "quantized_normal", "lognormal", "smallint", "mix2",
             "constant"]
    arrays, ks = [], []
    for i in range(count):
        n = i + 1 if i < 4 else int(np.floor(10 ** rng.uniform(0, np.log10(max_size))))
        arrays.append(workloads.single_array(dists[i % len(dists)], n, np.float32,
                                             seed=seed * 1000 + i, tag="gpu-batched"))
        ks.append([1, n, (n + 1) // 2, int(rng.integers(1, n + 1))][i % 4])
    return arrays, ks


def _run(replay, tmp_path, arrays, addrs, sizes, ks, ft=4096, hist_bits=12, side_bits=11):
    offs, blob, pos = [], [], 0
    for a in arrays:
        offs.append(pos)
        blob.append(a)
        pos += a.size
    data = np.concatenate(blob).astype(np.float32) if blob else np.zeros(0, np.float32)
    f = tmp_path / "desc.bin"
    with open(f, "wb") as fh:
        fh.write(struct.pack("<4q", len(arrays), ft, hist_bits, side_bits))
        for i in range(len(arrays)):
            fh.write(struct.pack("<Qqqq", addrs[i], sizes[i], ks[i], offs[i]))
        fh.write(struct.pack("<q", data.size))
        fh.write(data.tobytes())
    out = subprocess.run([str(replay), str(f)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    order, res = [], {}
    for line in out.stdout.splitlines():
        p = line.split()
        if p[0] == "order":
            order.append(int(p[2]))
        else:
            res[int(p[1])] = dict(status=int(p[2]), value=float(p[3]), less=int(p[4]),
                                  equal=int(p[5]), work_passes=int(p[6]))
    return order, res


def test_invalid_descriptor_batch_replay(replay, tmp_path, oracle_mod):
    from paper_1104_2732_amd import STATUS_BADARG
    arrays, ks = _mixed_batch(20, seed=3)
    sizes = [a.size for a in arrays]
    base = 0x7F00_0000_0000
    addrs = [base + 4096 * i for i in range(20)]  # aligned stand-ins for device pointers
    bad = {3: "k0", 5: "kbig", 7: "null", 9: "size0", 11: "unaligned"}
    ks[3] = 0
    ks[5] = sizes[5] + 1
    addrs[7] = 0
    sizes[9] = 0
    addrs[11] += 2
    order, res = _run(replay, tmp_path, arrays, addrs, sizes, ks)
    # every array taken once, largest first (ties by index)
    assert sorted(order) == list(range(20))
    want = sorted(range(20), key=lambda i: (-max(sizes[i], 0), i))
    assert order == want
    for i, (x, k) in enumerate(zip(arrays, ks)):
        if i in bad:
            assert res[i]["status"] == STATUS_BADARG, (i, bad[i], res[i])
            continue
        ref = oracle_mod.select_kth(x, k)
        assert res[i]["status"] == 0, (i, res[i])
        assert np.float32(res[i]["value"]) == np.float32(ref["value"]), (i, res[i], ref)
        assert (res[i]["less"], res[i]["equal"]) == (ref["less"], ref["equal"]), (i, res[i], ref)
        assert res[i]["work_passes"] <= 12, (i, res[i])


def test_full_batch_replay(replay, tmp_path, oracle_mod):
    """The 150-array mixed batches of the GPU parity test, through the same replay."""
    for seed in (0, 3, 11):
        arrays, ks = _mixed_batch(150, seed=seed)
        sizes = [a.size for a in arrays]
        addrs = [0x7F00_0000_0000 + 4096 * i for i in range(len(arrays))]
        order, res = _run(replay, tmp_path, arrays, addrs, sizes, ks)
        assert sorted(order) == list(range(len(arrays)))
        for i, (x, k) in enumerate(zip(arrays, ks)):
            ref = oracle_mod.select_kth(x, k)
            assert res[i]["status"] == 0, (seed, i, res[i])
            assert np.float32(res[i]["value"]) == np.float32(ref["value"]), (seed, i)
            assert (res[i]["less"], res[i]["equal"]) == (ref["less"], ref["equal"]), (seed, i)
