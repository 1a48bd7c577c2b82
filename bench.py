"""Benchmark: exact k-th element selection on one MI355X.

Workload (one "step"): every single-array case of the full-scale selection sweep,
    n in {2^24, 2^28} x {float32, float64}
      x {uniform[0,1), N(0,1), Cauchy(0,1), N(0,1) quantised to 1024 levels}
      x k in {1, floor(n/100), floor((n+1)/2), n-1},
i.e. 64 calls of select_kth on inputs already resident in HBM, enqueued
back to back on one stream.  The metric is exact-selection elements/s
(sum of n over the step's calls / step time); the JSON line also carries the
HBM roofline of the selection kernel and the CPU oracle timed on a bounded
sample of the same workload.  Further legs (their own keys in the line):
"small" (2^20 float32 uniform medians, seeds 0..9, default and cutting plane to
the end), "batched" (4096 lognormal arrays of log-uniform sizes in one
graph-captured launch vs a loop of single-array calls), "batched_large" (64
arrays of 2^22 elements, one or 16 workgroups per array), "lms" (1024
least-median-of-squares candidates over 2^20 rows, filtered and materialised
forms, their results compared), "lts" and "knn" (Section 6's
trimmed squares at the LMS shape; 1024 queries over 2^20 points), "transform"
(2^26 values with 1e20 outliers, cutting plane on x and on the log transform),
"learned" (the learned bracket proposal vs the plain method and the
sample-quantile baseline on 128 held-out 2^26-element mixture arrays; training
untimed) and "schedules" (the method under four schedules of its compaction:
cutting-plane passes to the end, split after one evaluation, split at the first
trial point, and the default).  --legs and --no-sweep select legs for profiling.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]

HBM traffic of the selection kernel comes from two rocprofv3 counter runs of
this same program with --copy-calibration (FETCH_SIZE, then WRITE_SIZE), each
scaled by what the counter reads for dispatches of known traffic in the same run:
the selection kernel's own pass 0 over 2^28 float32 values (1 GiB read with its
nontemporal loads) for FETCH_SIZE, a plain elementwise copy of 2^28 float32
values (1 GiB written) for WRITE_SIZE:
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR_F -- python3 bench.py \
        --steps 1 --warmup 0 --no-cpu-baseline --copy-calibration
    rocprofv3 --pmc WRITE_SIZE ... (same, into DIR_W)
    python bench.py --traffic-from DIR_F DIR_W   # writes the traffic record
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SIZES = (24, 28)
DTYPES = (np.float32, np.float64)
DISTS = ("uniform", "normal", "cauchy", "quantized_normal")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cp_select_kernel_traffic.json")
LEGS = ("small", "batched", "batched_large", "lms", "lts_knn", "transform", "learned",
        "schedules")
EPOCHS = 20  # training epochs of the learned proposal (untimed setup)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1104_2732_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(fn.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, if still current."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def _counter_rows(directory: str, counter: str):
    """(kernel name, value in KiB) per dispatch from a rocprofv3 counter-collection CSV tree."""
    import csv
    rows = []
    for root, _, files in os.walk(directory):
        for fn in files:
            if not fn.endswith("counter_collection.csv"):
                continue
            with open(os.path.join(root, fn), newline="") as f:
                for r in csv.DictReader(f):
                    if r.get("Counter_Name") == counter:
                        rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def traffic_from(fetch_dir: str, write_dir: str) -> dict:
    """Calibrate FETCH_SIZE and WRITE_SIZE on dispatches of known traffic and scale the
    selection kernel's per-dispatch readings; writes and returns the traffic record.
    FETCH_SIZE is scaled by what it reads for the selection kernel's own pass 0 over 2^28
    float32 values (rank 1 of an input with a unique minimum: one nontemporal read of 1 GiB,
    the first two selection dispatches of the run); the plain copy's factor is reported
    beside it.  WRITE_SIZE is scaled by the copy's (1 GiB written)."""
    gib = float(4 << 28)
    out = {"kernel_source_hash": kernel_source_hash(), "kernel": "cp_select_kernel"}
    per_launch = 0.0
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(d, counter)
        copies = [v for (name, v) in rows if "neg_kernel" in name]
        sel = [v for (name, v) in rows if "cp_select_kernel" in name]
        if not copies or len(sel) < 3:
            raise SystemExit(f"{counter}: no calibration dispatches or no selection dispatch in {d}")
        cal, sweep = sel[:2], sel[2:]
        copy_factor = gib / (float(np.mean(copies)) * 1024.0)
        rec = {"copy_KiB": float(np.mean(copies)), "copy_factor": copy_factor}
        if counter == "FETCH_SIZE":
            factor = gib / (float(np.mean(cal)) * 1024.0)
            rec["pass0_read_KiB"] = float(np.mean(cal))
            rec["pass0_read_factor"] = factor
        else:
            factor = copy_factor
        kib = float(np.mean(sweep))
        rec.update({"factor": factor, "select_KiB_per_dispatch": kib,
                    "select_dispatches": len(sweep), "bytes_per_launch": kib * 1024.0 * factor})
        out[counter] = rec
        per_launch += kib * 1024.0 * factor
    out["bytes_per_launch"] = per_launch
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    return out


def legs_traffic_from(fetch_dir: str, write_dir: str) -> dict:
    """HBM bytes of the batched and least-median-of-squares kernels from two counter runs of
    `bench.py --no-sweep --legs batched,lms --copy-calibration`: the last dispatch of each
    kernel (the batched leg ends with an eager call of its tuned options; the LMS leg's last
    calls of each form are ordinary ones), each counter scaled as in traffic_from (FETCH_SIZE
    by the selection kernel's pass 0 over 1 GiB, WRITE_SIZE by the copy's 1 GiB written)."""
    gib = float(4 << 28)
    kernels = {"batched_select_kernel<float": "batched float32 (4096 lognormal arrays)",
               "batched_select_kernel<double": "batched float64 (LMS medians, materialised form)",
               "lms_residual_rows_kernel<8, 2, false>": "LMS residuals (materialised form)",
               "lms_filter_kernel": "LMS filter (filtered form)",
               "lms_gather_kernel": "LMS packing and select (filtered form)"}
    out = {"kernel_source_hash": kernel_source_hash()}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(d, counter)
        if counter == "FETCH_SIZE":
            cal = [v for (name, v) in rows if "cp_select_kernel" in name][:2]
        else:
            cal = [v for (name, v) in rows if "neg_kernel" in name]
        if not cal:
            raise SystemExit(f"{counter}: no calibration dispatch in {d}")
        factor = gib / (float(np.mean(cal)) * 1024.0)
        out[counter + "_factor"] = factor
        for key, label in kernels.items():
            sel = [v for (name, v) in rows if key in name]
            if sel:
                out.setdefault(label, {})[counter + "_bytes"] = sel[-1] * 1024.0 * factor
    return out


def _time_ms(torch, fn, reps: int) -> float:
    """Mean device time of fn() over reps calls, bracketed by events on the current stream."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batched_leg(sel, cps, torch, reps: int = 5) -> dict:
    """4096 lognormal float32 arrays, sizes log-uniform in [1e3, 1e6], median ranks: one
    autotuned, graph-captured persistent launch against a loop of single-array calls."""
    import workloads
    arrays, sizes, ks = workloads.batched_arrays(4096, seed=0)
    dev = [torch.from_numpy(a).cuda() for a in arrays]
    del arrays
    ptrs, szs, kk, code = sel.batch_descriptors(dev, ks)
    out = sel.new_results(len(dev))
    best, tuned_ms = sel.autotune_batched(ptrs, szs, kk, len(dev), code, out)
    sel.reserve_batched(code)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            sel.select_kth_batched_async(ptrs, szs, kk, len(dev), code, out)
    torch.cuda.current_stream().wait_stream(stream)
    graph_ms = _time_ms(torch, g.replay, reps)
    res_b = out.cpu().numpy().view(cps.RESULT_DTYPE).copy()
    outs1 = sel.new_results(len(dev))
    views = [outs1[i * 48:(i + 1) * 48] for i in range(len(dev))]
    for d in dev:
        sel.reserve(d.numel(), code)

    def loop():
        for d, k, o in zip(dev, ks, views):
            sel.select_kth_async(d, int(k), o)
    loop_ms = _time_ms(torch, loop, 2)
    res_p = outs1.cpu().numpy().view(cps.RESULT_DTYPE)
    same = bool(np.array_equal(res_b["value_bits"], res_p["value_bits"]) and
                np.array_equal(res_b["less"], res_p["less"]) and
                np.array_equal(res_b["equal"], res_p["equal"]) and np.all(res_b["status"] == 0))
    total = int(np.sum(sizes))
    passes = res_b["passes"].astype(np.float64)
    # the same batch from [min, max] without the sampled bracket (the paper's start)
    o_plain = cps.default_batch_options(block_threads=best.block_threads, proposal=0)
    nobr_ms = _time_ms(torch, lambda: sel.select_kth_batched_async(ptrs, szs, kk, len(dev), code,
                                                                   out, o_plain), reps)
    # last: one eager call of the tuned options (the dispatch the counter runs read)
    sel.select_kth_batched_async(ptrs, szs, kk, len(dev), code, out, best)
    torch.cuda.synchronize()
    del dev
    return {"workload": "4096 lognormal(0,1) float32 arrays, sizes log-uniform in [1e3, 1e6], "
                        "median ranks (one persistent launch, captured in a graph)",
            "elements": total, "graph_ms": graph_ms, "elements_per_s": total / (graph_ms * 1e-3),
            "alg_GBps_one_read": total * 4 / (graph_ms * 1e-3) / 1e9,
            "passes_per_array_mean": float(passes.mean()),
            "passes_per_array_size_weighted": float((passes * sizes).sum() / sizes.sum()),
            "tuned": {"block_threads": best.block_threads, "split_capacity": best.split_capacity,
                      "partition_fraction": best.partition_fraction,
                      "count_first": best.count_first, "proposal": best.proposal,
                      "blocks_per_array": best.blocks_per_array,
                      "elements_per_block": best.elements_per_block},
            "without_sampled_bracket_ms": nobr_ms,
            "plain_loop_ms": loop_ms, "plain_loop_elements_per_s": total / (loop_ms * 1e-3),
            "speedup_vs_plain": loop_ms / graph_ms, "results_identical": same}


def batched_large_leg(sel, cps, torch, reps: int = 5) -> dict:
    """Few large arrays (64 lognormal float32 arrays of 2^22 elements, median ranks): one
    workgroup per array leaves most of the chip idle; split over 16 workgroups each they fill
    it.  The copy of each array's sampled-bracket interior gets room for 2^20 elements (the
    default 2^18 is sized for arrays of ~10^6 elements: an overflowing copy sends the array
    back over its full length with one workgroup, also timed); the autotuner sizes it from
    the batch itself."""
    g = torch.Generator(device="cuda")
    g.manual_seed(12345)
    x = torch.exp(torch.randn((64, 1 << 22), generator=g, device="cuda", dtype=torch.float32))
    dev = [x[i] for i in range(64)]
    ks = [((1 << 22) + 1) // 2] * 64
    ptrs, szs, kk, code = sel.batch_descriptors(dev, ks)
    out = sel.new_results(64)
    cases = {"one_workgroup_per_array": dict(team_capacity=1 << 20),
             "16_workgroups_per_array": dict(blocks_per_array=16, elements_per_block=1 << 18,
                                             team_capacity=1 << 20),
             "16_workgroups_per_array_default_capacity": dict(blocks_per_array=16,
                                                              elements_per_block=1 << 18),
             "without_sampled_bracket": dict(proposal=0)}
    tuner = cps.Selector(0)  # a handle of its own: the tuned choice stays out of later legs
    try:
        best, _ = tuner.autotune_batched(ptrs, szs, kk, 64, code, out)
    finally:
        tuner.close()
    cases["autotuned"] = {f: getattr(best, f) for f, _ in cps.BatchOptions._fields_}
    res = {}
    ref = None
    for name, kw in cases.items():
        o = cps.default_batch_options(**kw)
        ms = _time_ms(torch, lambda: sel.select_kth_batched_async(ptrs, szs, kk, 64, code, out, o), reps)
        r = out.cpu().numpy().view(cps.RESULT_DTYPE).copy()
        ref = r if ref is None else ref
        res[name] = {"ms": round(ms, 4), "elements_per_s": 64 * (1 << 22) / (ms * 1e-3),
                     "passes_per_array_mean": float(r["passes"].mean()),
                     "identical": bool(np.array_equal(r["value_bits"], ref["value_bits"]))}
    res["autotuned"]["options"] = {f: cases["autotuned"][f] for f in
                                   ("block_threads", "proposal", "blocks_per_array",
                                    "elements_per_block", "team_capacity")}
    del x, dev
    return {"workload": "64 lognormal(0,1) float32 arrays of 2^22 elements, median ranks",
            "cases": res}


def lts_knn_leg(sel, torch, reps: int = 5) -> dict:
    """Section 6's other uses of the k-th order statistic: least trimmed squares at the
    least-median-of-squares shape, and k nearest neighbours."""
    import workloads
    n, p, m = 1 << 20, 8, 1024
    X, y, _, betas = workloads.lms_problem(n, p, m, seed=0)
    Xd, yd, bd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (X, y, betas))
    import paper_1104_2732_amd as cps
    out = torch.empty(m * cps.TRIM_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    lts_ms = _time_ms(torch, lambda: sel.lts_trimmed_sq_async(Xd, yd, bd, (n + 1) // 2, out), reps)
    lts_mat_ms = _time_ms(torch, lambda: sel.lts_trimmed_sq_async(Xd, yd, bd, (n + 1) // 2, out,
                                                                  cps.LMS_MATERIALISED), reps)
    del Xd, yd, bd
    nk, dim, nq, k = 1 << 20, 8, 1024, 64
    rng = np.random.default_rng(0)
    P = rng.standard_normal((nk, dim)).astype(np.float32)
    Q = rng.standard_normal((nq, dim)).astype(np.float32)
    f = (np.sin(P.sum(axis=1)) + 0.1 * rng.standard_normal(nk)).astype(np.float32)
    Pd, fd, Qd = (torch.from_numpy(a).cuda() for a in (P, f, Q))
    kout = torch.empty(nq * cps.KNN_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    knn_ms = _time_ms(torch, lambda: sel.knn_mean_async(Pd, fd, Qd, k, kout), reps)
    knn_mat_ms = _time_ms(torch, lambda: sel.knn_mean_async(Pd, fd, Qd, k, kout,
                                                            cps.LMS_MATERIALISED), reps)
    return {"lts": {"workload": "n=2^20 rows, p=8, 1024 candidates, h=floor((n+1)/2)",
                    "ms": lts_ms, "residuals_per_s": n * m / (lts_ms * 1e-3),
                    "materialised_ms": lts_mat_ms},
            "knn": {"workload": "2^20 points in 8 dimensions (N(0,1)), 1024 queries, k=64",
                    "ms": knn_ms, "distances_per_s": nk * nq / (knn_ms * 1e-3),
                    "materialised_ms": knn_mat_ms}}


def transform_leg(sel, cps, torch, reps: int = 3) -> dict:
    """Section 5.3's outliers: 2^26 float32 N(0,1) values with 64 of them near 1e20, the
    cutting plane to the end on x and on F(x) = log(1 + x - min x)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(777)
    n = 1 << 26
    x = torch.randn(n, generator=g, device="cuda", dtype=torch.float32)
    idx = torch.randint(0, n, (64,), generator=g, device="cuda")
    x[idx] = 1e20 * (1.0 + torch.rand(64, generator=g, device="cuda"))
    res = sel.new_results(1)
    stats = sel.new_stats()
    out = {"workload": "n=2^26 float32 N(0,1) with 64 values near 1e20, median rank", "cases": {}}
    for name, kw in {"cutting_plane_on_x": dict(partition_fraction=0.0, hist_bits=0),
                     "cutting_plane_on_log": dict(partition_fraction=0.0, hist_bits=0, transform=1),
                     "default_on_x": dict(), "default_on_log": dict(transform=1)}.items():
        o = cps.default_options(**kw)
        k = (n + 1) // 2
        ms = _time_ms(torch, lambda: sel.select_kth_async(x, k, res, options=o), reps)
        sel.select_kth_async(x, k, res, stats, options=o)
        torch.cuda.synchronize()
        st = stats.cpu().numpy().view(cps.STATS_DTYPE)[0]
        out["cases"][name] = {"ms": round(ms, 4), "work_passes": int(st["work_passes"]),
                              "kelley_steps": int(st["kelley_steps"]),
                              "value_bits": int(res.cpu().numpy().view(cps.RESULT_DTYPE)[0]["value_bits"])}
    vals = {c["value_bits"] for c in out["cases"].values()}
    out["results_identical"] = len(vals) == 1
    del x
    return out


def lms_leg(sel, cps, torch, reps: int = 5) -> dict:
    """Least median of squares: 2^20 rows, p = 8, 1024 candidates, 30 % of rows shifted; the
    filtered form (the default) and the materialised one, whose results must be identical."""
    import workloads
    n, p, m = 1 << 20, 8, 1024
    X, y, _, betas = workloads.lms_problem(n, p, m, seed=0)
    Xd, yd, bd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (X, y, betas))
    res = {}
    ms = {}
    for name, form in (("materialised", cps.LMS_MATERIALISED), ("filtered", cps.LMS_FILTERED)):
        out = sel.new_results(m)
        ms[name] = _time_ms(torch, lambda: sel.lms_median_sq_residuals_async(Xd, yd, bd, out, form),
                            reps)
        res[name] = out.cpu().numpy().view(cps.RESULT_DTYPE).copy()
    a, b = res["filtered"], res["materialised"]
    same = all(np.array_equal(a[f], b[f]) for f in ("value_bits", "less", "equal", "greater", "status"))
    passes = b["passes"].astype(np.float64)
    # the arithmetic every form must do: 2p - 1 products and sums, the difference and the
    # square per residual (fixed order, no fused multiply-add: one instruction each), against
    # the double-precision vector issue rate (256 CUs x 64 lanes x 2.4 GHz, FMA counted once)
    ops = (2 * p + 1) * n * m
    peak_ops = 256 * 64 * 2.4e9
    return {"workload": "n=2^20 rows, p=8, 1024 candidates (residuals fixed order, no FMA)",
            "ms": ms["filtered"], "residuals_per_s": n * m / (ms["filtered"] * 1e-3),
            "fp64_valu": {"ops_per_residual": 2 * p + 1, "ops_per_s": ops / (ms["filtered"] * 1e-3),
                          "peak_ops_per_s": peak_ops,
                          "frac": ops / (ms["filtered"] * 1e-3) / peak_ops},
            "materialised_ms": ms["materialised"], "forms_identical": bool(same),
            "materialised_passes_per_candidate_mean": float(passes.mean()),
            "residual_bytes_one_write_one_read": 2 * n * m * 8}


def learned_leg(sel, cps, torch, held_out: int = 128, chunk: int = 8) -> dict:
    """The learned proposal on held-out float32 mixture arrays of n = 2^26 with uniform ranks,
    against the plain method and the non-learned sample-quantile proposal on the same arrays
    (training untimed).  Arrays are generated on the device in chunks; every call is timed on
    its own with events on the launch stream (the mean of three runs)."""
    P = sel.new_params()
    t0 = time.time()
    rep = sel.mlp_train(P, seed=1, n_arrays=100_000, array_size=1 << 18, epochs=EPOCHS,
                        batch=256, lr=2e-3, holdout=4096, holdout_seed=2)
    train_s = time.time() - t0
    n = 1 << 26
    sel.reserve(n, cps.CPS_F32)
    names = ("plain", "learned", "sampled")
    ms = {k: [] for k in names}
    passes = {k: [] for k in names}
    same = True
    outs = {k: sel.new_results(1) for k in names}
    stream = torch.cuda.current_stream()

    def call(name, row, k):
        if name == "plain":
            sel.select_kth_async(row, k, outs[name])
        elif name == "learned":
            sel.select_kth_learned_async(row, k, P, outs[name])
        else:
            sel.select_kth_sampled_async(row, k, outs[name], 4.0)

    for c0 in range(0, held_out, chunk):
        x, ks = sel.mixture_generate(3, c0, chunk, n)
        ks = [int(v) for v in ks.cpu().numpy()]
        for a in range(chunk):
            row, k = x[a], ks[a]
            bits = set()
            for name in names:
                call(name, row, k)  # warm
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(3)]
                for e0, e1 in ev:
                    e0.record(stream)
                    call(name, row, k)
                    e1.record(stream)
                torch.cuda.synchronize()
                ms[name].append(float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev])))
                r = outs[name].cpu().numpy().view(cps.RESULT_DTYPE)[0]
                passes[name].append(int(r["passes"]))
                bits.add((int(r["value_bits"]), int(r["less"]), int(r["equal"]), int(r["status"])))
            same &= len(bits) == 1
        del x
    out = {"workload": f"{held_out} held-out mixture arrays (1-4 Gaussian/lognormal/uniform "
                       "components), float32, n=2^26, k uniform in [1, n]",
           "results_identical": bool(same)}
    for name in names:
        a, p = np.array(ms[name]), np.array(passes[name])
        out[name] = {"ms_mean": round(float(a.mean()), 4), "ms_median": round(float(np.median(a)), 4),
                     "passes_over_x_mean": float(p.mean()),
                     "passes_over_x_median": float(np.median(p))}
    t_plain, t_learned, t_sampled = (np.array(ms[k]) for k in names)
    out["learned_faster_than_plain"] = int(np.sum(t_learned < t_plain))
    out["learned_faster_than_sampled"] = int(np.sum(t_learned < t_sampled))
    out["learned_fewer_reads_than_sampled"] = int(np.sum(np.array(passes["learned"]) <
                                                         np.array(passes["sampled"])))
    out["speedup_vs_plain"] = float(t_plain.mean() / t_learned.mean())
    out["sampled_note"] = ("non-learned baseline: order statistics of the same stride sample "
                           "(radix-selected), +-4 sd of the sample rank")
    out["train_s"] = round(train_s, 2)
    out["train"] = {"arrays": 100_000, "array_size": 1 << 18, "epochs": EPOCHS,
                    "first_loss": rep["first_loss"], "final_loss": rep["final_loss"],
                    "holdout_coverage": rep["holdout_coverage"],
                    "holdout_width": rep["holdout_width"]}
    return out


def schedules_leg(sel, cps, torch, reps: int = 3) -> dict:
    """The same selections under four schedules of the method on 2^28 normal arrays:
    cutting-plane passes until the bracket holds at most the final threshold, then the
    gather and the exact select (no split, no histograms); the split after one evaluation
    pass (partition fraction 0.75); the split at the first trial point (both sides
    written and counted); and the default (the first evaluation counts both sides in key
    bins, the next pass over x compacts the bin of the rank)."""
    import workloads
    scheds = {"cutting_plane_to_the_end": dict(partition_fraction=0.0, hist_bits=0),
              "split_after_one_evaluation": dict(partition_fraction=0.75, count_first=0),
              "split_at_first_trial_point": dict(count_first=0),
              "default_count_at_first_trial_point": dict()}
    out = {"workload": "n=2^28 N(0,1), k in {n/100, median}", "cases": {}}
    evals = []
    res = sel.new_results(1)
    stats = sel.new_stats()
    for dtype in DTYPES:
        n = 1 << 28
        x = workloads.single_array("normal", n, dtype, seed=0, tag="bench")
        xt = torch.from_numpy(x).cuda()
        del x
        for k in (n // 100, (n + 1) // 2):
            for name, kw in scheds.items():
                o = cps.default_options(**kw)
                ms = _time_ms(torch, lambda: sel.select_kth_async(xt, k, res, options=o), reps)
                sel.select_kth_async(xt, k, res, stats, options=o)
                torch.cuda.synchronize()
                st = stats.cpu().numpy().view(cps.STATS_DTYPE)[0]
                case = {"ms": round(ms, 4), "passes_over_x": int(st["passes"]),
                        "work_passes": int(st["work_passes"]),
                        "kelley_steps": int(st["kelley_steps"])}
                if name == "cutting_plane_to_the_end":
                    # the iterated fused evaluation (Section 4, Algorithm 1): each pass's time
                    # from the publication of the state before it to the last workgroup's
                    # arrival after it (device clock, 100 MHz), n * sizeof(T) bytes per pass
                    np_ = min(int(st["work_passes"]), cps.STATS_MAX_PASSES)
                    us = [(int(st["t_arrive"][i]) - int(st["t_publish"][i - 1])) * 1e-2
                          for i in range(1, np_) if st["kind"][i] == cps.PASS_EVAL
                          and st["working"][i] == n]
                    gbps = [n * np.dtype(dtype).itemsize / (u * 1e-6) / 1e9 for u in us]
                    case["eval_passes"] = len(us)
                    case["eval_pass_us_mean"] = round(float(np.mean(us)), 2)
                    case["eval_pass_GBps_mean"] = round(float(np.mean(gbps)), 1)
                    case["eval_pass_frac_of_peak"] = round(float(np.mean(gbps)) / HBM_PEAK_GBS, 3)
                    evals.extend(gbps)
                out["cases"][f"{np.dtype(dtype).name} k={k} {name}"] = case
        del xt
        torch.cuda.empty_cache()
    # the fused evaluation pass iterated by the cutting plane, over the whole 2^28 array: its
    # own roofline (per-pass algorithmic bytes n * sizeof(T) over the per-pass device time)
    out["iterated_eval_pass"] = {
        "passes": len(evals), "GBps_mean": round(float(np.mean(evals)), 1),
        "frac_of_peak": round(float(np.mean(evals)) / HBM_PEAK_GBS, 3),
        "note": "evaluation passes of the cutting-plane-to-the-end schedule, both dtypes"}
    return out


def small_leg(sel, cps, torch, seeds=range(10), reps: int = 10) -> dict:
    """n = 2^20 float32 uniform[0,1), median rank: the plain method from the full [min, max]
    bracket plus the exact finish, on seeds 0..9 (each timed over `reps` calls with events on
    the launch stream), checked against the oracle per seed."""
    import oracle
    import workloads
    n = 1 << 20
    k = (n + 1) // 2
    out = {"workload": "n=2^20 float32 uniform[0,1), k=(n+1)/2, seeds 0..9", "cases": {}}
    res = sel.new_results(1)
    stats = sel.new_stats()
    scheds = {"default": None,
              "cutting_plane_to_the_end": cps.default_options(partition_fraction=0.0,
                                                              hist_bits=0)}
    ok = True
    for name, o in scheds.items():
        per_seed, passes = [], []
        for seed in seeds:
            x = workloads.single_array("uniform", n, np.float32, seed=seed, tag="bench-small")
            xt = torch.from_numpy(x).cuda()
            ms = _time_ms(torch, lambda: sel.select_kth_async(xt, k, res, options=o), reps)
            sel.select_kth_async(xt, k, res, stats, options=o)
            torch.cuda.synchronize()
            r = res.cpu().numpy().view(cps.RESULT_DTYPE)[0]
            ref = oracle.select_kth(x, k)
            ok &= bool(r["status"] == 0 and int(r["value_bits"]) == ref["value_bits"] and
                       int(r["less"]) == ref["less"] and int(r["equal"]) == ref["equal"])
            per_seed.append(ms)
            passes.append(int(stats.cpu().numpy().view(cps.STATS_DTYPE)[0]["passes"]))
        a = np.array(per_seed)
        out["cases"][name] = {"ms_mean": round(float(a.mean()), 4),
                              "ms_median": round(float(np.median(a)), 4),
                              "ms_min": round(float(a.min()), 4),
                              "elements_per_s_mean": n / (a.mean() * 1e-3),
                              "passes_over_x_mean": float(np.mean(passes))}
    out["parity_ok"] = ok
    out["parity_checked"] = len(scheds) * len(list(seeds))
    return out


def host_info() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(budget_s: float = 20.0):
    """The CPU oracle on a bounded sample of the same workload, one thread, ~budget_s seconds:
    the 32 n=2^24 cases, then n=2^28 float32 cases while the budget lasts."""
    import oracle
    import workloads
    elems = 0
    spent = 0.0
    done = 0
    results = {}  # (lg, dtype name, dist, k) -> the oracle's result, for the parity check
    for lg, dtypes in ((24, DTYPES), (28, (np.float32,))):
        for dtype in dtypes:
            for dist in DISTS:
                if spent > budget_s:
                    break
                x = workloads.single_array(dist, 1 << lg, dtype, seed=0, tag="bench")
                for k in workloads.ks_for(x.size):
                    t0 = time.perf_counter()
                    r = oracle.select_kth(x, k)
                    spent += time.perf_counter() - t0
                    elems += x.size
                    done += 1
                    results[(lg, np.dtype(dtype).name, dist, int(k))] = r
                del x
    line = {"value": elems / spent, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} of the 64 calls (all n=2^24, then n=2^28 float32 until "
                      f"~{budget_s:.0f} s), single-threaded quickselect with its counting scan, "
                      f"{spent:.1f} s",
            "host": host_info()}
    return line, results


def calibration_dispatches(sel, torch, dev) -> None:
    """Dispatches of known HBM traffic for the counter runs: a plain copy of 2^28 float32
    values (1 GiB read and written), then two selections of rank 1 on a 2^28 float32 input
    whose minimum is unique: pass 0 alone, one read of 1 GiB with the selection kernel's own
    nontemporal loads, and nothing written."""
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst
    cal = torch.arange(1 << 28, dtype=torch.float32, device=dev)
    cal_out = sel.new_results(1)
    for _ in range(2):
        sel.select_kth_async(cal, 1, cal_out)
    torch.cuda.synchronize()
    del cal


def run_legs(sel, cps, torch, legs, line: dict) -> None:
    """The extra legs named in `legs` (all of LEGS by default), each under its own key."""
    table = {"small": lambda: small_leg(sel, cps, torch),
             "batched": lambda: batched_leg(sel, cps, torch),
             "batched_large": lambda: batched_large_leg(sel, cps, torch),
             "lms": lambda: lms_leg(sel, cps, torch),
             "lts_knn": lambda: lts_knn_leg(sel, torch),
             "transform": lambda: transform_leg(sel, cps, torch),
             "learned": lambda: learned_leg(sel, cps, torch),
             "schedules": lambda: schedules_leg(sel, cps, torch)}
    for name in LEGS:
        if name not in legs:
            continue
        torch.cuda.empty_cache()
        r = table[name]()
        if name == "lts_knn":
            line.update(r)
        else:
            line[name] = r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched, least-median-of-squares and learned-proposal legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB elementwise copy first (counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the traffic record from two rocprofv3 counter runs and exit")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated extra legs to run (default: all of " + ",".join(LEGS) + ")")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the single-array sweep and print only the extra legs (profiling)")
    ap.add_argument("--legs-traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the batched and LMS kernels' traffic from two counter runs of "
                         "--no-sweep --legs batched,lms --copy-calibration and exit")
    args = ap.parse_args()
    if args.traffic_from:
        print(json.dumps(traffic_from(*args.traffic_from)))
        return
    if args.legs_traffic_from:
        print(json.dumps(legs_traffic_from(*args.legs_traffic_from)))
        return
    legs = [l for l in args.legs.split(",") if l]
    unknown = [l for l in legs if l not in LEGS]
    if unknown:
        ap.error(f"unknown legs {unknown}; known: {list(LEGS)}")
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs each selection on a single "
              "MI355X.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1104_2732_amd as cps
    import workloads

    dev = torch.device("cuda", 0)
    sel = cps.Selector(0)
    if args.no_sweep:
        line = {"legs_only": True}
        if args.copy_calibration:
            calibration_dispatches(sel, torch, dev)
        run_legs(sel, cps, torch, legs, line)
        print(json.dumps(line), flush=True)
        sel.close()
        return

    # ---- resident inputs
    t_gen = time.time()
    inputs = []  # (tensor, n, k, dtype)
    keys = []    # (lg, dtype name, distribution, k) of each call
    for lg in SIZES:
        n = 1 << lg
        for dtype in DTYPES:
            for dist in DISTS:
                x = workloads.single_array(dist, n, dtype, seed=0, tag="bench")
                xt = torch.from_numpy(x).to(dev)
                del x
                for k in workloads.ks_for(n):
                    inputs.append((xt, n, k, np.dtype(dtype)))
                    keys.append((lg, np.dtype(dtype).name, dist, int(k)))
    for dtype in DTYPES:
        sel.reserve(1 << max(SIZES), cps.CPS_F32 if dtype == np.float32 else cps.CPS_F64)
    torch.cuda.synchronize()
    gen_s = time.time() - t_gen

    if args.copy_calibration:
        calibration_dispatches(sel, torch, dev)

    outs = sel.new_results(len(inputs))
    res_views = [outs[i * 48:(i + 1) * 48] for i in range(len(inputs))]

    # ---- algorithmic traffic per call from the kernel's own trace (untimed run)
    stats_buf = sel.new_stats()
    alg_bytes = []
    for (xt, n, k, dt), out in zip(inputs, res_views):
        sel.select_kth_async(xt, k, out, stats_buf)
        torch.cuda.synchronize()
        st = stats_buf.cpu().numpy().view(cps.STATS_DTYPE)[0]
        alg_bytes.append(int(st["elements_read"] + st["elements_written"]) * dt.itemsize)
    res = outs.cpu().numpy().view(cps.RESULT_DTYPE)
    assert np.all(res["status"] == 0), "a selection reported a non-zero status"

    def step(events=None):
        for i, ((xt, n, k, dt), out) in enumerate(zip(inputs, res_views)):
            if events is not None:
                events[i][0].record()
            sel.select_kth_async(xt, k, out)
            if events is not None:
                events[i][1].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in inputs] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    kern_ms = np.array([[a.elapsed_time(b) for (a, b) in evs] for evs in ev])  # steps x calls
    per_call_ms = kern_ms.mean(axis=0)
    elems_per_step = sum(n for (_, n, _, _) in inputs)
    ms_per_step = wall * 1e3 / args.steps
    value = elems_per_step * args.steps / wall

    # roofline of the selection kernel: algorithmic bytes per launch / launch duration
    bytes_per_launch = float(np.mean(alg_bytes))
    avg_launch_ms = float(per_call_ms.mean())
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    big = [i for i, (_, n, _, _) in enumerate(inputs) if n == 1 << max(SIZES)]
    big_gbs = float(np.sum([alg_bytes[i] for i in big]) / (np.sum(per_call_ms[big]) * 1e-3) / 1e9)
    traffic = load_traffic()

    detail = {}
    for lg in SIZES:
        for dt in DTYPES:
            idx = [i for i, (_, n, _, d) in enumerate(inputs) if n == 1 << lg and d == np.dtype(dt)]
            t_ms = float(np.sum(per_call_ms[idx]))
            detail[f"{np.dtype(dt).name}_2^{lg}"] = {
                "ms_per_call": round(t_ms / len(idx), 4),
                "elements_per_s": (1 << lg) * len(idx) / (t_ms * 1e-3),
                "alg_GBps": float(np.sum([alg_bytes[i] for i in idx]) / (t_ms * 1e-3) / 1e9),
                "passes_over_x": float(np.mean(res["passes"][idx])),
            }

    line = {
        "metric": "exact-selection elements/s",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded Philox; uniform, normal, Cauchy, 1024-level quantised normal)",
        "config": {"workload": "single-array select_kth sweep: n in {2^24, 2^28} x {f32, f64} x "
                               "{uniform, normal, cauchy, quantized normal} x k in {1, n/100, "
                               "median, n-1} (64 calls per step)",
                   "calls_per_step": len(inputs), "elements_per_step": elems_per_step},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "cp_select_kernel", "avg_launch_ms": avg_launch_ms,
                     "alg_bytes_per_launch": bytes_per_launch,
                     "n2^28_only_GBps": big_gbs},
        "detail": detail,
        "setup_s": round(gen_s, 1),
    }
    # parity of every call of the sweep at full size: the defining property of x_(k)
    # (Section 1: #(x < m) < k <= #(x <= m) with m an element of x), counted on the host
    inv_ok, inv_checked = True, 0
    for xt in {id(t): t for (t, _, _, _) in inputs}.values():
        xh = xt.cpu().numpy()
        for i, (t, n, k, dt) in enumerate(inputs):
            if t is not xt:
                continue
            v = np.array([res[i]["value"]], dtype=dt)[0]
            less = int(np.count_nonzero(xh < v))
            eq = int(np.count_nonzero(xh == v))
            inv_ok &= bool(eq >= 1 and less < k <= less + eq and
                           (int(res[i]["less"]), int(res[i]["equal"])) == (less, eq))
            inv_checked += 1
        del xh
    line["parity"] = {"invariant_checked": inv_checked, "invariant_ok": inv_ok,
                      "note": "every call of the sweep: #(x<m) < k <= #(x<=m), m in x, and "
                              "the reported counts, on the host copy of each input"}
    if not args.no_extras:
        del inputs
        run_legs(sel, cps, torch, legs, line)
    if not args.no_cpu_baseline:
        line["cpu_baseline"], oracle_res = cpu_baseline()
        # the oracle's own results on the calls it timed, against the GPU's
        ok = True
        for i, key in enumerate(keys):
            ref = oracle_res.get(key)
            if ref is None:
                continue
            ok &= bool(int(res[i]["value_bits"]) == ref["value_bits"] and
                       int(res[i]["less"]) == ref["less"] and
                       int(res[i]["equal"]) == ref["equal"] and res[i]["status"] == 0)
        line["parity"]["oracle_checked"] = len(oracle_res)
        line["parity"]["oracle_ok"] = ok
    print(json.dumps(line), flush=True)
    sel.close()


if __name__ == "__main__":
    main()
