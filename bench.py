#!/usr/bin/env python3
"""Benchmark of the plain product over Z/pZ on one MI355X, with the GCD
workloads reported beside it. Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Headline (value, ms_per_step): mulmods/s of the plain product of two dense
polynomials of degree 65535 over p = 469762049 (4,294,967,296 products of
coefficients per step), inputs resident in HBM, one step = one complete
product (all kernels of the call), timed with events on the launch stream
over K steps after W warm-up steps (defaults 200 and 1000: the shader clock
takes tens of milliseconds of sustained load to reach its steady rate).

Beside it, in the same line:
  roofline      the dominant kernel of the engine that ran (matrix cores:
                mulx_kernel, the method's work of one multiply-add (2
                operations) per coefficient product against the dense int8
                MFMA peak, and apart from it the MFMA digit utilisation (16
                int8 digit products per coefficient product); VALU tiles:
                mul_tile_kernel, one 32x32->64-bit multiply-add per
                coefficient product against the VALU multiply-add peak):
                algorithmic operations per launch over its average duration
                (HIP events around each launch on its stream, same timed
                steps), and the measured HBM traffic over the algorithmic
                bytes;
  cpu_baseline  the CPU oracle timed on this host on a bounded sample of the
                same product (single thread), with the CPU model and counts;
  cpu_baselines the oracle on the other workloads: the gcd and division
                (one thread), the batched products and the served gcds
                (one thread on a sample, and a thread pool over instances);
  batched_4096  4096 independent products (degrees log-uniform in [32, 8192])
                as one prepared batch replayed from a captured graph (the
                larger items on the matrix cores, the rest on the VALU tiles
                beside them; tile shape from the autotuner), beside the same
                products as 4096 separate calls on the same stream;
  product_2048  the degree-2047 product: single-call host latency, and the
                steady rate of 100 calls captured in one graph and replayed;
  divrem_65536  Euclidean division with a long quotient: degree 65535 by
                degree 32767 (32769 quotient terms) at the default s;
  gcd_32768     Euclidean division and remainder-sequence gcd of the degree
                32768 / 32767 pair with a planted degree-1000 gcd (time per
                division step, grid syncs, updates/s against the VALU peak),
                and the extended gcd (Bezout cofactors) of the same pair;
  batched_gcd   the same 2048 gcd requests as one prepared batch (s from the
                autotuner) replayed from a captured graph, beside one call per
                request on a sample;
  served        a Poisson stream of 2048 gcd requests (degrees log-uniform
                in [64, 16384], planted gcd, three primes) through the
                continuous-batching server: saturated GCDs/s, then p50/p99
                latency at 0.8 of that rate (and at 0.5, 1.0, 1.2), beside
                the same trace served one synchronous call per request (FIFO)
                at 0.8;
  served_mixed  the same kind of trace with a quarter of the requests
                Euclidean divisions: saturated requests/s, p50/p99 of each.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "mulmods/s in plain poly multiply; batched GCDs/s + p99 vs one-call-per-instance"
# VALU peak for one exact 32x32->64-bit multiply-add per lane per clock
# (v_mad_u64_u32 issues at the full rate on gfx950): 256 CUs x 64 lanes x 2.4 GHz.
PEAK_MULMOD_PER_S = 256 * 64 * 2.4e9
# Published dense int8 matrix-core peak of MI355X (operations: 2 per multiply-add).
PEAK_INT8_OPS_PER_S = 5.0e15
# int8 digit products per coefficient product on the matrix cores (4 x 4 digits)
DIGIT_PRODUCTS = 16
# HBM bytes the degree-65535 product must move: both inputs read, f written once
ALGO_BYTES_65536 = 4 * (65536 + 65536 + 131071)
KERNEL_SOURCES = {"mulx_kernel": ("mul_mfma.hip", "common.hpp", "internal.hpp"),
                  "mul_tile_kernel": ("mul.hip", "common.hpp", "internal.hpp")}


def traffic_file(kernel: str) -> str:
    return os.path.join(ROOT, "profiles", "traffic_%s_product_65536.json" % kernel)


def source_digest(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1402_0264_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str):
    """HBM bytes per launch of the kernel from the committed counter
    summary, or None when its source changed since the counters were taken."""
    try:
        with open(traffic_file(kernel)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("source_digest") != source_digest(kernel):
        return None
    return rec.get("bytes_per_launch")


def tune_summary(rec: dict) -> dict:
    out = {"engine": rec["engine"], "ms": rec["ms"], "cached": rec.get("cached", False)}
    if rec["engine"] == "valu":
        out.update({"r": rec["r"], "s": rec["kc"]})
    return out


def time_steps(fn, steps: int, warmup: int):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def cpu_info() -> dict:
    """The host the CPU baselines ran on: model name, logical CPUs, the
    CPUs this process may use, and the pool size the baselines use (the
    box's thread budget, OMP_NUM_THREADS, when set)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    pool = int(os.environ.get("OMP_NUM_THREADS") or 0) or avail
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_available": avail, "pool_threads": min(pool, avail)}


def _pool_map(fn, items, threads: int):
    """fn over items on a thread pool (the oracle's ctypes calls release
    the GIL, so the threads run on separate cores)."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, items))


def cpu_baselines(reqs, threads: int) -> dict:
    """The oracle (plain C, no tuning) on the other workloads: one thread,
    and a pool of `threads` threads over independent instances (batched
    products, served gcds). Bounded samples where the whole would take
    minutes; each entry says what it timed."""
    import oracle
    from paper_1402_0264_amd import gen
    oracle.lib()
    out = {}
    pl = gen.gcd_32768()
    p = pl.p
    a, b = oracle.mul(pl.g, pl.u, p), oracle.mul(pl.g, pl.v, p)
    t0 = time.perf_counter()
    g, degs, stats = oracle.gcd(a, b, p, with_info=True)
    t = time.perf_counter() - t0
    out["gcd_32768"] = {"kind": "oracle", "threads": 1, "ms": round(t * 1e3, 1), "gcds_per_s": round(1 / t, 3),
                        "updates": int(stats.updates), "updates_per_s": round(stats.updates / t, 1),
                        "sample": "the whole gcd (Euclid, one remainder at a time)"}
    st = gen.Stream(gen.SEED_BASE + 6)
    da, db = st.uniform_poly(65535, gen.P_A), st.uniform_poly(32767, gen.P_A)
    t0 = time.perf_counter()
    oracle.divrem(da, db, gen.P_A)
    t = time.perf_counter() - t0
    upd = (da.size - db.size + 1) * db.size
    out["divrem_65536"] = {"kind": "oracle", "threads": 1, "ms": round(t * 1e3, 1),
                           "updates_per_s": round(upd / t, 1), "sample": "the whole division"}
    bt = gen.batch_products()
    pairs = list(zip(bt.a, bt.b))
    sample = pairs[::16]
    work = float(sum(x.size * y.size for x, y in sample))
    t0 = time.perf_counter()
    for x, y in sample:
        oracle.mul(x, y, bt.p)
    t1 = time.perf_counter() - t0
    work_all = float(sum(x.size * y.size for x, y in pairs))
    t0 = time.perf_counter()
    _pool_map(lambda xy: oracle.mul(xy[0], xy[1], bt.p), pairs, threads)
    tp = time.perf_counter() - t0
    out["batched_4096"] = {"kind": "oracle",
                           "single_thread": {"mulmods_per_s": round(work / t1, 1),
                                             "sample": "every 16th of the 4096 products (%d), %.3g mulmods"
                                                       % (len(sample), work)},
                           "pool": {"threads": threads, "ms": round(tp * 1e3, 1),
                                    "mulmods_per_s": round(work_all / tp, 1), "sample": "all 4096 products"}}
    if reqs:
        one = reqs[:32]
        t0 = time.perf_counter()
        for x, y, q, *_ in one:
            oracle.gcd(x, y, q)
        t1 = time.perf_counter() - t0
        many = reqs[:512]
        t0 = time.perf_counter()
        _pool_map(lambda r: oracle.gcd(r[0], r[1], r[2]), many, threads)
        tp = time.perf_counter() - t0
        out["served"] = {"kind": "oracle",
                         "single_thread": {"gcds_per_s": round(len(one) / t1, 2),
                                           "sample": "the first %d requests of the trace, one after another" % len(one)},
                         "pool": {"threads": threads, "gcds_per_s": round(len(many) / tp, 2),
                                  "sample": "the first %d requests of the trace on the pool" % len(many)}}
    return out


def cpu_baseline(a, b, p: int, seconds: float) -> dict:
    """The oracle (plain C, one thread) on sampled output coefficients of the
    same product; each f_k is computed in full by the schoolbook definition."""
    import oracle
    from paper_1402_0264_amd import gen
    oracle.lib()
    na, nb = a.size, b.size
    st = gen.Stream(gen.SEED_BASE + 77)
    n = terms = 0
    t0 = time.perf_counter()
    while True:
        k = st.uniform_int(0, na + nb - 2)
        oracle.mul_coeff(a, b, p, k)
        terms += min(k, na - 1) - max(0, k - nb + 1) + 1
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    rec = {"value": terms / el, "unit": "mulmods/s", "cores": 1, "kind": "oracle",
           "sample": "%d output coefficients f_k of the degree-65535 product, k uniform, "
                     "%d coefficient products in %.1f s" % (n, terms, el)}
    rec.update(cpu_info())
    return rec


def bench_batched(reps: int) -> dict:
    import torch
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import gen, tune
    bt = gen.batch_products()
    p = bt.p
    items = [(pm.to_device(a), pm.to_device(b), p) for a, b in zip(bt.a, bt.b)]
    work = float(sum(a.size * b.size for a, b in zip(bt.a, bt.b)))
    t = tune.tune_mul_batch(items)
    batch = pm.MulBatch(items, t["r"], t["kc"])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.run()
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_batch = e0.elapsed_time(e1) / reps
    # the same products as one call each (the library's own per-call plan)
    outs = [torch.empty(a.numel() + b.numel() - 1, dtype=torch.int32, device="cuda") for a, b, _ in items]
    d_nf = torch.zeros(len(items), dtype=torch.int64, device="cuda")
    d_st = torch.zeros(len(items), dtype=torch.int32, device="cuda")

    def one_by_one():
        for i, (a, b, _) in enumerate(items):
            pm.mul_async(a, b, p, outs[i], d_nf[i:i + 1], d_st[i:i + 1])

    one_by_one()
    torch.cuda.synchronize()
    e0.record()
    one_by_one()
    e1.record()
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1)
    same = all(torch.equal(o, f) for o, f in zip(outs[::97], batch.outputs[::97]))
    batch.close()
    return {"workload": "4096 products, degrees log-uniform in [32, 8192], p=469762049",
            "mulmods": work, "ms": round(ms_batch, 4), "mulmods_per_s": round(work / (ms_batch * 1e-3), 1),
            "tuned": {"r": t["r"], "kc": t["kc"], "from_cache": t["cached"]},
            "one_call_per_instance_ms": round(ms_single, 4),
            "speedup_vs_one_call_per_instance": round(ms_single / ms_batch, 2),
            "graph_replays": reps, "matches_one_call_results": bool(same)}


def _pct(xs, q):
    xs = sorted(xs)
    return xs[max(0, min(len(xs) - 1, int(round(q * len(xs) + 0.5)) - 1))]


_SERVED = {}


def served_inputs(count: int):
    """The served trace's requests as host arrays; a = g*u and b = g*v are
    formed with the library's batched product (built once per count)."""
    if count in _SERVED:
        return _SERVED[count]
    _SERVED[count] = _served_inputs(count)
    return _SERVED[count]


def _served_inputs(count: int):
    import torch
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import gen
    trace = gen.served_trace(count, rate=1.0)
    items = []
    for r in trace:
        g = pm.to_device(r.factors.g)
        items.append((g, pm.to_device(r.factors.u), r.p))
        items.append((g, pm.to_device(r.factors.v), r.p))
    out = []
    for lo in range(0, len(items), 1024):
        b = pm.MulBatch(items[lo:lo + 1024])
        b.run()
        torch.cuda.synchronize()
        out += [pm.to_numpy(f) for f in b.outputs]
        b.close()
    reqs = [(out[2 * i], out[2 * i + 1], r.p, r.arrival, r.D, r.k) for i, r in enumerate(trace)]
    return reqs


def bench_batched_gcd(reqs, one_call_sample: int = 256, reps: int = 3, served=None) -> dict:
    """The served trace's requests as one prepared batch (pm_gcd_batch_*):
    s picked by the autotuner, the run captured in a CUDA graph and
    replayed; beside it, the first requests of the same list as one
    synchronous poly_gcd_modp call each."""
    import numpy as np
    import torch
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import tune
    items = [(pm.to_device(a), pm.to_device(b), p) for a, b, p, *_ in reqs]
    t = tune.tune_gcd_batch(items)
    batch = pm.GcdBatch(items, t["s"])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch.run(stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.run()
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    res = batch.results()
    ok = all(r["status"] == 0 for _, r in res)
    # the same requests one call each (the single-instance cooperative path),
    # on a sample; the sampled gcds must equal the batch's
    k = min(one_call_sample, len(items))
    t_one = same = None
    if k > 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        singles = [pm.gcd(a, b, p) for a, b, p in items[:k]]
        torch.cuda.synchronize()
        t_one = (time.perf_counter() - t0) / k
        same = all(torch.equal(g1, res[i][0]) for i, g1 in enumerate(singles))
    # every gcd the server returned for the same requests equals the batch's
    served_same = None
    if served is not None:
        served_same = len(served) == len(res) and all(
            np.array_equal(served[i], pm.to_numpy(g)) for i, (g, _) in enumerate(res))
    batch.close()
    updates = sum(r["updates"] for _, r in res)
    return {"workload": "the served trace's %d requests (D log-uniform in [64, 16384], three primes) "
                        "in one prepared batch replayed from a CUDA graph" % len(items),
            "s": t["s"], "tune_trials": t["trials"], "model_s_star": t["model_s_star"], "ms": round(ms, 3),
            "gcds_per_s": round(len(items) / (ms * 1e-3), 1), "updates_per_s": round(updates / (ms * 1e-3), 1),
            "one_call_per_instance_gcds_per_s": round(1.0 / t_one, 1) if t_one else None, "one_call_sample": k,
            "speedup_vs_one_call_per_instance": round((len(items) / (ms * 1e-3)) * t_one, 1) if t_one else None,
            "all_ok": ok, "sample_equals_one_call": same, "served_results_equal_batch": served_same}


def _round_or_none(x, nd: int = 1):
    return None if x is None else round(x, nd)


def run_server_trace(reqs, scale: float, keep: bool = False, stats=None, **opts):
    """Submit each request at arrival * scale seconds (the requests that have
    arrived by each pass of the loop go in one submit_many call); returns
    latencies (ms, in completion order, with each one's op), the span from
    the first arrival to the last completion, and with `keep` the
    completions by request index. A request is (a, b, p, arrival, D, k) for
    a gcd, with a seventh element True for a division. `stats` (a dict)
    receives the completion rate over the arrival window: the requests done
    between the first and the last submission over that time, which a short
    trace's n / span understates (its span ends with the drain of the
    largest requests, each one CU's step chain)."""
    import paper_1402_0264_amd as pm
    srv = pm.Server(**opts)
    t0 = time.perf_counter()
    i = done = 0
    lat = []
    first = last = None
    kept = {}
    marks = []
    deadline = time.perf_counter() + 600.0
    while done < len(reqs):
        now = time.perf_counter() - t0
        if time.perf_counter() > deadline:
            raise TimeoutError("served trace did not finish")
        due = []
        while i < len(reqs) and reqs[i][3] * scale <= now:  # every request that has arrived, one call
            r = reqs[i]
            due.append((r[0], r[1], r[2], i, len(r) > 6 and r[6]))
            i += 1
        srv.submit_many(due)
        for c in srv.poll():
            if c["status"] != 0:
                raise RuntimeError("served request %d failed: %d" % (c["tag"], c["status"]))
            lat.append((c["t_done_ms"] - c["t_submit_ms"], c["op"]))
            marks.append((c["t_submit_ms"], c["t_done_ms"]))
            first = c["t_submit_ms"] if first is None else min(first, c["t_submit_ms"])
            last = c["t_done_ms"] if last is None else max(last, c["t_done_ms"])
            if keep:
                kept[c["tag"]] = c
            done += 1
    srv.close()
    if stats is not None:
        s0 = min(m[0] for m in marks)
        s1 = max(m[0] for m in marks)
        n_in = sum(1 for m in marks if m[1] <= s1)
        stats["window_ms"] = s1 - s0
        stats["window_rate"] = n_in / ((s1 - s0) / 1e3) if s1 > s0 else None
    return lat, (last - first) / 1e3, kept


def run_one_call_trace(reqs, scale: float):
    """The same trace, one synchronous poly_gcd_modp call per request in
    arrival order (host copy in, gcd, copy out)."""
    import paper_1402_0264_amd as pm
    t0 = time.perf_counter()
    lat = []
    for a, b, p, arr, _, _ in reqs:
        t_arr = arr * scale
        while time.perf_counter() - t0 < t_arr:
            pass
        g = pm.gcd(pm.to_device(a), pm.to_device(b), p)
        pm.to_numpy(g)
        lat.append((time.perf_counter() - t0 - t_arr) * 1e3)
    span = time.perf_counter() - t0 - reqs[0][3] * scale
    return lat, span


def bench_served(n_req: int, warm: int, load: float, baseline: bool, loads=(0.5, 1.0, 1.2)) -> dict:
    import torch
    reqs = served_inputs(n_req + warm)
    warm_reqs, reqs = reqs[:warm], reqs[warm:]
    t_first = reqs[0][3]
    reqs = [(a, b, p, arr - t_first, D, k) for a, b, p, arr, D, k in reqs]
    run_server_trace(warm_reqs, 0.0)
    lat_sat, span_sat, kept = run_server_trace(reqs, 0.0, keep=True)  # everything arrives at once
    sat = len(reqs) / span_sat
    # the same, with the inputs read by the workers from pinned host memory
    # instead of copied to the device arena
    _, span_host, _ = run_server_trace(reqs, 0.0, staging=2)
    mean_gap = reqs[-1][3] / max(len(reqs) - 1, 1)         # of the rate-1 trace
    rate = load * sat
    scale = 1.0 / (rate * mean_gap)
    st = {}
    lat, span, _ = run_server_trace(reqs, scale, stats=st)
    lat = [x for x, _ in lat]
    out = {"workload": "%d gcd requests, D log-uniform in [64, 16384], deg b = D-1, planted gcd degree "
                       "uniform in [0, D/4], p in {469762049, 998244353, 167772161}" % len(reqs),
           "saturated_gcds_per_s": round(sat, 1),
           "saturated_gcds_per_s_inputs_in_host_memory": round(len(reqs) / span_host, 1),
           "offered_rate_per_s": round(rate, 1), "load": load,
           "gcds_per_s": round(len(reqs) / span, 1),
           "gcds_per_s_in_arrival_window": _round_or_none(st["window_rate"]),
           "arrival_window_ms": round(st["window_ms"], 2),
           "p50_ms": round(_pct(lat, 0.50), 3), "p99_ms": round(_pct(lat, 0.99), 3),
           "max_ms": round(max(lat), 3)}
    sweep = [{"load": load, "gcds_per_s": out["gcds_per_s"],
              "gcds_per_s_in_arrival_window": out["gcds_per_s_in_arrival_window"],
              "p50_ms": out["p50_ms"], "p99_ms": out["p99_ms"]}]
    for ld in loads:
        sc = 1.0 / (ld * sat * mean_gap)
        st2 = {}
        l2, sp2, _ = run_server_trace(reqs, sc, stats=st2)
        l2 = [x for x, _ in l2]
        sweep.append({"load": ld, "gcds_per_s": round(len(reqs) / sp2, 1),
                      "gcds_per_s_in_arrival_window": _round_or_none(st2["window_rate"]),
                      "p50_ms": round(_pct(l2, 0.50), 3), "p99_ms": round(_pct(l2, 0.99), 3)})
    out["loads"] = sorted(sweep, key=lambda x: x["load"])
    if baseline:
        run_one_call_trace(warm_reqs[:16], 0.0)
        lat1, span1 = run_one_call_trace(reqs, scale)
        out["one_call_per_instance"] = {"gcds_per_s": round(len(reqs) / span1, 1),
                                        "p50_ms": round(_pct(lat1, 0.50), 3),
                                        "p99_ms": round(_pct(lat1, 0.99), 3)}
        out["throughput_ratio"] = round(out["gcds_per_s"] / out["one_call_per_instance"]["gcds_per_s"], 2)
        out["p99_ratio_one_call_over_served"] = round(out["one_call_per_instance"]["p99_ms"] / out["p99_ms"], 2)
    torch.cuda.synchronize()
    out["_results"] = {t: c["g"] for t, c in kept.items()}  # checked against the batch, then dropped
    return out


def bench_served_mixed(n_req: int, warm: int, load: float) -> dict:
    """A Poisson stream of gcd and division requests (a quarter divisions:
    a of degree D, b of degree D/2) through the same server: saturated
    requests/s, then p50/p99 per kind at `load` of that rate. Every
    division is checked against the oracle (on a thread pool), every gcd
    against the prepared batch's result for the same pair."""
    import numpy as np
    import torch
    import oracle
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import gen
    trace = gen.served_mixed_trace(n_req + warm, rate=1.0)
    gi = [i for i, r in enumerate(trace) if isinstance(r, gen.Request)]
    items = []
    for i in gi:
        g = pm.to_device(trace[i].factors.g)
        items += [(g, pm.to_device(trace[i].factors.u), trace[i].p), (g, pm.to_device(trace[i].factors.v), trace[i].p)]
    prods = []
    for lo in range(0, len(items), 1024):
        b = pm.MulBatch(items[lo:lo + 1024])
        b.run()
        torch.cuda.synchronize()
        prods += [pm.to_numpy(f) for f in b.outputs]
        b.close()
    reqs = []
    j = 0
    for r in trace:
        if isinstance(r, gen.Request):
            reqs.append((prods[2 * j], prods[2 * j + 1], r.p, r.arrival, r.D, r.k, False))
            j += 1
        else:
            reqs.append((r.a, r.b, r.p, r.arrival, r.D, 0, True))
    warm_reqs, reqs = reqs[:warm], reqs[warm:]
    t_first = reqs[0][3]
    reqs = [(a, b, p, arr - t_first, D, k, d) for a, b, p, arr, D, k, d in reqs]
    run_server_trace(warm_reqs, 0.0)
    lat_sat, span_sat, kept = run_server_trace(reqs, 0.0, keep=True)
    sat = len(reqs) / span_sat
    mean_gap = reqs[-1][3] / max(len(reqs) - 1, 1)
    st = {}
    lat, span, _ = run_server_trace(reqs, 1.0 / (load * sat * mean_gap), stats=st)
    gl = [x for x, op in lat if op != pm.PM_OP_DIVREM]
    dl = [x for x, op in lat if op == pm.PM_OP_DIVREM]
    # checks: divisions against the oracle, gcds against the prepared batch
    divs = [i for i, r in enumerate(reqs) if r[6]]
    threads = cpu_info()["pool_threads"]
    want = _pool_map(lambda i: oracle.divrem(reqs[i][0], reqs[i][1], reqs[i][2]), divs, threads)
    div_ok = all(np.array_equal(kept[i]["q"], w[0]) and np.array_equal(kept[i]["r"], w[1])
                 for i, w in zip(divs, want))
    gcds = [i for i, r in enumerate(reqs) if not r[6]]
    res = pm.gcd_batch([(pm.to_device(reqs[i][0]), pm.to_device(reqs[i][1]), reqs[i][2]) for i in gcds])
    gcd_ok = all(r["status"] == 0 and np.array_equal(kept[i]["g"], pm.to_numpy(g)) for i, (g, r) in zip(gcds, res))
    return {"workload": "%d requests, a quarter of them divisions (deg a = D, deg b = D/2) and the rest gcds as "
                        "in the served trace, D log-uniform in [64, 16384], three primes" % len(reqs),
            "divisions": len(divs), "gcds": len(gcds),
            "saturated_requests_per_s": round(sat, 1), "load": load,
            "requests_per_s": round(len(reqs) / span, 1),
            "requests_per_s_in_arrival_window": _round_or_none(st["window_rate"]),
            "gcd_p50_ms": round(_pct(gl, 0.50), 3), "gcd_p99_ms": round(_pct(gl, 0.99), 3),
            "divrem_p50_ms": round(_pct(dl, 0.50), 3), "divrem_p99_ms": round(_pct(dl, 0.99), 3),
            "divisions_equal_oracle": bool(div_ok), "gcds_equal_batch": bool(gcd_ok)}


def bench_product_2048(reps: int) -> dict:
    """The degree-2047 product: host wall time of one synchronous call
    (launch-latency bound), and the steady rate of 100 asynchronous calls
    captured in one graph and replayed."""
    import torch
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import gen
    a_np, b_np = gen.product_2048()
    p = gen.P_A
    a, b = pm.to_device(a_np), pm.to_device(b_np)
    work = float(a_np.size) * float(b_np.size)
    pm.mul(a, b, p)
    torch.cuda.synchronize()
    lat = []
    for _ in range(reps):
        t0 = time.perf_counter()
        pm.mul(a, b, p)
        lat.append((time.perf_counter() - t0) * 1e3)
    stream = torch.cuda.Stream()
    f = torch.empty(a_np.size + b_np.size - 1, dtype=torch.int32, device="cuda")
    d_nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    d_st = torch.zeros(1, dtype=torch.int32, device="cuda")
    calls = 100
    with torch.cuda.stream(stream):
        for _ in range(3):          # scratch and plan exist before the capture
            pm.mul_async(a, b, p, f, d_nf, d_st)
    stream.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        for _ in range(calls):
            pm.mul_async(a, b, p, f, d_nf, d_st)
    graph.replay()
    torch.cuda.synchronize()
    ok = int(d_st.item()) == 0 and int(d_nf.item()) == a_np.size + b_np.size - 1
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    per = e0.elapsed_time(e1) / (10 * calls)
    return {"workload": "product_2048: deg 2047 x deg 2047 over p=469762049",
            "single_call_ms_median": round(sorted(lat)[len(lat) // 2], 4), "single_call_ms_min": round(min(lat), 4),
            "graph_ms_per_product": round(per, 5), "graph_mulmods_per_s": round(work / (per * 1e-3), 1),
            "graph_calls": calls, "device_checks_ok": ok}


def bench_gcd(reps: int) -> dict:
    import numpy as np
    import torch
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import gen
    pl = gen.gcd_32768()
    p = pl.p
    g = pm.to_device(pl.g)
    a = pm.mul(g, pm.to_device(pl.u), p)   # inputs formed on the GPU
    b = pm.mul(g, pm.to_device(pl.v), p)
    pm.divrem(a, b, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        q, r = pm.divrem(a, b, p)
    t_div = (time.perf_counter() - t0) / reps
    pm.gcd(a, b, p)
    best = None
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = pm.gcd(a, b, p)
        times.append(time.perf_counter() - t0)
    st = pm.last_gcd_stats()
    t_gcd = sorted(times)[len(times) // 2]
    ok = bool(np.array_equal(pm.to_numpy(out), pl.g))
    # the extended gcd (Bezout cofactors) on the same pair
    gx, sx, tx = pm.xgcd(a, b, p)
    xtimes = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gx, sx, tx = pm.xgcd(a, b, p)
        xtimes.append(time.perf_counter() - t0)
    t_xgcd = sorted(xtimes)[len(xtimes) // 2]
    ok_x = bool(np.array_equal(pm.to_numpy(gx), pl.g))
    return {"workload": "deg a 32768, deg b 32767, planted monic gcd of degree 1000, p=469762049",
            "divrem_ms": round(t_div * 1e3, 4), "quotient_terms": int(q.numel()),
            "gcd_ms_median": round(t_gcd * 1e3, 4), "gcd_ms_min": round(min(times) * 1e3, 4),
            "gcds_per_s": round(1.0 / t_gcd, 2), "division_steps": st["steps"], "updates": st["updates"],
            "updates_per_s": round(st["updates"] / t_gcd, 1), "chunks": st["chunks"],
            "ns_per_division_step": round(t_gcd * 1e9 / max(st["steps"], 1), 1),
            "grid_syncs": st["chunks"],
            "updates_frac_of_valu_peak": round(st["updates"] / t_gcd / PEAK_MULMOD_PER_S, 5),
            "gcd_equals_planted": ok,
            "xgcd_ms_median": round(t_xgcd * 1e3, 4), "xgcd_cofactor_terms": [int(sx.numel()), int(tx.numel())],
            "xgcd_gcd_equals_planted": ok_x}


def bench_divrem(reps: int) -> dict:
    """Euclidean division with a long quotient: a of degree 65535 by b of
    degree 32767 (32769 quotient terms), at the default s; median of reps
    synchronous calls (both host reads of the call included)."""
    import torch
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import gen
    st = gen.Stream(gen.SEED_BASE + 6)
    a_np, b_np = st.uniform_poly(65535, gen.P_A), st.uniform_poly(32767, gen.P_A)
    a, b = pm.to_device(a_np), pm.to_device(b_np)
    pm.divrem(a, b, gen.P_A)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q, r = pm.divrem(a, b, gen.P_A)
        times.append(time.perf_counter() - t0)
    t = sorted(times)[len(times) // 2]
    mu, db = int(q.numel()), b_np.size - 1
    updates = mu * (db + 1)
    return {"workload": "deg a 65535 / deg b 32767 over p=469762049 (the s sweep's division)",
            "s": pm.get_params()["div_s"] or 64, "divrem_ms_median": round(t * 1e3, 4),
            "divrem_ms_min": round(min(times) * 1e3, 4), "quotient_terms": mu, "remainder_terms": int(r.numel()),
            "updates": updates, "updates_per_s": round(updates / t, 1)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    # the shader clock ramps up over the first tens of milliseconds of
    # sustained matrix-core load (per-step time of the degree-65535 product
    # over consecutive 200-step windows from a cold start: 64.4, 61.0, 60.0,
    # 59.8 us); 1000 warm-up steps (about 60 ms) reach the steady rate
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gcd", action="store_true")
    ap.add_argument("--gcd-reps", type=int, default=5)
    ap.add_argument("--no-div", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-batched-gcd", action="store_true", help="skip the prepared gcd batch")
    ap.add_argument("--one-call-sample", type=int, default=256,
                    help="gcd batch: requests also run as one poly_gcd_modp call each (0: none)")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=2048)
    ap.add_argument("--no-served-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--mul-r", type=int, default=0, help="force the product's outputs per thread (skips tuning)")
    ap.add_argument("--mul-s", type=int, default=0, help="force the product's b-chunk s (skips tuning)")
    ap.add_argument("--engine", choices=("auto", "mfma", "valu"), default="auto",
                    help="product engine (auto: the autotuner's pick)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import gen

    torch.cuda.set_device(0)
    pm.lib()
    a_np, b_np = gen.product_65536()
    p = gen.P_A
    a, b = pm.to_device(a_np), pm.to_device(b_np)
    nf = a_np.size + b_np.size - 1
    f = torch.empty(nf, dtype=torch.int32, device="cuda")
    d_nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    d_st = torch.zeros(1, dtype=torch.int32, device="cuda")

    tuned = None
    if args.engine == "valu" or args.mul_r or args.mul_s:
        pm.set_params(mul_r=args.mul_r, mul_s=args.mul_s, mul_engine=pm.MUL_VALU)
    elif args.engine == "mfma":
        pm.set_params(mul_engine=pm.MUL_MFMA)
    elif not args.no_tune:
        from paper_1402_0264_amd import tune
        tuned = tune.tune_mul(a, b, p)
        pm.set_params(**tune.params_of(tuned))
    mfma = pm.get_params()["mul_engine"] == pm.MUL_MFMA or (
        pm.get_params()["mul_engine"] == pm.MUL_AUTO and not (pm.get_params()["mul_r"] or pm.get_params()["mul_s"]))
    kernel = "mulx_kernel" if mfma else "mul_tile_kernel"
    reduce_kernel = "mulx_reduce_kernel" if mfma else "mul_reduce_kernel"

    def step():
        pm.mul_async(a, b, p, f, d_nf, d_st)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    pm.timing_reset()
    pm.timing_enable(True)
    ms = time_steps(step, args.steps, 0)
    pm.timing_enable(False)
    n_tile, ms_tile = pm.timing_read(kernel)
    n_red, ms_red = pm.timing_read(reduce_kernel)
    assert n_tile == args.steps, "the product did not run %s once per step" % kernel
    pm.timing_reset()
    assert int(d_st.item()) == 0 and int(d_nf.item()) == nf, "product failed its device checks"
    work = float(a_np.size) * float(b_np.size)
    ms_per_step = ms / args.steps
    value = work / (ms_per_step * 1e-3)
    tile_avg_ms = ms_tile / max(n_tile, 1)
    achieved = work / (tile_avg_ms * 1e-3)
    if mfma:
        # the method's work: one multiply-add (2 operations) per coefficient
        # product, against the dense int8 matrix-core peak; the matrix cores
        # spend 16 int8 digit products on each, reported apart as their use
        ops = 2.0 * work
        roof = {"bound": "mfma", "achieved": round(ops / (tile_avg_ms * 1e-3) / 1e12, 2),
                "peak": round(PEAK_INT8_OPS_PER_S / 1e12, 1), "unit": "TOP/s",
                "frac": round(ops / (tile_avg_ms * 1e-3) / PEAK_INT8_OPS_PER_S, 4),
                "mfma_digit_utilisation": round(2.0 * DIGIT_PRODUCTS * work / (tile_avg_ms * 1e-3)
                                                / PEAK_INT8_OPS_PER_S, 4),
                # the kernel's coefficient products per second over the VALU's
                # (one 32x32->64 multiply-add per lane per clock): above 1, the
                # matrix cores beat any VALU mulmod kernel
                "kernel_over_valu_mulmod_peak": round(achieved / PEAK_MULMOD_PER_S, 3)}
    else:
        roof = {"bound": "alu", "achieved": round(achieved / 1e12, 3),
                "peak": round(PEAK_MULMOD_PER_S / 1e12, 3), "unit": "Tmulmod/s",
                "frac": round(achieved / PEAK_MULMOD_PER_S, 4)}
    traffic = traffic_for(kernel)
    roof.update({"traffic": traffic, "kernel": kernel, "kernel_avg_ms": round(tile_avg_ms, 5),
                 "kernel_Tmulmod_per_s": round(achieved / 1e12, 2), "launches": n_tile,
                 "algorithmic_bytes": ALGO_BYTES_65536,
                 "traffic_over_algorithmic": round(traffic / ALGO_BYTES_65536, 2) if traffic else None})
    if n_red:  # the VALU engine's addition phase carries timing events; the matrix cores' does not
        roof["reduce_avg_ms"] = round(ms_red / n_red, 5)
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "mulmods/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded uniform residues)",
        "config": {"workload": "product_65536: deg 65535 x deg 65535 over p=469762049",
                   "engine": "matrix cores (int8 digits)" if mfma else "VALU tiles",
                   "params": pm.get_params(), "tuned": tuned and tune_summary(tuned),
                   "parallelism": "single GPU"},
        "roofline": roof,
    }
    pm.set_params()
    out["product_2048"] = bench_product_2048(20)
    if not args.no_batched:
        out["batched_4096"] = bench_batched(10)
    if not args.no_div:
        out["divrem_65536"] = bench_divrem(5)
    if not args.no_gcd:
        out["gcd_32768"] = bench_gcd(args.gcd_reps)
    if not args.no_served:
        out["served"] = bench_served(args.served_requests, 128, 0.8, not args.no_served_baseline)
    if not args.no_served:
        out["served_mixed"] = bench_served_mixed(args.served_requests, 128, 0.8)
    if not args.no_batched and not args.no_batched_gcd:
        # the served measurement's requests (after its warm-up ones), so the
        # server's results can be compared one by one
        out["batched_gcd"] = bench_batched_gcd(served_inputs(args.served_requests + 128)[128:],
                                               one_call_sample=args.one_call_sample,
                                               served=out.get("served", {}).pop("_results", None))
    if "served" in out:
        out["served"].pop("_results", None)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a_np, b_np, p, args.cpu_seconds)
        reqs = None if args.no_served else served_inputs(args.served_requests + 128)[128:]
        out["cpu_baselines"] = cpu_baselines(reqs, out["cpu_baseline"]["pool_threads"])
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
