#!/usr/bin/env python3
"""Benchmark of the plain product over Z/pZ on one MI355X, with the GCD
workloads reported beside it. Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Headline (value, ms_per_step): mulmods/s of the plain product of two dense
polynomials of degree 65535 over p = 469762049 (4,294,967,296 products of
coefficients per step), inputs resident in HBM, one step = one complete
product (all kernels of the call), timed with events on the launch stream
over K steps after W warm-up steps.

Beside it, in the same line:
  roofline      the dominant kernel (mul_tile_kernel): algorithmic
                multiply-adds per launch over its average duration (HIP
                events around each launch on its stream, same timed steps),
                against the VALU multiply-add peak of the chip;
  cpu_baseline  the CPU oracle timed on this host on a bounded sample of the
                same product (single thread);
  batched_4096  4096 independent products (degrees log-uniform in [32, 8192])
                in one persistent launch replayed from a captured graph,
                tile shape from the autotuner, beside the same products as
                4096 separate calls on the same stream;
  gcd_32768     Euclidean division and remainder-sequence gcd of the degree
                32768 / 32767 pair with a planted degree-1000 gcd.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_product_65536.json")


def source_digest() -> str:
    h = hashlib.sha256()
    for f in ("mul.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_1402_0264_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(launch_bytes_alg: float):
    """HBM bytes per launch of mul_tile_kernel from the committed counter
    summary, or None when the kernel source changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest():
        return None
    return rec.get("bytes_per_launch")


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
    return {"value": terms / el, "unit": "mulmods/s", "cores": 1, "kind": "oracle",
            "sample": "%d output coefficients f_k of the degree-65535 product, k uniform, "
                      "%d coefficient products in %.1f s" % (n, terms, el)}


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
    return {"workload": "deg a 32768, deg b 32767, planted monic gcd of degree 1000, p=469762049",
            "divrem_ms": round(t_div * 1e3, 4), "quotient_terms": int(q.numel()),
            "gcd_ms_median": round(t_gcd * 1e3, 4), "gcd_ms_min": round(min(times) * 1e3, 4),
            "gcds_per_s": round(1.0 / t_gcd, 2), "division_steps": st["steps"], "updates": st["updates"],
            "updates_per_s": round(st["updates"] / t_gcd, 1), "chunks": st["chunks"],
            "gcd_equals_planted": ok}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gcd", action="store_true")
    ap.add_argument("--gcd-reps", type=int, default=5)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding paragraph of DESIGN.md); run with --gpus 1", file=sys.stderr)
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
    if not args.no_tune:
        from paper_1402_0264_amd import tune
        tuned = tune.tune_mul(a, b, p)
        pm.set_params(mul_r=tuned["r"], mul_s=tuned["kc"])

    def step():
        pm.mul_async(a, b, p, f, d_nf, d_st)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    pm.timing_reset()
    pm.timing_enable(True)
    ms = time_steps(step, args.steps, 0)
    pm.timing_enable(False)
    n_tile, ms_tile = pm.timing_read("mul_tile_kernel")
    n_red, ms_red = pm.timing_read("mul_reduce_kernel")
    pm.timing_reset()
    assert int(d_st.item()) == 0 and int(d_nf.item()) == nf, "product failed its device checks"
    work = float(a_np.size) * float(b_np.size)
    ms_per_step = ms / args.steps
    value = work / (ms_per_step * 1e-3)
    tile_avg_ms = ms_tile / max(n_tile, 1)
    achieved = work / (tile_avg_ms * 1e-3)
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
                   "params": pm.get_params(), "tuned": tuned and {"r": tuned["r"], "s": tuned["kc"]},
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 3),
                     "peak": round(PEAK_MULMOD_PER_S / 1e12, 3), "unit": "Tmulmod/s",
                     "frac": round(achieved / PEAK_MULMOD_PER_S, 4),
                     "traffic": traffic_for(work),
                     "kernel": "mul_tile_kernel", "kernel_avg_ms": round(tile_avg_ms, 5),
                     "launches": n_tile, "reduce_avg_ms": round(ms_red / max(n_red, 1), 5)},
    }
    pm.set_params()
    if not args.no_batched:
        out["batched_4096"] = bench_batched(10)
    if not args.no_gcd:
        out["gcd_32768"] = bench_gcd(args.gcd_reps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a_np, b_np, p, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
