"""Sweeps of the program parameter s beside the model's estimate: the plain
product (Sec. 5), Euclidean division with a large quotient (Sec. 3) and the
Euclidean gcd (Sec. 6), where s = 1 is the paper's naive kernel.

    python -m paper_1402_0264_amd.sweep [--op mul] [--n 65536] [--s 1,2,4,...,512] [--reps 5]
    python -m paper_1402_0264_amd.sweep --op div [--n 65536] [--s 1,2,...,64]
    python -m paper_1402_0264_amd.sweep --op gcd [--s 1,2,...,256]
    python -m paper_1402_0264_amd.sweep --op table2
    python -m paper_1402_0264_amd.sweep --op sort [--s 1,2,...,10]

Division: a of n terms and b of n/2 terms (quotient of n/2 + 1 terms, the
paper's n = 2m case); s is the number of division steps fused per pass over
the heads. The model's T(s) (Corollary 1 with the printed N, L, C of the
optimized division) decreases with s, so its prediction is "as large as
fits"; the paper's printed R = T_1/T_s at s = Z/7 is reported beside it.

Gcd: the degree 32768 / 32767 pair with a planted degree-1000 gcd; s caps
the division steps fused per chunk (one grid barrier each). The model's
T(s) is minimised at s* = sqrt(8U(2n+m)/3) (our derivation from the printed
N, L, C); the paper measured 4.24x from s = 1 to s = 512 at 10000 x 9000
(Table 2).

s keeps the paper's meaning: the number of coefficients of b that one
thread-block multiplies (so b is cut into m/s chunks and the partial sums
of each chunk form one row of the array M, n + s - 1 words long, which the
addition phase then adds). Each thread computes min(s, 16) consecutive
entries of its row (the paper's s entries per thread, capped at 16 so the
sums stay in registers). For each s the script prints one JSON line: the
measured time (median of reps, HIP events around the whole product), the
multiplication- and addition-phase kernel times, the bytes of M written
and read, and the model's Corollary-1 estimate T(s) normalised to s = 1.
A last row times the matrix-core engine (its s is fixed at 4096) on the
same inputs, and a final line names the measured optimum of the VALU engine,
the model's (s = 1: its estimate grows with s), the paper's own
measurement (s = 4) and the matrix-core time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# threads per block of the naive kernels (the paper's l)
ELL = 256


def _median_ms(fn, reps: int) -> float:
    import time
    import torch
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    times.sort()
    return times[len(times) // 2]


def sweep_div(args) -> int:
    import torch
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import gen, mmm
    torch.cuda.set_device(0)
    n, m = args.n, args.n // 2
    st = gen.Stream(gen.SEED_BASE + 6)
    a_np, b_np = st.uniform_poly(n - 1, gen.P_A), st.uniform_poly(m - 1, gen.P_A)
    a, b = pm.to_device(a_np), pm.to_device(b_np)
    svals = [int(x) for x in (args.s or "1,2,4,8,16,32,64").split(",")]
    ref = None
    rows = []
    t1 = mmm.div_time(n, m, 1, mmm.U_THROUGHPUT)
    tn = mmm.div_time_naive(n, m, mmm.U_THROUGHPUT, ELL)
    for s in svals:
        pm.set_params(div_s=s)
        q, r = pm.divrem(a, b, gen.P_A)
        torch.cuda.synchronize()
        if ref is None:
            ref = (q.clone(), r.clone())
        same = bool(torch.equal(q, ref[0]) and torch.equal(r, ref[1]))
        ms = _median_ms(lambda: pm.divrem(a, b, gen.P_A), args.reps)
        rec = {"op": "divrem", "kernel": "fused", "s": s, "ms": round(ms, 4), "quotient_terms": int(q.numel()),
               "model_T_over_T1": round(mmm.div_time(n, m, s, mmm.U_THROUGHPUT) / t1, 4),
               "model_T_over_Tnaive": round(mmm.div_time(n, m, s, mmm.U_THROUGHPUT) / tn, 4),
               "identical_to_first": same}
        rows.append(rec)
        print(json.dumps(rec), flush=True)
    pm.set_params()
    if args.no_naive:
        return 0
    # the naive algorithm (one division step per launch), the s0 end
    q, r = pm.divrem(a, b, gen.P_A, naive=True)
    torch.cuda.synchronize()
    same = bool(torch.equal(q, ref[0]) and torch.equal(r, ref[1]))
    ms_n = _median_ms(lambda: pm.divrem(a, b, gen.P_A, naive=True), max(1, args.reps // 2))
    print(json.dumps({"op": "divrem", "kernel": "naive", "s": 1, "ms": round(ms_n, 4), "launches": n - m + 1,
                      "us_per_step": round(ms_n * 1e3 / (n - m + 1), 3), "model_T_over_Tnaive": 1.0,
                      "identical_to_first": same}), flush=True)
    best = min(rows, key=lambda x: x["ms"])
    print(json.dumps({"summary": True, "op": "divrem", "n": n, "m": m, "measured_best_s": best["s"],
                      "measured_T1_over_Tbest": round(rows[0]["ms"] / best["ms"], 3),
                      "measured_Tnaive_over_Tbest": round(ms_n / best["ms"], 3),
                      "model_best_s": min(rows, key=lambda x: x["model_T_over_T1"])["s"],
                      "model_Tnaive_over_T_at_measured_best": round(1.0 / best["model_T_over_Tnaive"], 3),
                      "paper_R_printed_at_Z": round(mmm.div_ratio_printed(mmm.Z_MI355X, mmm.U_THROUGHPUT), 3),
                      "all_identical": all(x["identical_to_first"] for x in rows) and same}), flush=True)
    return 0


def sweep_gcd(args) -> int:
    import numpy as np
    import torch
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import gen, mmm
    torch.cuda.set_device(0)
    pl = gen.gcd_32768()
    p = pl.p
    g = pm.to_device(pl.g)
    a = pm.mul(g, pm.to_device(pl.u), p)
    b = pm.mul(g, pm.to_device(pl.v), p)
    n, m = a.numel() - 1, b.numel() - 1
    svals = [int(x) for x in (args.s or "1,2,4,8,16,32,64,128,256").split(",")]
    rows = []
    t1 = mmm.gcd_time(n, m, 1, mmm.U_THROUGHPUT)
    tn = mmm.gcd_time_naive(n, m, mmm.U_THROUGHPUT, ELL)
    for s in svals:
        pm.set_params(gcd_s=s)
        out = pm.gcd(a, b, p)
        torch.cuda.synchronize()
        ok = bool(np.array_equal(pm.to_numpy(out), pl.g))
        ms = _median_ms(lambda: pm.gcd(a, b, p), args.reps)
        stt = pm.last_gcd_stats()
        rec = {"op": "gcd", "kernel": "fused", "s": s, "ms": round(ms, 3), "chunks": stt["chunks"],
               "steps": stt["steps"], "ns_per_step": round(ms * 1e6 / max(stt["steps"], 1), 1),
               "model_T_over_T1": round(mmm.gcd_time(n, m, s, mmm.U_THROUGHPUT) / t1, 4),
               "model_T_over_Tnaive": round(mmm.gcd_time(n, m, s, mmm.U_THROUGHPUT) / tn, 4),
               "gcd_equals_planted": ok}
        rows.append(rec)
        print(json.dumps(rec), flush=True)
    pm.set_params()
    if args.no_naive:
        return 0
    # the naive algorithm (one division step per launch), the s0 end
    out = pm.gcd(a, b, p, naive=True)
    torch.cuda.synchronize()
    ok_n = bool(np.array_equal(pm.to_numpy(out), pl.g))
    ms_n = _median_ms(lambda: pm.gcd(a, b, p, naive=True), max(1, args.reps // 2))
    stt = pm.last_gcd_stats()
    print(json.dumps({"op": "gcd", "kernel": "naive", "s": 1, "ms": round(ms_n, 3), "steps": stt["steps"],
                      "ns_per_step": round(ms_n * 1e6 / max(stt["steps"], 1), 1), "model_T_over_Tnaive": 1.0,
                      "gcd_equals_planted": ok_n}), flush=True)
    best = min(rows, key=lambda x: x["ms"])
    print(json.dumps({"summary": True, "op": "gcd", "n": n, "m": m, "measured_best_s": best["s"],
                      "measured_T1_over_Tbest": round(rows[0]["ms"] / best["ms"], 3),
                      "measured_Tnaive_over_Tbest": round(ms_n / best["ms"], 3),
                      "model_s_star": round(mmm.gcd_s_star(n, m, mmm.U_THROUGHPUT), 1),
                      "model_T1_over_T_at_best": round(1.0 / min(x["model_T_over_T1"] for x in rows), 3),
                      "model_Tnaive_over_T_at_measured_best": round(1.0 / best["model_T_over_Tnaive"], 3),
                      "paper_R_printed": round(mmm.gcd_ratio_printed(n, mmm.Z_MI355X, mmm.U_THROUGHPUT), 3),
                      "paper_table2_s1_over_s512": 4.24,
                      "all_correct": all(x["gcd_equals_planted"] for x in rows) and ok_n}), flush=True)
    return 0


# The (n, m) pairs of Table 2 (term counts; deg a = n - 1, deg b = m - 1) and
# the times the paper printed there, in seconds, for s = 1 and s = 512 on its
# own GPU: context for the shape of the ratio, not a target.
TABLE2 = ((2000, 1500, 0.058, 0.024), (3000, 2500, 0.108, 0.039), (4000, 3500, 0.158, 0.053),
          (5000, 4500, 0.203, 0.069), (6000, 5000, 0.235, 0.056), (7000, 6000, 0.282, 0.066),
          (8000, 7000, 0.324, 0.076), (9000, 8000, 0.367, 0.087), (10000, 9000, 0.411, 0.097))


def table2(args) -> int:
    """The shape of Table 2 on this GPU: for each (n, m) pair, a uniform
    random a of n terms and b of m terms over p_A (coprime with high
    probability, so the remainder sequence runs to the end), timed with the
    naive gcd (one step per launch) and the fused gcd at its default s."""
    import torch
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import gen, mmm
    torch.cuda.set_device(0)
    p = gen.P_A
    pm.set_params()
    gs = pm.get_params()["gcd_s"] or 128
    ratios = []
    for k, (n, m, t1_paper, t512_paper) in enumerate(TABLE2):
        st = gen.Stream(gen.SEED_BASE + 40 + k)
        a = pm.to_device(st.uniform_poly(n - 1, p))
        b = pm.to_device(st.uniform_poly(m - 1, p))
        g_f = pm.gcd(a, b, p)
        torch.cuda.synchronize()
        ms_f = _median_ms(lambda: pm.gcd(a, b, p), args.reps)
        steps_f = pm.last_gcd_stats()["steps"]
        g_n = pm.gcd(a, b, p, naive=True)
        torch.cuda.synchronize()
        ms_n = _median_ms(lambda: pm.gcd(a, b, p, naive=True), args.reps)
        steps_n = pm.last_gcd_stats()["steps"]
        same = bool(torch.equal(g_f, g_n)) and steps_f == steps_n
        model = mmm.gcd_time_naive(n - 1, m - 1, mmm.U_THROUGHPUT, ELL) / mmm.gcd_time(n - 1, m - 1, gs,
                                                                                         mmm.U_THROUGHPUT)
        rec = {"op": "table2", "n": n, "m": m, "naive_ms": round(ms_n, 3), "fused_ms": round(ms_f, 3),
               "fused_s": gs, "steps": steps_f, "gcd_degree": int(g_f.numel()) - 1,
               "measured_Tnaive_over_Tfused": round(ms_n / ms_f, 2),
               "model_Tnaive_over_Ts": round(model, 2),
               "paper_s1_s": t1_paper, "paper_s512_s": t512_paper,
               "paper_s1_over_s512": round(t1_paper / t512_paper, 2),
               "naive_equals_fused": same}
        ratios.append(rec["measured_Tnaive_over_Tfused"])
        print(json.dumps(rec), flush=True)
    print(json.dumps({"summary": True, "op": "table2", "measured_ratio_min": min(ratios),
                      "measured_ratio_max": max(ratios),
                      "paper_ratio_min": round(min(r[2] / r[3] for r in TABLE2), 2),
                      "paper_ratio_max": round(max(r[2] / r[3] for r in TABLE2), 2),
                      "model_R_limit": round((3 + 5 * mmm.U_THROUGHPUT) * mmm.Z_MI355X
                                             / (3 * (mmm.Z_MI355X + 16 * mmm.U_THROUGHPUT)), 2)}), flush=True)
    return 0


def sweep_sort(args) -> int:
    """The radix sort of Sec. 4 over its digit width s: 2^26 uniform 32-bit
    keys (keys only), s = 1..10, beside the model's T_s/T_1 and the printed
    R = T_1/T_s at l = 256 threads per block."""
    import torch
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import gen, mmm
    torch.cuda.set_device(0)
    n = args.n if args.n != 65536 else 1 << 26
    st = gen.Stream(gen.SEED_BASE + 9)
    keys = pm.to_device(st.raw(n).astype("uint32"))
    ko = torch.empty(n, dtype=torch.int32, device="cuda")
    svals = [int(x) for x in (args.s or "1,2,3,4,5,6,7,8,9,10").split(",")]
    ref = None
    rows = []
    t1 = mmm.sort_time(n, 32, 1, mmm.U_THROUGHPUT)
    for sv in svals:
        pm.radix_sort(keys, s=sv, out=(ko, None))
        torch.cuda.synchronize()
        if ref is None:
            ref = ko.clone()
        same = bool(torch.equal(ko, ref))
        times = []
        for _ in range(args.reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            pm.radix_sort(keys, s=sv, out=(ko, None))
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        times.sort()
        ms = times[len(times) // 2]
        passes = (32 + sv - 1) // sv
        moved = passes * 12.0 * n   # per pass: keys read twice (histogram, scatter), written once
        rec = {"op": "sort", "s": sv, "passes": passes, "ms": round(ms, 4), "keys_per_s": round(n / (ms * 1e-3), 1),
               "GB_per_s_at_12B_per_key_per_pass": round(moved / (ms * 1e-3) / 1e9, 1),
               "model_T_over_T1": round(mmm.sort_time(n, 32, sv, mmm.U_THROUGHPUT) / t1, 4),
               "paper_R_printed": round(mmm.sort_ratio_printed(sv, mmm.U_THROUGHPUT), 3),
               "identical_to_first": same}
        rows.append(rec)
        print(json.dumps(rec), flush=True)
    best = min(rows, key=lambda x: x["ms"])
    model_best = max(range(1, 17), key=lambda sv: mmm.sort_ratio_printed(sv, mmm.U_THROUGHPUT))
    print(json.dumps({"summary": True, "op": "sort", "n": n, "key_bits": 32, "measured_best_s": best["s"],
                      "measured_T1_over_Tbest": round(rows[0]["ms"] / best["ms"], 3) if rows[0]["s"] == 1 else None,
                      "model_best_s_1_to_16": model_best,
                      "model_R_at_measured_best": round(mmm.sort_ratio_printed(best["s"], mmm.U_THROUGHPUT), 3),
                      "threads_per_block": 256, "log2_l": 8,
                      "all_identical": all(x["identical_to_first"] for x in rows)}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--op", choices=("mul", "div", "gcd", "table2", "sort"), default="mul")
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--s", default=None)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--no-naive", action="store_true", help="division and gcd: skip the naive kernels")
    args = ap.parse_args()
    if args.op == "div":
        return sweep_div(args)
    if args.op == "gcd":
        return sweep_gcd(args)
    if args.op == "table2":
        return table2(args)
    if args.op == "sort":
        return sweep_sort(args)
    if args.s is None:
        args.s = "1,2,4,8,16,32,64,128,256,512,1024,2048,4096"
    import torch
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import gen, mmm

    torch.cuda.set_device(0)
    a_np, b_np = gen.mul_pair(args.n, args.n, gen.P_A, seed=gen.SEED_BASE + 3)
    p = gen.P_A
    a, b = pm.to_device(a_np), pm.to_device(b_np)
    nf = 2 * args.n - 1
    f = torch.empty(nf, dtype=torch.int32, device="cuda")
    d_nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    d_st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ref = None
    rows = []
    svals = [int(x) for x in args.s.split(",")]
    t1_model = mmm.mul_time(args.n, args.n, 1, mmm.U_THROUGHPUT)
    for s in svals:
        r = min(s, 16)
        pm.set_params(mul_r=r, mul_s=s, mul_engine=pm.MUL_VALU)
        pm.mul_async(a, b, p, f, d_nf, d_st)
        torch.cuda.synchronize()
        if ref is None:
            ref = f.clone()
        same = bool(torch.equal(f, ref)) and int(d_st.item()) == 0
        times = []
        pm.timing_reset()
        pm.timing_enable(True)
        for _ in range(args.reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            pm.mul_async(a, b, p, f, d_nf, d_st)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        pm.timing_enable(False)
        nt, mt = pm.timing_read("mul_tile_kernel")
        nr, mr = pm.timing_read("mul_reduce_kernel")
        pm.timing_reset()
        times.sort()
        ms = times[len(times) // 2]
        rows_m = (args.n + s - 1) // s if s < args.n else 1
        m_bytes = 0 if rows_m <= 1 else 2 * 4 * rows_m * (args.n + s - 1)
        rec = {"s": s, "r": r, "ms": round(ms, 4), "mulmods_per_s": round(args.n * args.n / (ms * 1e-3), 1),
               "mult_phase_ms": round(mt / max(nt, 1), 4), "add_phase_ms": round(mr / max(nr, 1), 4),
               "M_bytes_written_and_read": m_bytes,
               "model_T_over_T1": round(mmm.mul_time(args.n, args.n, s, mmm.U_THROUGHPUT) / t1_model, 3),
               "identical_to_s1": same}
        rows.append(rec)
        print(json.dumps(rec), flush=True)
    # the matrix-core engine (its s is fixed: 4096 b-coefficients per stage)
    pm.set_params(mul_engine=pm.MUL_MFMA)
    pm.mul_async(a, b, p, f, d_nf, d_st)
    torch.cuda.synchronize()
    same = bool(torch.equal(f, ref)) and int(d_st.item()) == 0
    times = []
    for _ in range(args.reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        pm.mul_async(a, b, p, f, d_nf, d_st)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    ms = times[len(times) // 2]
    mx = {"engine": "mfma", "s": 4096, "ms": round(ms, 4), "mulmods_per_s": round(args.n * args.n / (ms * 1e-3), 1),
          "identical_to_s1": same}
    print(json.dumps(mx), flush=True)
    pm.set_params()
    best = min(rows, key=lambda x: x["ms"])
    print(json.dumps({"summary": True, "n": args.n, "measured_best_s": best["s"], "measured_best_ms": best["ms"],
                      "mfma_engine_ms": mx["ms"],
                      "model_best_s": min(rows, key=lambda x: x["model_T_over_T1"])["s"],
                      "paper_measured_best_s": 4, "U": round(mmm.U_THROUGHPUT, 3), "Z": mmm.Z_MI355X,
                      "all_identical": all(x["identical_to_s1"] for x in rows) and mx["identical_to_s1"]}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
