"""Sweep of the program parameter s for the plain product (Sec. 5), beside
the model's estimate.

    python -m paper_1402_0264_amd.sweep [--n 65536] [--s 1,2,4,...,512] [--reps 5]

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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--s", default="1,2,4,8,16,32,64,128,256,512,1024,2048,4096")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
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
