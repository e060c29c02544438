"""Calibration runs for the rooflines (not part of the library's interface).

    python3 -m paper_1402_0264_amd.calib            # the HBM byte counters' copy
    python3 -m paper_1402_0264_amd.calib valu       # VALU multiply-add and HBM latency

copy: a plain device-to-device copy of a known size (256 MiB read, 256 MiB
written per copy, 5 copies), so that FETCH_SIZE and WRITE_SIZE as reported
by the profiler can be scaled to bytes (factor = known bytes / counter
bytes per dispatch), e.g.

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_1402_0264_amd.calib

valu: the kernels of calib_src/valu_peak.hip (libpolymodp_calib.so, built by
paper_1402_0264_amd.build): the exact 32x32->64-bit multiply-add rate, the
rate of complete lazy-folded mulmods, and the cycles of one dependent HBM
load (a random cycle through 1 GiB, beyond the 256 MiB last-level cache).
Prints one JSON line.
"""
import ctypes
import json
import os
import sys

BYTES = 256 << 20
PKG = os.path.dirname(os.path.abspath(__file__))
CALIB_LIB = os.path.join(PKG, "libpolymodp_calib.so")


def copy_run() -> int:
    import torch
    torch.cuda.set_device(0)
    src = torch.randint(0, 1 << 30, (BYTES // 4,), dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copied %d bytes x 5" % BYTES, flush=True)
    return 0


def _fold_every(p: int) -> int:
    c32 = (1 << 32) % p
    after = 0xFFFFFFFF * c32 + 0xFFFFFFFF
    return min(((1 << 64) - 1 - after) // ((p - 1) ** 2), 1 << 30)


def valu_run() -> int:
    import time
    import torch
    torch.cuda.set_device(0)
    if not os.path.exists(CALIB_LIB):
        raise ImportError("libpolymodp_calib.so is not built; run `python -m paper_1402_0264_amd.build`")
    L = ctypes.CDLL(CALIB_LIB)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    L.calib_mad.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, vp]
    L.calib_mulmod.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32,
                               ctypes.c_uint64, ctypes.c_int, vp]
    L.calib_chase.argtypes = [vp, i64, vp, vp]
    L.calib_wall_khz.argtypes = [ctypes.POINTER(ctypes.c_int)]
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    stream = torch.cuda.current_stream().cuda_stream
    inp = torch.randint(1, 1 << 30, (1024,), dtype=torch.int32, device="cuda")
    blocks = cus * 16                      # 16 waves per CU: issue-bound, not latency-bound
    out = torch.empty(blocks * 256, dtype=torch.int64, device="cuda")
    iters = 4096
    lanes = blocks * 256

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = float("inf")
        for _ in range(5):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best * 1e-3

    t_mad = timed(lambda: L.calib_mad(inp.data_ptr(), out.data_ptr(), blocks, iters, stream))
    mads = lanes * iters * 8.0
    p = 469762049
    fold = _fold_every(p)
    mu = ((1 << 64) - 1) // p
    t_mm = timed(lambda: L.calib_mulmod(inp.data_ptr(), out.data_ptr(), blocks, iters, p, (1 << 32) % p, mu,
                                        fold, stream))
    # dependent loads over a 1 GiB random cycle (x -> a x + c mod 2^28 is one cycle of all 2^28 indexes)
    n = 1 << 28
    idx = torch.arange(n, dtype=torch.int64, device="cuda")
    nxt = ((idx * 1103515245 + 12345) % n).to(torch.int32)
    del idx
    res = torch.zeros(3, dtype=torch.int64, device="cuda")
    steps = 200000
    L.calib_chase(nxt.data_ptr(), 1000, res.data_ptr(), stream)   # warm the code, not the data
    torch.cuda.synchronize()
    L.calib_chase(nxt.data_ptr(), steps, res.data_ptr(), stream)
    torch.cuda.synchronize()
    cyc, wall, _ = res.tolist()
    khz = ctypes.c_int(0)
    L.calib_wall_khz(ctypes.byref(khz))
    ns = wall / (khz.value * 1e3) * 1e9 / steps if khz.value > 0 else None
    clock_mhz = props.clock_rate / 1e3 if hasattr(props, "clock_rate") else None
    peak_ref = cus * 64 * 2.4e9
    rec = {
        "device": props.name, "cus": cus,
        "mad_u64_u32_per_s": mads / t_mad, "mad_lane_ops_per_cu_per_clock_at_2.4GHz": mads / t_mad / cus / 2.4e9,
        "mad_frac_of_256x64x2.4GHz": mads / t_mad / peak_ref,
        "mulmod_per_s": mads / t_mm, "mulmod_frac_of_256x64x2.4GHz": mads / t_mm / peak_ref,
        "mulmod_fold_every": fold, "p": p,
        "hbm_dependent_load_cycles": cyc / steps, "hbm_dependent_load_ns": ns,
        "chase_buffer_bytes": 4 * n, "chase_steps": steps,
        "shader_clock_mhz_reported": clock_mhz,
        "U_latency_view_cycles_at_2.4GHz": (ns * 2.4) if ns else None,
        "U_throughput_view": 64.0 / (8e12 / 4 / cus / 2.4e9),
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "valu":
        sys.exit(valu_run())
    sys.exit(copy_run())
