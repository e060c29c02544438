"""Autotuner for the product kernels: engine and tile shape.

For the batched product the tunable shape is (r, kc): r outputs per thread
(a thread-block owns 256*r outputs) and kc coefficients of b staged per
pass, which is the paper's program parameter s for the product (Sec. 5:
b-coefficients handled per thread-block). For the single large product the
same pair picks the split into b-chunks. Each candidate is timed with HIP
events on the real inputs; the fastest is kept in a JSON cache keyed by a
workload signature and the device name.

The model of the paper predicts the opposite direction for the product (its
estimate grows with s, so s should be as small as possible; mmm.py), while
the paper measured its best s at 4. The tuner's choice is reported beside
both.
"""
from __future__ import annotations

import json
import os

BATCH_CANDIDATES = [(4, 256), (4, 512), (4, 1024), (8, 256), (8, 512), (8, 1024), (8, 2048),
                    (16, 256), (16, 512), (16, 1024), (16, 2048)]
SINGLE_CANDIDATES = [(8, 512), (8, 1024), (8, 2048), (16, 512), (16, 1024), (16, 2048), (16, 4096)]


def cache_path() -> str:
    p = os.environ.get("PM_TUNE_CACHE")
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "polymodp", "tune.json")


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(key: str, rec: dict) -> None:
    d = _load()
    d[key] = rec
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(d, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only costs the cache


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).name or "gpu"


def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def batch_signature(items) -> str:
    """items: list of (a, b, p) with tensor/array a, b."""
    degs = [(len(a) if not hasattr(a, "numel") else a.numel()) for a, _, _ in items]
    degs += [(len(b) if not hasattr(b, "numel") else b.numel()) for _, b, _ in items]
    pbits = sorted({int(p).bit_length() for _, _, p in items})
    work = sum((a.numel() if hasattr(a, "numel") else len(a)) * (b.numel() if hasattr(b, "numel") else len(b))
               for a, b, _ in items)
    return "mul_batch:n%d:deg%d-%d:work%.3g:pbits%s" % (len(items), min(degs), max(degs), work,
                                                         "-".join(map(str, pbits)))


def tune_mul_batch(items, candidates=BATCH_CANDIDATES, reps: int = 3, use_cache: bool = True) -> dict:
    """Pick (r, kc) for a batch of products (list of (a, b, p) device
    tensors). Returns {"r", "kc", "ms", "trials", "cached"}."""
    import paper_1402_0264_amd as pm
    key = batch_signature(items) + ":" + _device_name()
    if use_cache:
        rec = _load().get(key)
        if rec:
            rec = dict(rec)
            rec["cached"] = True
            return rec
    trials = []
    for r, kc in candidates:
        b = pm.MulBatch(items, r, kc)
        ms = _time(b.run, reps)
        b.close()
        trials.append({"r": r, "kc": kc, "ms": round(ms, 5)})
    best = min(trials, key=lambda t: t["ms"])
    rec = {"r": best["r"], "kc": best["kc"], "ms": best["ms"], "trials": trials}
    _store(key, rec)
    rec = dict(rec)
    rec["cached"] = False
    return rec


GCD_S_CANDIDATES = (16, 32, 64, 128, 256)


def tune_gcd_batch(items, candidates=GCD_S_CANDIDATES, reps: int = 2, use_cache: bool = True) -> dict:
    """Pick s (division steps per chunk) for a batch of gcds (list of (a, b,
    p) device tensors), beside the model's s* for the batch's largest
    instance (the minimiser of the printed T_s over real s; its optimised
    gcd needs 6s <= Z words of local memory). Returns {"s", "ms", "trials",
    "model_s_star", "model_s_feasible_max", "cached"}."""
    import paper_1402_0264_amd as pm
    from paper_1402_0264_amd import mmm
    sig = batch_signature(items).replace("mul_batch", "gcd_batch")
    key = sig + ":" + _device_name()
    if use_cache:
        rec = _load().get(key)
        if rec:
            rec = dict(rec)
            rec["cached"] = True
            return rec
    trials = []
    for sv in candidates:
        b = pm.GcdBatch(items, sv)
        ms = _time(b.run, reps)
        b.close()
        trials.append({"s": sv, "ms": round(ms, 4)})
    best = min(trials, key=lambda t: t["ms"])
    n = max(max(a.numel(), b.numel()) for a, b, _ in items) - 1
    rec = {"s": best["s"], "ms": best["ms"], "trials": trials,
           "model_s_star": round(mmm.gcd_s_star(n, n - 1, mmm.U_THROUGHPUT), 1),
           "model_s_feasible_max": mmm.Z_MI355X // 6}
    _store(key, rec)
    rec = dict(rec)
    rec["cached"] = False
    return rec


PARAM_NAMES = ("mul_s", "mul_r", "div_s", "gcd_s", "mul_engine")


def save_params(path: str, params: dict) -> None:
    """Write tuned parameters (pm_params names, e.g. params_of(tune_mul(...)))
    as the text file the library's pm_autotune_load applies."""
    lines = ["# polymodp parameters (pm_autotune_load): name value"]
    for k, v in params.items():
        if k not in PARAM_NAMES:
            raise ValueError("unknown parameter %r" % k)
        lines.append("%s %d" % (k, int(v)))
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    os.replace(tmp, path)


def params_of(rec: dict) -> dict:
    """pm.set_params keywords for a tune_mul result."""
    import paper_1402_0264_amd as pm
    if rec["engine"] == "mfma":
        return {"mul_engine": pm.MUL_MFMA}
    return {"mul_engine": pm.MUL_VALU, "mul_r": rec["r"], "mul_s": rec["kc"]}


def tune_mul(a, b, p: int, candidates=SINGLE_CANDIDATES, reps: int = 3, use_cache: bool = True) -> dict:
    """Pick the engine for one product of device tensors a, b: the matrix
    cores, or the VALU tiles with their best (mul_r, mul_s). Returns
    {"engine": "mfma" | "valu", "r", "kc", "ms", "trials", "cached"}."""
    import torch
    import paper_1402_0264_amd as pm
    key = "mul2:%d:%d:pbits%d:%s" % (a.numel(), b.numel(), int(p).bit_length(), _device_name())
    if use_cache:
        rec = _load().get(key)
        if rec:
            rec = dict(rec)
            rec["cached"] = True
            return rec
    n = a.numel() + b.numel() - 1
    f = torch.empty(n, dtype=torch.int32, device=a.device)
    d_nf = torch.zeros(1, dtype=torch.int64, device=a.device)
    d_st = torch.zeros(1, dtype=torch.int32, device=a.device)
    saved = pm.get_params()
    trials = []
    try:
        pm.set_params(div_s=saved["div_s"], gcd_s=saved["gcd_s"], mul_engine=pm.MUL_MFMA)
        ms = _time(lambda: pm.mul_async(a, b, p, f, d_nf, d_st), reps)
        trials.append({"engine": "mfma", "r": 0, "kc": 0, "ms": round(ms, 5)})
        for r, kc in candidates:
            pm.set_params(mul_r=r, mul_s=kc, div_s=saved["div_s"], gcd_s=saved["gcd_s"], mul_engine=pm.MUL_VALU)
            ms = _time(lambda: pm.mul_async(a, b, p, f, d_nf, d_st), reps)
            trials.append({"engine": "valu", "r": r, "kc": kc, "ms": round(ms, 5)})
    finally:
        pm.set_params(**saved)
    best = min(trials, key=lambda t: t["ms"])
    rec = {"engine": best["engine"], "r": best["r"], "kc": best["kc"], "ms": best["ms"], "trials": trials}
    _store(key, rec)
    rec = dict(rec)
    rec["cached"] = False
    return rec
