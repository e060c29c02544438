"""Dense univariate polynomial arithmetic over Z/pZ on AMD MI355X (gfx950).

Python binding of libpolymodp (C ABI in include/polymodp.h): argument
marshalling only. Every step of the computation runs in the library's HIP
kernels; PyTorch provides device memory and streams. There is no CPU
fallback: if the library is not built, loading it raises.

Polynomials are torch tensors of dtype int32 or uint32 on a ROCm device,
holding uint32 coefficient bit patterns (index = exponent). Results come
back as int32 tensors of the same bit patterns; ``to_numpy`` views them as
numpy uint32.
"""
from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpolymodp.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "polymodp.h")

PM_OK, PM_EINVAL, PM_EMODULUS, PM_ERANGE, PM_EDIVZERO, PM_ENOMEM, PM_EDEVICE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "PM_OK", -1: "PM_EINVAL", -2: "PM_EMODULUS", -3: "PM_ERANGE", -4: "PM_EDIVZERO",
                -5: "PM_ENOMEM", -6: "PM_EDEVICE"}


class PolyModPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("mul_s", ctypes.c_int32), ("mul_r", ctypes.c_int32),
                ("div_s", ctypes.c_int32), ("gcd_s", ctypes.c_int32), ("mul_engine", ctypes.c_int32)]


class GcdItem(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p), ("na", ctypes.c_int64), ("b", ctypes.c_void_p), ("nb", ctypes.c_int64),
                ("p", ctypes.c_uint32), ("g", ctypes.c_void_p), ("g_cap", ctypes.c_int64)]


class GcdResult(ctypes.Structure):
    _fields_ = [("ng", ctypes.c_int64), ("steps", ctypes.c_int64), ("updates", ctypes.c_int64),
                ("chunks", ctypes.c_int64), ("status", ctypes.c_int32), ("done", ctypes.c_int32),
                ("nr", ctypes.c_int64)]


GCD_BATCH_MAX = 17408
NOALLOC_SCRATCH_WORDS = 1 << 24


class MulItem(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p), ("na", ctypes.c_int64), ("b", ctypes.c_void_p), ("nb", ctypes.c_int64),
                ("p", ctypes.c_uint32), ("f", ctypes.c_void_p), ("f_cap", ctypes.c_int64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_int32), ("large_blocks", ctypes.c_int32), ("arena_words", ctypes.c_int64),
                ("s", ctypes.c_int32), ("small_blocks", ctypes.c_int32), ("staging", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class GcdRequest(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p), ("na", ctypes.c_int64), ("b", ctypes.c_void_p), ("nb", ctypes.c_int64),
                ("p", ctypes.c_uint32), ("g", ctypes.c_void_p), ("g_cap", ctypes.c_int64),
                ("tag", ctypes.c_uint64), ("op", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("r", ctypes.c_void_p), ("r_cap", ctypes.c_int64)]


# pm_gcd_request as a numpy record (same field offsets as GcdRequest)

def _req_dtype():
    import numpy as np
    return np.dtype({"names": ["a", "na", "b", "nb", "p", "g", "g_cap", "tag", "op", "r", "r_cap"],
                     "formats": ["<u8", "<i8", "<u8", "<i8", "<u4", "<u8", "<i8", "<u8", "<i4", "<u8", "<i8"],
                     "offsets": [GcdRequest.a.offset, GcdRequest.na.offset, GcdRequest.b.offset,
                                 GcdRequest.nb.offset, GcdRequest.p.offset, GcdRequest.g.offset,
                                 GcdRequest.g_cap.offset, GcdRequest.tag.offset, GcdRequest.op.offset,
                                 GcdRequest.r.offset, GcdRequest.r_cap.offset],
                     "itemsize": ctypes.sizeof(GcdRequest)})


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("op", ctypes.c_int32), ("ng", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("updates", ctypes.c_int64), ("t_submit_ms", ctypes.c_double), ("t_start_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double), ("nr", ctypes.c_int64)]


class MulPlanInfo(ctypes.Structure):
    _fields_ = [("engine", ctypes.c_int32), ("r", ctypes.c_int32), ("s", ctypes.c_int64),
                ("scratch_words", ctypes.c_int64), ("work_groups", ctypes.c_int64),
                ("max_share_groups", ctypes.c_int64)]


PM_OP_MUL, PM_OP_DIVREM, PM_OP_GCD = 0, 1, 2


class GcdStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("updates", ctypes.c_int64), ("chunks", ctypes.c_int64)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)


def lib() -> ctypes.CDLL:
    """Load libpolymodp.so; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libpolymodp.so is not built; run `python -m paper_1402_0264_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.poly_mul_modp.argtypes = [_vp, _i64, _vp, _i64, ctypes.c_uint32, _vp, _i64, _i64p, _vp]
    L.poly_mul_modp.restype = ctypes.c_int32
    L.poly_mul_modp_async.argtypes = [_vp, _i64, _vp, _i64, ctypes.c_uint32, _vp, _i64, _vp, _vp, _vp]
    L.poly_mul_modp_async.restype = ctypes.c_int32
    L.poly_mul_modp_noalloc.argtypes = L.poly_mul_modp_async.argtypes
    L.poly_mul_modp_noalloc.restype = ctypes.c_int32
    L.poly_divrem_modp.argtypes = [_vp, _i64, _vp, _i64, ctypes.c_uint32, _vp, _i64, _i64p, _vp, _i64,
                                   _i64p, _vp]
    L.poly_divrem_modp.restype = ctypes.c_int32
    L.poly_gcd_modp.argtypes = [_vp, _i64, _vp, _i64, ctypes.c_uint32, _vp, _i64, _i64p, _vp]
    L.poly_gcd_modp.restype = ctypes.c_int32
    L.poly_divrem_modp_naive.argtypes = L.poly_divrem_modp.argtypes
    L.poly_divrem_modp_naive.restype = ctypes.c_int32
    L.poly_gcd_modp_naive.argtypes = L.poly_gcd_modp.argtypes
    L.poly_gcd_modp_naive.restype = ctypes.c_int32
    L.poly_xgcd_modp.argtypes = [_vp, ctypes.c_int64, _vp, ctypes.c_int64, ctypes.c_uint32,
                                 _vp, ctypes.c_int64, _i64p, _vp, ctypes.c_int64, _i64p,
                                 _vp, ctypes.c_int64, _i64p, _vp]
    L.poly_xgcd_modp.restype = ctypes.c_int32
    L.poly_gcd_modp_degrees.argtypes = [_vp, _i64, _vp, _i64, ctypes.c_uint32, _vp, _i64, _i64p, _i64p, _i64,
                                        _i64p, _vp]
    L.poly_gcd_modp_degrees.restype = ctypes.c_int32
    L.poly_euclid_steps_modp.argtypes = [_vp, _i64, _vp, _i64, ctypes.c_uint32, _i64, _vp, _i64, _i64p, _vp,
                                         _i64, _i64p, _i64p, _vp]
    L.poly_euclid_steps_modp.restype = ctypes.c_int32
    L.pm_radix_sort_u32.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp]
    L.pm_radix_sort_u32.restype = ctypes.c_int32
    L.poly_gcd_modp_batch.argtypes = [ctypes.POINTER(GcdItem), ctypes.c_int32, ctypes.POINTER(GcdResult), _vp]
    L.pm_gcd_batch_create.argtypes = [ctypes.POINTER(GcdItem), ctypes.c_int32, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_void_p)]
    L.pm_gcd_batch_create.restype = ctypes.c_int32
    L.pm_gcd_batch_run.argtypes = [ctypes.c_void_p, _vp]
    L.pm_gcd_batch_run.restype = ctypes.c_int32
    L.pm_gcd_batch_results.argtypes = [ctypes.c_void_p, ctypes.POINTER(GcdResult), _vp]
    L.pm_gcd_batch_results.restype = ctypes.c_int32
    L.pm_gcd_batch_destroy.argtypes = [ctypes.c_void_p]
    L.pm_gcd_batch_destroy.restype = None
    L.poly_gcd_modp_batch.restype = ctypes.c_int32
    L.pm_mul_batch_create.argtypes = [ctypes.POINTER(MulItem), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_void_p)]
    L.pm_mul_batch_create.restype = ctypes.c_int32
    L.pm_mul_batch_run.argtypes = [ctypes.c_void_p, _vp, _vp]
    L.pm_mul_batch_run.restype = ctypes.c_int32
    L.pm_mul_batch_destroy.argtypes = [ctypes.c_void_p]
    L.pm_mul_batch_destroy.restype = None
    L.poly_mul_modp_batch.argtypes = [ctypes.POINTER(MulItem), ctypes.c_int32, _vp, _vp]
    L.poly_mul_modp_batch.restype = ctypes.c_int32
    L.pm_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(ctypes.c_void_p)]
    L.pm_server_create.restype = ctypes.c_int32
    L.pm_server_submit.argtypes = [ctypes.c_void_p, ctypes.POINTER(GcdRequest), ctypes.POINTER(ctypes.c_uint64)]
    L.pm_server_submit.restype = ctypes.c_int32
    L.pm_server_submit_batch.argtypes = [ctypes.c_void_p, ctypes.POINTER(GcdRequest), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_uint64)]
    L.pm_server_submit_batch.restype = ctypes.c_int32
    L.pm_server_poll.argtypes = [ctypes.c_void_p, ctypes.POINTER(Completion), ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_int32)]
    L.pm_server_poll.restype = ctypes.c_int32
    L.pm_server_pending.argtypes = [ctypes.c_void_p]
    L.pm_server_pending.restype = ctypes.c_int64
    L.pm_server_destroy.argtypes = [ctypes.c_void_p]
    L.pm_server_destroy.restype = None
    L.pm_last_gcd_stats.argtypes = [ctypes.POINTER(GcdStats)]
    L.pm_last_gcd_stats.restype = None
    L.pm_set_params.argtypes = [ctypes.POINTER(Params)]
    L.pm_set_params.restype = ctypes.c_int32
    L.pm_get_params.argtypes = [ctypes.POINTER(Params)]
    L.pm_get_params.restype = None
    L.pm_timing_enable.argtypes = [ctypes.c_int]
    L.pm_timing_enable.restype = None
    L.pm_timing_reset.argtypes = []
    L.pm_timing_reset.restype = None
    L.pm_timing_read.argtypes = [ctypes.c_char_p, _i64p, ctypes.POINTER(ctypes.c_double)]
    L.pm_timing_read.restype = ctypes.c_int32
    L.poly_divrem_modp_async.argtypes = [_vp, _i64, _vp, _i64, ctypes.c_uint32, _vp, _i64, _vp, _vp, _i64, _vp, _vp,
                                         _vp]
    L.poly_divrem_modp_async.restype = ctypes.c_int32
    L.poly_gcd_modp_async.argtypes = [_vp, _i64, _vp, _i64, ctypes.c_uint32, _vp, _i64, _vp, _vp, _vp]
    L.poly_gcd_modp_async.restype = ctypes.c_int32
    L.pm_workspace_size.argtypes = [ctypes.c_int32, _i64, _i64, _i64p]
    L.pm_workspace_size.restype = ctypes.c_int32
    L.pm_set_workspace.argtypes = [_vp, _vp, _i64]
    L.pm_set_workspace.restype = ctypes.c_int32
    L.pm_mul_plan.argtypes = [_i64, _i64, ctypes.POINTER(MulPlanInfo)]
    L.pm_mul_plan.restype = ctypes.c_int32
    L.pm_autotune_load.argtypes = [ctypes.c_char_p]
    L.pm_autotune_load.restype = ctypes.c_int32
    L.pm_release.argtypes = []
    L.pm_release.restype = None
    L.pm_last_error.argtypes = []
    L.pm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def declared_symbols() -> list:
    """Function names declared in include/polymodp.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) - {"if", "sizeof"})


def _check(st: int):
    if st != PM_OK:
        raise PolyModPError(st, lib().pm_last_error().decode(errors="replace"))


def last_error() -> str:
    return lib().pm_last_error().decode(errors="replace")


# ----------------------------------------------------------------- torch glue
def _torch():
    import torch
    return torch


def _dev_ptr(t) -> int:
    return t.data_ptr() if t.numel() else 0


def _as_u32_tensor(x, device=None):
    torch = _torch()
    if isinstance(x, torch.Tensor):
        if x.dtype == torch.uint32:
            x = x.view(torch.int32)
        if x.dtype != torch.int32:
            raise TypeError("coefficient tensors must be int32 or uint32")
        if not x.is_cuda:
            raise ValueError("coefficient tensors must live on the GPU")
        return x.contiguous()
    import numpy as np
    arr = np.ascontiguousarray(np.asarray(x, dtype=np.uint32)).view(np.int32)
    return torch.from_numpy(arr.copy()).to(device or "cuda")


def to_device(x, device=None):
    """numpy/list of uint32 coefficients -> int32 tensor on the GPU."""
    return _as_u32_tensor(x, device)


def to_numpy(t):
    """int32 coefficient tensor -> numpy uint32 array."""
    import numpy as np
    return t.detach().cpu().numpy().view(np.uint32).copy()


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def mul(a, b, p: int, stream=None):
    """Product a*b mod p; returns an int32 tensor of length deg a + deg b + 1."""
    torch = _torch()
    a, b = _as_u32_tensor(a), _as_u32_tensor(b, None)
    na, nb = a.numel(), b.numel()
    n = na + nb - 1 if na and nb else 0
    f = torch.empty(max(n, 1), dtype=torch.int32, device=a.device if na else b.device)
    nf = ctypes.c_int64(0)
    _check(lib().poly_mul_modp(_dev_ptr(a), na, _dev_ptr(b), nb, p, f.data_ptr(), n, ctypes.byref(nf),
                               _stream_handle(stream)))
    return f[:nf.value]


def mul_async(a, b, p: int, f, d_nf, d_status, stream=None):
    """Enqueue f = a*b; d_nf (int64, 1 element) and d_status (int32,
    1 element) are device tensors written by the launch."""
    a, b = _as_u32_tensor(a), _as_u32_tensor(b)
    _check(lib().poly_mul_modp_async(_dev_ptr(a), a.numel(), _dev_ptr(b), b.numel(), p, f.data_ptr(),
                                     f.numel(), d_nf.data_ptr(), d_status.data_ptr(), _stream_handle(stream)))


def mul_noalloc(a, b, p: int, f, d_nf=None, d_status=None, stream=None):
    """Enqueue f = a*b with the library's static scratch
    (poly_mul_modp_noalloc: nothing is allocated); d_nf (int64) and
    d_status (int32), one element each, are optional device tensors."""
    a, b = _as_u32_tensor(a), _as_u32_tensor(b)
    _check(lib().poly_mul_modp_noalloc(_dev_ptr(a), a.numel(), _dev_ptr(b), b.numel(), p, f.data_ptr(),
                                       f.numel(), d_nf.data_ptr() if d_nf is not None else None,
                                       d_status.data_ptr() if d_status is not None else None,
                                       _stream_handle(stream)))


def divrem(a, b, p: int, stream=None, naive: bool = False):
    """(q, r) with a = q*b + r, deg r < deg b. ``naive``: one division step
    per launch (poly_divrem_modp_naive)."""
    torch = _torch()
    a, b = _as_u32_tensor(a), _as_u32_tensor(b)
    na, nb = a.numel(), b.numel()
    qcap = max(na - nb + 1, 0) if nb else 0
    qcap = max(qcap, na)  # the true quotient may be longer when b has high zeros
    rcap = max(nb, na, 1)
    dev = a.device if na else b.device
    q = torch.empty(max(qcap, 1), dtype=torch.int32, device=dev)
    r = torch.empty(rcap, dtype=torch.int32, device=dev)
    nq, nr = ctypes.c_int64(0), ctypes.c_int64(0)
    fn = lib().poly_divrem_modp_naive if naive else lib().poly_divrem_modp
    _check(fn(_dev_ptr(a), na, _dev_ptr(b), nb, p, q.data_ptr(), qcap, ctypes.byref(nq), r.data_ptr(), rcap,
              ctypes.byref(nr), _stream_handle(stream)))
    return q[:nq.value], r[:nr.value]


def divrem_async(a, b, p: int, q, r, d_nq=None, d_nr=None, d_status=None, stream=None):
    """Enqueue the division into the device tensors q (at least
    na - nb + 1 words) and r (at least min(na, nb - 1) words)
    (poly_divrem_modp_async; b must have a non-zero top coefficient).
    d_nq, d_nr (int64) and d_status (int32), one element each, are
    optional device tensors written by the launch."""
    a, b = _as_u32_tensor(a), _as_u32_tensor(b)
    ptr = lambda t: t.data_ptr() if t is not None else None
    _check(lib().poly_divrem_modp_async(_dev_ptr(a), a.numel(), _dev_ptr(b), b.numel(), p, _dev_ptr(q), q.numel(),
                                        ptr(d_nq), _dev_ptr(r), r.numel(), ptr(d_nr), ptr(d_status),
                                        _stream_handle(stream)))


def gcd_async(a, b, p: int, g, d_ng=None, d_status=None, stream=None):
    """Enqueue the monic gcd into the device tensor g (poly_gcd_modp_async);
    d_ng (int64) and d_status (int32) are optional device tensors."""
    a, b = _as_u32_tensor(a), _as_u32_tensor(b)
    ptr = lambda t: t.data_ptr() if t is not None else None
    _check(lib().poly_gcd_modp_async(_dev_ptr(a), a.numel(), _dev_ptr(b), b.numel(), p, _dev_ptr(g), g.numel(),
                                     ptr(d_ng), ptr(d_status), _stream_handle(stream)))


def workspace_size(op: int, na: int, nb: int) -> int:
    """Words of workspace the asynchronous entry point of op (PM_OP_MUL,
    PM_OP_DIVREM, PM_OP_GCD) needs at these sizes (pm_workspace_size)."""
    w = ctypes.c_int64(0)
    _check(lib().pm_workspace_size(op, na, nb, ctypes.byref(w)))
    return w.value


def set_workspace(buf, stream=None):
    """Give the stream a caller-owned workspace (an int32 device tensor,
    256-byte aligned), or return it to the library's pool with None
    (pm_set_workspace)."""
    if buf is None:
        _check(lib().pm_set_workspace(_stream_handle(stream), None, 0))
    else:
        _check(lib().pm_set_workspace(_stream_handle(stream), buf.data_ptr(), buf.numel()))


def mul_plan(na: int, nb: int) -> dict:
    """The product plan for na x nb terms (pm_mul_plan; no device work)."""
    info = MulPlanInfo()
    _check(lib().pm_mul_plan(na, nb, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in MulPlanInfo._fields_}


def autotune_load(path: str) -> None:
    """Apply a parameter file written by tune.save_params (pm_autotune_load)."""
    _check(lib().pm_autotune_load(os.fsencode(path)))


def gcd(a, b, p: int, stream=None, naive: bool = False):
    """Monic gcd(a, b) mod p. ``naive``: one division step per launch
    (poly_gcd_modp_naive)."""
    torch = _torch()
    a, b = _as_u32_tensor(a), _as_u32_tensor(b)
    na, nb = a.numel(), b.numel()
    cap = max(na, nb, 1)
    g = torch.empty(cap, dtype=torch.int32, device=a.device if na else b.device)
    ng = ctypes.c_int64(0)
    fn = lib().poly_gcd_modp_naive if naive else lib().poly_gcd_modp
    _check(fn(_dev_ptr(a), na, _dev_ptr(b), nb, p, g.data_ptr(), cap, ctypes.byref(ng), _stream_handle(stream)))
    return g[:ng.value]


def gcd_degrees(a, b, p: int, stream=None):
    """(g, degs): the monic gcd and the degree sequence of the Euclidean
    remainder sequence (deg r0, deg r1, ..., -1), rebuilt from the kernel's
    step log (poly_gcd_modp_degrees)."""
    import numpy as np
    torch = _torch()
    a, b = _as_u32_tensor(a), _as_u32_tensor(b)
    na, nb = a.numel(), b.numel()
    cap = max(na, nb, 1)
    g = torch.empty(cap, dtype=torch.int32, device=a.device if na else b.device)
    degs = np.zeros(na + nb + 4, dtype=np.int64)
    ng, nd = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().poly_gcd_modp_degrees(_dev_ptr(a), na, _dev_ptr(b), nb, p, g.data_ptr(), cap, ctypes.byref(ng),
                                       degs.ctypes.data_as(_i64p), degs.size, ctypes.byref(nd),
                                       _stream_handle(stream)))
    return g[:ng.value], degs[:nd.value].copy()


def euclid_steps(a, b, p: int, k: int, stream=None):
    """(x, y, taken): the pair after the first k steps of the naive
    Euclidean algorithm (poly_euclid_steps_modp), each made monic."""
    torch = _torch()
    a, b = _as_u32_tensor(a), _as_u32_tensor(b)
    na, nb = a.numel(), b.numel()
    dev = a.device if na else b.device
    x = torch.empty(max(na, 1), dtype=torch.int32, device=dev)
    y = torch.empty(max(nb, 1), dtype=torch.int32, device=dev)
    nx, ny, taken = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().poly_euclid_steps_modp(_dev_ptr(a), na, _dev_ptr(b), nb, p, k, x.data_ptr(), na,
                                        ctypes.byref(nx), y.data_ptr(), nb, ctypes.byref(ny), ctypes.byref(taken),
                                        _stream_handle(stream)))
    return x[:nx.value], y[:ny.value], taken.value


def xgcd(a, b, p: int, stream=None):
    """(g, s, t) with s a + t b = g, g = monic gcd(a, b) mod p, and the
    unique cofactors with deg s < deg b - deg g (s = 0 when deg g = deg b;
    s = 1/lc(a), t = 0 when b = 0)."""
    torch = _torch()
    a, b = _as_u32_tensor(a), _as_u32_tensor(b)
    na, nb = a.numel(), b.numel()
    cap = max(na, nb, 1)
    dev = a.device if na else b.device
    g = torch.empty(cap, dtype=torch.int32, device=dev)
    s = torch.empty(cap, dtype=torch.int32, device=dev)
    t = torch.empty(cap, dtype=torch.int32, device=dev)
    ng, ns, nt = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().poly_xgcd_modp(_dev_ptr(a), na, _dev_ptr(b), nb, p, g.data_ptr(), cap, ctypes.byref(ng),
                                s.data_ptr(), cap, ctypes.byref(ns), t.data_ptr(), cap, ctypes.byref(nt),
                                _stream_handle(stream)))
    return g[:ng.value], s[:ns.value], t[:nt.value]


def radix_sort(keys, values=None, s: int = 0, key_bits: int = 32, stream=None, out=None):
    """Stable LSD radix sort of uint32 keys (int32 tensors holding the bit
    patterns) on their low key_bits bits with s-bit digits (pm_radix_sort_u32);
    returns (keys, values) sorted, values None when not given. ``out``:
    optional (keys_out, values_out) tensors to write into."""
    torch = _torch()
    k = _as_u32_tensor(keys)
    n = k.numel()
    v = _as_u32_tensor(values) if values is not None else None
    if out is not None:
        ko, vo = out
    else:
        ko = torch.empty(n, dtype=torch.int32, device=k.device)
        vo = torch.empty(n, dtype=torch.int32, device=k.device) if v is not None else None
    _check(lib().pm_radix_sort_u32(_dev_ptr(k), _dev_ptr(v) if v is not None else None, n, key_bits, s,
                                   _dev_ptr(ko), _dev_ptr(vo) if vo is not None else None, _stream_handle(stream)))
    return ko, vo


class MulBatch:
    """Prepared batch of products (pm_mul_batch_*). ``items`` is a list of
    (a, b, p) with a, b device tensors; outputs are allocated here and
    returned by ``outputs``. ``run`` enqueues one persistent launch (graph
    capturable)."""

    def __init__(self, items, r: int = 0, kc: int = 0):
        torch = _torch()
        self.keep, self.outputs = [], []
        arr = (MulItem * max(len(items), 1))()
        for i, (a, b, p) in enumerate(items):
            a, b = _as_u32_tensor(a), _as_u32_tensor(b)
            n = a.numel() + b.numel() - 1 if a.numel() and b.numel() else 0
            f = torch.zeros(max(n, 1), dtype=torch.int32, device=a.device if a.numel() else b.device)
            self.keep += [a, b]
            self.outputs.append(f[:n])
            arr[i] = MulItem(_dev_ptr(a), a.numel(), _dev_ptr(b), b.numel(), p, f.data_ptr(), n)
        self.count = len(items)
        self.handle = ctypes.c_void_p()
        _check(lib().pm_mul_batch_create(arr, self.count, r, kc, ctypes.byref(self.handle)))

    def run(self, d_status=None, stream=None):
        _check(lib().pm_mul_batch_run(self.handle, d_status.data_ptr() if d_status is not None else None,
                                      _stream_handle(stream)))

    def close(self):
        if self.handle:
            lib().pm_mul_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GcdBatch:
    """Prepared batch of gcds (pm_gcd_batch_*). ``items`` is a list of
    (a, b, p) with a, b device tensors; outputs are allocated here. ``run``
    enqueues at most two launches and may be captured in a CUDA graph;
    ``results`` returns [(g, result dict)] of the last run."""

    def __init__(self, items, s: int = 0):
        torch = _torch()
        self.keep, self.gs = [], []
        self.count = len(items)
        arr = (GcdItem * max(self.count, 1))()
        for i, (a, b, p) in enumerate(items):
            a, b = _as_u32_tensor(a), _as_u32_tensor(b)
            cap = max(a.numel(), b.numel(), 1)
            g = torch.empty(cap, dtype=torch.int32, device=a.device if a.numel() else b.device)
            self.keep += [a, b]
            self.gs.append(g)
            arr[i] = GcdItem(_dev_ptr(a), a.numel(), _dev_ptr(b), b.numel(), p, g.data_ptr(), cap)
        self.handle = ctypes.c_void_p()
        _check(lib().pm_gcd_batch_create(arr, self.count, s, ctypes.byref(self.handle)))

    def run(self, stream=None):
        _check(lib().pm_gcd_batch_run(self.handle, _stream_handle(stream)))

    def results(self, stream=None):
        res = (GcdResult * max(self.count, 1))()
        _check(lib().pm_gcd_batch_results(self.handle, res, _stream_handle(stream)))
        out = []
        for i in range(self.count):
            r = res[i]
            out.append((self.gs[i][:r.ng], {"status": r.status, "ng": r.ng, "steps": r.steps,
                                            "updates": r.updates, "chunks": r.chunks}))
        return out

    def close(self):
        if self.handle:
            lib().pm_gcd_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mul_batch(items, d_status=None, stream=None):
    """One-shot batched products; returns the list of outputs."""
    b = MulBatch(items, get_params()["mul_r"] if get_params()["mul_r"] in (4, 8, 16) else 0,
                 get_params()["mul_s"])
    b.run(d_status, stream)
    _torch().cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    out = b.outputs
    b.close()
    return out


def gcd_batch(pairs, stream=None):
    """Monic gcds of many (a, b, p) triples in one launch; returns a list of
    (g, result dict). Inputs are device tensors (or arrays moved there)."""
    torch = _torch()
    n = len(pairs)
    items = (GcdItem * max(n, 1))()
    results = (GcdResult * max(n, 1))()
    keep = []
    outs = []
    for i, (a, b, p) in enumerate(pairs):
        a, b = _as_u32_tensor(a), _as_u32_tensor(b)
        cap = max(a.numel(), b.numel(), 1)
        g = torch.empty(cap, dtype=torch.int32, device=a.device if a.numel() else b.device)
        keep += [a, b]
        outs.append(g)
        items[i] = GcdItem(_dev_ptr(a), a.numel(), _dev_ptr(b), b.numel(), p, g.data_ptr(), cap)
    _check(lib().poly_gcd_modp_batch(items, n, results, _stream_handle(stream)))
    ret = []
    for i in range(n):
        r = results[i]
        ret.append((outs[i][:r.ng], {"status": r.status, "ng": r.ng, "steps": r.steps, "updates": r.updates,
                                     "chunks": r.chunks}))
    return ret


class Server:
    """Continuous-batching server of gcd and division requests (pm_server_*).
    Inputs and outputs are host numpy arrays; ``submit`` returns a ticket,
    ``poll`` returns the finished requests as dicts: the monic gcd ``g``, or
    for a division (``divrem=True``) the quotient ``q`` and remainder ``r``."""

    def __init__(self, max_inflight: int = 0, large_blocks: int = 0, arena_words: int = 0, s: int = 0,
                 small_blocks: int = 0, staging: int = 0):
        self.handle = ctypes.c_void_p()
        _check(lib().pm_server_create(ctypes.byref(ServerOpts(max_inflight, large_blocks, arena_words, s,
                                                              small_blocks, staging, 0)),
                                      ctypes.byref(self.handle)))
        self._out = {}
        self._buf = (Completion * 512)()

    def submit(self, a, b, p: int, tag: int = 0, divrem: bool = False) -> int:
        return self.submit_many([(a, b, p, tag, divrem)])[0]

    def submit_many(self, reqs) -> list:
        """Submits [(a, b, p, tag[, divrem]), ...] in one call; returns the
        tickets. The request records are built as one numpy array with the
        layout of pm_gcd_request, and the outputs are views of one buffer
        (g, or q then r: max(na, nb) words each)."""
        import numpy as np
        n = len(reqs)
        if n == 0:
            return []
        ins = []
        for r in reqs:
            a, b = r[0], r[1]
            if not (isinstance(a, np.ndarray) and a.dtype == np.uint32 and a.flags.c_contiguous):
                a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
            if not (isinstance(b, np.ndarray) and b.dtype == np.uint32 and b.flags.c_contiguous):
                b = np.ascontiguousarray(np.asarray(b, dtype=np.uint32))
            ins.append((a, b))
        na = np.fromiter((x[0].size for x in ins), dtype=np.int64, count=n)
        nb = np.fromiter((x[1].size for x in ins), dtype=np.int64, count=n)
        div = np.fromiter((bool(r[4]) if len(r) > 4 else False for r in reqs), dtype=bool, count=n)
        cap = np.maximum(np.maximum(na, nb), 1)
        words = np.where(div, 2 * cap, cap)
        offs = np.zeros(n, dtype=np.int64)
        np.cumsum(words[:-1], out=offs[1:])
        gbuf = np.zeros(int(offs[-1] + words[-1]), dtype=np.uint32)
        rec = np.zeros(n, dtype=_req_dtype())
        rec["a"] = np.fromiter((x[0].ctypes.data if x[0].size else 0 for x in ins), dtype=np.uint64, count=n)
        rec["na"] = na
        rec["b"] = np.fromiter((x[1].ctypes.data if x[1].size else 0 for x in ins), dtype=np.uint64, count=n)
        rec["nb"] = nb
        rec["p"] = np.fromiter((r[2] for r in reqs), dtype=np.uint32, count=n)
        base = np.uint64(gbuf.ctypes.data)
        rec["g"] = base + 4 * offs.astype(np.uint64)
        rec["g_cap"] = cap
        rec["tag"] = np.fromiter((r[3] for r in reqs), dtype=np.uint64, count=n)
        rec["op"] = np.where(div, PM_OP_DIVREM, PM_OP_GCD)
        rec["r"] = np.where(div, base + 4 * (offs + cap).astype(np.uint64), np.uint64(0))
        rec["r_cap"] = np.where(div, cap, 0)
        tickets = np.zeros(n, dtype=np.uint64)
        _check(lib().pm_server_submit_batch(self.handle, ctypes.cast(rec.ctypes.data, ctypes.POINTER(GcdRequest)),
                                            n, ctypes.cast(tickets.ctypes.data, ctypes.POINTER(ctypes.c_uint64))))
        for i in range(n):
            o, c = int(offs[i]), int(cap[i])
            self._out[int(tickets[i])] = (gbuf[o:o + c], gbuf[o + c:o + 2 * c] if div[i] else None)
        return [int(t) for t in tickets]

    def poll(self) -> list:
        n = ctypes.c_int32(0)
        _check(lib().pm_server_poll(self.handle, self._buf, len(self._buf), ctypes.byref(n)))
        done = []
        for i in range(n.value):
            c = self._buf[i]
            g, r = self._out.pop(c.ticket)
            d = {"ticket": c.ticket, "tag": c.tag, "status": c.status, "op": c.op, "steps": c.steps,
                 "updates": c.updates, "t_submit_ms": c.t_submit_ms, "t_start_ms": c.t_start_ms,
                 "t_done_ms": c.t_done_ms}
            if c.op == PM_OP_DIVREM:
                d["q"] = g[:c.ng].copy()
                d["r"] = r[:c.nr].copy()
            else:
                d["g"] = g[:c.ng].copy()
            done.append(d)
        return done

    def pending(self) -> int:
        return int(lib().pm_server_pending(self.handle))

    def drain(self, timeout_s: float = 300.0) -> list:
        """Poll until every submitted request has finished (raises
        TimeoutError after timeout_s)."""
        import time
        out = []
        t_end = time.monotonic() + timeout_s
        while self.pending():
            out += self.poll()
            if time.monotonic() > t_end:
                raise TimeoutError("server did not finish its requests in %.0f s" % timeout_s)
        return out

    def close(self):
        if self.handle:
            lib().pm_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def last_gcd_stats() -> dict:
    st = GcdStats()
    lib().pm_last_gcd_stats(ctypes.byref(st))
    return {"steps": st.steps, "updates": st.updates, "chunks": st.chunks}


MUL_AUTO, MUL_VALU, MUL_MFMA = 0, 1, 2


def set_params(mul_s: int = 0, mul_r: int = 0, div_s: int = 0, gcd_s: int = 0, mul_engine: int = MUL_AUTO):
    _check(lib().pm_set_params(ctypes.byref(Params(mul_s, mul_r, div_s, gcd_s, mul_engine))))


def get_params() -> dict:
    pp = Params()
    lib().pm_get_params(ctypes.byref(pp))
    return {"mul_s": pp.mul_s, "mul_r": pp.mul_r, "div_s": pp.div_s, "gcd_s": pp.gcd_s,
            "mul_engine": pp.mul_engine}


def timing_enable(on: bool = True):
    lib().pm_timing_enable(1 if on else 0)


def timing_reset():
    lib().pm_timing_reset()


def timing_read(kernel: str):
    """(launches, total_ms) of the recorded launches of one kernel."""
    n, ms = ctypes.c_int64(0), ctypes.c_double(0)
    _check(lib().pm_timing_read(kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def release():
    lib().pm_release()
