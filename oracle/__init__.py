"""CPU oracle for dense polynomial arithmetic over Z/pZ.

TEST INFRASTRUCTURE ONLY: the plain C reference in ``polymodp_oracle.c``
(schoolbook product, long division, Euclidean and extended Euclidean
remainder sequences) behind a ctypes wrapper. Only the tests, the smoke
check and the CPU-baseline leg of the benchmark use it; the GPU library
neither imports nor links it, and the two share no code.

Every function takes and returns numpy uint32 coefficient arrays (index =
exponent); outputs are normalised (no high zeros, zero polynomial = empty).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "polymodp_oracle.c")
_LIB = os.path.join(_HERE, "libpolymodp_oracle.so")

_u32p = ctypes.POINTER(ctypes.c_uint32)
_i64p = ctypes.POINTER(ctypes.c_int64)


class Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("updates", ctypes.c_int64),
                ("divisions", ctypes.c_int64)]


def build(force: bool = False) -> str:
    """Compile the oracle with the host C compiler (plain -O2, no SIMD
    intrinsics, no threads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        L.orc_is_prime.argtypes = [ctypes.c_uint32]
        L.orc_is_prime.restype = ctypes.c_int
        L.orc_inv.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.orc_inv.restype = ctypes.c_uint32
        L.orc_mul.argtypes = [_u32p, ctypes.c_int64, _u32p, ctypes.c_int64, ctypes.c_uint32, _u32p]
        L.orc_mul.restype = ctypes.c_int64
        L.orc_mul_coeff.argtypes = [_u32p, ctypes.c_int64, _u32p, ctypes.c_int64, ctypes.c_uint32,
                                    ctypes.c_int64]
        L.orc_mul_coeff.restype = ctypes.c_uint32
        L.orc_divrem.argtypes = [_u32p, ctypes.c_int64, _u32p, ctypes.c_int64, ctypes.c_uint32,
                                 _u32p, _i64p, _u32p, _i64p]
        L.orc_divrem.restype = ctypes.c_int
        L.orc_gcd.argtypes = [_u32p, ctypes.c_int64, _u32p, ctypes.c_int64, ctypes.c_uint32,
                              _u32p, _i64p, ctypes.c_int64, _i64p, ctypes.POINTER(Stats)]
        L.orc_gcd.restype = ctypes.c_int64
        L.orc_radix_sort.argtypes = [_u32p, _u32p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _u32p, _u32p]
        L.orc_radix_sort.restype = ctypes.c_int
        L.orc_xgcd.argtypes = [_u32p, ctypes.c_int64, _u32p, ctypes.c_int64, ctypes.c_uint32,
                               _u32p, _i64p, _u32p, _i64p, _u32p, _i64p]
        L.orc_xgcd.restype = ctypes.c_int
        L.orc_euclid_step.argtypes = [_u32p, _i64p, _u32p, _i64p, ctypes.c_uint32]
        L.orc_euclid_step.restype = ctypes.c_int
        _lib = L
    return _lib


def _arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint32))


def _ptr(x: np.ndarray):
    return x.ctypes.data_as(_u32p)


def is_prime(p: int) -> bool:
    return bool(lib().orc_is_prime(p))


def inv(x: int, p: int) -> int:
    return int(lib().orc_inv(x, p))


def mul(a, b, p: int) -> np.ndarray:
    a, b = _arr(a), _arr(b)
    f = np.zeros(max(a.size + b.size - 1, 1), dtype=np.uint32)
    nf = lib().orc_mul(_ptr(a), a.size, _ptr(b), b.size, p, _ptr(f))
    return f[:nf].copy()


def mul_coeff(a, b, p: int, k: int) -> int:
    """f_k of the product a*b (no normalisation of the inputs)."""
    a, b = _arr(a), _arr(b)
    return int(lib().orc_mul_coeff(_ptr(a), a.size, _ptr(b), b.size, p, k))


def divrem(a, b, p: int):
    a, b = _arr(a), _arr(b)
    q = np.zeros(max(a.size, 1), dtype=np.uint32)
    r = np.zeros(max(a.size, b.size, 1), dtype=np.uint32)
    nq, nr = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = lib().orc_divrem(_ptr(a), a.size, _ptr(b), b.size, p, _ptr(q), ctypes.byref(nq),
                          _ptr(r), ctypes.byref(nr))
    if rc != 0:
        raise ZeroDivisionError("division by the zero polynomial")
    return q[:nq.value].copy(), r[:nr.value].copy()


def gcd(a, b, p: int, with_info: bool = False):
    """Monic gcd. With ``with_info`` also returns (degree sequence, Stats)."""
    a, b = _arr(a), _arr(b)
    cap = max(a.size, b.size, 1)
    g = np.zeros(cap, dtype=np.uint32)
    dcap = a.size + b.size + 4
    degs = np.zeros(dcap, dtype=np.int64)
    nd = ctypes.c_int64(0)
    st = Stats()
    ng = lib().orc_gcd(_ptr(a), a.size, _ptr(b), b.size, p, _ptr(g),
                       degs.ctypes.data_as(_i64p), dcap, ctypes.byref(nd), ctypes.byref(st))
    g = g[:ng].copy()
    if with_info:
        return g, degs[:nd.value].copy(), st
    return g


def xgcd(a, b, p: int):
    """(g, s, t) with s*a + t*b = g monic."""
    a, b = _arr(a), _arr(b)
    cap = a.size + b.size + 2
    g, s, t = (np.zeros(cap, dtype=np.uint32) for _ in range(3))
    ng, ns, nt = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    lib().orc_xgcd(_ptr(a), a.size, _ptr(b), b.size, p, _ptr(g), ctypes.byref(ng),
                   _ptr(s), ctypes.byref(ns), _ptr(t), ctypes.byref(nt))
    return g[:ng.value].copy(), s[:ns.value].copy(), t[:nt.value].copy()


def radix_sort(keys, vals=None, c: int = 32, s: int = 8):
    """Stable LSD radix sort of uint32 keys on their low c bits with s-bit
    digits (Sec. 4); returns (keys, vals) sorted (vals None when not given)."""
    k = _arr(keys)
    n = k.size
    ko = np.zeros(max(n, 1), dtype=np.uint32)
    v = _arr(vals) if vals is not None else None
    vo = np.zeros(max(n, 1), dtype=np.uint32) if v is not None else None
    null = ctypes.cast(None, _u32p)
    rc = lib().orc_radix_sort(_ptr(k) if n else null, _ptr(v) if v is not None and n else null, n, c, s,
                              _ptr(ko), _ptr(vo) if vo is not None else null)
    if rc != 0:
        raise ValueError("bad c or s")
    return ko[:n].copy(), (vo[:n].copy() if vo is not None else None)


def euclid_step(a: np.ndarray, da: int, b: np.ndarray, db: int, p: int):
    """One naive Euclidean step on copies of a, b (full-length buffers);
    returns (a', da', b', db', stepped)."""
    a, b = _arr(a).copy(), _arr(b).copy()
    xa, xb = ctypes.c_int64(da), ctypes.c_int64(db)
    stepped = lib().orc_euclid_step(_ptr(a), ctypes.byref(xa), _ptr(b), ctypes.byref(xb), p)
    return a, xa.value, b, xb.value, bool(stepped)
