"""Seeded synthetic inputs for the dense polynomial workloads over Z/pZ.

This module only draws random numbers. It holds none of the arithmetic of
the method (no products, divisions or remainders of polynomials): planted
inputs are returned as their factors (g, u, v) and the caller forms
a = g*u and b = g*v with a multiplication of its own choosing.

Every draw comes from ``numpy.random.PCG64(seed).random_raw()``; the raw
64-bit words of that bit generator are stable across numpy versions while
the ``Generator`` sampling methods are not. The recipes:

* uniform residue in [0, p): take the low 32 bits u of a raw word and
  accept when u < p * floor(2^32 / p); the value is u mod p (exact
  rejection sampling, no modulo bias);
* non-zero residue (leading coefficients): a uniform residue in
  [0, p - 1), plus one;
* log-uniform integer in [lo, hi]: x = (raw >> 11) / 2^53 and
  d = floor(exp(ln lo + x * (ln(hi + 1) - ln lo))), clamped to [lo, hi];
* exponential inter-arrival gap with rate lam: -ln(1 - x) / lam;
* uniform index in [0, k): rejection on the low 32 bits as above.

A polynomial is a numpy uint32 array of coefficients, index = exponent.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

P_A = 469762049   # 7 * 2^26 + 1
P_B = 998244353   # 119 * 2^23 + 1
P_C = 167772161   # 5 * 2^25 + 1
PRIMES = (P_A, P_B, P_C)

SEED_BASE = 1402026400


class Stream:
    """One sequential stream of raw 64-bit words."""

    def __init__(self, seed: int):
        self.bg = np.random.PCG64(seed)

    def raw(self, n: int) -> np.ndarray:
        return self.bg.random_raw(n).astype(np.uint64)

    def residues(self, n: int, lo_excl_top: int) -> np.ndarray:
        """n uniform integers in [0, m) with m = lo_excl_top < 2^32."""
        m = int(lo_excl_top)
        if n <= 0:
            return np.zeros(0, dtype=np.uint32)
        limit = m * ((1 << 32) // m)
        out = np.empty(n, dtype=np.uint64)
        got = 0
        while got < n:
            need = n - got
            w = self.raw(need + need // 8 + 8) & np.uint64(0xFFFFFFFF)
            w = w[w < np.uint64(limit)]
            take = min(need, w.size)
            out[got:got + take] = w[:take]
            got += take
        return (out % np.uint64(m)).astype(np.uint32)

    def uniform_poly(self, deg: int, p: int, monic: bool = False) -> np.ndarray:
        """Dense polynomial of exact degree deg: coefficients 0..deg-1
        uniform in [0, p), leading coefficient uniform non-zero (or 1)."""
        if deg < 0:
            return np.zeros(0, dtype=np.uint32)
        c = np.empty(deg + 1, dtype=np.uint32)
        c[:deg] = self.residues(deg, p)
        if monic:
            c[deg] = 1
        else:
            c[deg] = self.residues(1, p - 1)[0] + 1
        return c

    def unit(self) -> float:
        return float(int(self.raw(1)[0]) >> 11) / float(1 << 53)

    def log_uniform_int(self, lo: int, hi: int) -> int:
        x = self.unit()
        d = int(math.floor(math.exp(math.log(lo) + x * (math.log(hi + 1) - math.log(lo)))))
        return max(lo, min(hi, d))

    def uniform_int(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi]."""
        return lo + int(self.residues(1, hi - lo + 1)[0])

    def exponential(self, lam: float) -> float:
        return -math.log(1.0 - self.unit()) / lam

    def index(self, k: int) -> int:
        return int(self.residues(1, k)[0])


# ---------------------------------------------------------------------------
# Workloads. Each draws from one stream in the documented order.
# ---------------------------------------------------------------------------

def mul_pair(n_a: int, n_b: int, p: int = P_A, seed: int = SEED_BASE + 1):
    """Two dense polynomials with n_a and n_b terms (degrees n_a-1, n_b-1),
    uniform coefficients and non-zero leading coefficients: a then b."""
    st = Stream(seed)
    return st.uniform_poly(n_a - 1, p), st.uniform_poly(n_b - 1, p)


def product_2048(seed: int = SEED_BASE + 1):
    """Plain product of two degree-2047 polynomials over p = 469762049."""
    return mul_pair(2048, 2048, P_A, seed)


def product_65536(seed: int = SEED_BASE + 3):
    """Plain product of two degree-65535 polynomials over p = 469762049."""
    return mul_pair(65536, 65536, P_A, seed)


@dataclass
class PlantedGcd:
    p: int
    g: np.ndarray  # monic planted common factor
    u: np.ndarray  # cofactor of a
    v: np.ndarray  # cofactor of b


def planted_gcd(deg_a: int, deg_b: int, deg_g: int, p: int, st: Stream) -> PlantedGcd:
    """Factors of a = g*u, b = g*v with g monic of degree deg_g and u, v of
    degrees deg_a - deg_g and deg_b - deg_g. Draw order: g, u, v."""
    g = st.uniform_poly(deg_g, p, monic=True)
    u = st.uniform_poly(deg_a - deg_g, p)
    v = st.uniform_poly(deg_b - deg_g, p)
    return PlantedGcd(p, g, u, v)


def gcd_32768(seed: int = SEED_BASE + 2) -> PlantedGcd:
    """Division / remainder-sequence GCD workload: deg a = 32768,
    deg b = 32767, planted monic gcd of degree 1000, p = 469762049."""
    return planted_gcd(32768, 32767, 1000, P_A, Stream(seed))


@dataclass
class Batch:
    p: int
    a: list = field(default_factory=list)
    b: list = field(default_factory=list)


def batch_products(count: int = 4096, lo: int = 32, hi: int = 8192, p: int = P_A,
                   seed: int = SEED_BASE + 4) -> Batch:
    """Independent products: per instance deg a, deg b log-uniform in
    [lo, hi] (drawn in that order), then a, then b."""
    st = Stream(seed)
    out = Batch(p)
    for _ in range(count):
        da = st.log_uniform_int(lo, hi)
        db = st.log_uniform_int(lo, hi)
        out.a.append(st.uniform_poly(da, p))
        out.b.append(st.uniform_poly(db, p))
    return out


@dataclass
class Request:
    arrival: float  # seconds from the start of the trace
    p: int
    D: int          # deg a = D, deg b = D - 1
    k: int          # planted gcd degree
    factors: PlantedGcd


def served_trace(count: int, rate: float, lo: int = 64, hi: int = 16384,
                 seed: int = SEED_BASE + 5) -> list:
    """Poisson stream of GCD requests. Per request, in this order: the
    inter-arrival gap (rate ``rate`` per second), the prime index, D
    log-uniform in [lo, hi], k uniform in [0, floor(D/4)], then g (monic,
    degree k), u (degree D-k), v (degree D-1-k)."""
    st = Stream(seed)
    t = 0.0
    reqs = []
    for _ in range(count):
        t += st.exponential(rate)
        p = PRIMES[st.index(len(PRIMES))]
        D = st.log_uniform_int(lo, hi)
        k = st.uniform_int(0, D // 4)
        reqs.append(Request(t, p, D, k, planted_gcd(D, D - 1, k, p, st)))
    return reqs


@dataclass
class DivisionRequest:
    arrival: float
    p: int
    D: int          # deg a
    a: np.ndarray
    b: np.ndarray   # degree floor(D / 2)


def served_mixed_trace(count: int, rate: float, div_share: float = 0.25, lo: int = 64, hi: int = 16384,
                       seed: int = SEED_BASE + 7) -> list:
    """Poisson stream of gcd and division requests. Per request, in this
    order: the inter-arrival gap, the prime index, the kind (a division with
    probability div_share), D log-uniform in [lo, hi]; then for a gcd the
    draws of served_trace (k, g, u, v), for a division a of degree D and b
    of degree floor(D/2), uniform with non-zero leading coefficients."""
    st = Stream(seed)
    t = 0.0
    reqs = []
    for _ in range(count):
        t += st.exponential(rate)
        p = PRIMES[st.index(len(PRIMES))]
        div = st.unit() < div_share
        D = st.log_uniform_int(lo, hi)
        if div:
            a = st.uniform_poly(D, p)
            reqs.append(DivisionRequest(t, p, D, a, st.uniform_poly(D // 2, p)))
        else:
            k = st.uniform_int(0, D // 4)
            reqs.append(Request(t, p, D, k, planted_gcd(D, D - 1, k, p, st)))
    return reqs
