"""Running-time estimates of the many-core machine model for the three
case studies, used to state the range of the program parameter s that the
model predicts and to set it beside the measured optimum.

Corollary 1 bounds the running time of a program by (N/K + L) * C, where N
is the number of thread-blocks, L the length of the longest path of
kernels, C the largest per-block span plus overhead, and K the largest
number of blocks in an anti-chain (here: the block count of the widest
kernel). The per-algorithm N, L, C below are the ones the paper prints for
the optimized algorithms (the naive ones are the same formulas at s = 1 for
the product, and the separately printed N_1, L_1, C_1 for division and gcd).
U is the cost of one word transferred between global and local memory, in
units of one local operation; Z the local-memory size in words.

Machine constants for MI355X (stated, not measured here):
  Z = 160 KiB of LDS per CU / 4 bytes = 40960 words;
  U (throughput view) = VALU lane-ops per CU per clock over HBM words per CU
    per clock = 64 / (8e12 B/s / 4 B / 256 CUs / 2.4e9 Hz) ~ 19.7;
  U (latency view) = the paper's 400-800 cycles of global-memory latency.
"""
from __future__ import annotations

import math

Z_MI355X = 160 * 1024 // 4
U_THROUGHPUT = 64.0 / (8e12 / 4 / 256 / 2.4e9)
U_LATENCY = (400.0, 800.0)


# -------------------------------------------------------------- product
def mul_terms(n: float, m: float, s: float, U: float, ell: float):
    """(N_s, L_s, C_s, K_s) of the plain multiplication (Sec. 5):
    N_s = (n+s-1)(2m-s)/(s^2 l), L_s = log2(m/s) + 1,
    C_s = s(2s-1) + 2U(s+1); K_s = blocks of the multiplication kernel,
    x*y/(s l) with x = m/s and y = n+s-1."""
    N = (n + s - 1) * (2 * m - s) / (s * s * ell)
    L = math.log2(m / s) + 1
    C = s * (2 * s - 1) + 2 * U * (s + 1)
    K = (m / s) * (n + s - 1) / (s * ell)
    return N, L, C, K


def mul_time(n: float, m: float, s: float, U: float, ell: float = 256) -> float:
    """Corollary 1 estimate; equals (3 - s/m + log2(m/s)) * C_s."""
    N, L, C, K = mul_terms(n, m, s, U, ell)
    return (N / K + L) * C


def mul_ratio_printed(n: float, s: float, U: float) -> float:
    """The paper's printed R = T_1 / T_s for m = n (Sec. 5)."""
    return ((n * math.log2(n) + 3 * n - 1) * (1 + 4 * U)) / (
        (n * math.log2(n / s) + 3 * n - s) * (2 * U * s + 2 * U + 2 * s * s - s))


# ------------------------------------------------------------- division
def div_time_naive(n: float, m: float, U: float, ell: float) -> float:
    """T_1 = (N_1/K_1 + L_1) C_1 with N_1 = (n-m+1)m/l, K_1 = m/l,
    L_1 = n-m+1, C_1 = 3+5U (Sec. 3.1, 3.3)."""
    N, K, L, C = (n - m + 1) * m / ell, m / ell, n - m + 1, 3 + 5 * U
    return (N / K + L) * C


def div_time(n: float, m: float, s: float, U: float) -> float:
    """T_s = (N_s/K_s + L_s) C_s with N_s = (n-m+1)m/(2s^2), K_s = m/(2s),
    L_s = (n-m+1)/s, C_s = 3s+9U (Sec. 3.2, 3.3)."""
    N, K, L, C = (n - m + 1) * m / (2 * s * s), m / (2 * s), (n - m + 1) / s, 3 * s + 9 * U
    return (N / K + L) * C


def div_ratio_printed(Z: float, U: float) -> float:
    """R = (3+5U) Z / (3 (Z + 21U)) with l = Z/2, s = Z/7 (Sec. 3.3)."""
    return (3 + 5 * U) * Z / (3 * (Z + 21 * U))


# ------------------------------------------------------------------ gcd
def gcd_time_naive(n: float, m: float, U: float, ell: float) -> float:
    """N_1 = m(n+l+1)/l, K_1 = m/l, L_1 = m+n-2, C_1 = 3+5U (Sec. 6.1)."""
    N, K, L, C = m * (n + ell + 1) / ell, m / ell, m + n - 2, 3 + 5 * U
    return (N / K + L) * C


def gcd_time(n: float, m: float, s: float, U: float) -> float:
    """N_s = mn/s^2 + m/s, K_s = m/s, L_s = n/s + m/s, C_s = 3s+8U (Sec. 6.2)."""
    N, K, L, C = m * n / (s * s) + m / s, m / s, n / s + m / s, 3 * s + 8 * U
    return (N / K + L) * C


def gcd_ratio_printed(n: float, Z: float, U: float) -> float:
    """R = (6n-2+Z)(3+5U) Z / ((18n+Z)(Z+16U)) with m = n, l = Z/2,
    s = Z/6 (Sec. 6.3)."""
    return (6 * n - 2 + Z) * (3 + 5 * U) * Z / ((18 * n + Z) * (Z + 16 * U))


def gcd_s_star(n: float, m: float, U: float) -> float:
    """Minimiser of gcd_time over real s: ((2n+m)/s + 1)(3s + 8U) is least
    at s = sqrt(8U(2n+m)/3) (our derivation from the printed N, L, C)."""
    return math.sqrt(8 * U * (2 * n + m) / 3)


# ----------------------------------------------------------- radix sort
def sort_terms(n: float, c: float, s: float, U: float, ell: float = 256):
    """(N_s, L_s, C_s, K_s) of the radix sort (Sec. 4): N_s = (c/s)(1/(2l) +
    2^s/(8 l^2)) n, L_s = 5c/s, C_s = s(41 + 8 log2 l) + 12 + 9U; K_s = the
    blocks of one pass's widest kernel, one per tile of 4l keys."""
    N = (c / s) * (1 / (2 * ell) + 2 ** s / (8 * ell * ell)) * n
    L = 5 * c / s
    C = s * (41 + 8 * math.log2(ell)) + 12 + 9 * U
    K = n / (4 * ell)
    return N, L, C, K


def sort_time(n: float, c: float, s: float, U: float, ell: float = 256) -> float:
    """Corollary 1 estimate (N_s/K_s + L_s) C_s; s = 1 is the naive sort."""
    N, L, C, K = sort_terms(n, c, s, U, ell)
    return (N / K + L) * C


def sort_ratio_printed(s: float, U: float, ell: float = 256) -> float:
    """The paper's printed R = T_1/T_s of the radix sort (Sec. 4)."""
    lg = math.log2(ell)
    return (14 * ell + 2) * (53 + 8 * lg + 9 * U) * s / ((14 * ell + 2 ** s) * (41 * s + 8 * s * lg + 12 + 9 * U))


def argmin(fn, candidates):
    best = min(candidates, key=fn)
    return best, fn(best)


def predicted_ranges(n_mul: int = 65536, n_gcd: int = 32769, U: float = U_THROUGHPUT,
                     Z: int = Z_MI355X) -> dict:
    """The s the model favours for each case study at the given sizes,
    over the powers of two that fit the local memory."""
    ss = [2 ** k for k in range(0, 14)]
    mul_ok = [s for s in ss if 2 * s * 256 + 2 * s - 1 <= Z]   # 2 s l + 2 s - 1 <= Z
    div_ok = [s for s in ss if 7 * s <= Z and 3 * s <= 1024]   # 7s <= Z, 3s threads
    gcd_ok = [s for s in ss if 6 * s <= Z and 3 * s <= 1024]
    mul_best, _ = argmin(lambda s: mul_time(n_mul, n_mul, s, U), mul_ok)
    div_best, _ = argmin(lambda s: div_time(2 * n_gcd, n_gcd, s, U), div_ok)
    gcd_best, _ = argmin(lambda s: gcd_time(n_gcd, n_gcd - 1, s, U), gcd_ok)
    return {"U": U, "Z": Z,
            "mul": {"argmin_s": mul_best, "note": "T(s) increases with s: s as small as possible"},
            "div": {"argmin_s": div_best, "note": "T(s) decreases with s: as large as fits"},
            "gcd": {"argmin_s": gcd_best, "s_star_real": gcd_s_star(n_gcd, n_gcd - 1, U)}}
