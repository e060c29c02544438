"""Independent checks used to pin the oracle. None of these calls the oracle
or the GPU library; each is a different route to the same exact answer:
Horner evaluation, Kronecker substitution through Python big integers, a
textbook number-theoretic transform, synthetic division, Gaussian
elimination of the Sylvester matrix, and sympy over GF(p)."""
from __future__ import annotations

import numpy as np


def trim(c) -> list:
    c = [int(x) for x in c]
    while c and c[-1] == 0:
        c.pop()
    return c


def horner(c, x: int, p: int) -> int:
    acc = 0
    for coef in reversed([int(v) for v in c]):
        acc = (acc * x + coef) % p
    return acc


def kronecker_mul(a, b, p: int, slot_bits: int = 80) -> list:
    """Exact integer product by packing coefficients into slot_bits-bit
    fields of one big integer; each field of the product holds an exact
    convolution sum (< min(na, nb) * (p-1)^2 < 2^slot_bits for the sizes
    used here), which is then reduced mod p."""
    a, b = trim(a), trim(b)
    if not a or not b:
        return []
    n = min(len(a), len(b))
    assert n * (p - 1) ** 2 < (1 << slot_bits)
    A = int.from_bytes(b"".join(int(x).to_bytes(slot_bits // 8, "little") for x in a), "little")
    B = int.from_bytes(b"".join(int(x).to_bytes(slot_bits // 8, "little") for x in b), "little")
    C = A * B
    nb = slot_bits // 8
    raw = C.to_bytes(nb * (len(a) + len(b)), "little")
    out = [int.from_bytes(raw[i * nb:(i + 1) * nb], "little") % p for i in range(len(a) + len(b) - 1)]
    return trim(out)


def _primitive_root_of_unity(p: int, n: int) -> int:
    # p - 1 = c * 2^k with n | 2^k; 3 generates (Z/pZ)* for the NTT primes used here
    assert (p - 1) % n == 0
    return pow(3, (p - 1) // n, p)


def ntt(x: np.ndarray, p: int, invert: bool = False) -> np.ndarray:
    """Iterative radix-2 number-theoretic transform (Cooley-Tukey), values
    in uint64 with products below 2^60."""
    n = x.size
    x = x.astype(np.uint64).copy()
    bits = n.bit_length() - 1
    rev = np.zeros(n, dtype=np.int64)
    i = np.arange(n, dtype=np.int64)
    for k in range(bits):
        rev |= ((i >> k) & 1) << (bits - 1 - k)
    x = x[rev]
    length = 2
    P = np.uint64(p)
    while length <= n:
        w = _primitive_root_of_unity(p, length)
        if invert:
            w = pow(w, p - 2, p)
        half = length // 2
        tw = np.array([pow(w, k, p) for k in range(half)], dtype=np.uint64)
        xr = x.reshape(-1, length)
        u = xr[:, :half].copy()
        v = (xr[:, half:] * tw) % P
        xr[:, :half] = (u + v) % P
        xr[:, half:] = (u + P - v) % P
        x = xr.reshape(-1)
        length *= 2
    if invert:
        ninv = pow(n, p - 2, p)
        x = (x * np.uint64(ninv)) % P
    return x


def ntt_mul(a, b, p: int) -> list:
    a, b = trim(a), trim(b)
    if not a or not b:
        return []
    m = len(a) + len(b) - 1
    n = 1
    while n < m:
        n *= 2
    A = np.zeros(n, dtype=np.uint64); A[:len(a)] = a
    B = np.zeros(n, dtype=np.uint64); B[:len(b)] = b
    C = ntt((ntt(A, p) * ntt(B, p)) % np.uint64(p), p, invert=True)
    return trim(C[:m].tolist())


def synthetic_division(a, c: int, p: int):
    """Divide a by (X - c): Horner's scheme gives the quotient coefficients
    and the remainder a(c)."""
    a = trim(a)
    if not a:
        return [], 0
    n = len(a)
    q = [0] * (n - 1)
    acc = 0
    for i in range(n - 1, -1, -1):
        acc = (acc * c + a[i]) % p
        if i > 0:
            q[i - 1] = acc
    return trim(q), acc


def rank_mod_p(rows: list, p: int) -> int:
    m = [list(r) for r in rows]
    rank = 0
    ncols = len(m[0]) if m else 0
    for col in range(ncols):
        piv = None
        for r in range(rank, len(m)):
            if m[r][col] % p:
                piv = r
                break
        if piv is None:
            continue
        m[rank], m[piv] = m[piv], m[rank]
        iv = pow(m[rank][col], p - 2, p)
        m[rank] = [(v * iv) % p for v in m[rank]]
        for r in range(len(m)):
            if r != rank and m[r][col] % p:
                f = m[r][col]
                m[r] = [(x - f * y) % p for x, y in zip(m[r], m[rank])]
        rank += 1
    return rank


def sylvester_gcd_degree(a, b, p: int) -> int:
    """deg gcd(a, b) = deg a + deg b - rank Syl(a, b), for a, b non-constant."""
    a, b = trim(a), trim(b)
    da, db = len(a) - 1, len(b) - 1
    n = da + db
    rows = []
    for i in range(db):
        row = [0] * n
        for j, c in enumerate(reversed(a)):
            row[i + j] = c
        rows.append(row)
    for i in range(da):
        row = [0] * n
        for j, c in enumerate(reversed(b)):
            row[i + j] = c
        rows.append(row)
    return n - rank_mod_p(rows, p)


def sympy_poly(c, p: int):
    import sympy
    X = sympy.Symbol("X")
    c = trim(c)
    return sympy.Poly(list(reversed(c)) if c else [0], X, modulus=p, symmetric=False)


def from_sympy(P) -> list:
    co = [int(v) % P.get_modulus() for v in P.all_coeffs()]
    return trim(list(reversed(co)))


def det_mod_p(rows: list, p: int) -> int:
    """Determinant of a square matrix over GF(p) by Gaussian elimination."""
    m = [[int(v) % p for v in r] for r in rows]
    n = len(m)
    det = 1
    for col in range(n):
        piv = next((r for r in range(col, n) if m[r][col]), None)
        if piv is None:
            return 0
        if piv != col:
            m[col], m[piv] = m[piv], m[col]
            det = -det
        det = det * m[col][col] % p
        iv = pow(m[col][col], p - 2, p)
        for r in range(col + 1, n):
            if m[r][col]:
                f = m[r][col] * iv % p
                m[r] = [(x - f * y) % p for x, y in zip(m[r], m[col])]
    return det % p


def subresultant_degrees(a, b, p: int) -> list:
    """The degrees j < deg b at which the j-th principal subresultant
    coefficient of (a, b), deg a >= deg b >= 1, is non-zero, from highest to
    lowest. psc_j is the determinant of the (m + n - 2j)-square matrix whose
    rows are x^(n-j-1-i) a (i < n - j) and x^(m-j-1-i) b (i < m - j), each
    written by the coefficients of degrees m + n - j - 1 down to j. By the
    fundamental theorem of subresultants these are exactly the degrees of
    the Euclidean remainders after a and b (linear algebra only: no
    division of polynomials)."""
    a, b = trim(a), trim(b)
    m, n = len(a) - 1, len(b) - 1
    assert m >= n >= 1
    out = []
    for j in range(n - 1, -1, -1):
        size = m + n - 2 * j
        rows = []
        for poly, deg, count in ((a, m, n - j), (b, n, m - j)):
            for i in range(count):
                shift = count - 1 - i
                row = [0] * size
                for e, c in enumerate(poly):
                    col = (m + n - j - 1) - (e + shift)
                    if 0 <= col < size:
                        row[col] = c
                rows.append(row)
        if det_mod_p(rows, p):
            out.append(j)
    return out


def sympy_remainder_degrees(a, b, p: int) -> list:
    """deg r0, deg r1, ..., -1 of the Euclidean remainder sequence, formed
    with sympy's remainder over GF(p) (r0 the operand of higher degree, a on
    equal degrees)."""
    A, B = sympy_poly(a, p), sympy_poly(b, p)

    def deg(P):
        return -1 if P.is_zero else P.degree()

    if deg(A) < deg(B):
        A, B = B, A
    out = [deg(A), deg(B)]
    while not B.is_zero:
        A, B = B, A.rem(B)
        out.append(deg(B))
    return out
