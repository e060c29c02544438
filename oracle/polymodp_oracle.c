/*
 * polymodp_oracle.c -- plain, slow, obviously correct CPU reference for dense
 * univariate polynomial arithmetic over Z/pZ.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the oracle that the GPU library is
 * checked against. It shares no code, header, table or helper with the GPU
 * path, and the product path never links or calls it: only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * Conventions (Sec. 3 of the paper, problem statement): a polynomial is an
 * array of coefficients indexed by exponent; n terms means degree n - 1.
 * Inputs may carry high zero coefficients; every output is normalised (its
 * leading coefficient is non-zero) and its length is returned; the zero
 * polynomial has length 0. The field is Z/pZ with p prime, 2 <= p < 2^31;
 * coefficients are canonical residues in [0, p).
 *
 * Arithmetic: every product is formed in 64 or 128 bits and reduced with the
 * C remainder operator, so there is no modular trick here to get wrong.
 *
 * The radix-sort case study (Sec. 4) has its plain stable LSD radix sort at
 * the end of the file.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* Number of terms once high zero coefficients are dropped. */
static int64_t trimmed(const uint32_t *a, int64_t n)
{
    while (n > 0 && a[n - 1] == 0)
        n--;
    return n;
}

/* Trial division; p fits in 32 bits so this is quick enough. */
int orc_is_prime(uint32_t p)
{
    if (p < 2)
        return 0;
    for (uint64_t d = 2; d * d <= p; d++)
        if (p % d == 0)
            return 0;
    return 1;
}

/* Inverse of x modulo p by the extended Euclidean algorithm on integers.
 * Returns 0 when x = 0 mod p (no inverse). */
uint32_t orc_inv(uint32_t x, uint32_t p)
{
    int64_t r0 = p, r1 = x % p, s0 = 0, s1 = 1;
    if (r1 == 0)
        return 0;
    while (r1 != 0) {
        int64_t q = r0 / r1, t;
        t = r0 - q * r1; r0 = r1; r1 = t;
        t = s0 - q * s1; s0 = s1; s1 = t;
    }
    /* r0 = gcd(x, p) = 1 and s0 * x = 1 (mod p) */
    s0 %= (int64_t)p;
    if (s0 < 0)
        s0 += p;
    return (uint32_t)s0;
}

/*
 * Product f = a * b (Sec. 5): f_k = sum over i of a_i * b_{k-i}, for
 * k = 0 .. na + nb - 2. Each f_k is summed exactly in 128 bits and reduced
 * once. f needs room for na + nb - 1 words; entries past the returned length
 * are written as zero. Returns the normalised length of f.
 */
int64_t orc_mul(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb,
                uint32_t p, uint32_t *f)
{
    int64_t nf = (na > 0 && nb > 0) ? na + nb - 1 : 0;
    for (int64_t k = 0; k < nf; k++) {
        int64_t lo = k - (nb - 1) > 0 ? k - (nb - 1) : 0;
        int64_t hi = k < na - 1 ? k : na - 1;
        u128 acc = 0;
        for (int64_t i = lo; i <= hi; i++)
            acc += (u128)((uint64_t)a[i] * (uint64_t)b[k - i]);
        f[k] = (uint32_t)(acc % p);
    }
    return trimmed(f, nf);
}

/* One coefficient of the product, f_k, by the same definition as orc_mul
 * (for spot checks of products too large to form here). */
uint32_t orc_mul_coeff(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb,
                       uint32_t p, int64_t k)
{
    if (na <= 0 || nb <= 0 || k < 0 || k > na + nb - 2)
        return 0;
    int64_t lo = k - (nb - 1) > 0 ? k - (nb - 1) : 0;
    int64_t hi = k < na - 1 ? k : na - 1;
    u128 acc = 0;
    for (int64_t i = lo; i <= hi; i++)
        acc += (u128)((uint64_t)a[i] * (uint64_t)b[k - i]);
    return (uint32_t)(acc % p);
}

/* Statistics of one long division or one remainder sequence. */
typedef struct {
    int64_t steps;    /* division steps (one quotient coefficient each)   */
    int64_t updates;  /* coefficient updates, (deg divisor + 1) per step  */
    int64_t divisions;/* Euclidean divisions (remainders formed)          */
} orc_stats;

/*
 * Long division of w (nw terms, modified in place) by the normalised b
 * (nb >= 1 terms), in the step order of the naive division (Sec. 3.1,
 * Algorithms 1 and 2): for i = nw-1 down to nb-1, the multiplier is
 * c = w_i * lc(b)^{-1}; it is the quotient coefficient of X^{i-nb+1}, and
 * c * X^{i-nb+1} * b is subtracted from w. A zero w_i gives c = 0 and the
 * step changes nothing. Afterwards w holds the remainder in its low nb-1
 * entries. q (optional) receives nw - nb + 1 quotient coefficients.
 */
static void long_division(uint32_t *w, int64_t nw, const uint32_t *b, int64_t nb,
                          uint32_t p, uint32_t *q, orc_stats *st)
{
    uint64_t inv = orc_inv(b[nb - 1], p);
    for (int64_t i = nw - 1; i >= nb - 1; i--) {
        uint64_t c = ((uint64_t)w[i] * inv) % p;
        int64_t sh = i - (nb - 1);
        if (q)
            q[sh] = (uint32_t)c;
        for (int64_t j = 0; j < nb; j++) {
            uint64_t prod = (c * b[j]) % p;
            w[sh + j] = (uint32_t)(((uint64_t)w[sh + j] + p - prod) % p);
        }
        if (st) {
            st->steps += 1;
            st->updates += nb;
        }
    }
}

/*
 * Euclidean division (Sec. 3, problem statement): the unique (q, r) with
 * a = q*b + r and deg r < deg b. b must be non-zero (returns -4 otherwise).
 * q needs room for max(na' - nb' + 1, 0) words and r for max(nb' - 1, 0)
 * words, where na', nb' are the trimmed lengths; when deg a < deg b the
 * quotient is zero and r = a (then r needs na' words). Lengths go to *nq
 * and *nr. Returns 0.
 */
int orc_divrem(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb,
               uint32_t p, uint32_t *q, int64_t *nq, uint32_t *r, int64_t *nr)
{
    na = trimmed(a, na);
    nb = trimmed(b, nb);
    if (nb == 0)
        return -4;
    if (na < nb) {
        memcpy(r, a, (size_t)na * sizeof(uint32_t));
        *nq = 0;
        *nr = na;
        return 0;
    }
    uint32_t *w = (uint32_t *)malloc((size_t)na * sizeof(uint32_t));
    memcpy(w, a, (size_t)na * sizeof(uint32_t));
    long_division(w, na, b, nb, p, q, NULL);
    *nq = trimmed(q, na - nb + 1);
    *nr = trimmed(w, nb - 1);
    memcpy(r, w, (size_t)(*nr) * sizeof(uint32_t));
    free(w);
    return 0;
}

/* Multiply the n coefficients of x by the inverse of its leading one. */
static void make_monic(uint32_t *x, int64_t n, uint32_t p)
{
    if (n == 0)
        return;
    uint64_t inv = orc_inv(x[n - 1], p);
    for (int64_t i = 0; i < n; i++)
        x[i] = (uint32_t)(((uint64_t)x[i] * inv) % p);
}

/*
 * Monic gcd of a and b by the Euclidean remainder sequence (Sec. 6):
 * r0 = a, r1 = b (the one of higher degree first; on equal degrees a is the
 * dividend, as in the naive Euclidean kernel), then (r0, r1) <- (r1, r0 mod r1)
 * until r1 = 0. The last non-zero remainder, made monic, is the gcd; a
 * non-zero constant remainder gives gcd 1, and gcd(0, 0) = 0.
 * g needs room for max(na', nb') words. degs (optional, capacity degs_cap)
 * receives the degree sequence deg r0, deg r1, ..., ending with -1;
 * *n_degs its full length. st (optional) receives the step counts.
 * Returns the length of g.
 */
int64_t orc_gcd(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb,
                uint32_t p, uint32_t *g, int64_t *degs, int64_t degs_cap,
                int64_t *n_degs, orc_stats *st)
{
    na = trimmed(a, na);
    nb = trimmed(b, nb);
    int64_t cap = na > nb ? na : nb;
    uint32_t *x = (uint32_t *)malloc((size_t)(cap + 1) * sizeof(uint32_t));
    uint32_t *y = (uint32_t *)malloc((size_t)(cap + 1) * sizeof(uint32_t));
    int64_t nx, ny;
    if (na >= nb) {
        memcpy(x, a, (size_t)na * 4); nx = na;
        memcpy(y, b, (size_t)nb * 4); ny = nb;
    } else {
        memcpy(x, b, (size_t)nb * 4); nx = nb;
        memcpy(y, a, (size_t)na * 4); ny = na;
    }
    int64_t nd = 0;
    if (st)
        memset(st, 0, sizeof(*st));
#define PUSH_DEG(d) do { if (degs && nd < degs_cap) degs[nd] = (d); nd++; } while (0)
    PUSH_DEG(nx - 1);
    PUSH_DEG(ny - 1);
    while (ny > 0) {
        long_division(x, nx, y, ny, p, NULL, st);
        if (st)
            st->divisions += 1;
        int64_t nr = trimmed(x, ny - 1);
        /* (x, y) <- (y, x mod y) */
        uint32_t *t = x; x = y; y = t;
        nx = ny;
        ny = nr;
        PUSH_DEG(ny - 1);
    }
#undef PUSH_DEG
    make_monic(x, nx, p);
    memcpy(g, x, (size_t)nx * 4);
    if (n_degs)
        *n_degs = nd;
    free(x);
    free(y);
    return nx;
}

/* dst = dst - c * src (lengths: dst has room for max(nd, ns)); returns the
 * normalised length. */
static int64_t sub_mul(uint32_t *dst, int64_t nd, const uint32_t *src, int64_t ns,
                       uint32_t p)
{
    for (int64_t i = nd; i < ns; i++)
        dst[i] = 0;
    int64_t n = nd > ns ? nd : ns;
    for (int64_t i = 0; i < ns; i++)
        dst[i] = (uint32_t)(((uint64_t)dst[i] + p - src[i]) % p);
    return trimmed(dst, n);
}

/*
 * Extended Euclidean algorithm: monic g = gcd(a, b) and cofactors s, t with
 * s*a + t*b = g (the Bezout certificate of the gcd). Buffers: g and s and t
 * each need room for na' + nb' + 1 words. Returns 0, or -1 when both inputs
 * are zero (then g = s = t = 0).
 */
int orc_xgcd(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb,
             uint32_t p, uint32_t *g, int64_t *ng, uint32_t *s, int64_t *ns,
             uint32_t *t, int64_t *nt)
{
    na = trimmed(a, na);
    nb = trimmed(b, nb);
    int64_t cap = na + nb + 2;
    uint32_t *r0 = calloc(cap, 4), *r1 = calloc(cap, 4);
    uint32_t *s0 = calloc(cap, 4), *s1 = calloc(cap, 4);
    uint32_t *t0 = calloc(cap, 4), *t1 = calloc(cap, 4);
    uint32_t *q = calloc(cap, 4), *rr = calloc(cap, 4), *tmp = calloc(2 * cap, 4);
    int64_t n_r0 = na, n_r1 = nb, n_s0 = 1, n_s1 = 0, n_t0 = 0, n_t1 = 1;
    memcpy(r0, a, (size_t)na * 4);
    memcpy(r1, b, (size_t)nb * 4);
    s0[0] = 1;
    t1[0] = 1;
    while (n_r1 > 0) {
        int64_t nq, nr;
        orc_divrem(r0, n_r0, r1, n_r1, p, q, &nq, rr, &nr);
        /* (r0, r1) <- (r1, rr) */
        memcpy(r0, r1, (size_t)n_r1 * 4); n_r0 = n_r1;
        memset(r1, 0, (size_t)cap * 4);
        memcpy(r1, rr, (size_t)nr * 4); n_r1 = nr;
        /* (s0, s1) <- (s1, s0 - q*s1) and likewise for t */
        int64_t nm = orc_mul(q, nq, s1, n_s1, p, tmp);
        n_s0 = sub_mul(s0, n_s0, tmp, nm, p);
        { uint32_t *z = s0; s0 = s1; s1 = z; int64_t m = n_s0; n_s0 = n_s1; n_s1 = m; }
        nm = orc_mul(q, nq, t1, n_t1, p, tmp);
        n_t0 = sub_mul(t0, n_t0, tmp, nm, p);
        { uint32_t *z = t0; t0 = t1; t1 = z; int64_t m = n_t0; n_t0 = n_t1; n_t1 = m; }
    }
    int rc = 0;
    if (n_r0 == 0) {
        *ng = *ns = *nt = 0;
        rc = -1;
    } else {
        uint64_t inv = orc_inv(r0[n_r0 - 1], p);
        for (int64_t i = 0; i < n_r0; i++) g[i] = (uint32_t)((r0[i] * inv) % p);
        for (int64_t i = 0; i < n_s0; i++) s[i] = (uint32_t)((s0[i] * inv) % p);
        for (int64_t i = 0; i < n_t0; i++) t[i] = (uint32_t)((t0[i] * inv) % p);
        *ng = n_r0;
        *ns = n_s0;
        *nt = n_t0;
    }
    free(r0); free(r1); free(s0); free(s1); free(t0); free(t1);
    free(q); free(rr); free(tmp);
    return rc;
}

/*
 * One step of the naive Euclidean kernel (Sec. 6.1, Algorithm 9), for
 * step-level checks: with da = deg a and db = deg b (-1 for zero), if
 * da >= db >= 0 then a <- a - (lc a / lc b) X^(da-db) b, else if
 * 0 <= da < db then b <- b - (lc b / lc a) X^(db-da) a. The multiplier is
 * taken before any coefficient changes. Degrees are rescanned afterwards.
 * Returns 1 if a step was taken, 0 if one operand is already zero.
 */
int orc_euclid_step(uint32_t *a, int64_t *da, uint32_t *b, int64_t *db, uint32_t p)
{
    uint32_t *x, *y;
    int64_t *dx, *dy;
    if (*da >= *db && *db >= 0) {
        x = a; dx = da; y = b; dy = db;
    } else if (*da >= 0 && *da < *db) {
        x = b; dx = db; y = a; dy = da;
    } else {
        return 0;
    }
    uint64_t c = ((uint64_t)x[*dx] * orc_inv(y[*dy], p)) % p;
    int64_t sh = *dx - *dy;
    for (int64_t j = 0; j <= *dy; j++) {
        uint64_t prod = (c * y[j]) % p;
        x[sh + j] = (uint32_t)(((uint64_t)x[sh + j] + p - prod) % p);
    }
    while (*dx >= 0 && x[*dx] == 0)
        (*dx)--;
    return 1;
}

/*
 * Radix sort (Sec. 4): the stable least-significant-digit sort of n keys
 * of c bits (1 <= c <= 32; only the low c bits of a key are its sort key)
 * with digits of s bits (1 <= s <= 16), in ceil(c/s) passes from the low
 * digit up. Each pass is one counting sort on its digit: the histogram of
 * the digit values, its exclusive prefix sum (where each value's run
 * starts), and a scatter in input order, which keeps equal digits in their
 * previous order. vals (may be NULL, then vals_out is ignored) moves with
 * its key. Returns 0, or -1 for bad c or s.
 */
int orc_radix_sort(const uint32_t *keys, const uint32_t *vals, int64_t n, int c, int s,
                   uint32_t *keys_out, uint32_t *vals_out)
{
    if (c < 1 || c > 32 || s < 1 || s > 16)
        return -1;
    uint32_t *k0 = malloc((size_t)(n > 0 ? n : 1) * 4), *k1 = malloc((size_t)(n > 0 ? n : 1) * 4);
    uint32_t *v0 = malloc((size_t)(n > 0 ? n : 1) * 4), *v1 = malloc((size_t)(n > 0 ? n : 1) * 4);
    int64_t *count = malloc(((size_t)1 << s) * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) {
        k0[i] = keys[i];
        v0[i] = vals ? vals[i] : 0;
    }
    for (int shift = 0; shift < c; shift += s) {
        int bits = c - shift < s ? c - shift : s;
        uint32_t mask = (uint32_t)((1ull << bits) - 1);
        int64_t r = (int64_t)1 << bits;
        for (int64_t d = 0; d < r; d++)
            count[d] = 0;
        for (int64_t i = 0; i < n; i++)
            count[(k0[i] >> shift) & mask]++;
        int64_t run = 0;  /* exclusive prefix sum: start of each digit's run */
        for (int64_t d = 0; d < r; d++) {
            int64_t c_d = count[d];
            count[d] = run;
            run += c_d;
        }
        for (int64_t i = 0; i < n; i++) {
            int64_t at = count[(k0[i] >> shift) & mask]++;
            k1[at] = k0[i];
            v1[at] = v0[i];
        }
        uint32_t *t = k0; k0 = k1; k1 = t;
        t = v0; v0 = v1; v1 = t;
    }
    for (int64_t i = 0; i < n; i++) {
        keys_out[i] = k0[i];
        if (vals && vals_out)
            vals_out[i] = v0[i];
    }
    free(k0); free(k1); free(v0); free(v1); free(count);
    return 0;
}
