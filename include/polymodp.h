/*
 * polymodp.h -- C ABI of libpolymodp: dense univariate polynomial arithmetic
 * over the prime field Z/pZ on AMD Instinct MI355X (gfx950).
 *
 * The operations are the ones whose many-core algorithms the paper "A
 * Many-core Machine Model for Designing Algorithms with Minimum Parallelism
 * Overheads" (Haque, Moreno Maza, Xie) studies: the plain product (Sec. 5),
 * Euclidean division (Sec. 3) and the Euclidean gcd (Sec. 6).
 *
 * Conventions for every entry point
 *  - A polynomial is an array of uint32 coefficients indexed by exponent; its
 *    length is its number of terms (degree + 1). High zero coefficients in
 *    inputs are allowed and ignored; the zero polynomial has length 0.
 *    Outputs are normalised: their reported length ends at a non-zero
 *    coefficient.
 *  - Coefficient and output arrays are DEVICE pointers (memory of the
 *    current HIP device). Length and status pointers named d_* are device
 *    pointers too; the other int64_t* outputs are host pointers.
 *  - p must be a prime with 2 <= p < 2^30, and every input coefficient must
 *    be a canonical residue in [0, p).
 *  - `stream` is a hipStream_t (NULL = the default stream). Work is enqueued
 *    on it in order; synchronous entry points wait for it before returning.
 *  - Ownership: the caller owns every buffer. Inputs are read only. Outputs
 *    (over their capacity) must not overlap inputs or each other: PM_EINVAL.
 *    Scratch memory belongs to the library (one pool per device and stream,
 *    grown on demand and kept until pm_release) unless the caller sets a
 *    workspace for the stream (pm_set_workspace).
 *  - Errors: checks that need no device access (null pointers, negative
 *    lengths, capacities smaller than the given lengths require, outputs
 *    overlapping inputs, a modulus that is not a prime below 2^30) are made
 *    before anything is enqueued.
 *    Checks that need the data (coefficients >= p, a zero divisor, a
 *    capacity below what the true degrees require) are made on the device:
 *    synchronous calls return them, asynchronous calls write them to
 *    d_status. Nothing is thrown across the ABI. pm_last_error() describes
 *    the last failure of the calling thread.
 */
#ifndef POLYMODP_H
#define POLYMODP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pm_status;
enum {
    PM_OK = 0,
    PM_EINVAL = -1,    /* null pointer, negative length, capacity too small */
    PM_EMODULUS = -2,  /* p not prime, or p >= 2^30                          */
    PM_ERANGE = -3,    /* an input coefficient is >= p                       */
    PM_EDIVZERO = -4,  /* division by the zero polynomial                    */
    PM_ENOMEM = -5,    /* device or host memory could not be allocated       */
    PM_EDEVICE = -6    /* a HIP runtime error or a broken device invariant   */
};
/* No C++ exception leaves a function of this interface: one raised inside
 * (host memory exhaustion, a thread that cannot start) becomes PM_ENOMEM or
 * PM_EDEVICE, with its message in pm_last_error(); the functions that
 * return nothing swallow it. */

/*
 * Product f = a * b (Sec. 5, plain multiplication: every coefficient of a
 * is multiplied with every coefficient of b and the products of equal degree
 * are added), f_k = sum_i a_i b_{k-i} mod p.
 *   a, na / b, nb : inputs (device), lengths >= 0
 *   f, f_cap      : output (device), f_cap >= na + nb - 1 when na, nb > 0
 *   nf            : host; normalised length of f (0 if a or b is zero)
 * f[0 .. na+nb-2] is written in full; entries past *nf are zero.
 */
pm_status poly_mul_modp(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb, uint32_t p,
                        uint32_t *f, int64_t f_cap, int64_t *nf, void *stream);

/*
 * Asynchronous product: same computation, nothing waits for the device and
 * nothing is allocated when the plan's scratch is already in the pool (a
 * plan with a single b-chunk needs none). d_nf (int64) and d_status (int32)
 * are device pointers written by the launch. Safe to capture in a hipGraph
 * once the same sizes ran once outside capture.
 */
pm_status poly_mul_modp_async(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb, uint32_t p,
                              uint32_t *f, int64_t f_cap, int64_t *d_nf, int32_t *d_status, void *stream);

/*
 * The asynchronous product for callers that cannot allocate device memory
 * (code under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc): arguments, result and device-side checks as
 * poly_mul_modp_async, but no call allocates or frees anything. The
 * kernels' scratch (the partial sums of the addition phase) is a static
 * device array of PM_NOALLOC_SCRATCH_WORDS words (64 MiB) that every device
 * the library runs on holds until the process ends. The engine is the one
 * poly_mul_modp_async picks, or else the VALU tiles, whichever plan's
 * scratch fits; a product no plan fits returns PM_EINVAL before anything is
 * enqueued (the matrix cores fit every square product up to about 300000
 * terms per operand). All calls on one device share that device's array:
 * two calls that overlap in time on one device (two streams, or two host
 * threads) race and give wrong results; calls in order on one stream are
 * safe. d_nf and d_status may be NULL.
 */
#define PM_NOALLOC_SCRATCH_WORDS (1 << 24)
pm_status poly_mul_modp_noalloc(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb, uint32_t p,
                                uint32_t *f, int64_t f_cap, int64_t *d_nf, int32_t *d_status, void *stream);

/*
 * Batched products: many independent f_i = a_i * b_i (mixed lengths and
 * primes) in ONE persistent launch. The work is cut into output tiles of
 * 256*r coefficients, each summed over the whole of b_i in chunks of kc
 * coefficients of b (kc is the paper's s); thread-blocks take tiles from a
 * queue, longest first.
 *   items  : host array; a, b, f are device pointers, f_cap >= na + nb - 1
 *   r, kc  : tile shape (r in {4, 8, 16}; kc >= r); 0 = defaults
 * pm_mul_batch_create checks every item on the host, builds the task
 * table and uploads it (allocates device memory; not graph-capturable).
 * pm_mul_batch_run enqueues the batch: no allocation, no host sync, and it
 * may be captured in a hipGraph and replayed. Item coefficients must be
 * canonical residues; when d_status (device, count int32) is given, an
 * extra launch checks them and writes PM_OK or PM_ERANGE per item. f_i is
 * written in full (na_i + nb_i - 1 words). A batch object must not run on
 * two streams at once.
 */
typedef struct {
    const uint32_t *a;
    int64_t na;
    const uint32_t *b;
    int64_t nb;
    uint32_t p;
    uint32_t *f;
    int64_t f_cap;
} pm_mul_item;
typedef struct pm_mul_batch pm_mul_batch;
pm_status pm_mul_batch_create(const pm_mul_item *items, int32_t count, int32_t r, int32_t kc,
                              pm_mul_batch **out);
pm_status pm_mul_batch_run(pm_mul_batch *batch, int32_t *d_status, void *stream);
void pm_mul_batch_destroy(pm_mul_batch *batch);
/* create + run + wait + destroy */
pm_status poly_mul_modp_batch(const pm_mul_item *items, int32_t count, int32_t *d_status, void *stream);

/*
 * Euclidean division (Sec. 3, problem statement): the unique q, r with
 * a = q*b + r and deg r < deg b, for b != 0.
 *   q, q_cap : quotient (device); needs deg a - deg b + 1 words (0 when
 *              deg a < deg b); q_cap >= na - nb + 1 is checked on the host
 *              when nb > 0, the true requirement on the device
 *   r, r_cap : remainder (device); needs deg b words, or deg a + 1 when
 *              deg a < deg b
 *   nq, nr   : host; normalised lengths
 * The quotient comes from the top deg a - deg b + 1 coefficients of a, s
 * division steps per chunk (pm_params.div_s), on up to one cooperating
 * thread-block per CU; the library's scratch holds 3 na words for it.
 * Returns PM_EDIVZERO when b is the zero polynomial, PM_ERANGE for a
 * coefficient >= p.
 */
pm_status poly_divrem_modp(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb, uint32_t p,
                           uint32_t *q, int64_t q_cap, int64_t *nq, uint32_t *r, int64_t r_cap, int64_t *nr,
                           void *stream);

/*
 * Asynchronous division: the q and r of poly_divrem_modp with nothing
 * waiting for the device. The launch shapes are planned from the given
 * lengths, so b must come without high zero coefficients (b[nb - 1] != 0,
 * checked on the device: PM_EINVAL in d_status); a may have them.
 *   q_cap >= na - nb + 1, r_cap >= min(na, nb - 1) (checked on the host);
 *   q[deg a - deg b + 1 .. na - nb] is zeroed, r[0 .. min(na, nb - 1) - 1]
 *   is written in full
 *   d_nq, d_nr (int64), d_status (int32): device pointers, each may be
 *   NULL, written by the last launch; lengths are 0 after an error
 * nb = 0 returns PM_EDIVZERO before anything is enqueued; a coefficient
 * >= p gives PM_ERANGE in d_status. No host synchronisation; no allocation
 * once the stream's scratch exists (see pm_set_workspace).
 */
pm_status poly_divrem_modp_async(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb, uint32_t p,
                                 uint32_t *q, int64_t q_cap, int64_t *d_nq, uint32_t *r, int64_t r_cap,
                                 int64_t *d_nr, int32_t *d_status, void *stream);

/*
 * Greatest common divisor by the Euclidean remainder sequence (Sec. 6),
 * returned monic; gcd(a, 0) = a made monic, gcd(0, 0) = 0.
 *   g, g_cap : output (device); needs deg gcd + 1 words, at most
 *              max(deg a, deg b) + 1 (checked on the device)
 *   ng       : host; length of g
 * Up to s division steps per chunk (pm_params.gcd_s) on one cooperating
 * thread-block per 512 positions. When the degrees differ by 128 or more,
 * the first division of the sequence runs as one poly_divrem_modp-style
 * division (the chunks would take each step of a long quotient alone);
 * pm_last_gcd_stats counts its steps position by position all the same.
 * Returns PM_ERANGE for a coefficient >= p.
 */
pm_status poly_gcd_modp(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb, uint32_t p,
                        uint32_t *g, int64_t g_cap, int64_t *ng, void *stream);

/*
 * Asynchronous gcd: the monic g of poly_gcd_modp with nothing waiting for
 * the device. d_ng (int64) and d_status (int32) are device pointers (each
 * may be NULL); the length is 0 after an error. Every step runs in the
 * fused chunks: there is no leading division, so a degree gap of k costs
 * about k chunks (poly_gcd_modp divides first when k >= 128). No host
 * synchronisation; no allocation once the stream's scratch exists (see
 * pm_set_workspace).
 */
pm_status poly_gcd_modp_async(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb, uint32_t p,
                              uint32_t *g, int64_t g_cap, int64_t *d_ng, int32_t *d_status, void *stream);

/*
 * The gcd of poly_gcd_modp together with the degree sequence of its
 * Euclidean remainder sequence (Sec. 6): degs[0] = deg r0 (the operand of
 * higher degree, a on equal degrees), degs[1] = deg r1, then the degree of
 * each later remainder, ending with -1 for the zero remainder; with a zero
 * operand it is (deg of the other, -1), and (-1, -1) for two zeros.
 *   degs, degs_cap : host array; the first min(*n_degs, degs_cap) entries
 *                    are written
 *   n_degs         : host; the full length of the sequence
 * The kernel logs the shift and the reduced operand of every division step
 * it runs (Alg. 9's rule: the operand of higher degree, a on a tie); the
 * host rebuilds each step's degrees from the log and checks them
 * (PM_EDEVICE if the log is inconsistent). The remainders of the paper's
 * step sequence are associates of the textbook ones with the same degrees,
 * so this is the sequence of every correct Euclidean algorithm. Scratch:
 * about 12 (na + nb) words for the log. Synchronous.
 */
pm_status poly_gcd_modp_degrees(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb, uint32_t p,
                                uint32_t *g, int64_t g_cap, int64_t *ng, int64_t *degs, int64_t degs_cap,
                                int64_t *n_degs, void *stream);

/*
 * The first k division steps of the naive Euclidean algorithm (Sec. 6.1,
 * Alg. 9), fused s at a time as in poly_gcd_modp: a step reduces the
 * operand of higher degree (a on equal degrees) by the other,
 * X <- X - (lc X / lc Y) x^(deg X - deg Y) Y; positions whose coefficient is
 * already zero are skipped, not counted. Both operands after the steps are
 * returned made monic (the steps' own scaling is a unit, so this is
 * canonical): x from a, y from b.
 *   k          : steps to run (>= 0); fewer when an operand becomes zero
 *   x, x_cap / y, y_cap : outputs (device), each needs deg + 1 words of its
 *                operand after the steps (at most na and nb)
 *   nx, ny     : host; their lengths (0 for a zero operand)
 *   taken      : host; the steps run
 * No leading division is taken apart (unlike poly_gcd_modp): every step is
 * one of the fused chunks. Synchronous.
 */
pm_status poly_euclid_steps_modp(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb, uint32_t p,
                                 int64_t k, uint32_t *x, int64_t x_cap, int64_t *nx, uint32_t *y, int64_t y_cap,
                                 int64_t *ny, int64_t *taken, void *stream);

/*
 * Extended Euclidean algorithm (the Bezout certificate of Sec. 6's gcd):
 * monic g = gcd(a, b) and cofactors s, t with s a + t b = g. Of all such
 * pairs it returns the unique one with deg s < deg b - deg g (s = 0 when
 * deg g = deg b); for b = 0, s = 1/lc(a) and t = 0; gcd(0, 0) gives three
 * empty outputs.
 *   g, s, t  : outputs (device), with capacities g_cap, s_cap, t_cap; each
 *              needs at most max(deg a, deg b) + 1 words (checked)
 *   ng, ns, nt : host; normalised lengths
 * The remainder sequence is poly_gcd_modp's, with the cofactor of a taken
 * through every chunk's matrix; the cofactor is then reduced modulo b/g
 * when needed, and t = (g - s a)/b is one exact division (PM_EDEVICE if it
 * is not exact: an internal invariant). Host reads: a few per call.
 * Returns PM_ERANGE for a coefficient >= p.
 */
pm_status poly_xgcd_modp(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb, uint32_t p,
                         uint32_t *g, int64_t g_cap, int64_t *ng, uint32_t *s, int64_t s_cap, int64_t *ns,
                         uint32_t *t, int64_t t_cap, int64_t *nt, void *stream);

/*
 * The naive algorithms of the paper, for the s = 1 end of the sweeps over s:
 * one division step per kernel launch, each launch a global synchronisation
 * (Sec. 3, naive division, Alg. 1/2; Sec. 6, naive gcd, Alg. 8/9, with the
 * exact inverse of the divisor's leading coefficient at every step).
 * Arguments, results and errors as poly_divrem_modp and poly_gcd_modp.
 * The library's scratch holds a working copy of the inputs. They cost
 * deg a - deg b + 1 launches (division) and about 2 (deg a + deg b)
 * launches (gcd), and are not meant for production use.
 */
pm_status poly_divrem_modp_naive(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb, uint32_t p,
                                 uint32_t *q, int64_t q_cap, int64_t *nq, uint32_t *r, int64_t r_cap, int64_t *nr,
                                 void *stream);
pm_status poly_gcd_modp_naive(const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb, uint32_t p,
                              uint32_t *g, int64_t g_cap, int64_t *ng, void *stream);

/*
 * Many independent gcds in one launch (one thread-block per instance, both
 * polynomials resident in LDS for the whole remainder sequence). Items may
 * mix degrees and primes; each needs max(na, nb) <= PM_GCD_BATCH_MAX.
 *   items   : host array of `count` descriptors; a, b, g are device pointers
 *   results : host array of `count` results, filled when the call returns
 * Host checks (per item: prime, lengths, pointers) fail the whole call
 * before any device work; device checks are reported per item in
 * results[i].status. Synchronous.
 */
#define PM_GCD_BATCH_MAX 17408
typedef struct {
    const uint32_t *a;
    int64_t na;
    const uint32_t *b;
    int64_t nb;
    uint32_t p;
    uint32_t *g;
    int64_t g_cap;
} pm_gcd_item;
typedef struct {
    int64_t ng;       /* length of the monic gcd                          */
    int64_t steps;    /* Euclidean division steps                         */
    int64_t updates;  /* coefficient updates, (deg divisor + 1) per step  */
    int64_t chunks;   /* fused chunks                                     */
    int32_t status;   /* PM_OK or the item's device-side error            */
    int32_t done;     /* 1 once the item finished                         */
    int64_t nr;       /* 0 (the server's division requests use it)        */
} pm_gcd_result;
pm_status poly_gcd_modp_batch(const pm_gcd_item *items, int32_t count, pm_gcd_result *results, void *stream);
/*
 * The same batch prepared once and run many times (for hipGraph capture):
 * pm_gcd_batch_create checks every item on the host, orders the items
 * longest first within each of the two block shapes, and uploads the job
 * table (allocates device memory, synchronous; not graph-capturable).
 * s: division steps per chunk, 0..256 (0 = 128).
 * pm_gcd_batch_run enqueues one launch per block shape (at most two): no
 * allocation, no host work, no memset, so it may be captured in a hipGraph
 * and replayed; every run rewrites each item's g and result in full.
 * pm_gcd_batch_results copies the results of the last run to the host
 * (synchronous). A batch object must not run on two streams at once.
 */
typedef struct pm_gcd_batch pm_gcd_batch;
pm_status pm_gcd_batch_create(const pm_gcd_item *items, int32_t count, int32_t s, pm_gcd_batch **out);
pm_status pm_gcd_batch_run(pm_gcd_batch *batch, void *stream);
pm_status pm_gcd_batch_results(pm_gcd_batch *batch, pm_gcd_result *results, void *stream);
void pm_gcd_batch_destroy(pm_gcd_batch *batch);

/*
 * Server with continuous batching of gcd and division requests. Requests
 * of mixed degree (up to PM_GCD_BATCH_MAX terms per operand), prime and
 * kind are queued by pm_server_submit (inputs are copied; the caller may
 * reuse its arrays at once). pm_server_submit and pm_server_poll admit
 * queued requests in arrival order while a slot (max_inflight) and room in
 * the device-memory arena (arena_words) for the request's inputs, and in
 * the host output arena for its outputs, are free. An admitted request's
 * inputs are copied into the device arena (one copy per contiguous run of
 * an admission pass, on an SDMA engine, so that the copies need no CU);
 * the request is published to the GPU once its copy has completed.
 * pm_server_poll returns the requests that finished since the last poll.
 * Two persistent worker kernels run the published requests, one thread-
 * block each, taking the next one as soon as one finishes, so requests
 * join and leave the GPU individually: blocks of 1024 threads (one per
 * CU) take any request, and when large_blocks leaves CUs free, blocks of
 * 256 threads (several per CU) take those whose operands fit 4096 terms.
 * Each request's remainder sequence
 * (or division) stays in its block's LDS until its results are written to
 * the caller's host buffers (done by the time the completion is returned).
 * The workers stop by themselves after an idle period and are relaunched
 * when work arrives (the 1024-thread worker first, so that the other
 * fills the CUs it leaves); pm_server_destroy stops them and waits.
 * Not thread-safe: one host thread drives a server. Times are milliseconds
 * on the server's steady clock.
 */
typedef struct pm_server pm_server;
typedef struct {
    int32_t max_inflight;  /* requests admitted at once (0 = 4096)                       */
    int32_t large_blocks;  /* blocks of the 1024-thread worker (0 = one per CU)          */
    int64_t arena_words;   /* device words for resident inputs (0 = 32 Mi, or less when
                            * the device has less than 8 times that free); the host
                            * output arena has as many words                              */
    int32_t s;             /* Euclidean steps fused per chunk (0 = 128)                   */
    int32_t small_blocks;  /* blocks of the 256-thread worker (0 = fill the other CUs,
                            * -1 = none: every request on the 1024-thread worker)         */
    int32_t staging;       /* where the workers read inputs: 0 = the device arena when an
                            * SDMA engine can fill it, else pinned host memory; 1 = the
                            * device arena (PM_EDEVICE without an SDMA engine); 2 = the
                            * pinned host mirror, read over the bus                        */
    int32_t reserved;
} pm_server_opts;
/* A request: op PM_OP_GCD (or 0) asks for the monic gcd of a and b, written
 * to g; PM_OP_DIVREM asks for the division of a by b (Sec. 3's problem:
 * a = q b + r, deg r < deg b), q written to g and r to r. */
typedef struct {
    const uint32_t *a;     /* host arrays */
    int64_t na;
    const uint32_t *b;
    int64_t nb;
    uint32_t p;
    uint32_t *g;           /* host output, g_cap words: the gcd, or q      */
    int64_t g_cap;
    uint64_t tag;          /* returned in the completion */
    int32_t op;            /* PM_OP_GCD (0 also) or PM_OP_DIVREM          */
    int32_t reserved;
    uint32_t *r;           /* division: host output r, r_cap words        */
    int64_t r_cap;
} pm_gcd_request;
typedef pm_gcd_request pm_request;
typedef struct {
    uint64_t ticket;
    uint64_t tag;
    int32_t status;
    int32_t op;            /* the request's op                           */
    int64_t ng;            /* length of the gcd, or of q                 */
    int64_t steps;
    int64_t updates;
    double t_submit_ms;    /* pm_server_submit                          */
    double t_start_ms;     /* published to the GPU                      */
    double t_done_ms;      /* seen finished by pm_server_poll           */
    int64_t nr;            /* division: length of r                     */
} pm_completion;
pm_status pm_server_create(const pm_server_opts *opts, pm_server **out);
/* Errors found on the host (bad buffers, a request above PM_GCD_BATCH_MAX
 * terms or above the whole arena, a modulus that is not a prime below 2^30,
 * b = 0 with nb = 0 for a division) return at once and queue nothing;
 * errors found on the device (a coefficient >= p, a zero divisor, outputs
 * too short for the true degrees) come back in the completion's status. */
pm_status pm_server_submit(pm_server *srv, const pm_gcd_request *req, uint64_t *ticket);
/* count requests in one call (tickets: count entries, or NULL); all are
 * checked first, so an error queues none of them. The requests of one call
 * are queued longest first (by na * nb; equal ones in the given order), so
 * their tickets need not increase in the given order. */
pm_status pm_server_submit_batch(pm_server *srv, const pm_gcd_request *reqs, int32_t count, uint64_t *tickets);
pm_status pm_server_poll(pm_server *srv, pm_completion *out, int32_t max, int32_t *n);
int64_t pm_server_pending(pm_server *srv);   /* queued + on the device */
void pm_server_destroy(pm_server *srv);

/* Statistics of the last poly_gcd_modp call on this thread. */
typedef struct {
    int64_t steps;    /* Euclidean division steps                        */
    int64_t updates;  /* coefficient updates, (deg divisor + 1) per step */
    int64_t chunks;   /* fused chunks, one grid barrier each             */
} pm_gcd_stats;
void pm_last_gcd_stats(pm_gcd_stats *out);

/*
 * Tuning (the paper's program parameter s).
 *   mul_s   : b-coefficients per thread-block in the product (0 = default)
 *   mul_r   : outputs per thread in the product (1,2,4,8,16,32; 0 = default)
 *   div_s   : division steps fused per chunk of the quotient (1..64; 0 = 64)
 *   gcd_s   : Euclidean steps fused per chunk (1..256; 0 = 128)
 *   mul_engine : which kernels compute a product (poly_mul_modp and
 *             poly_mul_modp_async): 0 = automatic (the matrix cores for
 *             products with n_a * n_b >= 40e6 and min(n_a, n_b) >= 256
 *             unless mul_s or mul_r is set), 1 = the VALU tile kernels
 *             (Sec. 5's layout, tuned by mul_s and mul_r), 2 = the matrix
 *             cores (int8 digit products; s fixed at 4096). The matrix
 *             cores take a product only where their int32 digit sums stay
 *             exact (pm_mul_plan); the VALU tiles take the rest. Results
 *             are identical.
 * The settings are per process and apply to later calls.
 */
typedef struct {
    int32_t mul_s;
    int32_t mul_r;
    int32_t div_s;
    int32_t gcd_s;
    int32_t mul_engine;
} pm_params;
pm_status pm_set_params(const pm_params *params);
void pm_get_params(pm_params *params);

/*
 * Loads tuned parameters from a text file (paper_1402_0264_amd.tune writes
 * one): lines "name value" (or "name = value") for any of mul_s, mul_r,
 * div_s, gcd_s and mul_engine; '#' starts a comment; names not given keep
 * their current values. The values are checked as pm_set_params checks
 * them, and on any error (unreadable file, unknown name, bad value) nothing
 * changes and PM_EINVAL is returned.
 */
pm_status pm_autotune_load(const char *path);

/*
 * The plan poly_mul_modp and poly_mul_modp_async take for a product of
 * na x nb terms on the current device under the current pm_params
 * (diagnostics; nothing is enqueued): the engine (PM_MUL_VALU or
 * PM_MUL_MFMA, 0 when an operand is empty); for the VALU tiles the outputs
 * per thread r and the b-chunk s; for the matrix cores s = 4096, the
 * work-groups and the most groups of 8 block offsets one work-group sums
 * (at most 64, the bound that keeps the int32 digit sums exact); and the
 * scratch words.
 */
enum { PM_MUL_AUTO = 0, PM_MUL_VALU = 1, PM_MUL_MFMA = 2 };
typedef struct {
    int32_t engine;
    int32_t r;
    int64_t s;
    int64_t scratch_words;
    int64_t work_groups;
    int64_t max_share_groups;
} pm_mul_plan_info;
pm_status pm_mul_plan(int64_t na, int64_t nb, pm_mul_plan_info *out);

/*
 * Caller workspace. pm_set_workspace gives a stream on the current device
 * a device buffer of `words` uint32 words (256-byte aligned, at least 64
 * words) from which every later call on that stream takes its scratch and
 * its device-side result record instead of the library's pool; a call that
 * needs more returns PM_ENOMEM and allocates nothing. With a workspace of
 * pm_workspace_size(op, na, nb) words (for the largest sizes to come) set,
 * poly_mul_modp_async (PM_OP_MUL), poly_divrem_modp_async (PM_OP_DIVREM)
 * and poly_gcd_modp_async (PM_OP_GCD) allocate nothing, also on their
 * first call (inside hipGraph capture, for instance). The synchronous entry
 * points still copy their results through a pinned host record, and the
 * extended gcd, the gcd's step log and its leading division keep auxiliary
 * buffers of the library. The sizes follow the current device and
 * pm_params. pm_set_workspace waits for the stream and zeroes the first 64
 * words; the caller keeps the buffer alive, and used by nothing else, while
 * it is set. d_words = NULL with words = 0 returns the stream to the pool;
 * pm_release drops every workspace.
 */
enum { PM_OP_MUL = 0, PM_OP_DIVREM = 1, PM_OP_GCD = 2 };
pm_status pm_workspace_size(int32_t op, int64_t na, int64_t nb, int64_t *words);
pm_status pm_set_workspace(void *stream, void *d_words, int64_t words);

/*
 * Kernel timing (diagnostics). While enabled, every kernel launch of the
 * library is bracketed by two HIP events recorded on its launch stream
 * (no host synchronisation). pm_timing_read waits for the recorded launches
 * of the kernel with the given function name (e.g. "mul_tile_kernel",
 * "mul_reduce_kernel", "gcd_kernel") and returns their count and total
 * elapsed milliseconds. pm_timing_reset drops the records.
 */
void pm_timing_enable(int on);
pm_status pm_timing_read(const char *kernel, int64_t *launches, double *total_ms);
void pm_timing_reset(void);

/* Frees the scratch pool of every device and stream, including buffers that
 * larger calls outgrew (they are kept until here, since a captured graph
 * may still use them), and drops every caller workspace. */
void pm_release(void);

/* Thread-local description of the last non-OK status. */
const char *pm_last_error(void);

/*
 * Radix sort (Sec. 4, the paper's third case study): the stable sort of n
 * uint32 keys on their low key_bits bits (1..32), least significant digit
 * first with digits of s bits (1..10; 0 = 8), in ceil(key_bits/s) passes.
 * Each pass is a digit histogram per tile of 4096 keys, an exclusive prefix
 * sum over the histograms (digit-major), and a stable scatter through LDS.
 *   keys, vals       : input (device), n words each; vals may be NULL
 *   keys_out, vals_out : output (device), n words each; vals_out is needed
 *                    when vals is given; no output may overlap an input or
 *                    the other output
 * n <= 2^32 - 1. Asynchronous on the stream: no host read; the library's
 * scratch holds (1 or 2) n + 2^s n / 4096 words. Returns PM_EINVAL for bad
 * arguments.
 */
pm_status pm_radix_sort_u32(const uint32_t *keys, const uint32_t *vals, int64_t n, int32_t key_bits, int32_t s,
                            uint32_t *keys_out, uint32_t *vals_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* POLYMODP_H */
