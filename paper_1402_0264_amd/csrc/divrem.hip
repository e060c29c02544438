// divrem.hip -- Euclidean division of dense polynomials over Z/pZ on gfx950
// (Sec. 3: naive and optimized division).
//
// The quotient q depends only on the top mu = deg a - deg b + 1 coefficients
// of a (the head) and on b: step i of the long division takes the current
// leading coefficient of the head, multiplies it by lc(b)^{-1} to get one
// quotient coefficient, and subtracts that multiple of the shifted b. As in
// the paper's optimized division the steps are fused s at a time (a chunk):
// the s quotient terms of a chunk depend only on the chunk's s-head, and are
// then applied to the rest of the head at once.
//
// Inside a chunk the s steps form a triangular Toeplitz system: with
// beta_d = b[deg b - d] (0 beyond deg b), the chunk's head values v_j and its
// quotient terms q_j satisfy sum_{i<=j} beta_{j-i} q_i = v_j. So
// q = G * v mod x^s, where G is the inverse of sum_d beta_d x^d modulo x^64;
// G is computed once per division (64 serial steps on one wave), and every
// chunk's s steps become one lower-triangular product with no serial chain.
//
// The head is cut into tiles of s positions (tile c is chunk c's s-head) and
// runs of K tiles; run r belongs to block r mod B. A block keeps its runs up
// to date by applying published quotient terms; when all chunks above its
// next run are applied it leads that run: it computes the run's chunks one
// after the other, applying each to the rest of the run at once, and
// publishes every quotient term. Blocks meet only through these published
// terms (64-bit words whose high word marks them written), so there is no
// grid-wide barrier, and one block's K chunks pass without any hand-off.
//
// The part of a below deg b only ever receives updates, never feeds a
// decision, so it is done afterwards in one fully parallel launch:
// r_k = a_k - sum_t q_t b_{k-t} for k < deg b, a product with a subtracting
// epilogue (mul_mfma.hip or mul.hip).
#include "internal.hpp"

namespace pm {
namespace {

// Degrees (largest non-zero index) of a and b, by two waves scanning from
// the top; resets the call's results. The range check runs in
// zero_check_kernel, next in the stream, on many blocks.
__global__ __launch_bounds__(256) void degrees_kernel(const uint32_t* a, int64_t na, const uint32_t* b,
                                                      int64_t nb, CallInfo* info) {
    const int wave = threadIdx.x >> 6;
    if (wave < 2) {
        const int64_t d = top_nonzero_wave(wave == 0 ? a : b, wave == 0 ? na : nb);
        if ((threadIdx.x & 63) == 0) {
            if (wave == 0) info->deg_a = d;
            else info->deg_b = d;
        }
    }
    if (threadIdx.x == 0) {
        info->status = 0;
        info->flags = 0;
        info->n0 = info->n1 = 0;
        info->steps = info->chunks = info->updates = 0;
    }
}

// Clears the published-term words and checks every coefficient of a and b
// against p (info->flags = 1 when one is not a residue).
__global__ __launch_bounds__(256) void zero_check_kernel(uint64_t* qlog, int64_t nq, const uint32_t* a, int64_t na,
                                                         const uint32_t* b, int64_t nb, uint32_t p, CallInfo* info) {
    int bad = 0;
    const int64_t n = nq > na ? (nq > nb ? nq : nb) : (na > nb ? na : nb);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        if (i < nq) qlog[i] = 0;
        if (i < na) bad |= a[i] >= p;
        if (i < nb) bad |= b[i] >= p;
    }
    bad = __syncthreads_or(bad);
    if (bad && threadIdx.x == 0) atomicOr(&info->flags, 1);
}

constexpr int DIVF_QB = 4096;                   // quotient terms one batch holds in LDS
constexpr int DIVF_RUN = 384;                   // head positions per run, rounded up to whole tiles
constexpr int DIVF_RMAX = DIVF_RUN + 64;        // most positions of a run
constexpr int DIVF_BW = DIVF_QB + DIVF_RMAX + 8;  // distance window of one batch
constexpr int DIVF_GRP = 8;                     // products summed between folds (p < 2^30)

struct DivFlow {
    const uint32_t* a;
    const uint32_t* b;
    Field F;
    uint32_t* q;
    int64_t q_cap, r_cap;
    uint32_t* h;        // head of a, updated in place; a run is touched by its owner only
    uint64_t* qlog;     // published quotient terms: (1 << 32) | q[y]; 0 = not yet
    CallInfo* info;
    int S, K;           // chunk (tile) size, tiles per run
};

__device__ __forceinline__ uint64_t qlog_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void qlog_store(uint64_t* p, uint32_t v) {
    __hip_atomic_store(p, (1ull << 32) | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Geometry of the head: tile t holds head indices lo(t) .. hi(t), from the
// top down (tile t is chunk t's s-head); run r holds tiles rK .. rK+K-1.
struct DivGeom {
    int64_t mu, nt, runs;
    int S, K;
    __device__ int64_t hi(int64_t t) const { return mu - 1 - t * S; }
    __device__ int64_t lo(int64_t t) const {
        int64_t l = mu - (t + 1) * S;
        return l < 0 ? 0 : l;
    }
    __device__ int64_t run_end(int64_t r) const {
        int64_t e = (r + 1) * K;
        return e < nt ? e : nt;
    }
};

// The two sums over k = k0 .. k1 of sQ[k] beta(dd - k) and sQ[k] beta(dd + 1
// - k), where beta(d) = w[d] (w points at beta(0) of a staged window): the
// updates of two neighbouring positions x and x - 1 with dd = yhi - x, one
// window read per two products. Even and odd k go to separate lazy sums
// (four independent chains), each folded after at most DIVF_GRP products.
__device__ __forceinline__ void pair_sums(const uint32_t* sQ, const uint32_t* w, int64_t dd, int k0, int k1,
                                          const Field& F, uint32_t& r0, uint32_t& r1) {
    const uint32_t* wd = w + dd;  // wd[-k] = beta(dd - k)
    uint32_t hi = wd[1 - k0];
    uint64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    int k = k0;
    for (; k + 2 * DIVF_GRP <= k1 + 1; k += 2 * DIVF_GRP) {
#pragma unroll
        for (int u = 0; u < 2 * DIVF_GRP; u++) {
            const uint32_t lo = wd[-(k + u)];
            const uint32_t qv = sQ[k + u];
            if (u & 1) {
                b0 += (uint64_t)qv * lo;
                b1 += (uint64_t)qv * hi;
            } else {
                a0 += (uint64_t)qv * lo;
                a1 += (uint64_t)qv * hi;
            }
            hi = lo;
        }
        a0 = fold(a0, F.c32);
        a1 = fold(a1, F.c32);
        b0 = fold(b0, F.c32);
        b1 = fold(b1, F.c32);
    }
    for (int u = 0; k <= k1; k++, u ^= 1) {  // fewer than 2 DIVF_GRP left
        const uint32_t lo = wd[-k];
        const uint32_t qv = sQ[k];
        if (u) {
            b0 += (uint64_t)qv * lo;
            b1 += (uint64_t)qv * hi;
        } else {
            a0 += (uint64_t)qv * lo;
            a1 += (uint64_t)qv * hi;
        }
        hi = lo;
    }
    r0 = reduce64(fold(a0, F.c32) + fold(b0, F.c32), F);
    r1 = reduce64(fold(a1, F.c32) + fold(b1, F.c32), F);
}

// h[x] -= sum_{y = ylo..yhi} q[y] beta(y - x) for xlo <= x <= xhi (all below
// ylo), sQ[k] = q[yhi - k], h in device memory: the distances the batch
// spans are staged in sBw first. Called by the whole block; ends
// synchronized.
__device__ void apply_batch(uint32_t* h, const uint32_t* b, int64_t db, const uint32_t* sQ, uint32_t* sBw,
                            int64_t xlo, int64_t xhi, int64_t ylo, int64_t yhi, const Field& F) {
    const int tid = threadIdx.x;
    const int64_t dbase = ylo - xhi;
    const int64_t n = yhi - xlo + 2 - dbase;
    for (int64_t j = tid; j < n; j += DIV_THREADS) {
        const int64_t d = dbase + j;
        sBw[j] = d <= db ? b[db - d] : 0u;
    }
    __syncthreads();
    const uint32_t* w = sBw - dbase;
    const int k1 = (int)(yhi - ylo);
    for (int64_t x = xhi - 2 * tid; x >= xlo; x -= 2 * DIV_THREADS) {
        const int64_t dd = yhi - x;
        const int64_t k0 = dd - db > 0 ? dd - db : 0;  // beyond deg b: no update
        if (k0 > k1) continue;
        uint32_t r0, r1;
        pair_sums(sQ, w, dd, (int)k0, k1, F, r0, r1);
        h[x] = submod(h[x], r0, F.p);
        if (x - 1 >= xlo) h[x - 1] = submod(h[x - 1], r1, F.p);
    }
    __syncthreads();
}

// Copies the published terms of chunks c0 .. cmax-1 into sQ (sQ[k] = q[hi(c0)
// - k]) and returns the end of the prefix of complete chunks (c0 if chunk c0
// is not complete yet). Loads DIV_THREADS words per round and stops after
// the first round with a missing word. Called by the whole block; ends
// synchronized.
__device__ int64_t take_terms(const uint64_t* qlog, const DivGeom& G, int64_t c0, int64_t cmax, uint32_t* sQ,
                              int* s_word) {
    const int tid = threadIdx.x;
    const int64_t top = G.hi(c0);
    const int64_t n = top - G.lo(cmax - 1) + 1;  // words of chunks c0 .. cmax-1
    if (tid == 0) *s_word = 0x7fffffff;
    __syncthreads();
    int64_t first = n;
    for (int64_t k0 = 0; k0 < n; k0 += DIV_THREADS) {
        const int64_t k = k0 + tid;
        if (k < n) {
            const uint64_t w = qlog_load(qlog + top - k);
            if ((w >> 32) == 0) atomicMin(s_word, (int)k);
            sQ[k] = (uint32_t)w;
        }
        __syncthreads();
        const int sw = *s_word;
        __syncthreads();  // every wave has read it before the next round may lower it
        if (sw != 0x7fffffff) {
            first = sw;
            break;
        }
    }
    return first >= n ? cmax : c0 + first / G.S;
}

// sum_{i < 8 NG} x[i] y[i] for a register row x and a row y broadcast from
// LDS (zero past the values in use): up to four independent lazy sums, one
// per group of DIVF_GRP products in turn, each folded after its group.
template <int NG>
__device__ __forceinline__ uint32_t dot_groups(const uint32_t (&x)[64], const uint32_t* y, const Field& F) {
    constexpr int A = NG < 4 ? NG : 4;
    uint64_t acc[A];
#pragma unroll
    for (int j = 0; j < A; j++) acc[j] = 0;
#pragma unroll
    for (int g = 0; g < NG; g++) {
#pragma unroll
        for (int u = 0; u < DIVF_GRP; u++)
            acc[g % A] += (uint64_t)x[g * DIVF_GRP + u] * y[g * DIVF_GRP + u];
        acc[g % A] = fold(acc[g % A], F.c32);
    }
    // folded sums are below 2^32 p < 2^62: pairwise folds keep the total in range
    uint64_t t = acc[0];
#pragma unroll
    for (int j = 1; j < A; j++) t = fold(t + acc[j], F.c32);
    return reduce64(t, F);
}

// Leads run f (tiles t0 .. t1-1, head values in sH[i] = h[hi(t0) - i]) from
// chunk cstart: t0 itself for the first run, else t0 - 1, whose published
// terms the caller has put in sQ[0 .. S-1]. Every iteration c: wave 0 puts
// chunk c into tile c+1 (the only tile the next terms need) and computes
// tile c+1's terms; waves 1-3 meanwhile apply chunk c to the tiles below.
template <int NG>
__device__ void lead_run(const DivFlow& D, const DivGeom& G, const Field& F, int64_t db, int64_t t0, int64_t t1,
                         int64_t cstart, int rlen, uint32_t* sH, uint32_t* sQ, uint32_t* sV, const uint32_t* sGp,
                         const uint32_t* sBr) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int S = G.S;
    const int64_t rhi = G.hi(t0);
    uint32_t greg[64], breg[64];
    if (wave == 0) {
#pragma unroll
        for (int i = 0; i < 8 * NG; i++) {
            greg[i] = sGp[64 + lane - i];  // G_{lane - i}, zero above the diagonal
            breg[i] = sBr[S - i + lane];   // beta(S + lane - k): chunk c to tile c+1
        }
        if (cstart == t0) {
            const int cs = (int)(rhi - G.lo(t0) + 1);
            sV[lane] = lane < cs ? sH[lane] : 0u;
            const uint32_t qj = dot_groups<NG>(greg, sV, F);
            if (lane < cs) {
                D.q[rhi - lane] = qj;
                qlog_store(D.qlog + rhi - lane, qj);
            }
            sQ[lane] = lane < cs ? qj : 0u;  // whole groups of 8 read past cs
        } else if (lane >= S) {
            sQ[lane] = 0;
        }
    }
    __syncthreads();
    for (int64_t c = cstart; c + 1 < t1; c++) {
        const int ic = (int)(c - t0) * S;  // sH index of chunk c's top (-S for t0 - 1)
        const uint32_t* qc = sQ + ((c - cstart) & 1) * 64;
        uint32_t* qn = sQ + ((c + 1 - cstart) & 1) * 64;
        if (wave == 0) {
            const int64_t top = G.hi(c + 1);
            const int cs = (int)(top - G.lo(c + 1) + 1);
            const uint32_t upd = dot_groups<NG>(breg, qc, F);  // qc is zero past S
            sV[lane] = lane < cs ? submod(sH[ic + S + lane], upd, F.p) : 0u;
            const uint32_t qj = dot_groups<NG>(greg, sV, F);
            if (lane < cs) {
                D.q[top - lane] = qj;
                qlog_store(D.qlog + top - lane, qj);
            }
            qn[lane] = lane < cs ? qj : 0u;
        } else {
            // chunk c to the run's positions from tile c+2 on, within deg b
            int iend = ic + S + (int)(db < DIVF_RMAX ? db : DIVF_RMAX) + 1;
            if (iend > rlen) iend = rlen;
            for (int i = ic + 2 * S + 2 * (tid - 64); i < iend; i += 2 * (DIV_THREADS - 64)) {
                uint32_t r0, r1;
                pair_sums(qc, sBr, i - ic, 0, S - 1, F, r0, r1);
                sH[i] = submod(sH[i], r0, F.p);
                if (i + 1 < rlen) sH[i + 1] = submod(sH[i + 1], r1, F.p);
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(DIV_THREADS) void divrem_flow_kernel(DivFlow D) {
    __shared__ uint32_t sGp[128];                 // sGp[64 + k] = G_k, zeros below
    __shared__ uint32_t sBrp[64 + DIVF_RMAX + 72];  // zeros, then beta(d) for the distances of a lead
    uint32_t* const sBr = sBrp + 64;
    __shared__ uint32_t sH[DIVF_RMAX];       // the run being led: sH[i] = h[hi(first tile) - i]
    __shared__ uint32_t sV[64];
    __shared__ uint32_t sQ[DIVF_QB];
    __shared__ uint32_t sBw[DIVF_BW];
    __shared__ int s_word;
    const Field F = D.F;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    CallInfo* info = D.info;
    const int64_t da = info->deg_a, db = info->deg_b;  // from degrees_kernel
    int status = info->flags ? -3 /* PM_ERANGE */ : info->status;
    if (status == 0 && db < 0) status = -4;                  // PM_EDIVZERO
    const int64_t mu = (status == 0 && da >= db) ? da - db + 1 : 0;
    const int64_t nr_max = (da < db) ? da + 1 : db;          // room the remainder may need
    if (status == 0 && (mu > D.q_cap || nr_max > D.r_cap)) status = -1;  // PM_EINVAL
    DivGeom G;
    G.mu = mu;
    G.S = D.S;
    G.K = D.K;
    G.nt = (mu + G.S - 1) / G.S;
    G.runs = (G.nt + G.K - 1) / G.K;
    if (blockIdx.x == 0 && tid == 0) {
        info->status = status;
        info->n0 = status == 0 ? mu : 0;
        info->n1 = 0;
        info->chunks = status == 0 ? G.nt : 0;
        info->steps = status == 0 ? mu : 0;
        info->updates = status == 0 ? mu * (db + 1) : 0;
    }
    if (status != 0 || mu == 0) return;
    const int64_t B = gridDim.x, me = blockIdx.x;
    if (me >= G.runs) return;
    const int S = G.S;
    const int KS = G.K * S;  // <= DIVF_RMAX - 1

    // the head of a over this block's runs: h[x] = a[deg b + x]
    for (int64_t r = me; r < G.runs; r += B) {
        const int64_t xlo = G.lo(G.run_end(r) - 1), xhi = G.hi(r * G.K);
        for (int64_t x = xlo + tid; x <= xhi; x += DIV_THREADS) D.h[x] = D.a[db + x];
    }
    for (int d = tid; d < KS + S + 2; d += DIV_THREADS) sBr[d] = d <= db ? D.b[db - d] : 0u;
    if (tid < 64) {
        sBrp[tid] = 0;
        sGp[tid] = 0;
    }
    __syncthreads();
    // G = (sum_{d<64} beta_d x^d)^{-1} mod x^64 by 64 division steps on the
    // series 1: lane k holds the pending coefficient of x^k
    if (wave == 0) {
        const uint32_t inv = invmod(sBr[0], F);
        uint32_t val = lane == 0 ? 1u : 0u;
        for (int j = 0; j < 64; j++) {
            const uint32_t gj = mulmod((uint32_t)__builtin_amdgcn_readlane((int)val, j), inv, F);
            if (lane > j) val = submod(val, mulmod(gj, sBr[lane - j], F), F.p);
            if (lane == j) sGp[64 + j] = gj;
        }
    }
    __syncthreads();

    int64_t f = me;       // front run: the next one this block leads
    int64_t cf = 0;       // chunks applied to the front run
    int64_t cr = 0;       // chunks applied to every later run of this block
    bool staged = false;  // the front run is in sH (its turn is next)
    const int64_t sub = (DIVF_RUN + S - 1) / S;  // chunks per batch for the later runs
    const int64_t qb_chunks = DIVF_QB / S;
    while (f < G.runs) {
        const int64_t t0 = f * G.K, t1 = G.run_end(f);
        const int64_t rlo = G.lo(t1 - 1), rhi = G.hi(t0);
        const int rlen = (int)(rhi - rlo + 1);
        bool lead = cf == t0;  // the first run
        if (!lead && staged && cf == t0 - 1)
            lead = take_terms(D.qlog, G, cf, t0, sQ, &s_word) == t0;  // the last terms of the run above
        if (lead) {
            if (!staged)
                for (int i = tid; i < rlen; i += DIV_THREADS) sH[i] = D.h[rhi - i];
            staged = false;
            __syncthreads();
            const int64_t cstart = cf;
            switch ((S + DIVF_GRP - 1) / DIVF_GRP) {
                case 1: lead_run<1>(D, G, F, db, t0, t1, cstart, rlen, sH, sQ, sV, sGp, sBr); break;
                case 2: lead_run<2>(D, G, F, db, t0, t1, cstart, rlen, sH, sQ, sV, sGp, sBr); break;
                case 3:
                case 4: lead_run<4>(D, G, F, db, t0, t1, cstart, rlen, sH, sQ, sV, sGp, sBr); break;
                default: lead_run<8>(D, G, F, db, t0, t1, cstart, rlen, sH, sQ, sV, sGp, sBr); break;
            }
            f += B;
            cf = cr;  // the new front is a later run: it has the chunks before cr
            continue;
        }
        if (staged && cf == t0 - 1) {
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        if (!staged && cf >= t0 - G.K) {
            // only the run just above is left: move the front run and the
            // distances its last updates span (below 2 K s + 2) into LDS,
            // so that the hand-off needs no memory round trip but the terms
            for (int i = tid; i < rlen; i += DIV_THREADS) sH[i] = D.h[rhi - i];
            for (int d = tid; d < 2 * KS + 2; d += DIV_THREADS) sBw[d] = d <= db ? D.b[db - d] : 0u;
            staged = true;
            __syncthreads();
        }
        // chunks published by other blocks, for the front run
        int64_t cmax = cf + qb_chunks < t0 ? cf + qb_chunks : t0;
        if (!staged && cmax > t0 - G.K) cmax = t0 - G.K;  // reach the hand-off staged
        if (staged && cmax > t0 - 1) cmax = t0 - 1;         // the lead takes the last chunk
        int64_t c1 = take_terms(D.qlog, G, cf, cmax, sQ, &s_word);
        if (c1 > cf) {
            if (staged) {
                const int64_t yhi = G.hi(cf);
                const int k1 = (int)(yhi - G.lo(c1 - 1));
                for (int i = 2 * tid; i < rlen; i += 2 * DIV_THREADS) {
                    const int64_t dd = yhi - rhi + i;  // distance of position rhi - i to yhi
                    const int64_t k0 = dd - db > 0 ? dd - db : 0;
                    if (k0 > k1) continue;
                    uint32_t r0, r1;
                    pair_sums(sQ, sBw, dd, (int)k0, k1, F, r0, r1);
                    sH[i] = submod(sH[i], r0, F.p);
                    if (i + 1 < rlen) sH[i + 1] = submod(sH[i + 1], r1, F.p);
                }
                __syncthreads();
            } else {
                apply_batch(D.h, D.b, db, sQ, sBw, rlo, rhi, G.lo(c1 - 1), G.hi(cf), F);
            }
            cf = c1;
            continue;
        }
        // nothing new: bring the later runs forward while the front's turn is far
        if (cr < cf && t0 - cf > 2 * G.K && f + B < G.runs) {
            cmax = cr + sub < cf ? cr + sub : cf;
            c1 = take_terms(D.qlog, G, cr, cmax, sQ, &s_word);  // all published: c1 = cmax
            for (int64_t r = f + B; r < G.runs; r += B)
                apply_batch(D.h, D.b, db, sQ, sBw, G.lo(G.run_end(r) - 1), G.hi(r * G.K), G.lo(c1 - 1), G.hi(cr),
                            F);
            cr = c1;
            continue;
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

// out = r + q_0 y over n terms (r has nr <= n terms): what remains of the
// dividend when the division steps stop one position early, above the
// divisor's degree instead of at it (the gcd's tie rule, Sec. 6).
__global__ __launch_bounds__(256) void fold_q0_kernel(const uint32_t* r, int64_t nr, const uint32_t* q,
                                                      const uint32_t* y, int64_t n, uint32_t* out, Field F) {
    const uint32_t q0 = q[0];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint32_t ri = i < nr ? r[i] : 0u;
        out[i] = addmod(ri, mulmod(q0, y[i], F), F.p);
    }
}

// out[i] = -x[i] for i < n; out[0] = 0 when drop0 (the cofactor of a in
// b - (q - q_0) a after the gcd's leading division)
__global__ __launch_bounds__(256) void negate_kernel(const uint32_t* x, int64_t n, uint32_t* out, uint32_t p,
                                                     int drop0) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = (drop0 && i == 0) ? 0u : submod(0u, x[i], p);
}

// out[i] = x[i] - y[i] for i < n, x read as zero past nx and y past ny
__global__ __launch_bounds__(256) void sub_kernel(const uint32_t* x, int64_t nx, const uint32_t* y, int64_t ny,
                                                  int64_t n, uint32_t* out, uint32_t p) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = submod(i < nx ? x[i] : 0u, i < ny ? y[i] : 0u, p);
}

// Between the quotient and the remainder product of the asynchronous
// division, whose product shape is planned from the given lengths: q is
// zeroed past the true quotient length up to the q_plan words the product
// reads, and a divisor whose given top coefficient b[nb - 1] is zero is
// refused (the product would miss the true degree of b).
__global__ __launch_bounds__(256) void divrem_async_fix_kernel(uint32_t* q, int64_t q_plan, const uint32_t* b,
                                                               int64_t nb, CallInfo* info) {
    const int64_t mu = info->n0;  // 0 after an error
    for (int64_t i = mu + (int64_t)blockIdx.x * 256 + threadIdx.x; i < q_plan; i += (int64_t)gridDim.x * 256)
        q[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0 && info->status == 0 && nb > 0 && b[nb - 1] == 0u)
        info->status = -1;  // PM_EINVAL
}

// An asynchronous call's results, from the call's device record to the
// caller's device words (any of them may be null); lengths are 0 on error.
__global__ void info_export_kernel(const CallInfo* info, int64_t* d_n0, int64_t* d_n1, int32_t* d_status) {
    const int32_t st = info->status;
    if (d_status) *d_status = st;
    if (d_n0) *d_n0 = st == 0 ? info->n0 : 0;
    if (d_n1) *d_n1 = st == 0 ? info->n1 : 0;
}

__global__ __launch_bounds__(256) void trim_kernel(const uint32_t* r, int64_t n, CallInfo* info) {
    if (threadIdx.x < 64) {
        int64_t d = top_nonzero_wave(r, n);
        if (threadIdx.x == 0) info->n1 = d + 1;
    }
}

}  // namespace

hipError_t divrem_head_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, const Field& F,
                              uint32_t* q, int64_t q_cap, int64_t r_cap, uint32_t* head, CallInfo* info,
                              int s, int num_cus, hipStream_t stream) {
    if (s < 1) s = 1;
    if (s > 64) s = 64;
    const int64_t words = na > 0 ? na : 1;
    DivFlow D;
    D.a = a;
    D.b = b;
    D.F = F;
    D.q = q;
    D.q_cap = q_cap;
    D.r_cap = r_cap;
    D.h = head;
    D.qlog = (uint64_t*)(head + ((words + 1) & ~1LL));
    D.info = info;
    D.S = s;
    D.K = (DIVF_RUN + s - 1) / s;  // runs of about DIVF_RUN head positions
    // blocks: one per run of the head when b has a non-zero top coefficient
    // (the device finds the true degrees; a longer head only gives a block
    // more runs)
    const int64_t mu_plan = na - nb + 1;
    int64_t runs = mu_plan > 0 ? ((mu_plan + s - 1) / s + D.K - 1) / D.K : 1;
    int blocks = (int)(runs < num_cus ? runs : num_cus);
    if (blocks < 1) blocks = 1;
    {
        TimingScope ts("degrees_kernel", stream);
        hipLaunchKernelGGL(degrees_kernel, dim3(1), dim3(256), 0, stream, a, na, b, nb, info);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        const int64_t n = words > nb ? words : nb;
        int zb = (int)((n + 1023) / 1024);
        if (zb > 2048) zb = 2048;
        if (zb < 1) zb = 1;
        TimingScope ts("zero_check_kernel", stream);
        hipLaunchKernelGGL(zero_check_kernel, dim3(zb), dim3(256), 0, stream, D.qlog, words, a, na, b, nb, F.p,
                           info);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    TimingScope ts("divrem_flow_kernel", stream);
    if (blocks == 1) {
        hipLaunchKernelGGL(divrem_flow_kernel, dim3(1), dim3(DIV_THREADS), 0, stream, D);
        return hipGetLastError();
    }
    void* args[] = {&D};
    return hipLaunchCooperativeKernel((const void*)divrem_flow_kernel, dim3(blocks), dim3(DIV_THREADS), args, 0,
                                      stream);
}

hipError_t fold_q0_launch(const uint32_t* r, int64_t nr, const uint32_t* q, const uint32_t* y, int64_t n,
                          uint32_t* out, const Field& F, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int64_t grid = (n + 255) / 256;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(fold_q0_kernel, dim3((unsigned)grid), dim3(256), 0, stream, r, nr, q, y, n, out, F);
    return hipGetLastError();
}

namespace {
unsigned elementwise_grid(int64_t n) {
    int64_t grid = (n + 255) / 256;
    return (unsigned)(grid < 1 ? 1 : grid > 1024 ? 1024 : grid);
}
}  // namespace

hipError_t negate_launch(const uint32_t* x, int64_t n, uint32_t* out, uint32_t p, bool drop0,
                         hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(negate_kernel, dim3(elementwise_grid(n)), dim3(256), 0, stream, x, n, out, p,
                       drop0 ? 1 : 0);
    return hipGetLastError();
}

hipError_t sub_launch(const uint32_t* x, int64_t nx, const uint32_t* y, int64_t ny, int64_t n, uint32_t* out,
                      uint32_t p, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(sub_kernel, dim3(elementwise_grid(n)), dim3(256), 0, stream, x, nx, y, ny, n, out, p);
    return hipGetLastError();
}

hipError_t divrem_async_fix_launch(uint32_t* q, int64_t q_plan, const uint32_t* b, int64_t nb, CallInfo* info,
                                   hipStream_t stream) {
    hipLaunchKernelGGL(divrem_async_fix_kernel, dim3(elementwise_grid(q_plan)), dim3(256), 0, stream, q, q_plan, b,
                       nb, info);
    return hipGetLastError();
}

hipError_t info_export_launch(const CallInfo* info, int64_t* d_n0, int64_t* d_n1, int32_t* d_status,
                              hipStream_t stream) {
    if (!d_n0 && !d_n1 && !d_status) return hipSuccess;
    hipLaunchKernelGGL(info_export_kernel, dim3(1), dim3(1), 0, stream, info, d_n0, d_n1, d_status);
    return hipGetLastError();
}

hipError_t trim_launch(const uint32_t* r, int64_t n, CallInfo* info, hipStream_t stream) {
    TimingScope ts("trim_kernel", stream);
    hipLaunchKernelGGL(trim_kernel, dim3(1), dim3(64), 0, stream, r, n, info);
    return hipGetLastError();
}

}  // namespace pm
