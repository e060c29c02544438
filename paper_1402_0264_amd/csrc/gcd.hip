// gcd.hip -- Euclidean remainder-sequence gcd of dense polynomials over
// Z/pZ on gfx950 (Sec. 6: naive and optimized Euclidean algorithm).
//
// Two kernels share the fused chunk of gcd_core.hpp (heads -> recorded
// steps -> matrix M -> one independent sum per coefficient):
//
//  * gcd_pipe_kernel, for one large instance: a cooperative persistent
//    grid; every block owns a slice of coefficient positions of both
//    polynomials. Each chunk, every block recomputes the same steps and the
//    same M from the heads, applies the previous chunk's M to its slice
//    meanwhile, and meets the others at one split grid barrier. No other
//    communication: the heads are the only cross-block state, as the
//    paper's s-heads are. Its extended variant also carries the cofactor of
//    a through every M.
//  * gcd_batch_kernel, for many instances: one block per instance, both
//    polynomials resident in LDS for the whole remainder sequence; each
//    chunk computes the new coefficients into registers, then overwrites the
//    LDS copy after a block barrier.
//
// Both end with the last non-zero remainder made monic (one Fermat inverse).
#include "gcd_core.hpp"
#include "internal.hpp"

namespace pm {
namespace {

struct GcdArgs {
    const uint32_t* a;
    const uint32_t* b;
    int64_t na, nb;
    uint32_t* buf;     // A0 | B0 | A1 | B1, N words each
    uint32_t* flags;   // one word per block
    int64_t N;
    uint32_t* g;
    int64_t g_cap;
    Field F;
    CallInfo* info;
    int groups, slice, s;
    // extended variant: the cofactor of the caller's a in both operands,
    // carried through every chunk by the same M (A = S_A a + T_A b, and
    // likewise for B); its degree never exceeds deg b (s_deg_cap)
    uint32_t* sbuf;  // SA0 | SB0 | SA1 | SB1, N words each
    const uint32_t* sa0;
    const uint32_t* sb0;
    int64_t nsa, nsb;
    int64_t s_deg_cap;
    uint32_t* s_res;  // N words: the cofactor of the last non-zero remainder, scaled as g is
    // diagnostics (GcdTrace): step log written by block 0, and a step limit
    // after which both operands are written made monic (A to g, B to b_out)
    int32_t* tlog;
    int64_t tchunk_cap, tstep_cap;
    int64_t max_steps;
    uint32_t* b_out;
    int64_t b_cap;
};

// Block 0 records a chunk whose head run is over (desc[0 .. n) final, behind
// a block barrier): its starting degrees and its steps. Called by every
// thread of every block with the same arguments; nrec and nst are the
// block's running counts.
__device__ __forceinline__ void trace_chunk(const GcdArgs& G, int32_t& nrec, int32_t& nst, int64_t dA, int64_t dB,
                                            const StepDesc* desc, int n) {
    if (!G.tlog || blockIdx.x != 0) return;
    int32_t* hdr = G.tlog;
    int32_t* rec = G.tlog + GCD_TRACE_HDR;
    int32_t* stp = rec + 4 * G.tchunk_cap;
    if (nrec >= G.tchunk_cap || (int64_t)nst + n > G.tstep_cap) {
        if (threadIdx.x == 0) hdr[2] = 1;  // overflow: the log is incomplete
        return;
    }
    if (threadIdx.x == 0) {
        rec[4 * nrec + 0] = (int32_t)dA;
        rec[4 * nrec + 1] = (int32_t)dB;
        rec[4 * nrec + 2] = nst;
        rec[4 * nrec + 3] = n;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        stp[2 * (nst + i) + 0] = desc[i].d;
        stp[2 * (nst + i) + 1] = desc[i].which & 1;  // 2: the first step of a round, X = A
    }
    nrec++;
    nst += n;
}

// Steps the next head run may take under the step limit (G.s without one).
__device__ __forceinline__ int steps_allowed(const GcdArgs& G, int64_t done) {
    if (G.max_steps < 0) return G.s;
    const int64_t left = G.max_steps - done;
    return left <= 0 ? 0 : (left < G.s ? (int)left : G.s);
}

// The heads of A and B in the head run's interleaved layout: entry i (the
// coefficient of x^(deg - i)) in lane i / E of element i % E.
template <int E>
__device__ __forceinline__ void load_heads(const uint32_t* A, const uint32_t* B, int64_t dA, int64_t dB,
                                           uint32_t (&hA)[E], uint32_t (&hB)[E]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int64_t i = E * lane + e;
        hA[e] = dA - i >= 0 ? A[dA - i] : 0u;
        hB[e] = dB - i >= 0 ? B[dB - i] : 0u;
    }
}

// ------------------------------------------------------- pipelined grid
// The arrive half of a grid barrier, called by each of the block's nwaves
// arriving waves once they are done with the chunk-start operands (and
// their writes of the new ones are issued): the last of them to arrive (an
// LDS counter) arrives for the block. A wave that wrote device memory
// (wrote = true) first waits until its stores have reached the L2; the
// last arriver then releases the whole block's stores with one agent-scope
// fence. (A fence per wave costs far more: each writes back the XCD's whole
// L2, and those of all the waves on an XCD queue behind each other.) A wave
// that only read (its loads already consumed) needs no wait.
__device__ __forceinline__ void arrive_by_waves(CallInfo* info, unsigned nblocks, uint32_t* s_arrive, int nwaves,
                                                bool wrote) {
    if (wrote) __builtin_amdgcn_s_waitcnt(0);
    if ((threadIdx.x & 63) == 0) {
        const uint32_t before = atomicAdd(s_arrive, 1u);
        if (before == (uint32_t)nwaves - 1) {
            *s_arrive = 0u;  // every apply wave has counted; reused after the block barrier
            if (nblocks > 1) {
                __threadfence();
                const unsigned arrived = atomicAdd(&info->bar_count, 1u);
                if (arrived == nblocks - 1) {
                    atomicExch(&info->bar_count, 0u);
                    __threadfence();
                    atomicAdd(&info->bar_gen, 1u);
                }
            }
        }
    }
}

// The wait half: thread 0 waits until every block has arrived for
// generation gen. Called by all threads of the block. Thread 0 polls with
// plain coherent loads and then acquires once at agent scope; that acquire
// is the block's: the block barrier orders every other thread after it (no
// fence per wave).
__device__ __forceinline__ void wait_grid(CallInfo* info, unsigned nblocks, unsigned& gen) {
    if (nblocks > 1) {
        if (threadIdx.x == 0) {
            while (__hip_atomic_load(&info->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen)
                __builtin_amdgcn_s_sleep(1);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        gen++;
    }
    __syncthreads();
}

// The top 64 E entries of both operands after a chunk, from the chunk-start
// operands A, B (device memory) and the chunk's M: the next chunk's heads.
// The whole block: it stages four windows of 64 E + 64 words (A and B
// below each new degree), then wave w computes head vector w (A's entries
// 0-63 and 64-127, then B's) into hbuf. Ends with the block's barrier.
template <int E>
__device__ void heads_after_chunk(const uint32_t* A, const uint32_t* B, int64_t ndA, int64_t ndB, int S,
                                  const uint32_t* Mc, const Field& F, uint32_t* hw, uint32_t* hbuf) {
    static_assert(2 * E == GCD_THREADS / 64, "one head vector per wave");
    constexpr int WH = 64 * E + 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t baseA = ndA - WH + 1, baseB = ndB - WH + 1;
    // every load of a thread is issued before the first is waited for: the
    // windows were just written by other blocks, so each is a full trip to
    // memory, and this is on the path of every chunk
    constexpr int PER = (4 * WH + GCD_THREADS - 1) / GCD_THREADS;
    uint32_t v[PER];
#pragma unroll
    for (int j = 0; j < PER; j++) {
        const int x = tid + j * GCD_THREADS;
        const int win = x / WH, off = x - win * WH;
        const int64_t P = (win < 2 ? baseA : baseB) + off;
        const uint32_t* src = (win & 1) ? B : A;
        v[j] = (x < 4 * WH && P >= 0) ? src[P] : 0u;
    }
#pragma unroll
    for (int j = 0; j < PER; j++) {
        const int x = tid + j * GCD_THREADS;
        if (x < 4 * WH) hw[x] = v[j];
    }
    __syncthreads();
    const int row = wave / E, e = wave - row * E;  // row 0: A, 1: B
    const int i = lane + 64 * e;
    const int64_t nd = row ? ndB : ndA;
    const uint32_t* w = hw + 2 * WH * row;
    hbuf[wave * 64 + lane] =
        nd - i >= 0 ? apply_row_at(w, w + WH, WH - 1 - i, S, Mc + 128 * row, Mc + 128 * row + 64, F) : 0u;
    __syncthreads();
}

// The cooperative gcd with the chunks overlapped: while the apply waves
// (2 and 3) of every block apply chunk c to their halves of the block's
// slice, wave 0 computes chunk c+1's heads from the chunk-start operands
// and chunk c's M and runs chunk c+1's steps, which wave 1 composes into
// the other M. The grid barrier is split: the apply waves arrive as soon
// as their writes are out, wave 0 as soon as it has read the chunk-start
// operands it needs (another block may overwrite that half of the double
// buffer once the barrier completes), and the block waits only after the
// head run.
// A chunk that ends in an unknown degree or a single big step is followed
// by the serial path (barrier, rescan, heads from device memory).
template <int E, bool XG>
__global__ __launch_bounds__(GCD_THREADS) void gcd_pipe_kernel(GcdArgs G) {
    static_assert(GCD_THREADS == 256, "waves 0 and 1 run the steps and M, waves 2 and 3 apply");
    constexpr int NAPPLY = 2;
    constexpr int NARRIVE = NAPPLY + 1;  // the apply waves and wave 0
    constexpr int WH = 64 * E + 64;
    extern __shared__ uint32_t smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int slice = G.slice;
    const int half = slice / NAPPLY;
    const int64_t N = G.N;
    const int64_t lo = (int64_t)blockIdx.x * slice;
    const int64_t hi = lo + slice;
    uint32_t* stage = smem;                                  // NAPPLY x 2 x (half + 64)
    uint32_t* hw = stage + NAPPLY * 2 * (half + 64);         // 4 x WH
    uint32_t* hbuf = hw + 4 * WH;                            // 2 x 64 E: the next heads
    uint32_t* Mbuf = hbuf + 128 * E;                         // 2 x 256
    StepDesc* desc = (StepDesc*)(Mbuf + 512);                // GCD_MAXSTEPS
    __shared__ ChunkOut s_out[2];
    __shared__ int64_t s_deg[2];
    __shared__ StepLog s_log;
    __shared__ uint32_t s_arrive;
    const Field F = G.F;
    unsigned gen = __hip_atomic_load(&G.info->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t* const A0 = G.buf;
    uint32_t* const B0 = G.buf + N;
    uint32_t* const A1 = G.buf + 2 * N;
    uint32_t* const B1 = G.buf + 3 * N;

    if (tid == 0) {
        steplog_reset(&s_log);
        s_arrive = 0u;
    }
    int bad = 0;
    for (int64_t i = lo + tid; i < hi; i += GCD_THREADS) {
        uint32_t x = i < G.na ? G.a[i] : 0u;
        uint32_t y = i < G.nb ? G.b[i] : 0u;
        bad |= (x >= F.p) | (y >= F.p);
        A0[i] = x;
        B0[i] = y;
    }
    if constexpr (XG) {
        for (int64_t i = lo + tid; i < hi; i += GCD_THREADS) {
            G.sbuf[i] = i < G.nsa ? G.sa0[i] : 0u;
            G.sbuf[N + i] = i < G.nsb ? G.sb0[i] : 0u;
            G.sbuf[2 * N + i] = 0u;  // a block's slice of the other half is read
            G.sbuf[3 * N + i] = 0u;  // before its first write once the degree grows
        }
    }
    bad = __syncthreads_or(bad);
    if (tid == 0) G.flags[blockIdx.x] = (uint32_t)bad;
    if (wave < 2) {
        int64_t d = top_nonzero_wave(wave == 0 ? G.a : G.b, wave == 0 ? G.na : G.nb);
        if (lane == 0) s_deg[wave] = d;
    }
    grid_sync(G.info, G.groups, gen);
    int anybad = 0;
    for (int i = tid; i < G.groups; i += GCD_THREADS) anybad |= (int)G.flags[i];
    anybad = __syncthreads_or(anybad);
    if (anybad) {
        if (blockIdx.x == 0 && tid == 0) {
            G.info->status = -3;  // PM_ERANGE
            G.info->n0 = 0;
        }
        return;
    }
    int64_t dA = uni(s_deg[0]), dB = uni(s_deg[1]);
    // bound on the cofactors' degree; grows by each chunk's shift
    int64_t cdeg = XG ? uni((G.nsa > G.nsb ? G.nsa : G.nsb) - 1) : 0;
    int cur = 0, mb = 0;
    int64_t steps = 0, chunks = 0, updates = 0;
    int64_t run = 0;              // steps with a non-zero multiplier applied so far
    int32_t t_rec = 0, t_st = 0;  // trace counts (block 0)
    const int64_t max_chunks = (dA > 0 ? dA : 0) + (dB > 0 ? dB : 0) + 4;
    bool ok = true;
    // chunk 0's steps and M, from the input operands
    if (dA >= 0 && dB >= 0) {
        if (wave == 0) {
            uint32_t hA[E], hB[E];
            load_heads<E>(A0, B0, dA, dB, hA, hB);
            int nst, big;
            head_run_log<E>(hA, hB, (int)dA, (int)dB, steps_allowed(G, 0), F, desc, &s_log, &s_out[0], nst, big);
        } else if (wave == 1) {
            m_build_live(desc, &s_log, F, Mbuf);
        }
        __syncthreads();
        if (tid == 0) steplog_reset(&s_log);
        __syncthreads();
        trace_chunk(G, t_rec, t_st, dA, dB, desc, uni(s_out[0].nsteps));
    }
    for (;;) {
        // state_c (cur) is complete; chunk c's steps are in s_out[mb], M[mb]
        if (dA < 0 || dB < 0) break;
        // a chunk without steps only follows the step limit
        if (G.max_steps >= 0 && uni(s_out[mb].nsteps) == 0) break;
        if (chunks >= max_chunks) { ok = false; break; }
        chunks++;
        const uint32_t* Acur = cur ? A1 : A0;
        const uint32_t* Bcur = cur ? B1 : B0;
        uint32_t* Anext = cur ? A0 : A1;
        uint32_t* Bnext = cur ? B0 : B1;
        ChunkOut res = s_out[mb];
        res.dA = uni(res.dA);
        res.dB = uni(res.dB);
        res.upd = uni(res.upd);
        res.nsteps = uni(res.nsteps);
        res.S = uni(res.S);
        res.unkA = uni(res.unkA);
        res.unkB = uni(res.unkB);
        res.big = uni(res.big);
        const uint32_t* Mc = Mbuf + 256 * mb;
        uint32_t* Mn = Mbuf + 256 * (mb ^ 1);
        const bool pipe = !res.big && !res.unkA && !res.unkB && res.dA >= 0 && res.dB >= 0;
        const int64_t top = dA > dB ? dA : dB;
        int64_t cdn = 0;
        if constexpr (XG) {
            cdn = cdeg + (res.big ? (int64_t)desc[0].d : (int64_t)res.S);
            if (cdn > G.s_deg_cap) cdn = G.s_deg_cap;
            cdn = uni(cdn);
        }
        if (pipe) heads_after_chunk<E>(Acur, Bcur, res.dA, res.dB, res.S, Mc, F, hw, hbuf);
        if (wave == 0) {
            // done with state c (the windows were read before the block's
            // barrier); wave 0 wrote nothing here
            arrive_by_waves(G.info, G.groups, &s_arrive, NARRIVE, false);
            if (pipe) {
                uint32_t hA[E], hB[E];
#pragma unroll
                for (int e = 0; e < E; e++) {
                    hA[e] = hbuf[E * lane + e];
                    hB[e] = hbuf[64 * E + E * lane + e];
                }
                int nst, big;
                head_run_log<E>(hA, hB, (int)res.dA, (int)res.dB, steps_allowed(G, run + res.nsteps), F, desc,
                                &s_log, &s_out[mb ^ 1], nst, big);
            }
        } else if (wave == 1) {
            if (pipe) m_build_live(desc, &s_log, F, Mn);
        } else {
            const int w = wave - 2;
            const int64_t wlo = lo + (int64_t)w * half;
            uint32_t* la = stage + w * 2 * (half + 64);
            uint32_t* lb = la + half + 64;
            if (wlo <= top) {
                if (!res.big) {
                    const int S = res.S;
                    // the extended variant (twice the apply) takes M's rows from
                    // registers and reads only its windows from LDS; measured, the
                    // plain one runs faster with M read from LDS
                    uint32_t mreg[4];
#pragma unroll
                    for (int r = 0; r < 4; r++) mreg[r] = XG ? Mc[64 * r + lane] : 0u;
                    stage_pair(la, lb, Acur, Bcur, wlo - S, half + S);
                    __builtin_amdgcn_wave_barrier();
                    // half is a multiple of 256: four positions per lane at a time
                    for (int x0 = 0; x0 < half; x0 += 256) {
                        uint32_t na_[4], nb_[4];
                        apply_m_strided<4, XG>(la, lb, x0 + lane + S, 64, x0 + lane + S + 192, S, Mc, F, na_, nb_, mreg);
#pragma unroll
                        for (int j = 0; j < 4; j++) {
                            const int64_t P = wlo + x0 + lane + 64 * j;
                            Anext[P] = P <= res.dA ? na_[j] : 0u;
                            Bnext[P] = P <= res.dB ? nb_[j] : 0u;
                        }
                    }
                } else {
                    const StepDesc D = desc[0];
                    const uint32_t* Xc = D.which ? Bcur : Acur;
                    const uint32_t* Yc = D.which ? Acur : Bcur;
                    uint32_t* Xn = D.which ? Bnext : Anext;
                    uint32_t* Yn = D.which ? Anext : Bnext;
                    const int64_t bX = D.which ? res.dB : res.dA;
                    const int64_t bY = D.which ? res.dA : res.dB;
                    for (int x = lane; x < half; x += 64) {
                        const int64_t P = wlo + x;
                        uint32_t y = P - D.d >= 0 ? Yc[P - D.d] : 0u;
                        uint32_t nx = redc((uint64_t)D.m1 * Xc[P] + (uint64_t)D.m2 * y, F);
                        Xn[P] = P <= bX ? nx : 0u;
                        Yn[P] = P <= bY ? Yc[P] : 0u;
                    }
                }
            }
            if constexpr (XG) {
                // the cofactors take the same M; a wave computes its whole
                // half once the bound reaches it (values past the true
                // degree come out zero)
                const uint32_t* SAc = G.sbuf + (cur ? 2 * N : 0);
                const uint32_t* SBc = SAc + N;
                uint32_t* SAn = G.sbuf + (cur ? 0 : 2 * N);
                uint32_t* SBn = SAn + N;
                if (wlo <= cdn) {
                    if (!res.big) {
                        const int S = res.S;
                        uint32_t mreg[4];
#pragma unroll
                        for (int r = 0; r < 4; r++) mreg[r] = Mc[64 * r + lane];
                        __builtin_amdgcn_wave_barrier();
                        stage_pair(la, lb, SAc, SBc, wlo - S, half + S);
                        __builtin_amdgcn_wave_barrier();
                        for (int x0 = 0; x0 < half; x0 += 256) {
                            uint32_t sa_[4], sb_[4];
                            apply_m_strided<4, true>(la, lb, x0 + lane + S, 64, x0 + lane + S + 192, S, Mc, F, sa_, sb_, mreg);
#pragma unroll
                            for (int j = 0; j < 4; j++) {
                                SAn[wlo + x0 + lane + 64 * j] = sa_[j];
                                SBn[wlo + x0 + lane + 64 * j] = sb_[j];
                            }
                        }
                    } else {
                        const StepDesc D = desc[0];
                        const uint32_t* Xc = D.which ? SBc : SAc;
                        const uint32_t* Yc = D.which ? SAc : SBc;
                        uint32_t* Xn = D.which ? SBn : SAn;
                        uint32_t* Yn = D.which ? SAn : SBn;
                        for (int x = lane; x < half; x += 64) {
                            const int64_t P = wlo + x;
                            uint32_t y = P - D.d >= 0 ? Yc[P - D.d] : 0u;
                            Xn[P] = redc((uint64_t)D.m1 * Xc[P] + (uint64_t)D.m2 * y, F);
                            Yn[P] = Yc[P];
                        }
                    }
                }
            }
            arrive_by_waves(G.info, G.groups, &s_arrive, NARRIVE, true);
        }
        __syncthreads();
        if (tid == 0) steplog_reset(&s_log);
        wait_grid(G.info, G.groups, gen);
        cur ^= 1;
        dA = res.dA;
        dB = res.dB;
        cdeg = cdn;
        steps += res.nsteps + res.zsteps;
        run += res.nsteps;
        updates += res.upd;
        if (pipe) trace_chunk(G, t_rec, t_st, dA, dB, desc, uni(s_out[mb ^ 1].nsteps));
        if (!pipe) {
            const uint32_t* An = cur ? A1 : A0;
            const uint32_t* Bn = cur ? B1 : B0;
            if (res.unkA || res.unkB) {
                if (wave == 0) {
                    int64_t x = res.unkA ? top_nonzero_wave(An, dA + 1) : dA;
                    int64_t y = res.unkB ? top_nonzero_wave(Bn, dB + 1) : dB;
                    if (lane == 0) { s_deg[0] = x; s_deg[1] = y; }
                }
                __syncthreads();
                dA = uni(s_deg[0]);
                dB = uni(s_deg[1]);
                // the zero steps after the step whose new degree was unknown
                const int64_t zY = uni(s_out[mb].zY);
                const int64_t z = zero_steps(uni(s_out[mb].zX), zY, res.unkA ? dA : dB);
                steps += z;
                updates += z * (zY + 1);
            }
            if (dA >= 0 && dB >= 0) {
                if (wave == 0) {
                    uint32_t hA[E], hB[E];
                    load_heads<E>(An, Bn, dA, dB, hA, hB);
                    int nst, big;
                    head_run_log<E>(hA, hB, (int)dA, (int)dB, steps_allowed(G, run), F, desc, &s_log,
                                    &s_out[mb ^ 1], nst, big);
                } else if (wave == 1) {
                    m_build_live(desc, &s_log, F, Mn);
                }
                __syncthreads();
                if (tid == 0) steplog_reset(&s_log);
            }
            __syncthreads();
            if (dA >= 0 && dB >= 0) trace_chunk(G, t_rec, t_st, dA, dB, desc, uni(s_out[mb ^ 1].nsteps));
        }
        mb ^= 1;
    }
    if (G.tlog && blockIdx.x == 0 && tid == 0) {
        // the end record (final degrees, no steps) and the header
        if (t_rec < G.tchunk_cap) {
            int32_t* rec = G.tlog + GCD_TRACE_HDR + 4 * t_rec;
            rec[0] = (int32_t)dA;
            rec[1] = (int32_t)dB;
            rec[2] = t_st;
            rec[3] = 0;
            t_rec++;
        } else {
            G.tlog[2] = 1;
        }
        G.tlog[0] = t_rec;
        G.tlog[1] = t_st;
    }

    // The last non-zero remainder, made monic.
    const uint32_t* Acur = cur ? A1 : A0;
    const uint32_t* Bcur = cur ? B1 : B0;
    const uint32_t* Rp = dA >= 0 ? Acur : Bcur;
    const int64_t dR = dA >= 0 ? dA : dB;
    int status = ok ? 0 : -6;  // PM_EDEVICE on a broken invariant
    if (G.max_steps >= 0) {
        // the pair after the limited steps, each made monic
        if (status == 0 && (dA + 1 > G.g_cap || dB + 1 > G.b_cap)) status = -1;
        if (status == 0 && dA >= 0) {
            const uint32_t inv = invmod(Acur[dA], F);
            for (int64_t P = lo + tid; P < hi && P <= dA; P += GCD_THREADS) G.g[P] = mulmod(Acur[P], inv, F);
        }
        if (status == 0 && dB >= 0) {
            const uint32_t inv = invmod(Bcur[dB], F);
            for (int64_t P = lo + tid; P < hi && P <= dB; P += GCD_THREADS) G.b_out[P] = mulmod(Bcur[P], inv, F);
        }
        if (blockIdx.x == 0 && tid == 0) {
            G.info->status = status;
            G.info->n0 = status == 0 ? dA + 1 : 0;
            G.info->n1 = status == 0 ? dB + 1 : 0;
            G.info->steps = steps;
            G.info->chunks = chunks;
            G.info->updates = updates;
            G.info->run_steps = run;
        }
        return;
    }
    if (status == 0 && dR + 1 > G.g_cap) status = -1;  // PM_EINVAL: g too small
    if (status == 0 && dR >= 0) {
        const uint32_t inv = invmod(Rp[dR], F);
        for (int64_t P = lo + tid; P < hi && P <= dR; P += GCD_THREADS) G.g[P] = mulmod(Rp[P], inv, F);
    }
    if constexpr (XG) {
        // the cofactor of a in the last non-zero remainder, scaled as g is
        const uint32_t* SR = G.sbuf + (cur ? 2 * N : 0) + (dA >= 0 ? 0 : N);
        const uint32_t inv = (status == 0 && dR >= 0) ? invmod(Rp[dR], F) : 0u;
        for (int64_t P = lo + tid; P < hi; P += GCD_THREADS) G.s_res[P] = mulmod(SR[P], inv, F);
    }
    if (blockIdx.x == 0 && tid == 0) {
        G.info->status = status;
        G.info->n0 = status == 0 ? dR + 1 : 0;
        G.info->steps = steps;
        G.info->chunks = chunks;
        G.info->updates = updates;
        G.info->run_steps = run;
    }
}

// ------------------------------------------------------------------ batched
// One block per instance; A and B live in LDS at offset PADLO so that
// positions below 0 read as zero.
constexpr int PADLO = 64;

// One whole instance on the calling block (all NT threads).
template <int NT, int PPT, int E>
__device__ void gcd_instance(const GcdJob& J, int s, int64_t cap, uint32_t* smem) {
    static_assert(NT / 64 >= 2 * E, "a wave per head vector");
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const Field F = J.F;
    uint32_t* A = smem + PADLO;                 // cap words (+PADLO zeros below)
    uint32_t* B = A + cap + PADLO;
    uint32_t* Mbuf = B + cap;                   // 2 x 256: M of this chunk and of the next
    uint32_t* hbuf = Mbuf + 512;                // 2 x 64 E: the next chunk's heads
    StepDesc* desc = (StepDesc*)(hbuf + 128 * E); // GCD_MAXSTEPS
    __shared__ ChunkOut s_out[2];
    __shared__ int64_t s_deg[2];
    __shared__ StepLog s_log;
    // wave 0 runs the heads, wave 1 composes M, waves 2.. own the positions.
    // The 1024-thread shape gives each lane four consecutive positions per
    // pass (NP passes) and slides a window down A and B (apply_m_window4:
    // its apply is bound by VALU, not LDS, reads). The 256-thread shape
    // keeps the strided passes of AG positions, which need fewer registers
    // and so let two blocks share a CU.
    constexpr int NA = NT - 128;
    constexpr bool WIN = NT > 256;
    constexpr int NP = (NT * PPT + 4 * NA - 1) / (4 * NA);
    constexpr int AG = 4;
    constexpr int PPA = WIN ? 4 * NP : (NT * PPT + NA - 1) / NA;

    const int64_t n = J.na > J.nb ? J.na : J.nb;
    // (the window apply reads B in 16-byte pieces: B's offset, cap + PADLO
    // words past A, must be a multiple of 4, as the capacities are)
    const bool badcap = WIN && (cap & 3) != 0;
    int bad = n > cap || badcap;
    if (tid < PADLO) { A[tid - PADLO] = 0u; B[tid - PADLO] = 0u; }
    if (tid == 0) steplog_reset(&s_log);
    if (J.fresh) {
        for (int64_t i = tid; i < cap; i += NT) {
            uint32_t x = i < J.na ? __hip_atomic_load(J.a + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : 0u;
            uint32_t y = i < J.nb ? __hip_atomic_load(J.b + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : 0u;
            bad |= (x >= F.p) | (y >= F.p);
            A[i] = x;
            B[i] = y;
        }
    } else {
        for (int64_t i = tid; i < cap; i += NT) {
            uint32_t x = i < J.na ? J.a[i] : 0u;
            uint32_t y = i < J.nb ? J.b[i] : 0u;
            bad |= (x >= F.p) | (y >= F.p);
            A[i] = x;
            B[i] = y;
        }
    }
    bad = __syncthreads_or(bad);
    if (bad) {
        if (tid == 0) {
            J.out->status = (n > cap || badcap) ? -1 : -3;
            J.out->ng = 0;
            J.out->steps = J.out->updates = J.out->chunks = 0;
            __threadfence_system();
            __hip_atomic_store(&J.out->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        return;
    }
    if (wave < 2) {
        int64_t d = top_nonzero_wave(wave == 0 ? A : B, cap);
        if (lane == 0) s_deg[wave] = d;
    }
    __syncthreads();
    int64_t dA = uni(s_deg[0]), dB = uni(s_deg[1]);
    int64_t steps = 0, chunks = 0, updates = 0;
    const int64_t max_chunks = (dA > 0 ? dA : 0) + (dB > 0 ? dB : 0) + 4;
    bool ok = true;
    int mb = 0;
    // the first chunk's steps and M, from the heads of the inputs
    if (dA >= 0 && dB >= 0) {
        if (wave == 0) {
            uint32_t hA[E], hB[E];
            load_heads<E>(A, B, dA, dB, hA, hB);
            int nst, big;
            head_run_log<E>(hA, hB, (int)dA, (int)dB, s, F, desc, &s_log, &s_out[0], nst, big);
        } else if (wave == 1) {
            m_build_live(desc, &s_log, F, Mbuf);
        }
        __syncthreads();
        if (tid == 0) steplog_reset(&s_log);
        __syncthreads();
    }
    // Each chunk: waves 2.. compute M * (A, B) at every position into
    // registers while wave 0 computes the top of the new pair (the next
    // chunk's heads) from the same chunk-start data and runs the next
    // chunk's steps, which wave 1 composes into the other M buffer; after a
    // barrier the new pair is written back. A chunk whose heads ran out (degree unknown) or that is
    // one big step is followed by the serial path: write, rescan, then heads.
    for (;;) {
        if (dA < 0 || dB < 0) break;
        if (chunks >= max_chunks) { ok = false; break; }
        chunks++;
        ChunkOut res = s_out[mb];
        res.dA = uni(res.dA);
        res.dB = uni(res.dB);
        res.upd = uni(res.upd);
        res.nsteps = uni(res.nsteps);
        res.S = uni(res.S);
        res.unkA = uni(res.unkA);
        res.unkB = uni(res.unkB);
        res.big = uni(res.big);
        const uint32_t* Mc = Mbuf + 256 * mb;
        uint32_t* Mn = Mbuf + 256 * (mb ^ 1);
        const bool pipe = !res.big && !res.unkA && !res.unkB && res.dA >= 0 && res.dB >= 0;
        const int top = (int)(dA > dB ? dA : dB);
        if (!res.big) {
            uint32_t nA[PPA], nB[PPA];
            if (pipe) {
                // the next chunk's heads from the chunk-start pair and M, one
                // 64-entry vector per wave (A's, then B's), off the chain
                if (wave < 2 * E) {
                    const int row = wave / E, e = wave - row * E;
                    const int P = (int)(row ? res.dB : res.dA) - (lane + 64 * e);
                    hbuf[wave * 64 + lane] =
                        P >= 0 ? apply_row_at(A, B, P, res.S, Mc + 128 * row, Mc + 128 * row + 64, F) : 0u;
                }
                __syncthreads();
            }
            if (wave == 0) {
                if (pipe) {
                    // the step chain bounds the chunk: its wave goes first on
                    // a SIMD it shares with apply waves
                    __builtin_amdgcn_s_setprio(3);
                    uint32_t hA[E], hB[E];
#pragma unroll
                    for (int e = 0; e < E; e++) {
                        hA[e] = hbuf[E * lane + e];
                        hB[e] = hbuf[64 * E + E * lane + e];
                    }
                    int nst, big;
                    head_run_log<E>(hA, hB, (int)res.dA, (int)res.dB, s, F, desc, &s_log, &s_out[mb ^ 1], nst, big);
                    __builtin_amdgcn_s_setprio(0);
                }
            } else if (wave == 1) {
                if (pipe) {
                    __builtin_amdgcn_s_setprio(2);
                    m_build_live(desc, &s_log, F, Mn);
                    __builtin_amdgcn_s_setprio(0);
                }
            } else if constexpr (WIN) {
#pragma unroll
                for (int t = 0; t < NP; t++) {
                    const int x = 4 * (tid - 128) + 4 * NA * t;
                    uint32_t ga[4] = {0u, 0u, 0u, 0u}, gb[4] = {0u, 0u, 0u, 0u};
                    if (x <= top) apply_m_window4(A, B, x, res.S, Mc, F, ga, gb);
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        nA[4 * t + j] = ga[j];
                        nB[4 * t + j] = gb[j];
                    }
                }
            } else {
                // AG positions at a time share each read of M (a position
                // above top is read at top; its sum is not stored)
#pragma unroll
                for (int j0 = 0; j0 < PPA; j0 += AG) {
                    const int P0 = (tid - 128) + j0 * NA;
                    uint32_t ga[AG], gb[AG];
#pragma unroll
                    for (int j = 0; j < AG; j++) ga[j] = gb[j] = 0u;
                    if (P0 <= top) apply_m_strided<AG>(A, B, P0, NA, (int)top, res.S, Mc, F, ga, gb);
#pragma unroll
                    for (int j = 0; j < AG && j0 + j < PPA; j++) {
                        nA[j0 + j] = ga[j];
                        nB[j0 + j] = gb[j];
                    }
                }
            }
            __syncthreads();
            if (tid == 0) steplog_reset(&s_log);  // the run above is over
            if (wave >= 2) {
#pragma unroll
                for (int j = 0; j < PPA; j++) {
                    // position of result j: four consecutive per pass, or strided
                    const int P = WIN ? 4 * (tid - 128) + 4 * NA * (j / 4) + (j % 4) : (tid - 128) + j * NA;
                    if (P <= top) {
                        A[P] = P <= res.dA ? nA[j] : 0u;
                        B[P] = P <= res.dB ? nB[j] : 0u;
                    }
                }
            }
        } else {
            const StepDesc D = desc[0];
            uint32_t* X = D.which ? B : A;
            const uint32_t* Y = D.which ? A : B;
            const int64_t bX = D.which ? res.dB : res.dA;
            // only X changes and Y is only read: in place
            for (int P = tid; P <= top; P += NT) {
                uint32_t y = P - D.d >= 0 ? Y[P - D.d] : 0u;
                uint32_t nx = redc((uint64_t)D.m1 * X[P] + (uint64_t)D.m2 * y, F);
                X[P] = P <= bX ? nx : 0u;
            }
        }
        __syncthreads();
        dA = res.dA;
        dB = res.dB;
        steps += res.nsteps + res.zsteps;
        updates += res.upd;
        if (!pipe) {
            if (res.unkA || res.unkB) {
                if (wave == 0) {
                    int64_t x = res.unkA ? top_nonzero_wave(A, dA + 1) : dA;
                    int64_t y = res.unkB ? top_nonzero_wave(B, dB + 1) : dB;
                    if (lane == 0) { s_deg[0] = x; s_deg[1] = y; }
                }
                __syncthreads();
                dA = uni(s_deg[0]);
                dB = uni(s_deg[1]);
                // the zero steps after the step whose new degree was unknown
                const int64_t zY = uni(s_out[mb].zY);
                const int64_t z = zero_steps(uni(s_out[mb].zX), zY, res.unkA ? dA : dB);
                steps += z;
                updates += z * (zY + 1);
            }
            if (dA >= 0 && dB >= 0) {
                if (wave == 0) {
                    uint32_t hA[E], hB[E];
                    load_heads<E>(A, B, dA, dB, hA, hB);
                    int nst, big;
                    head_run_log<E>(hA, hB, (int)dA, (int)dB, s, F, desc, &s_log, &s_out[mb ^ 1], nst, big);
                } else if (wave == 1) {
                    m_build_live(desc, &s_log, F, Mn);
                }
                __syncthreads();
                if (tid == 0) steplog_reset(&s_log);
                __syncthreads();
            }
        }
        mb ^= 1;
    }
    const uint32_t* R = dA >= 0 ? A : B;
    const int64_t dR = dA >= 0 ? dA : dB;
    int status = ok ? 0 : -6;
    if (status == 0 && dR + 1 > J.g_cap) status = -1;
    if (status == 0 && dR >= 0) {
        const uint32_t inv = invmod(R[dR], F);
        for (int64_t P = tid; P <= dR; P += NT) J.g[P] = mulmod(R[P], inv, F);
    }
    // g may live in host memory (the server's completion buffers): every
    // thread's stores are made visible before `done` is raised
    __threadfence_system();
    __syncthreads();
    if (tid == 0) {
        J.out->status = status;
        J.out->ng = status == 0 ? dR + 1 : 0;
        J.out->nr = 0;
        J.out->steps = steps;
        J.out->updates = updates;
        J.out->chunks = chunks;
        __threadfence_system();
        __hip_atomic_store(&J.out->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// One Euclidean division (Sec. 3) on the calling block, both operands in
// LDS (a request of the server). The quotient comes s = 64 terms per chunk,
// from the top down: the chunk's terms u_i = q_(jtop - i) solve the
// triangular system sum_(k<=i) beta_(i-k) u_k = v_i on the chunk's current
// head values v, with beta_d = b[deg b - d], so u = G v mod x^64 where G is
// the inverse of sum beta_d x^d (64 serial steps on one wave, once); then
// every position of a below the chunk takes the chunk's terms at once:
// a[x] -= sum_i u_i b[x - jtop + i]. What remains below deg b is r. Writes
// q to J.g, r to J.r and the result record (lengths, steps = the quotient's
// positions, updates = steps * (deg b + 1)).
template <int NT>
__device__ void div_instance(const GcdJob& J, int64_t cap, uint32_t* smem) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const Field F = J.F;
    uint32_t* A = smem + PADLO;      // cap words (+PADLO zeros below)
    uint32_t* B = A + cap + PADLO;   // cap words (+PADLO zeros below)
    uint32_t* sG = B + cap;          // 64: G_k
    uint32_t* sU = sG + 64;          // 64: the chunk's quotient terms
    __shared__ int64_t s_deg[2];
    const int64_t n = J.na > J.nb ? J.na : J.nb;
    int bad = n > cap;
    if (tid < PADLO) { A[tid - PADLO] = 0u; B[tid - PADLO] = 0u; }
    for (int64_t i = tid; i < cap; i += NT) {
        uint32_t x, y;
        if (J.fresh) {
            x = i < J.na ? __hip_atomic_load(J.a + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : 0u;
            y = i < J.nb ? __hip_atomic_load(J.b + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : 0u;
        } else {
            x = i < J.na ? J.a[i] : 0u;
            y = i < J.nb ? J.b[i] : 0u;
        }
        bad |= (x >= F.p) | (y >= F.p);
        A[i] = x;
        B[i] = y;
    }
    bad = __syncthreads_or(bad);
    int64_t da = -1, db = -1;
    if (!bad) {
        if (wave < 2) {
            const int64_t d = top_nonzero_wave(wave == 0 ? A : B, cap);
            if (lane == 0) s_deg[wave] = d;
        }
        __syncthreads();
        da = uni(s_deg[0]);
        db = uni(s_deg[1]);
    }
    int status = bad ? (n > cap ? -1 : -3) : 0;       // PM_EINVAL / PM_ERANGE
    if (status == 0 && db < 0) status = -4;           // PM_EDIVZERO
    const int64_t mu = (status == 0 && da >= db) ? da - db + 1 : 0;
    const int64_t nr_max = da < db ? da + 1 : db;
    if (status == 0 && (mu > J.g_cap || nr_max > J.r_cap)) status = -1;  // PM_EINVAL
    if (status == 0 && mu > 0) {
        // G = (sum_(d<64) beta_d x^d)^(-1) mod x^64: lane k holds the pending
        // coefficient of x^k of the series 1 being divided
        if (wave == 0) {
            const uint32_t beta = lane <= db ? B[db - lane] : 0u;
            sU[lane] = beta;
            const uint32_t inv = invmod(B[db], F);
            uint32_t val = lane == 0 ? 1u : 0u;
            for (int j = 0; j < 64; j++) {
                const uint32_t gj = mulmod((uint32_t)__builtin_amdgcn_readlane((int)val, j), inv, F);
                if (lane > j) val = submod(val, mulmod(gj, sU[lane - j], F), F.p);
                if (lane == j) sG[j] = gj;
            }
        }
        __syncthreads();
        const uint32_t half = F.fold_every / 2;
        for (int64_t jtop = mu - 1; jtop >= 0; jtop -= 64) {
            const int S = (int)(jtop + 1 < 64 ? jtop + 1 : 64);
            const int64_t top = jtop + db;  // a-position of q_jtop
            if (wave == 0) {
                // u_i = sum_(k<=i) G_(i-k) v_k, v_k = a[top - k]
                const uint32_t v = lane < S ? A[top - lane] : 0u;
                uint64_t acc = 0;
                uint32_t cnt = 0;
                for (int k = 0; k < S; k++) {
                    const uint32_t vk = (uint32_t)__builtin_amdgcn_readlane((int)v, k);
                    if (lane >= k) acc += (uint64_t)sG[lane - k] * vk;
                    if (++cnt == half) {
                        acc = fold(acc, F.c32);
                        cnt = 0;
                    }
                }
                const uint32_t u = lane < S ? reduce64(acc, F) : 0u;
                sU[lane] = u;
                if (lane < S) J.g[jtop - lane] = u;
            }
            __syncthreads();
            // positions jtop - S + 1 .. top - S below the chunk; b is zero
            // outside 0..db (PADLO zeros below, zeros loaded above)
            // the loop runs the same passes on every lane of a wave (the lane
            // reads of u need every lane active) and only the store is
            // guarded; a lane past the last position computes a clamped one
            const uint32_t u_reg = sU[lane];
            const int64_t lo = jtop - S + 1 > 0 ? jtop - S + 1 : 0, hi = top - S;
            for (int64_t x0 = lo + (tid - lane); x0 <= hi; x0 += NT) {
                const int64_t x = x0 + lane;
                const uint32_t* bw = B + ((x <= hi ? x : hi) - jtop);
                uint64_t acc = 0;
                uint32_t cnt = 0;
                for (int i = 0; i < S; i++) {
                    const uint32_t ui = (uint32_t)__builtin_amdgcn_readlane((int)u_reg, i);
                    acc += (uint64_t)ui * bw[i];
                    if (++cnt == half) {
                        acc = fold(acc, F.c32);
                        cnt = 0;
                    }
                }
                const uint32_t d = reduce64(acc, F);
                if (x <= hi) A[x] = submod(A[x], d, F.p);
            }
            __syncthreads();
        }
    }
    // r: what remains of a below deg b (all of a when deg a < deg b)
    int64_t nr = 0;
    if (status == 0) {
        if (wave == 0) {
            const int64_t d = top_nonzero_wave(A, nr_max);
            if (lane == 0) s_deg[0] = d;
        }
        __syncthreads();
        nr = uni(s_deg[0]) + 1;
        for (int64_t i = tid; i < nr; i += NT) J.r[i] = A[i];
    }
    // q and r may live in host memory (the server's completion buffers):
    // every thread's stores are made visible before `done` is raised
    __threadfence_system();
    __syncthreads();
    if (tid == 0) {
        J.out->status = status;
        J.out->ng = status == 0 ? mu : 0;
        J.out->nr = status == 0 ? nr : 0;
        J.out->steps = mu;
        J.out->updates = mu * (db + 1);
        J.out->chunks = (mu + 63) / 64;
        __threadfence_system();
        __hip_atomic_store(&J.out->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

template <int NT, int PPT, int E>
__global__ __launch_bounds__(NT) void gcd_batch_kernel(const GcdJob* jobs, const int32_t* order, int njobs,
                                                       int s, int64_t cap) {
    extern __shared__ __align__(16) uint32_t smem[];  // 16-byte reads of A and B
    if ((int)blockIdx.x >= njobs) return;
    const int jid = order ? order[blockIdx.x] : (int)blockIdx.x;
    const GcdJob J = jobs[jid];
    gcd_instance<NT, PPT, E>(J, s, cap, smem);
}

// Persistent worker for the server: each block claims the next published
// job (head < tail) and runs it, until `stop` is raised with nothing left,
// or nothing was published for `idle_ticks` of the constant-rate wall clock
// (the host relaunches the worker when new work arrives after that).
template <int NT, int PPT, int E>
__global__ __launch_bounds__(NT) void gcd_worker_kernel(const GcdJob* jobs, const uint32_t* order, uint32_t order_cap,
                                                        const uint32_t* tail, const uint32_t* stop, uint32_t* head,
                                                        uint32_t* started, int s, int64_t cap, uint64_t idle_ticks) {
    extern __shared__ __align__(16) uint32_t smem[];  // 16-byte reads of A and B
    __shared__ int64_t s_job;
    __shared__ GcdJob s_J;
    if (threadIdx.x == 0) __hip_atomic_fetch_add(started, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    for (;;) {
        if (threadIdx.x == 0) {
            int64_t got = -1;
            uint64_t idle_from = wall_clock64();
            for (;;) {
                const uint32_t t = __hip_atomic_load(tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                uint32_t h = __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (h < t) {
                    if (atomicCAS(head, h, h + 1) == h) { got = h; break; }
                    continue;
                }
                if (__hip_atomic_load(stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM)) break;
                if (wall_clock64() - idle_from > idle_ticks) break;
                __builtin_amdgcn_s_sleep(64);
            }
            s_job = got;
        }
        __syncthreads();
        const int64_t job = s_job;
        __syncthreads();
        if (job < 0) break;
        // the order ring and the job table live in host memory written by
        // the host after this kernel started: one thread reads them past
        // the caches and shares them
        if (threadIdx.x == 0) {
            const uint32_t slot =
                __hip_atomic_load(order + (job & (order_cap - 1)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            const uint64_t* src = (const uint64_t*)(jobs + slot);
            uint64_t* dst = (uint64_t*)&s_J;
            for (int w = 0; w < (int)(sizeof(GcdJob) / 8); w++)
                dst[w] = __hip_atomic_load(src + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        __syncthreads();
        const GcdJob J = s_J;
        if (J.op == JOB_DIVREM) div_instance<NT>(J, cap, smem);
        else gcd_instance<NT, PPT, E>(J, s, cap, smem);
        __syncthreads();
    }
}

template <int NT, int PPT, int E>
size_t batch_lds_bytes(int64_t cap) {
    return (size_t)(2 * (cap + PADLO) + 512 + 128 * E) * sizeof(uint32_t) + GCD_MAXSTEPS * sizeof(StepDesc);
}

}  // namespace

GcdPlan gcd_default_plan(int64_t n, int num_cus, int s) {
    GcdPlan P{};
    P.s = s > 0 ? s : 128;
    if (P.s > GCD_MAXSTEPS) P.s = GCD_MAXSTEPS;
    P.head = 128;  // a chunk has at most 2(S+1) <= 128 steps: about 64 entries of each head
    // 512 positions per block: fewer blocks make the per-chunk grid barrier
    // cheaper, while the apply (two positions per thread) stays short
    P.slice = 512;
    int64_t groups = (n + P.slice - 1) / P.slice;
    const int64_t max_groups = 2LL * num_cus;
    while (groups > max_groups) {
        P.slice *= 2;
        groups = (n + P.slice - 1) / P.slice;
    }
    if (groups < 1) groups = 1;
    P.groups = (int)groups;
    return P;
}

int64_t gcd_positions(const GcdPlan& plan) { return (int64_t)plan.groups * plan.slice; }

int64_t gcd_scratch_words(int64_t n, const GcdPlan& plan, bool cofactors) {
    int64_t N = gcd_positions(plan);
    if (N < n) N = n;
    const int64_t base = ((4 * N + plan.groups + 64) + 63) & ~63LL;
    return cofactors ? base + 4 * N : base;
}

hipError_t gcd_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, const Field& F, uint32_t* g,
                      int64_t g_cap, uint32_t* scratch, CallInfo* info, const GcdPlan& plan, hipStream_t stream,
                      const GcdCofactors* xg, const GcdTrace* tr) {
    // each apply wave takes half a slice, four positions per lane at a time
    if (plan.slice <= 0 || plan.slice % 512 != 0) return hipErrorInvalidValue;
    if (xg && tr) return hipErrorInvalidValue;  // the diagnostics are for the plain variant
    GcdArgs A{};
    A.a = a; A.b = b; A.na = na; A.nb = nb;
    A.N = gcd_positions(plan);
    A.buf = scratch;
    A.flags = scratch + 4 * A.N;
    A.g = g; A.g_cap = g_cap; A.F = F; A.info = info;
    A.groups = plan.groups; A.slice = plan.slice; A.s = plan.s;
    if (xg) {
        A.sbuf = scratch + (((4 * A.N + plan.groups + 64) + 63) & ~63LL);
        A.sa0 = xg->sa0; A.nsa = xg->nsa;
        A.sb0 = xg->sb0; A.nsb = xg->nsb;
        A.s_deg_cap = xg->deg_cap;
        A.s_res = xg->s_res;
    }
    A.max_steps = -1;
    if (tr) {
        A.tlog = tr->log;
        A.tchunk_cap = tr->chunk_cap;
        A.tstep_cap = tr->step_cap;
        A.max_steps = tr->max_steps;
        A.b_out = tr->b_out;
        A.b_cap = tr->b_cap;
    }
    constexpr int E = 2;  // 128-entry heads (GcdPlan::head)
    void* args[] = {&A};
    const int half = plan.slice / 2;
    const size_t lds = (size_t)(2 * 2 * (half + 64) + 4 * (64 * E + 64) + 128 * E + 512) * sizeof(uint32_t) +
                       GCD_MAXSTEPS * sizeof(StepDesc);
    TimingScope ts(xg ? "gcd_pipe_kernel_xg" : "gcd_pipe_kernel", stream);
    const void* fn = xg ? (const void*)gcd_pipe_kernel<E, true> : (const void*)gcd_pipe_kernel<E, false>;
    if (plan.groups == 1) {
        if (xg) hipLaunchKernelGGL((gcd_pipe_kernel<E, true>), dim3(1), dim3(GCD_THREADS), lds, stream, A);
        else hipLaunchKernelGGL((gcd_pipe_kernel<E, false>), dim3(1), dim3(GCD_THREADS), lds, stream, A);
        return hipGetLastError();
    }
    return hipLaunchCooperativeKernel(fn, dim3(plan.groups), dim3(GCD_THREADS), args, (unsigned)lds, stream);
}

int64_t gcd_batch_cap(int kind) { return kind == 0 ? 256 * 16 : 1024 * 17; }

int gcd_worker_blocks_per_cu(int kind) {
    int v = 0;
    hipError_t e;
    if (kind == 0)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, (const void*)gcd_worker_kernel<256, 16, 2>, 256,
                                                         batch_lds_bytes<256, 16, 2>(gcd_batch_cap(0)));
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, (const void*)gcd_worker_kernel<1024, 17, 2>, 1024,
                                                         batch_lds_bytes<1024, 17, 2>(gcd_batch_cap(1)));
    return e == hipSuccess && v > 0 ? v : 1;
}

hipError_t gcd_worker_launch(int kind, const GcdJob* jobs, const uint32_t* order, uint32_t order_cap,
                             const uint32_t* tail, const uint32_t* stop, uint32_t* head, uint32_t* started, int s,
                             int blocks, double idle_seconds, hipStream_t stream) {
    int dev = 0, khz = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
    const uint64_t ticks = (uint64_t)(idle_seconds * 1e3 * khz);
    // 128-entry heads for any s: a chunk has at most 2(S+1) <= 128 steps,
    // which consume about 64 entries of each head (a shorter run is still
    // exact); 1024 threads leave 128 VGPRs per lane
    if (kind == 0) {
        const int64_t cap = gcd_batch_cap(0);
        const size_t lds = batch_lds_bytes<256, 16, 2>(cap);
        hipLaunchKernelGGL((gcd_worker_kernel<256, 16, 2>), dim3(blocks), dim3(256), lds, stream, jobs, order,
                           order_cap, tail, stop, head, started, s, cap, ticks);
    } else {
        const int64_t cap = gcd_batch_cap(1);
        const size_t lds = batch_lds_bytes<1024, 17, 2>(cap);
        hipLaunchKernelGGL((gcd_worker_kernel<1024, 17, 2>), dim3(blocks), dim3(1024), lds, stream, jobs, order,
                           order_cap, tail, stop, head, started, s, cap, ticks);
    }
    return hipGetLastError();
}

hipError_t gcd_batch_launch(const GcdJob* d_jobs, const int32_t* d_order, int njobs, int kind, int s,
                            hipStream_t stream) {
    if (njobs <= 0) return hipSuccess;
    // 128-entry heads for any s (see gcd_worker_launch)
    if (kind == 0) {
        size_t lds = batch_lds_bytes<256, 16, 2>(gcd_batch_cap(0));
        TimingScope ts("gcd_batch_kernel", stream);
        hipLaunchKernelGGL((gcd_batch_kernel<256, 16, 2>), dim3(njobs), dim3(256), lds, stream, d_jobs, d_order,
                           njobs, s, gcd_batch_cap(0));
    } else {
        size_t lds = batch_lds_bytes<1024, 17, 2>(gcd_batch_cap(1));
        TimingScope ts("gcd_batch_kernel", stream);
        hipLaunchKernelGGL((gcd_batch_kernel<1024, 17, 2>), dim3(njobs), dim3(1024), lds, stream, d_jobs, d_order,
                           njobs, s, gcd_batch_cap(1));
    }
    return hipGetLastError();
}

}  // namespace pm
