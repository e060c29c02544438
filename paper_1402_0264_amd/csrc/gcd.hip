// gcd.hip -- Euclidean remainder-sequence gcd of dense polynomials over
// Z/pZ on gfx950 (Sec. 6: naive and optimized Euclidean algorithm).
//
// State: the two current polynomials A and B (the paper's a and b, updated
// in place by division steps) and their degrees (the paper's st). One
// division step reduces the operand of higher degree (A on ties, as in the
// naive Euclidean kernel):  A <- lc(B)*A - lc(A)*X^d*B with d = deg A - deg B.
// This is the paper's step multiplied by the unit lc(B), so no inverse sits
// on the dependent chain of steps; the Montgomery reduction used for the
// combination multiplies by one more unit, 2^-32. Remainders are therefore
// associates of the paper's, with the same degrees, and the final remainder
// is made monic with a single inverse.
//
// Fusion (the paper's s, Sec. 6.2): every thread-block loads the heads of A
// and B (their top H coefficients) and one wave runs up to s steps on the
// heads alone, recording each step's multipliers and shift; a head entry
// stays exact while everything it depends on was loaded, so the run stops
// when the next leading coefficient is no longer known. Then each block
// applies the recorded steps to its own slice of both polynomials, staged in
// LDS together with a halo below the slice that covers the total shift of
// the chunk; the top of the slice is exact at the end. Blocks exchange
// nothing but the slices themselves, through a double buffer in HBM, with
// one grid barrier per chunk. Every block computes the same step sequence
// from the same heads, so all of them leave the loop together.
#include "internal.hpp"

namespace pm {
namespace {

constexpr int MAXS = 256;  // descriptor slots per chunk

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
    int groups, slice, head, s, halo;
};

struct Desc {
    uint32_t m1;    // multiplier of the reduced operand X (lc of the other)
    uint32_t m2;    // multiplier of the shifted other operand Y (p - lc X)
    int32_t d;      // shift: deg X - deg Y
    int32_t which;  // 0: X = A, 1: X = B
};

struct ChunkResult {
    int64_t dA, dB;     // degrees after the chunk (upper bounds when unk*)
    int64_t upd;        // coefficient updates of the chunk
    int32_t nsteps;
    int32_t S;          // total shift
    int32_t unkA, unkB;
};

__device__ __forceinline__ void grid_sync(CallInfo* info, unsigned nblocks, unsigned& gen) {
    __threadfence();
    __syncthreads();
    if (nblocks > 1) {
        if (threadIdx.x == 0) {
            unsigned arrived = atomicAdd(&info->bar_count, 1u);
            if (arrived == nblocks - 1) {
                atomicExch(&info->bar_count, 0u);
                __threadfence();
                atomicAdd(&info->bar_gen, 1u);
            } else {
                while (__hip_atomic_load(&info->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen)
                    __builtin_amdgcn_s_sleep(1);
            }
        }
        gen++;
        __syncthreads();
        __threadfence();
    }
}

// Head phase, run by wave 0 (all 64 lanes). hA/hB: LDS arrays of H entries,
// entry i = coefficient of X^(deg - i).
__device__ void head_phase(const uint32_t* Acur, const uint32_t* Bcur, int64_t dA, int64_t dB, int H, int s,
                           int halo, const Field& F, uint32_t* hA, uint32_t* hB, Desc* desc, ChunkResult* out) {
    const int lane = threadIdx.x & 63;
    for (int i = lane; i < H; i += 64) {
        hA[i] = dA - i >= 0 ? Acur[dA - i] : 0u;
        hB[i] = dB - i >= 0 ? Bcur[dB - i] : 0u;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int vA = H, vB = H, S = 0, n = 0, unkA = 0, unkB = 0;
    int64_t upd = 0;
    while (n < s) {
        const bool redA = dA >= dB;
        uint32_t* X = redA ? hA : hB;
        uint32_t* Y = redA ? hB : hA;
        const int64_t dX = redA ? dA : dB, dY = redA ? dB : dA;
        const int vX = redA ? vA : vB, vY = redA ? vB : vA;
        const int64_t d64 = dX - dY;
        if (n > 0 && S + d64 > halo) break;
        const int d = (int)d64;
        const uint32_t lcX = X[0], lcY = Y[0];
        const uint32_t m1 = lcY, m2 = F.p - lcX;
        const int v = vX < vY ? vX : vY;
        // combine, keep the new values in registers (at most 4 per lane)
        uint32_t nv[4];
        unsigned long long nzm[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int i = lane + 64 * e;
            uint32_t x = 0;
            if (i < H && i < v) x = redc((uint64_t)m1 * X[i] + (uint64_t)m2 * Y[i], F);
            nv[e] = x;
            nzm[e] = __ballot(i >= 1 && i < v && x != 0);
        }
        if (lane == 0) desc[n] = Desc{m1, m2, d, redA ? 0 : 1};
        n++;
        S += d;
        upd += dY + 1;
        int delta = -1;
#pragma unroll
        for (int e = 0; e < 4; e++)
            if (delta < 0 && nzm[e]) delta = 64 * e + __builtin_ctzll(nzm[e]);
        int64_t ndX;
        int nvX;
        if (delta > 0) {
            ndX = dX - delta;
            nvX = v - delta;
            // shift the head: X[i] = new[i + delta]
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int i = lane + 64 * e;
                if (i < H) X[i] = nv[e];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            uint32_t sh[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int i = lane + 64 * e;
                sh[e] = (i < H && i + delta < H) ? X[i + delta] : 0u;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int i = lane + 64 * e;
                if (i < H) X[i] = sh[e];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            // every known entry below the old leading one vanished
            ndX = dX - v;
            nvX = 0;
            if (ndX < 0) ndX = -1;
            else if (redA) unkA = 1;
            else unkB = 1;
        }
        if (redA) { dA = ndX; vA = nvX; } else { dB = ndX; vB = nvX; }
        if (unkA || unkB || dA < 0 || dB < 0) break;
    }
    if (lane == 0) {
        out->dA = dA;
        out->dB = dB;
        out->upd = upd;
        out->nsteps = n;
        out->S = S;
        out->unkA = unkA;
        out->unkB = unkB;
    }
}

__global__ __launch_bounds__(GCD_THREADS) void gcd_kernel(GcdArgs G) {
    extern __shared__ uint32_t smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int slice = G.slice, halo = G.halo, H = G.head;
    const int64_t N = G.N;
    const int64_t lo = (int64_t)blockIdx.x * slice;
    const int64_t hi = lo + slice;
    uint32_t* la = smem;                       // slice + halo
    uint32_t* lb = la + slice + halo;          // slice + halo
    uint32_t* hA = lb + slice + halo;          // H
    uint32_t* hB = hA + H;                     // H
    Desc* desc = (Desc*)(hB + H);              // MAXS
    __shared__ ChunkResult s_res;
    __shared__ int64_t s_deg[2];
    const Field F = G.F;
    unsigned gen = __hip_atomic_load(&G.info->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t* const A0 = G.buf;
    uint32_t* const B0 = G.buf + N;
    uint32_t* const A1 = G.buf + 2 * N;
    uint32_t* const B1 = G.buf + 3 * N;

    // Stage the inputs into buffer 0 and check the range.
    int bad = 0;
    for (int64_t i = lo + tid; i < hi; i += GCD_THREADS) {
        uint32_t x = i < G.na ? G.a[i] : 0u;
        uint32_t y = i < G.nb ? G.b[i] : 0u;
        bad |= (x >= F.p) | (y >= F.p);
        A0[i] = x;
        B0[i] = y;
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
    int64_t dA = s_deg[0], dB = s_deg[1];
    int unkA = 0, unkB = 0;
    int cur = 0;
    int64_t steps = 0, chunks = 0, updates = 0;
    const int64_t max_chunks = (dA > 0 ? dA : 0) + (dB > 0 ? dB : 0) + 4;
    bool ok = true;
    for (;;) {
        const uint32_t* Acur = cur ? A1 : A0;
        const uint32_t* Bcur = cur ? B1 : B0;
        uint32_t* Anext = cur ? A0 : A1;
        uint32_t* Bnext = cur ? B0 : B1;
        if (unkA || unkB) {
            if (wave == 0) {
                int64_t x = unkA ? top_nonzero_wave(Acur, dA + 1) : dA;
                int64_t y = unkB ? top_nonzero_wave(Bcur, dB + 1) : dB;
                if (lane == 0) { s_deg[0] = x; s_deg[1] = y; }
            }
            __syncthreads();
            dA = s_deg[0];
            dB = s_deg[1];
            unkA = unkB = 0;
            __syncthreads();
        }
        if (dA < 0 || dB < 0) break;
        if (chunks >= max_chunks) { ok = false; break; }
        chunks++;
        if (wave == 0) head_phase(Acur, Bcur, dA, dB, H, G.s, halo, F, hA, hB, desc, &s_res);
        __syncthreads();
        const ChunkResult res = s_res;
        const int64_t top = dA > dB ? dA : dB;
        if (lo <= top) {
            const int S = res.S;
            if (S <= halo) {
                const int64_t base = lo - S;
                const int len = slice + S;
                for (int x = tid; x < len; x += GCD_THREADS) {
                    int64_t P = base + x;
                    la[x] = P >= 0 ? Acur[P] : 0u;
                    lb[x] = P >= 0 ? Bcur[P] : 0u;
                }
                __syncthreads();
                for (int k = 0; k < res.nsteps; k++) {
                    const Desc D = desc[k];
                    uint32_t* X = D.which ? lb : la;
                    const uint32_t* Y = D.which ? la : lb;
                    for (int x = tid; x < len; x += GCD_THREADS) {
                        uint32_t y = x - D.d >= 0 ? Y[x - D.d] : 0u;
                        X[x] = redc((uint64_t)D.m1 * X[x] + (uint64_t)D.m2 * y, F);
                    }
                    __syncthreads();
                }
                for (int x = tid; x < slice; x += GCD_THREADS) {
                    int64_t P = lo + x;
                    Anext[P] = P <= res.dA ? la[S + x] : 0u;
                    Bnext[P] = P <= res.dB ? lb[S + x] : 0u;
                }
            } else {
                // a single step with a shift beyond the halo: read the other
                // operand straight from the chunk-start buffer
                const Desc D = desc[0];
                const uint32_t* Xc = D.which ? Bcur : Acur;
                const uint32_t* Yc = D.which ? Acur : Bcur;
                uint32_t* Xn = D.which ? Bnext : Anext;
                uint32_t* Yn = D.which ? Anext : Bnext;
                const int64_t bX = D.which ? res.dB : res.dA;
                const int64_t bY = D.which ? res.dA : res.dB;
                for (int x = tid; x < slice; x += GCD_THREADS) {
                    int64_t P = lo + x;
                    uint32_t y = P - D.d >= 0 ? Yc[P - D.d] : 0u;
                    uint32_t nx = redc((uint64_t)D.m1 * Xc[P] + (uint64_t)D.m2 * y, F);
                    Xn[P] = P <= bX ? nx : 0u;
                    Yn[P] = P <= bY ? Yc[P] : 0u;
                }
            }
        }
        grid_sync(G.info, G.groups, gen);
        cur ^= 1;
        dA = res.dA;
        dB = res.dB;
        unkA = res.unkA;
        unkB = res.unkB;
        steps += res.nsteps;
        updates += res.upd;
    }

    // The last non-zero remainder, made monic.
    const uint32_t* Acur = cur ? A1 : A0;
    const uint32_t* Bcur = cur ? B1 : B0;
    const uint32_t* Rp = dA >= 0 ? Acur : Bcur;
    const int64_t dR = dA >= 0 ? dA : dB;
    int status = ok ? 0 : -6;  // PM_EDEVICE on a broken invariant
    if (status == 0 && dR + 1 > G.g_cap) status = -1;  // PM_EINVAL: g too small
    if (status == 0 && dR >= 0) {
        const uint32_t inv = invmod(Rp[dR], F);
        for (int64_t P = lo + tid; P < hi && P <= dR; P += GCD_THREADS) G.g[P] = mulmod(Rp[P], inv, F);
    }
    if (blockIdx.x == 0 && tid == 0) {
        G.info->status = status;
        G.info->n0 = status == 0 ? dR + 1 : 0;
        G.info->steps = steps;
        G.info->chunks = chunks;
        G.info->updates = updates;
    }
}

}  // namespace

GcdPlan gcd_default_plan(int64_t n, int num_cus, int s) {
    GcdPlan P{};
    P.head = 128;
    P.s = s > 0 ? s : 64;
    if (P.s > MAXS) P.s = MAXS;
    if (P.head < P.s + 64) P.head = ((P.s + 64) + 63) / 64 * 64;
    if (P.head > 256) P.head = 256;
    P.slice = 256;
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

int64_t gcd_scratch_words(int64_t n, const GcdPlan& plan) {
    int64_t N = (int64_t)plan.groups * plan.slice;
    if (N < n) N = n;
    return 4 * N + plan.groups + 64;
}

hipError_t gcd_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, const Field& F, uint32_t* g,
                      int64_t g_cap, uint32_t* scratch, CallInfo* info, const GcdPlan& plan, hipStream_t stream) {
    GcdArgs A{};
    A.a = a; A.b = b; A.na = na; A.nb = nb;
    A.N = (int64_t)plan.groups * plan.slice;
    A.buf = scratch;
    A.flags = scratch + 4 * A.N;
    A.g = g; A.g_cap = g_cap; A.F = F; A.info = info;
    A.groups = plan.groups; A.slice = plan.slice; A.head = plan.head; A.s = plan.s;
    A.halo = plan.s;  // generic chunks shift by about s/2
    size_t lds = (size_t)(2 * (plan.slice + A.halo) + 2 * plan.head) * sizeof(uint32_t) + MAXS * sizeof(Desc);
    void* args[] = {&A};
    if (plan.groups == 1) {
        hipLaunchKernelGGL(gcd_kernel, dim3(1), dim3(GCD_THREADS), lds, stream, A);
        return hipGetLastError();
    }
    return hipLaunchCooperativeKernel((const void*)gcd_kernel, dim3(plan.groups), dim3(GCD_THREADS), args,
                                      (unsigned)lds, stream);
}

}  // namespace pm
