// gcd_core.hpp -- the fused Euclidean chunk shared by the single-instance
// (multi-block) and the batched (one block per instance) gcd kernels.
//
// One division step reduces the operand X of higher degree (A on ties, the
// naive Euclidean kernel's rule) by the other operand Y:
//     X <- REDC(lc(Y)*X + (p - lc(X))*x^d*Y),   d = deg X - deg Y,
// i.e. the paper's step lc(X)/lc(Y) scaled by the unit lc(Y)*2^-32, so the
// degrees of all remainders are the paper's and no inverse is needed.
//
// A chunk (the paper's s steps per launch, Sec. 6.2) has three parts:
//  1. head_run: one wave runs up to s steps on the heads of A and B (their
//     top coefficients, held in registers, element e of lane l = index
//     l + 64e below the leading one). A head entry stays exact while every
//     entry it was computed from was loaded; the run stops before the next
//     leading coefficient would be unknown, or when the total shift of the
//     chunk would exceed MAXSHIFT. Each step is recorded (multipliers,
//     shift, operand).
//  2. build_m: one wave composes the recorded steps into the 2x2 matrix of
//     polynomials M = [[alpha, beta], [gamma, delta]] of degree <= the total
//     shift S, such that (A', B') = M * (A, B) for the chunk-start A, B.
//     Lane k holds coefficient k of each entry.
//  3. apply: every coefficient position P of the new polynomials is an
//     independent sum, A'[P] = sum_k alpha_k A[P-k] + beta_k B[P-k] (and
//     likewise B'), accumulated exactly in 64 bits with lazy folding and
//     reduced once (the same arithmetic as the plain product).
// Because REDC is exact modular arithmetic, M * (A, B) equals the result of
// applying the recorded steps one by one.
#pragma once

#include "common.hpp"

namespace pm {

constexpr int GCD_MAXSHIFT = 63;  // entries of M have at most 64 coefficients
constexpr int GCD_MAXSTEPS = 256;

struct StepDesc {
    uint32_t m1;    // multiplier of X: lc(Y)
    uint32_t m2;    // multiplier of x^d * Y: p - lc(X)
    int32_t d;      // shift
    int32_t which;  // 0: X = A, 1: X = B
};

struct ChunkOut {
    int64_t dA, dB;   // degrees after the chunk (upper bounds when unk*)
    int64_t upd;      // coefficient updates: sum of (deg Y + 1)
    int32_t nsteps;
    int32_t S;        // total shift = max degree of the entries of M
    int32_t unkA, unkB;
    int32_t big;      // 1: a single step whose shift exceeds GCD_MAXSHIFT
    int32_t pad;
};

// lane i <- lane i+1 of x (lane 63 <- `in63`)
__device__ __forceinline__ uint32_t lanes_down1(uint32_t x, uint32_t in63) {
    uint32_t y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
    return (threadIdx.x & 63) == 63 ? in63 : y;
}

// lane i <- lane i-1 of x (lane 0 <- 0)
__device__ __forceinline__ uint32_t lanes_up1(uint32_t x) {
    uint32_t y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
    return (threadIdx.x & 63) == 0 ? 0u : y;
}

// lane i <- lane i-d (0 for i < d), any 0 <= d < 64
__device__ __forceinline__ uint32_t lanes_up(uint32_t x, int d) {
    const int lane = threadIdx.x & 63;
    int src = lane - d;
    uint32_t y = (uint32_t)__builtin_amdgcn_ds_bpermute((src < 0 ? 0 : src) << 2, (int)x);
    return src < 0 ? 0u : y;
}

// Shift a strided head down by one entry: new[i] = old[i + 1] (0 enters at
// the end). Element e of lane l is entry l + 64e.
template <int E>
__device__ __forceinline__ void head_shift1(uint32_t (&h)[E]) {
#pragma unroll
    for (int e = 0; e < E; e++) {
        uint32_t next0 = e + 1 < E ? (uint32_t)__builtin_amdgcn_readlane((int)h[e + 1], 0) : 0u;
        h[e] = lanes_down1(h[e], next0);
    }
}

// One reduction of the head X by Y (in registers): X <- REDC(m1 X + m2 Y),
// entries at or beyond v cleared; returns delta, the index of the first
// non-zero entry after the leading one (the drop of deg X), or 0 when none
// is left among the first v.
template <int E>
__device__ __forceinline__ int head_reduce(uint32_t (&X)[E], const uint32_t (&Y)[E], uint32_t m1, uint32_t m2,
                                           int v, const Field& F) {
    const int lane = threadIdx.x & 63;
    unsigned long long m[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int i = lane + 64 * e;
        uint32_t x = redc((uint64_t)m1 * X[e] + (uint64_t)m2 * Y[e], F);
        x = i < v ? x : 0u;
        X[e] = x;
        m[e] = __ballot(x != 0);
    }
    m[0] &= ~1ull;  // entry 0 is the cancelled leading coefficient
#pragma unroll
    for (int e = 0; e < E; e++)
        if (m[e]) return 64 * e + (int)__builtin_ctzll(m[e]);
    return 0;
}

// Head run by one whole wave. hA/hB: the heads (entry i = coefficient of
// x^(deg - i)), exact for i < 64*E. Records the steps into desc[] (lane 0
// writes LDS), returns the chunk summary through *out (lane 0 writes) and
// the step count and big flag in n_out / big_out.
template <int E>
__device__ void head_run(uint32_t (&hA)[E], uint32_t (&hB)[E], int dA, int dB, int s, const Field& F,
                         StepDesc* desc, ChunkOut* out, int& n_out, int& big_out) {
    const int lane = threadIdx.x & 63;
    constexpr int H = 64 * E;
    dA = uni(dA);
    dB = uni(dB);
    s = uni(s);
    int vA = H, vB = H, S = 0, n = 0, unkA = 0, unkB = 0, big = 0;
    int64_t upd = 0;
    while (n < s && dA >= 0 && dB >= 0) {
        const bool redA = dA >= dB;
        const int d = redA ? dA - dB : dB - dA;
        if (S + d > GCD_MAXSHIFT) {
            if (n > 0) break;
            big = 1;  // one step alone, applied directly
        }
        const uint32_t lcA = (uint32_t)__builtin_amdgcn_readfirstlane((int)hA[0]);
        const uint32_t lcB = (uint32_t)__builtin_amdgcn_readfirstlane((int)hB[0]);
        const int v = vA < vB ? vA : vB;
        uint32_t m1, m2;
        int delta;
        if (redA) {
            m1 = lcB;
            m2 = F.p - lcA;
            delta = head_reduce<E>(hA, hB, m1, m2, v, F);
        } else {
            m1 = lcA;
            m2 = F.p - lcB;
            delta = head_reduce<E>(hB, hA, m1, m2, v, F);
        }
        if (lane == 0) desc[n] = StepDesc{m1, m2, d, redA ? 0 : 1};
        n++;
        if (!big) S += d;
        upd += (redA ? dB : dA) + 1;
        if (delta > 0) {
            for (int k = 0; k < delta; k++) {
                if (redA) head_shift1<E>(hA);
                else head_shift1<E>(hB);
            }
            if (redA) { dA -= delta; vA = v - delta; } else { dB -= delta; vB = v - delta; }
        } else {
            // the first v entries vanished: deg X <= old deg - v
            int nd = (redA ? dA : dB) - v;
            if (nd < 0) nd = -1;
            else if (redA) unkA = 1;
            else unkB = 1;
            if (redA) { dA = nd; vA = 0; } else { dB = nd; vB = 0; }
        }
        if (unkA | unkB | big) break;
    }
    n_out = n;
    big_out = big;
    if (lane == 0) {
        out->dA = dA;
        out->dB = dB;
        out->upd = upd;
        out->nsteps = n;
        out->S = S;
        out->unkA = unkA;
        out->unkB = unkB;
        out->big = big;
    }
}

// Compose the recorded steps into M (one wave; lane k = coefficient k).
// Writes M to LDS as 4 rows of 64 words: alpha, beta, gamma, delta.
// The descriptors are first spread over the lanes (lane j holds step j of
// each group of 64) so the sequential loop reads them with readlane.
__device__ __forceinline__ void build_m(const StepDesc* desc, int n, const Field& F, uint32_t* M) {
    const int lane = threadIdx.x & 63;
    n = uni(n);
    uint32_t al = lane == 0 ? 1u : 0u, be = 0u, ga = 0u, de = lane == 0 ? 1u : 0u;
    for (int k0 = 0; k0 < n; k0 += 64) {
        StepDesc mine = k0 + lane < n ? desc[k0 + lane] : StepDesc{0, 0, 0, 0};
        const uint32_t dw = (uint32_t)mine.d | ((uint32_t)mine.which << 31);
        const int kn = n - k0 < 64 ? n - k0 : 64;
        for (int k = 0; k < kn; k++) {
            const uint32_t m1 = (uint32_t)__builtin_amdgcn_readlane((int)mine.m1, k);
            const uint32_t m2 = (uint32_t)__builtin_amdgcn_readlane((int)mine.m2, k);
            const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)dw, k);
            const int d = (int)(w & 0x7fffffffu);
            if ((w >> 31) == 0) {  // (alpha, beta) <- REDC(m1*(alpha, beta) + m2*x^d*(gamma, delta))
                uint32_t sg = d == 0 ? ga : (d == 1 ? lanes_up1(ga) : lanes_up(ga, d));
                uint32_t sd = d == 0 ? de : (d == 1 ? lanes_up1(de) : lanes_up(de, d));
                al = redc((uint64_t)m1 * al + (uint64_t)m2 * sg, F);
                be = redc((uint64_t)m1 * be + (uint64_t)m2 * sd, F);
            } else {
                uint32_t sa = d == 0 ? al : (d == 1 ? lanes_up1(al) : lanes_up(al, d));
                uint32_t sb = d == 0 ? be : (d == 1 ? lanes_up1(be) : lanes_up(be, d));
                ga = redc((uint64_t)m1 * ga + (uint64_t)m2 * sa, F);
                de = redc((uint64_t)m1 * de + (uint64_t)m2 * sb, F);
            }
        }
    }
    M[lane] = al;
    M[64 + lane] = be;
    M[128 + lane] = ga;
    M[192 + lane] = de;
}

// New coefficients at one position: (A'[P], B'[P]) from the chunk-start
// values A[P-k], B[P-k], k = 0..S, read through la/lb at local index x
// (x - k >= 0 is guaranteed by the caller's staging).
__device__ __forceinline__ void apply_m_at(const uint32_t* la, const uint32_t* lb, int x, int S, const uint32_t* M,
                                           const Field& F, uint32_t& outA, uint32_t& outB) {
    uint64_t accA = 0, accB = 0;
    uint32_t cnt = 0;
    const uint32_t half = F.fold_every / 2;
    S = uni(S);
    for (int k = 0; k <= S; k++) {
        const uint32_t a = la[x - k], b = lb[x - k];
        accA += (uint64_t)M[k] * a;
        accA += (uint64_t)M[64 + k] * b;
        accB += (uint64_t)M[128 + k] * a;
        accB += (uint64_t)M[192 + k] * b;
        if (++cnt == half) {
            accA = fold(accA, F.c32);
            accB = fold(accB, F.c32);
            cnt = 0;
        }
    }
    outA = reduce64(accA, F);
    outB = reduce64(accB, F);
}

}  // namespace pm
