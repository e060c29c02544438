// gcd_core.hpp -- the fused Euclidean chunk shared by the single-instance
// (multi-block) and the batched (one block per instance) gcd kernels.
//
// One division step reduces the operand X of higher degree (A on ties, the
// naive Euclidean kernel's rule) by the other operand Y:
//     X <- REDC(lc(Y)*X + (p - lc(X))*x^d*Y),   d = deg X - deg Y,
// i.e. the paper's step lc(X)/lc(Y) scaled by the unit lc(Y)*2^-32, so the
// degrees of all remainders are the paper's and no inverse is needed.
//
// A chunk (the paper's s steps per launch, Sec. 6.2) has two parts:
//  1. head_run_log: one wave runs up to s steps on the heads of A and B
//     (their top coefficients, held in registers, element e of lane l =
//     index l + 64e below the leading one). A head entry stays exact while
//     every entry it was computed from was loaded; the run stops before the
//     next leading coefficient would be unknown, or when the total shift of
//     the chunk would exceed MAXSHIFT. Each step is recorded as it starts
//     and published with the next one (the last by the run's end count), and
//     a second wave (m_build_live) applies it to the 2x2 matrix of
//     polynomials M = [[alpha, beta], [gamma, delta]] (degree <= the total
//     shift S; lane k holds coefficient k of each entry), so that
//     (A', B') = M * (A, B) for the chunk-start A, B.
//  2. apply: every coefficient position P of the new polynomials is an
//     independent sum, A'[P] = sum_k alpha_k A[P-k] + beta_k B[P-k] (and
//     likewise B'), accumulated exactly in 64 bits with lazy folding and
//     reduced once (the same arithmetic as the plain product).
// Because REDC is exact modular arithmetic, M * (A, B) equals the result of
// applying the recorded steps one by one.
#pragma once

#include <type_traits>

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
    int64_t upd;      // coefficient updates: sum of (deg Y + 1) over all steps counted
    int32_t nsteps;   // steps run (records in desc[])
    int32_t S;        // total shift = max degree of the entries of M
    int32_t unkA, unkB;
    int32_t big;      // 1: a single step whose shift exceeds GCD_MAXSHIFT
    int32_t zsteps;   // steps with a zero multiplier, counted not run (see zero_steps)
    int64_t zX, zY;   // a step whose new degree is unknown (unk*): deg X and deg Y before it, else -1
};

// The long division visits every position from deg X down to deg Y
// (Alg. 1/2): after a step that leaves X with degree nd, the positions
// between are steps with a zero multiplier, each updating deg Y + 1
// coefficients with nothing. They are counted, not run.
__host__ __device__ __forceinline__ int64_t zero_steps(int64_t dX, int64_t dY, int64_t nd) {
    const int64_t fl = nd > dY - 1 ? nd : dY - 1;
    return dX - 1 - fl > 0 ? dX - 1 - fl : 0;
}

// lane i <- lane i+1 of x (lane 63 <- `in63`)
__device__ __forceinline__ uint32_t lanes_down1(uint32_t x, uint32_t in63) {
    uint32_t y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
    return (threadIdx.x & 63) == 63 ? in63 : y;
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

// Progress of a head run, read by the wave that composes M while the run
// goes on. Reset (prog = 0, end = -1) before every run, behind a barrier.
struct StepLog {
    int prog;  // steps published in desc[]
    int end;   // total steps once the run has finished, else -1
    int zs;    // zero-multiplier steps counted so far (written by the run's lane 0)
    int pad;
    int64_t zupd;  // their updates
};

__device__ __forceinline__ void steplog_reset(StepLog* L) {
    L->prog = 0;
    L->end = -1;
    L->zs = 0;
    L->zupd = 0;
}

// Adds the zero-multiplier steps of one step (X from degree dX to nd,
// divisor of degree dY) to the run's counts. One lane.
__device__ __forceinline__ void count_zero_steps(StepLog* L, int dX, int dY, int nd) {
    const int z = (int)zero_steps(dX, dY, nd);
    L->zs += z;
    L->zupd += (int64_t)z * (dY + 1);
}

// Head run in the heads' own layout (entry i = coefficient of x^(deg - i)),
// the form head_run_log takes for a first step whose shift exceeds
// GCD_MAXSHIFT (big): the two heads then cannot share one window. Each step
// reduces the operand of higher degree (A on a tie) and shifts the result
// by its degree drop. Same results and outputs as head_run_log.
template <int E>
__device__ void head_run_rel(const uint32_t (&hA)[E], const uint32_t (&hB)[E], int dA, int dB, int s,
                             const Field& F, StepDesc* desc, StepLog* L, ChunkOut* out, int& n_out,
                             int& big_out) {
    const int lane = threadIdx.x & 63;
    constexpr int H = 64 * E;
    s = uni(s);
    bool xa = uni(dA) >= uni(dB);
    uint32_t hX[E], hY[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        hX[e] = xa ? hA[e] : hB[e];
        hY[e] = xa ? hB[e] : hA[e];
    }
    // the run's state is wave-uniform and stays in scalar registers, so the
    // loop and its branches stay scalar (no exec masking)
    int dX = uni(xa ? dA : dB), dY = uni(xa ? dB : dA);
    int vX = H, vY = H, S = 0, n = 0, unkA = 0, unkB = 0, big = 0;
    uint32_t lcX = (uint32_t)__builtin_amdgcn_readfirstlane((int)hX[0]);
    uint32_t lcY = (uint32_t)__builtin_amdgcn_readfirstlane((int)hY[0]);
    int64_t upd = 0;
    // a first step whose shift alone exceeds MAXSHIFT is taken alone and
    // applied directly (big); later steps stop the run before such a shift
    if (s > 0 && dY >= 0 && dX - dY > GCD_MAXSHIFT) big = 1;
    // one exit test per step, at its end (a single scalar sign test: every
    // term is >= 0 exactly when the run goes on)
    if (s > 0 && dY >= 0) do {
        const int d = dX - dY;  // dX >= dY
        const uint32_t m1 = lcY;
        const uint32_t m2 = F.p - lcX;
        // publish the steps before this one, then record this one: the
        // release waits for this wave's LDS stores, and the last of them was
        // issued a whole step ago (publishing a step right after its record
        // would wait out the LDS write latency on every step)
        if (lane == 0) {
            __hip_atomic_store(&L->prog, n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            desc[n] = StepDesc{m1, m2, d, xa ? 0 : 1};
        }
        const int v = vX < vY ? vX : vY;
        // X <- REDC(m1 X + m2 Y) on the heads; entries at or beyond v cleared
        uint32_t x[E];
#pragma unroll
        for (int e = 0; e < E; e++) {
            const uint32_t t = redc((uint64_t)m1 * hX[e] + (uint64_t)m2 * hY[e], F);
            x[e] = lane + 64 * e < v ? t : 0u;
        }
        // entry 0 cancelled; entry 1 leads unless it vanished too
        const uint32_t next_lc = (uint32_t)__builtin_amdgcn_readlane((int)x[0], 1);
        n++;
        if (!big) S += d;
        upd += dY + 1;
        int nd, nv;
        uint32_t nlc;
        if (__builtin_expect(next_lc != 0u, 1)) {
            head_shift1<E>(x);
            nd = dX - 1;
            nv = v - 1;
            nlc = next_lc;
        } else {
            int delta = 0;
#pragma unroll
            for (int e = E - 1; e >= 0; e--) {
                unsigned long long msk = __ballot(x[e] != 0u);
                if (e == 0) msk &= ~1ull;
                if (msk) delta = 64 * e + (int)__builtin_ctzll(msk);
            }
            if (delta > 1) {
                // positions below deg X vanished too: shift them out, and
                // count the zero-multiplier steps among them (in LDS, so the
                // common path keeps no extra scalar state)
                for (int k = 0; k < delta; k++) head_shift1<E>(x);
                nd = dX - delta;
                nv = v - delta;
                nlc = (uint32_t)__builtin_amdgcn_readfirstlane((int)x[0]);
                if (lane == 0) count_zero_steps(L, dX, dY, nd);
            } else {
                // the first v entries vanished: deg X <= old deg - v
                nd = dX - v;
                nv = 0;
                nlc = 0u;
                if (nd < 0) {
                    nd = -1;
                    if (lane == 0) count_zero_steps(L, dX, dY, nd);
                } else {
                    if (xa) unkA = 1;
                    else unkB = 1;
                    if (lane == 0) {  // the zero steps wait for the true degree
                        out->zX = dX;
                        out->zY = dY;
                    }
                }
            }
        }
        // the next step reduces the operand of higher degree, A on a tie
        if (nd > dY || (nd == dY && xa)) {
#pragma unroll
            for (int e = 0; e < E; e++) hX[e] = x[e];
            dX = nd;
            vX = nv;
            lcX = nlc;
        } else {
#pragma unroll
            for (int e = 0; e < E; e++) {
                hX[e] = hY[e];
                hY[e] = x[e];
            }
            dX = dY;
            dY = nd;
            vX = vY;
            vY = nv;
            lcX = lcY;
            lcY = nlc;
            xa = !xa;
        }
    } while (((s - 1 - n) | dY | (GCD_MAXSHIFT - S - (dX - dY)) | -(unkA | unkB | big)) >= 0);
    n_out = n;
    big_out = big;
    if (lane == 0) {
        out->dA = xa ? dX : dY;
        out->dB = xa ? dY : dX;
        out->upd = upd + L->zupd;
        out->nsteps = n;
        out->S = S;
        out->unkA = unkA;
        out->unkB = unkB;
        out->big = big;
        out->zsteps = L->zs;
        if (!(unkA | unkB)) {
            out->zX = -1;
            out->zY = -1;
        }
        __hip_atomic_store(&L->end, n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// ---------------------------------------------------------------- windows
// A window of E registers holds 64E entries interleaved: entry i is in lane
// i / E of register i % E, so moving every entry by one place is a register
// rename plus one DPP lane shift.

// llvm.amdgcn.writelane: the value (uniform) into one lane (uniform) of old
extern "C" __device__ int pm_writelane_i32(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

__device__ __forceinline__ uint32_t writelane(uint32_t old, uint32_t value, int lane) {
    return (uint32_t)pm_writelane_i32((int)value, lane, (int)old);
}

// lane i <- lane i+1 of x (lane 63 <- 0)
__device__ __forceinline__ uint32_t lanes_next(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
}

// lane i <- lane i-1 of x (lane 0 <- 0)
__device__ __forceinline__ uint32_t lanes_prev(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
}

// A residue below 2p made canonical.
__device__ __forceinline__ uint32_t canon(uint32_t x, uint32_t p) {
    const uint32_t y = x - p;
    return y < x ? y : x;
}

// REDC without its final subtraction: x < p 2^32 gives a value < 2p
// congruent to x 2^-32 (for p = 2, x < 2^32: x mod 2, as redc).
__device__ __forceinline__ uint32_t redc_lazy(uint64_t x, const Field& F) {
    const uint32_t t = (uint32_t)x * F.pinv_neg;
    return (uint32_t)((x + (uint64_t)t * F.p) >> 32);
}

// out[i] = in[i + 1] (0 enters at the end)
template <int E>
__device__ __forceinline__ void window_next(const uint32_t (&in)[E], uint32_t (&out)[E]) {
#pragma unroll
    for (int e = 0; e + 1 < E; e++) out[e] = in[e + 1];
    out[E - 1] = lanes_next(in[0]);
}

// out[i] = in[i + delta], 0 where i + delta is outside the window
// (uniform delta, |delta| < 64E)
template <int E>
__device__ __forceinline__ void window_shift(const uint32_t (&in)[E], int delta, uint32_t (&out)[E]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int e = 0; e < E; e++) {
        // source entry E lane + e + delta = E (lane + q) + r
        const int t = e + delta;
        const int q = t >= 0 ? t / E : -((E - 1 - t) / E);
        const int r = t - E * q;
        uint32_t src = in[0];
#pragma unroll
        for (int j = 1; j < E; j++)
            if (r == j) src = in[j];
        const int sl = lane + q;
        const uint32_t v = (uint32_t)__builtin_amdgcn_ds_bpermute((sl & 63) << 2, (int)src);
        out[e] = (sl >= 0 && sl < 64) ? v : 0u;
    }
}

// Entry k (uniform, 0 <= k < 64E) of a window, to every lane.
template <int E>
__device__ __forceinline__ uint32_t window_at(const uint32_t (&r)[E], int k) {
    const unsigned u = (unsigned)k;
    uint32_t v = r[0];
#pragma unroll
    for (int e = 1; e < E; e++)
        if (u % E == (unsigned)e) v = r[e];
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)(u / E));
}

// The first entry k with lo < k < hi and r[k] != 0, or -1 (uniform bounds;
// canonical entries).
template <int E>
__device__ __forceinline__ int window_first_nonzero(const uint32_t (&r)[E], int lo, int hi) {
    const int lane = threadIdx.x & 63;
    int found = -1;
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int k = E * lane + e;
        const unsigned long long m = __ballot(r[e] != 0u && k > lo && k < hi);
        if (m) {
            const int c = E * (int)__builtin_ctzll(m) + e;
            found = (found < 0 || c < found) ? c : found;
        }
    }
    return found;
}

// Head run by one whole wave. hA/hB: the heads, entry i = coefficient of
// x^(deg - i) in the interleaved layout, exact for i < 64E. Each step
// reduces the operand of higher degree (A on a tie) by the other,
// X <- REDC(lc(Y) X + (p - lc(X)) x^d Y). The run holds both operands in one
// window, entry k being the coefficient of x^(base - k) with base the higher
// starting degree, so a step's shift d moves Y by d entries, the new leading
// coefficient is read in place and the roles change without moving data.
// An entry is exact below its operand's limit (V): X's new limit is
// min(V_X, V_Y - d). A step whose new leading coefficient lies at or beyond
// the limit ends the run with its degree unknown. Entries are kept below 2p
// (reduced lazily); leading coefficients and multipliers are canonical.
// The descriptors gather in lanes (step j in lane j mod 64) and go to
// desc[] every 8 steps or so, each flush published to the M builder on
// another wave (m_build_live) through L->prog, the last by L->end. A step
// recorded with which = 2 is an A step with d = 0 whose next record is a B
// step with d = 1 (a round, composed at once by the M builder).
// Returns the chunk summary through *out (lane 0 writes) and the step
// count and big flag in n_out / big_out; a big step is desc[0].
template <int E>
__device__ void head_run_log(const uint32_t (&hA)[E], const uint32_t (&hB)[E], int dA, int dB, int s,
                             const Field& F, StepDesc* desc, StepLog* L, ChunkOut* out, int& n_out,
                             int& big_out) {
    const int lane = threadIdx.x & 63;
    constexpr int H = 64 * E;
    s = uni(s);
    dA = uni(dA);
    dB = uni(dB);
    {
        const int dX = dA >= dB ? dA : dB, dY = dA >= dB ? dB : dA;
        if (s > 0 && dY >= 0 && dX - dY > GCD_MAXSHIFT) {
            // the relative form takes the heads with entry i in lane i mod 64
            // of register i / 64
            uint32_t cA[E], cB[E];
#pragma unroll
            for (int c = 0; c < E; c++) {
                const int i = lane + 64 * c;
                uint32_t va = 0u, vb = 0u;
#pragma unroll
                for (int j = 0; j < E; j++) {
                    const uint32_t a = (uint32_t)__builtin_amdgcn_ds_bpermute((i / E) << 2, (int)hA[j]);
                    const uint32_t b = (uint32_t)__builtin_amdgcn_ds_bpermute((i / E) << 2, (int)hB[j]);
                    va = i % E == j ? a : va;
                    vb = i % E == j ? b : vb;
                }
                cA[c] = va;
                cB[c] = vb;
            }
            head_run_rel<E>(cA, cB, dA, dB, s, F, desc, L, out, n_out, big_out);
            return;
        }
    }
    int n = 0, S = 0, unkA = 0, unkB = 0, flushed = 0;
    int64_t upd = 0;
    // Descriptors not yet flushed, step j in lane j mod 64: wm1 = m1 | kind
    // << 30 (m1 < p < 2^30), wm2 = m2, wd = d for kinds 0 and 1. Kinds: 0 X =
    // A, 1 X = B, 2 a round's A step (d = 0), 3 a round's B step (d = 1).
    uint32_t wm1 = 0u, wm2 = 0u, wd = 0u;
    uint32_t rA[E], rB[E];
    int VA = H, VB = H, base = 0;
    uint32_t lcA = (uint32_t)__builtin_amdgcn_readfirstlane((int)hA[0]);
    uint32_t lcB = (uint32_t)__builtin_amdgcn_readfirstlane((int)hB[0]);
    // The helpers below are lambdas over the run's state, all forced inline:
    // one left as a call-like closure keeps the windows (rA, rB) addressable,
    // and the compiler then mirrors them in scratch memory, storing them on
    // every round of the tie loop and reloading them (a wait on memory) each
    // time the loop is entered.
    // desc[j] for flushed <= j < upto, from lane j mod 64, then published
    auto flush = [&](int upto) __attribute__((always_inline)) {
        const int j = flushed + ((lane - flushed) & 63);
        if (j < upto) {
            const uint32_t kind = wm1 >> 30;
            const int which = kind == 2u ? 2 : (int)(kind & 1u);
            const int d = kind >= 2u ? (int)kind - 2 : (int)wd;
            desc[j] = StepDesc{wm1 & 0x3fffffffu, wm2, d, which};
        }
        flushed = upto;
        if (lane == 0) __hip_atomic_store(&L->prog, upto, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    if (s > 0 && dA >= 0 && dB >= 0) {
        // the window: the operand of higher degree as it is, the other moved
        // up by the degree gap
        base = dA >= dB ? dA : dB;
        if (dA >= dB) {
#pragma unroll
            for (int e = 0; e < E; e++) rA[e] = hA[e];
            window_shift<E>(hB, -(dA - dB), rB);
        } else {
#pragma unroll
            for (int e = 0; e < E; e++) rB[e] = hB[e];
            window_shift<E>(hA, -(dB - dA), rA);
        }
        // A step's new leading coefficient when entry kX + 1 did not give it
        // (it vanished, or it is not exact): the first non-zero exact entry
        // below the old leading one, X = 0, or an unknown degree (the run
        // ends). Sets dX, lcX and the zero-multiplier steps.
        auto resolve = [&](auto role, int dXo, int dY, int VX, int kX) __attribute__((always_inline)) {
            constexpr bool XA = decltype(role)::value;
            uint32_t(&X)[E] = XA ? rA : rB;
#pragma unroll
            for (int e = 0; e < E; e++) X[e] = canon(X[e], F.p);
            const int v = VX - kX;
            int nd;
            uint32_t nlc = 0u;
            const int k = window_first_nonzero<E>(X, kX + 1, VX);
            if (k >= 0) {
                nd = base - k;
                nlc = window_at<E>(X, k);
                if (lane == 0) count_zero_steps(L, dXo, dY, nd);
            } else {
                // every exact entry below the old leading one vanished
                nd = dXo - v;
                if (nd < 0) {
                    nd = -1;
                    if (lane == 0) count_zero_steps(L, dXo, dY, nd);
                } else {
                    (XA ? unkA : unkB) = 1;
                    if (lane == 0) {  // the zero steps wait for the true degree
                        out->zX = dXo;
                        out->zY = dY;
                    }
                }
            }
            (XA ? dA : dB) = nd;
            (XA ? lcA : lcB) = nlc;
        };
        // The step's descriptor into lane n mod 64 (d only for kinds 0, 1).
        auto record = [&](uint32_t m1, uint32_t m2, uint32_t kind) __attribute__((always_inline)) {
            const int l = n & 63;
            wm1 = writelane(wm1, m1 | (kind << 30), l);
            wm2 = writelane(wm2, m2, l);
        };
        // One step with X = A (XA) or X = B; d >= 0. Each role has its own
        // copy of the step, so a step moves no data between the operands.
        auto step = [&](auto role) __attribute__((always_inline)) {
            constexpr bool XA = decltype(role)::value;
            uint32_t(&X)[E] = XA ? rA : rB;
            const uint32_t(&Y)[E] = XA ? rB : rA;
            const int dX = XA ? dA : dB;
            const int dY = XA ? dB : dA;
            int& VX = XA ? VA : VB;
            const int VY = XA ? VB : VA;
            const uint32_t lcX = XA ? lcA : lcB;
            const uint32_t lcY = XA ? lcB : lcA;
            const int d = dX - dY;
            const uint32_t m1 = lcY;
            const uint32_t m2 = F.p - lcX;
            record(m1, m2, XA ? 0u : 1u);
            wd = writelane(wd, (uint32_t)d, n & 63);
            uint32_t ys[E];
            if (d == 0) {
#pragma unroll
                for (int e = 0; e < E; e++) ys[e] = Y[e];
            } else if (d == 1) {
                window_next<E>(Y, ys);
            } else {
                window_shift<E>(Y, d, ys);
            }
            // entries below 2p in, canonical out
#pragma unroll
            for (int e = 0; e < E; e++) X[e] = redc((uint64_t)m1 * X[e] + (uint64_t)m2 * ys[e], F);
            VX = VX < VY - d ? VX : VY - d;
            n++;
            S += d;
            upd += dY + 1;
            const int kX = base - dX;
            const int v = VX - kX;  // exact entries from the old leading one on
            const uint32_t nlc = v >= 2 ? window_at<E>(X, kX + 1) : 0u;
            if (__builtin_expect(nlc != 0u, 1)) {
                (XA ? dA : dB) = dX - 1;
                (XA ? lcA : lcB) = nlc;
            } else {
                resolve(role, dX, dY, VX, kX);
            }
        };
        for (;;) {
            // Rounds of the generic pattern from a tie deg A = deg B = D: A is
            // reduced by B (no shift) down to D - 1, then B by x A (shift 1)
            // down to D - 1, a tie again. A round takes 2 steps and 1 of the
            // shift budget; it is exact when its two new leading entries are
            // (k + 2 < min(V_A, V_B), k = base - D), and the counts of all its
            // rounds are settled at once. A vanishing leading entry ends the
            // rounds after its step, through resolve.
            if (dA == dB && dA >= 0) {
                const int D0 = dA;
                int k = base - D0;
                int rounds = 0;
                int why = 0;  // 1: A's new leading entry vanished, 2: B's
                uint32_t la = 0u;
                // Round r leaves V_A = minV0 - r and V_B = minV0 - r - 1, so
                // the limits on the rounds are known up front: the steps
                // left, the shift budget, and exactness (k + 2 < minV).
                const int minV0 = VA < VB ? VA : VB;
                int R = (s - n) / 2;
                R = R < GCD_MAXSHIFT - S ? R : GCD_MAXSHIFT - S;
                R = R < (minV0 - k - 1) / 2 ? R : (minV0 - k - 1) / 2;
                for (int r = 0; r < R; r++) {
                    const int minV = minV0 - r;
                    // A <- REDC(lcB A + (p - lcA) B)
                    const uint32_t m1 = uni(lcB), m2 = F.p - uni(lcA);
                    record(m1, m2, 2u);
#pragma unroll
                    for (int e = 0; e < E; e++) rA[e] = redc((uint64_t)m1 * rA[e] + (uint64_t)m2 * rB[e], F);
                    n++;
                    VA = minV;
                    la = window_at<E>(rA, k + 1);
                    if (__builtin_expect(la == 0u, 0)) {
                        why = 1;
                        break;
                    }
                    // B <- REDC(lcA B + (p - lcB) x A), deg B = deg A + 1
                    const uint32_t n2 = F.p - m1;
                    record(la, n2, 3u);
                    uint32_t xa[E];
                    window_next<E>(rA, xa);
#pragma unroll
                    for (int e = 0; e < E; e++) rB[e] = redc((uint64_t)la * rB[e] + (uint64_t)n2 * xa[e], F);
                    n++;
                    VB = minV - 1;
                    const uint32_t lb = window_at<E>(rB, k + 1);
                    lcA = la;
                    if (__builtin_expect(lb == 0u, 0)) {
                        why = 2;
                        break;
                    }
                    lcB = lb;
                    rounds++;
                    k++;
                    if (n - flushed >= 8) flush(n);
                }
                // the complete rounds: the sum over them of (D + 1) + D,
                // D = D0, D0 - 1, ...
                upd += (int64_t)rounds * (2 * D0 + 1) - (int64_t)rounds * (rounds - 1);
                S += rounds;
                const int D = D0 - rounds;
                dA = dB = D;
                if (why == 1) {
                    // the A step at the tie D stands alone (kind 0, d = 0)
                    wm1 = writelane(wm1, lcB, (n - 1) & 63);
                    wd = writelane(wd, 0u, (n - 1) & 63);
                    upd += D + 1;
                    resolve(std::true_type{}, D, D, VA, k);
                } else if (why == 2) {
                    // the round's A step (to D - 1), then B of degree D by
                    // x A of degree D - 1
                    upd += (D + 1) + D;
                    S += 1;
                    dA = D - 1;
                    resolve(std::false_type{}, D, D - 1, VB, k);
                }
                if (n - flushed >= 8) flush(n);
                const int ndX = dA >= dB ? dA : dB, ndY = dA >= dB ? dB : dA;
                if (((s - 1 - n) | ndY | (GCD_MAXSHIFT - S - (ndX - ndY)) | -(unkA | unkB)) < 0) break;
            }
            if (dA >= dB) step(std::true_type{});  // A on a tie
            else step(std::false_type{});
            if (n - flushed >= 8) flush(n);
            // the next step: steps left, both operands non-zero, its shift
            // within the chunk's matrix, and every degree known
            const int ndX = dA >= dB ? dA : dB, ndY = dA >= dB ? dB : dA;
            if (((s - 1 - n) | ndY | (GCD_MAXSHIFT - S - (ndX - ndY)) | -(unkA | unkB)) < 0) break;
        }
    }
    flush(n);
    n_out = n;
    big_out = 0;
    if (lane == 0) {
        out->dA = dA;
        out->dB = dB;
        out->upd = upd + L->zupd;
        out->nsteps = n;
        out->S = S;
        out->unkA = unkA;
        out->unkB = unkB;
        out->big = 0;
        out->zsteps = L->zs;
        if (!(unkA | unkB)) {
            out->zX = -1;
            out->zY = -1;
        }
        __hip_atomic_store(&L->end, n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// One step on M's rows: (P, Q) <- REDC(m1 (P, Q) + m2 x^d (R, T)); rows
// below 2p in, canonical out.
__device__ __forceinline__ void m_row_step(uint32_t& P, uint32_t& Q, uint32_t R, uint32_t T, uint32_t m1,
                                           uint32_t m2, int d, const Field& F) {
    if (d == 1) {
        R = lanes_prev(R);
        T = lanes_prev(T);
    } else if (d != 0) {
        R = lanes_up(R, d);
        T = lanes_up(T, d);
    }
    P = redc((uint64_t)m1 * P + (uint64_t)m2 * R, F);
    Q = redc((uint64_t)m1 * Q + (uint64_t)m2 * T, F);
}

// Composes M from the steps of a head run while it goes on (one whole
// wave, lane k = coefficient k of alpha, beta, gamma, delta): each published
// step (rows of X) <- REDC(m1 (rows of X) + m2 x^d (rows of Y)) is applied
// as soon as it appears, a round (a record with which = 2 and the next) as
// one update of both rows from the rows before it, with the head run's c1,
// c2. The published records are read a batch at a time, record k + j on
// lane j. Entries stay below 2p until the end. Writes M to LDS as 4 rows of
// 64 canonical words. Waits only on the head run, which never waits on it.
__device__ void m_build_live(const StepDesc* desc, StepLog* L, const Field& F, uint32_t* M) {
    const int lane = threadIdx.x & 63;
    uint32_t al = lane == 0 ? 1u : 0u, be = 0u, ga = 0u, de = lane == 0 ? 1u : 0u;
    int k = 0;
    for (;;) {
        // end, once set, publishes every step (the run's last step is
        // published by end alone); before that, prog is the count
        const int end = uni(__hip_atomic_load(&L->end, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
        const int avail =
            end >= 0 ? end : uni(__hip_atomic_load(&L->prog, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (k < avail) {
            const int cnt = avail - k < 64 ? avail - k : 64;
            StepDesc D{0u, 0u, 0, 0};
            if (lane < cnt) D = desc[k + lane];
            int i = 0;
            while (i < cnt) {
                const uint32_t m1 = (uint32_t)__builtin_amdgcn_readlane((int)D.m1, i);
                const uint32_t m2 = (uint32_t)__builtin_amdgcn_readlane((int)D.m2, i);
                const int w = __builtin_amdgcn_readlane(D.which, i);
                if (w == 2 && i + 1 < cnt) {
                    const uint32_t n1 = (uint32_t)__builtin_amdgcn_readlane((int)D.m1, i + 1);
                    const uint32_t n2 = (uint32_t)__builtin_amdgcn_readlane((int)D.m2, i + 1);
                    const uint32_t cv = redc((uint64_t)(lane == 0 ? m1 : m2) * n2, F);
                    const uint32_t c1 = (uint32_t)__builtin_amdgcn_readlane((int)cv, 0);
                    const uint32_t c2 = (uint32_t)__builtin_amdgcn_readlane((int)cv, 1);
                    const uint32_t xal = lanes_prev(al), xbe = lanes_prev(be);
                    const uint32_t xga = lanes_prev(ga), xde = lanes_prev(de);
                    const uint32_t nga = redc((uint64_t)n1 * ga + (uint64_t)c1 * xal + (uint64_t)c2 * xga, F);
                    const uint32_t nde = redc((uint64_t)n1 * de + (uint64_t)c1 * xbe + (uint64_t)c2 * xde, F);
                    al = redc_lazy((uint64_t)m1 * al + (uint64_t)m2 * ga, F);
                    be = redc_lazy((uint64_t)m1 * be + (uint64_t)m2 * de, F);
                    ga = nga;
                    de = nde;
                    i += 2;
                } else {
                    const int d = __builtin_amdgcn_readlane(D.d, i);
                    if ((w & 1) == 0) m_row_step(al, be, ga, de, m1, m2, d, F);
                    else m_row_step(ga, de, al, be, m1, m2, d, F);
                    i += 1;
                }
            }
            k += cnt;
        }
        if (end >= 0 && k >= end) break;
        if (k >= avail) __builtin_amdgcn_s_sleep(1);
    }
    M[lane] = canon(al, F.p);
    M[64 + lane] = canon(be, F.p);
    M[128 + lane] = canon(ga, F.p);
    M[192 + lane] = canon(de, F.p);
}

// New coefficients at G positions of one lane: (A'[P], B'[P]) is the sum
// over k = 0..S of M's coefficients k times the chunk-start A[P-k], B[P-k],
// read through la/lb at local index x + stride*j (j < G) clamped to xmax (a
// clamped position's sum is not used; the caller's staging or padding
// covers the indexes down to x - S). Each coefficient of M read from LDS
// serves all G positions, and the G sums give the loop independent work
// between its LDS reads.
// MREG: M's rows are taken from registers, mreg[r] holding row r's
// coefficient k on lane k, by a lane read per coefficient instead of an LDS
// read (M itself is then unused).
template <int G, bool MREG = false>
__device__ __forceinline__ void apply_m_strided(const uint32_t* la, const uint32_t* lb, int x, int stride, int xmax,
                                                int S, const uint32_t* M, const Field& F, uint32_t (&outA)[G],
                                                uint32_t (&outB)[G], const uint32_t* mreg = nullptr) {
    uint64_t accA[G], accB[G];
    int xs[G];
#pragma unroll
    for (int j = 0; j < G; j++) {
        accA[j] = accB[j] = 0;
        const int xj = x + stride * j;
        xs[j] = xj < xmax ? xj : xmax;
    }
    uint32_t cnt = 0;
    const uint32_t half = F.fold_every / 2;
    S = uni(S);
    for (int k = 0; k <= S; k++) {
        uint32_t ma, mb, mc, md;
        if constexpr (MREG) {
            ma = (uint32_t)__builtin_amdgcn_readlane((int)mreg[0], k);
            mb = (uint32_t)__builtin_amdgcn_readlane((int)mreg[1], k);
            mc = (uint32_t)__builtin_amdgcn_readlane((int)mreg[2], k);
            md = (uint32_t)__builtin_amdgcn_readlane((int)mreg[3], k);
        } else {
            ma = M[k];
            mb = M[64 + k];
            mc = M[128 + k];
            md = M[192 + k];
        }
#pragma unroll
        for (int j = 0; j < G; j++) {
            const uint32_t a = la[xs[j] - k], b = lb[xs[j] - k];
            accA[j] += (uint64_t)ma * a;
            accA[j] += (uint64_t)mb * b;
            accB[j] += (uint64_t)mc * a;
            accB[j] += (uint64_t)md * b;
        }
        if (++cnt == half) {
#pragma unroll
            for (int j = 0; j < G; j++) {
                accA[j] = fold(accA[j], F.c32);
                accB[j] = fold(accB[j], F.c32);
            }
            cnt = 0;
        }
    }
#pragma unroll
    for (int j = 0; j < G; j++) {
        outA[j] = reduce64(accA[j], F);
        outB[j] = reduce64(accB[j], F);
    }
}

// New coefficients at the four consecutive positions x..x+3 of one lane (x
// a multiple of 4, la and lb 16-byte aligned): (A'[P], B'[P]) is the sum
// over k of M's coefficients k times A[P-k], B[P-k]. The lane slides a
// window of eight values down each array, taking the next four with one
// 16-byte LDS read, so that each value read serves four positions (with
// consecutive lanes four words apart the reads are free of bank
// conflicts). k runs to S + 1 rounded up to 8: M's coefficients above S are
// zero. Words down to index x - 64 must be readable (zeros below position
// 0), and words up to x + 3 (those above the caller's top only feed sums it
// does not store).
__device__ __forceinline__ void apply_m_window4(const uint32_t* la, const uint32_t* lb, int x, int S,
                                                const uint32_t* M, const Field& F, uint32_t (&outA)[4],
                                                uint32_t (&outB)[4]) {
    uint64_t accA[4] = {0, 0, 0, 0}, accB[4] = {0, 0, 0, 0};
    // wa[4 + i] = A[x - k0 + i] and wa[i] = A[x - k0 - 4 + i], i < 4
    uint32_t wa[8], wb[8];
    {
        const uint4 a4 = *(const uint4*)(la + x), b4 = *(const uint4*)(lb + x);
        wa[4] = a4.x; wa[5] = a4.y; wa[6] = a4.z; wa[7] = a4.w;
        wb[4] = b4.x; wb[5] = b4.y; wb[6] = b4.z; wb[7] = b4.w;
    }
    const int kend = (uni(S) + 8) & ~7;
    uint32_t cnt = 0;
    const uint32_t half = F.fold_every / 2;
    for (int k0 = 0; k0 < kend; k0 += 4) {
        {
            const uint4 a4 = *(const uint4*)(la + x - k0 - 4), b4 = *(const uint4*)(lb + x - k0 - 4);
            wa[0] = a4.x; wa[1] = a4.y; wa[2] = a4.z; wa[3] = a4.w;
            wb[0] = b4.x; wb[1] = b4.y; wb[2] = b4.z; wb[3] = b4.w;
        }
#pragma unroll
        for (int kk = 0; kk < 4; kk++) {
            const int k = k0 + kk;
            const uint32_t ma = M[k], mb = M[64 + k], mc = M[128 + k], md = M[192 + k];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t a = wa[4 + j - kk], b = wb[4 + j - kk];
                accA[j] += (uint64_t)ma * a;
                accA[j] += (uint64_t)mb * b;
                accB[j] += (uint64_t)mc * a;
                accB[j] += (uint64_t)md * b;
            }
            if (++cnt == half) {
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    accA[j] = fold(accA[j], F.c32);
                    accB[j] = fold(accB[j], F.c32);
                }
                cnt = 0;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            wa[4 + i] = wa[i];
            wb[4 + i] = wb[i];
        }
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
        outA[j] = reduce64(accA[j], F);
        outB[j] = reduce64(accB[j], F);
    }
}

// One wave copies src[base + x] (0 below position 0) into l[x] for x < len,
// for two arrays at once; all of a lane's loads of a 256-word block are
// issued before the first is waited for.
__device__ __forceinline__ void stage_pair(uint32_t* la, uint32_t* lb, const uint32_t* A, const uint32_t* B,
                                           int64_t base, int len) {
    const int lane = threadIdx.x & 63;
    for (int x0 = 0; x0 < len; x0 += 256) {
        uint32_t va[4], vb[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int x = x0 + lane + 64 * j;
            const int64_t P = base + x;
            const bool in = x < len && P >= 0;
            va[j] = in ? A[P] : 0u;
            vb[j] = in ? B[P] : 0u;
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int x = x0 + lane + 64 * j;
            if (x < len) {
                la[x] = va[j];
                lb[x] = vb[j];
            }
        }
    }
}

// One new coefficient: sum_k Ma[k] la[x-k] + Mb[k] lb[x-k], k = 0..S (one
// row of M applied at local index x; x - k >= 0 guaranteed by the caller).
// Four accumulators (even and odd k, each row) keep the multiply-adds
// independent so the LDS reads of later terms overlap them; each is folded
// after fold_every products, and the four folded sums (each below 2^32 p,
// p < 2^30) add without overflow.
__device__ __forceinline__ uint32_t apply_row_at(const uint32_t* la, const uint32_t* lb, int x, int S,
                                                 const uint32_t* Ma, const uint32_t* Mb, const Field& F) {
    uint64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    uint32_t cnt = 0;
    const uint32_t fe = F.fold_every;
    int k = 0;
#pragma unroll 4
    for (; k + 1 <= S; k += 2) {
        a0 += (uint64_t)Ma[k] * la[x - k];
        b0 += (uint64_t)Mb[k] * lb[x - k];
        a1 += (uint64_t)Ma[k + 1] * la[x - k - 1];
        b1 += (uint64_t)Mb[k + 1] * lb[x - k - 1];
        if (++cnt == fe) {
            a0 = fold(a0, F.c32);
            b0 = fold(b0, F.c32);
            a1 = fold(a1, F.c32);
            b1 = fold(b1, F.c32);
            cnt = 0;
        }
    }
    if (k <= S) {  // after the loop cnt < fe: one more product fits
        a0 += (uint64_t)Ma[k] * la[x - k];
        b0 += (uint64_t)Mb[k] * lb[x - k];
    }
    return reduce64(fold(a0, F.c32) + fold(b0, F.c32) + fold(a1, F.c32) + fold(b1, F.c32), F);
}

}  // namespace pm
