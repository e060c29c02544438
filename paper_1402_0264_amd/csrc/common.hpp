// common.hpp -- field arithmetic over Z/pZ for gfx950 and the host-side
// constants it needs.
//
// The paper counts one machine-word operation per field operation (Sec. 3,
// problem statement). On CDNA4 the 32x32->64-bit multiply-add
// (v_mad_u64_u32) issues at the full VALU rate, so the hot loops here keep
// the exact 64-bit sums of products and reduce them rarely:
//
//  * lazy accumulation: acc += a*b in 64 bits; after at most `fold_every`
//    products the high word is folded back, acc = hi*(2^32 mod p) + lo, which
//    is one more multiply-add and keeps acc < 2^32*p;
//  * Barrett reduction of a 64-bit value (one 64x64 high product) when a
//    canonical residue is finally needed;
//  * Montgomery reduction (REDC) for the Euclidean steps, whose results only
//    matter up to a unit factor (the remainders are normalised at the end).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

// Constants of one prime, computed on the host (field_params in capi.cpp).
struct Field {
    uint32_t p;
    uint32_t c32;       // 2^32 mod p
    uint32_t pinv_neg;  // -p^{-1} mod 2^32
    uint32_t fold_every;// products that fit in a 64-bit accumulator after a fold
    uint64_t mu;        // floor((2^64 - 1) / p)
};

// x mod p for any 64-bit x. With mu = floor((2^64-1)/p) the estimate
// q = floor(x*mu / 2^64) is at most 2 below floor(x/p), so at most two
// corrections follow.
__device__ __forceinline__ uint32_t reduce64(uint64_t x, const Field& F) {
    uint64_t q = __umul64hi(x, F.mu);
    uint64_t r = x - q * (uint64_t)F.p;
    if (r >= F.p) r -= F.p;
    if (r >= F.p) r -= F.p;
    return (uint32_t)r;
}

__device__ __forceinline__ uint32_t mulmod(uint32_t a, uint32_t b, const Field& F) {
    return reduce64((uint64_t)a * b, F);
}

__device__ __forceinline__ uint32_t addmod(uint32_t a, uint32_t b, uint32_t p) {
    uint32_t s = a + b;
    return s >= p ? s - p : s;
}

__device__ __forceinline__ uint32_t submod(uint32_t a, uint32_t b, uint32_t p) {
    return a >= b ? a - b : a + p - b;
}

// Fold the high word of a lazy accumulator: returns a value congruent to acc
// and below 2^32 * p.
__device__ __forceinline__ uint64_t fold(uint64_t acc, uint32_t c32) {
    return (uint64_t)(uint32_t)(acc >> 32) * c32 + (uint32_t)acc;
}

// Montgomery reduction: returns x * 2^-32 mod p as a canonical residue for
// x < p * 2^32 (p < 2^30). Larger x below 6p^2 (the gcd's sums of three
// products of entries kept below 2p) give a congruent value below 1.5p. For
// p = 2 the host sets pinv_neg = 2^31, and the same steps return x mod 2 for
// x < 2^32 (the only unit mod 2 is 1, so that is the scaled step's value).
__device__ __forceinline__ uint32_t redc(uint64_t x, const Field& F) {
    uint32_t t = (uint32_t)x * F.pinv_neg;
    uint64_t s = x + (uint64_t)t * F.p;     // divisible by 2^32, no overflow
    uint32_t u = (uint32_t)(s >> 32);       // < 2p for x < p 2^32
    uint32_t v = u - F.p;                   // wraps above u when u < p
    return v < u ? v : u;
}

// x^e mod p by square and multiply (Fermat inverse: e = p - 2).
__device__ __forceinline__ uint32_t powmod(uint32_t x, uint32_t e, const Field& F) {
    uint32_t r = 1 % F.p;
    while (e) {
        if (e & 1u) r = mulmod(r, x, F);
        x = mulmod(x, x, F);
        e >>= 1;
    }
    return r;
}

__device__ __forceinline__ uint32_t invmod(uint32_t x, const Field& F) {
    return powmod(x, F.p - 2, F);
}

// Values the whole wave holds identically, moved to scalar registers so that
// loops and branches on them stay scalar (no exec masking).
__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Largest index i < n with v[i] != 0, or -1. Called by one whole wave, which
// scans 64 words at a time from the top; every lane gets the result.
__device__ inline int64_t top_nonzero_wave(const uint32_t* v, int64_t n) {
    const int lane = threadIdx.x & 63;
    for (int64_t hi = n - 1; hi >= 0; hi -= 64) {
        int64_t i = hi - lane;
        bool nz = i >= 0 && v[i] != 0;
        unsigned long long m = __ballot(nz);
        if (m) return hi - (int64_t)__builtin_ctzll(m);
    }
    return -1;
}

// Per-call results that live in device memory (async entry points return
// them there; the synchronous ones copy them back).
struct CallInfo {
    int64_t n0;         // length of the first output (f, q or g)
    int64_t n1;         // length of the second output (r)
    int32_t status;     // pm_status of the device-side checks
    int32_t flags;      // internal
    int64_t deg_a;      // trimmed degrees of the inputs (-1 = zero)
    int64_t deg_b;
    int64_t steps;      // Euclidean division steps (gcd)
    int64_t chunks;     // fused chunks (gcd / divrem)
    int64_t updates;    // coefficient updates, (deg divisor + 1) per step
    uint32_t bar_count; // grid barrier state (persistent kernels)
    uint32_t bar_gen;
    int64_t run_steps;  // gcd: steps with a non-zero multiplier that were run
    uint32_t mult;      // naive gcd: the multiplier of the next step
    uint32_t pad;
};

// Grid-wide barrier of a cooperative launch (all nblocks resident): one
// arrival counter and a generation word in device memory (CallInfo). gen
// is the caller's copy of the generation, read once at kernel start. Every
// wave waits for its own stores to reach the L2; thread 0 then releases the
// block's stores with one agent-scope fence (a fence per wave writes back
// the XCD's L2 once per wave, and those queue), arrives, polls with plain
// coherent loads and acquires once for the block.
__device__ __forceinline__ void grid_sync(CallInfo* info, unsigned nblocks, unsigned& gen) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (nblocks > 1) {
        if (threadIdx.x == 0) {
            __threadfence();
            unsigned arrived = atomicAdd(&info->bar_count, 1u);
            if (arrived == nblocks - 1) {
                atomicExch(&info->bar_count, 0u);
                __threadfence();
                atomicAdd(&info->bar_gen, 1u);
            } else {
                while (__hip_atomic_load(&info->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen)
                    __builtin_amdgcn_s_sleep(1);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
        }
        gen++;
        __syncthreads();
    }
}

}  // namespace pm
