// mul_mfma.hip -- the plain (schoolbook) product of Sec. 5 on the CDNA4
// matrix cores.
//
// The product f_k = sum_i a_i b_{k-i} is a dense contraction: cut a and the
// outputs into blocks of 64 positions; then output block K is
//
//     f[64K + u] = sum_J sum_v  b[64J + u - v] * a[64(K-J) + v],
//
// i.e. for each block offset J a 64x64 Toeplitz matrix of b times the column
// K-J of the 64 x (n_a/64) matrix of a-blocks. Every coefficient product of
// the schoolbook method appears exactly once, and nothing else.
//
// Exactness on int8 matrix cores. Each residue x < 2^30 is written in signed
// base-256 digits, x = sum_e d_e 256^e with d_0..d_2 in [-128, 127] and
// d_3 in [0, 64]; the digits come from two integer operations,
// (x + 0x808080) ^ 0x808080 read as four signed bytes. One coefficient
// product is then the 16 digit products d_j(b) d_i(a), weighted 256^(i+j).
// v_mfma_i32_16x16x64_i8 forms 64-term sums of digit products exactly in
// int32: |d d'| <= 2^14, so a sum over at most 512 block offsets (2^15
// terms) stays below 2^29. The 16 weighted sums are combined exactly in
// int64 and reduced modulo p once, when a work-group finishes an output
// range. All of it is exact, so the
// result is bit-identical to the plain definition.
//
// GEMM mapping for one 16x16x64 instruction: rows (u, j) = 4 outputs x 4
// digits of b (the Toeplitz side), columns (K, i) = 4 output blocks x 4
// digits of a, contraction over v in [0, 64).
//
//  * a work-group (8 waves, one per CU) owns 64 outputs u x 64 output
//    blocks K (4096 consecutive outputs, one "range" kr); wave w owns u in
//    [16(w mod 4), +16) (4 row tiles: u = 16(w mod 4) + 4t + ul) and the 32
//    blocks of half w div 4 (8 column tiles), 32 accumulator tiles. The two
//    waves on a SIMD belong to the same work-group and meet at every stage,
//    so they stay in step and finish together;
//  * b's digits are staged in LDS, reversed, in 4 copies shifted by 0..3
//    bytes. A lane reads the copy that cancels its ul, and then the four row
//    tiles of one offset J are 16-byte windows at dword steps inside one
//    16-byte-aligned 32-byte window: two LDS reads per step for all 4 tiles;
//  * a's digits are staged in LDS in 4 digit planes. Column tile m holds
//    blocks K0 + m + 8q (q = 0..3), so from one offset J to the next, tile m
//    becomes tile m-1 and tile 0 is tile 7 shifted by one q (a DPP row
//    shift) plus one new 16-byte read: the 8 column tiles form a register
//    ring that returns to its starting registers every 8 offsets;
//  * work is split stream-K in groups of 8 offsets: the (range, offset
//    group) iterations are cut into equal contiguous shares, one per
//    work-group; a work-group writes its partial sums (canonical residues) each
//    time it leaves a range, and mulx_reduce_kernel adds the partial sums of
//    each range (the paper's addition phase). Range bounds are rounded out to
//    whole groups; the extra offsets meet only zeros of a or b.
//
// The paper's parameter s (b-coefficients per thread-block) is the staging
// chunk here: JC offsets, i.e. 64*JC = 4096 coefficients of b per LDS stage.
#include "internal.hpp"

#include <hip/hip_ext.h>

#include <map>
#include <mutex>
#include <tuple>

namespace pm {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int MX_T = 64;            // positions per block
constexpr int MX_KW = 64;           // output blocks per range
constexpr int MX_RANGE = MX_T * MX_KW;  // outputs per range (4096)
constexpr int MX_GRP = 8;           // offsets per iteration (one turn of the ring)
constexpr int MX_JC = 64;           // block offsets per LDS stage
constexpr int MX_MAXGRP = 64;       // groups one share sums (512 offsets, |digit sum| < 2^29)
constexpr int MX_THREADS = 512;

// LDS layout (bytes).
constexpr int MX_ANEED = (MX_KW + MX_JC - 1) * MX_T;
constexpr int MX_APL = MX_ANEED + 16;  // a digit plane; /16 odd (conflict-free reads)
constexpr int MX_BPL = 4176;        // b plane (copy o, digit j): /16 odd, >= JC*64 + 64
constexpr int MX_BWORDS = MX_BPL / 4;
constexpr int MX_RAW = MX_BPL + 16; // packed b digits, reversed
constexpr int MX_LDS_A = 0;
constexpr int MX_LDS_B = MX_LDS_A + 4 * MX_APL;
constexpr int MX_LDS_RAW = MX_LDS_B + 16 * MX_BPL;
constexpr int MX_LDS_BYTES = MX_LDS_RAW + 4 * MX_RAW;

static_assert(MX_APL % 16 == 0 && (MX_APL / 16) % 2 == 1, "a plane");
static_assert(MX_BPL >= MX_JC * MX_T + 64 && (MX_BPL / 16) % 2 == 1, "b plane");
static_assert(MX_JC % MX_GRP == 0, "stage of whole groups");
static_assert(4 * (MX_BWORDS - 1) + 8 <= MX_RAW, "raw window");

}  // namespace

// Iteration space of one product (MxGeom in internal.hpp): ranges kr of
// 4096 outputs x block offsets J. Range kr needs the offsets
// [max(0, 64kr - nab_true + 1), min(nJ_true, 64kr + 64)); rounded out to
// whole groups of 8 this is [lo(kr), hi(kr)) with the same formulas on
// MxGeom's rounded nab and nJ. Iterations are counted in groups. Shared by
// the host planner and the kernels.
__host__ __device__ inline int64_t mx_lo(const MxGeom& g, int64_t r) {
    int64_t v = MX_KW * r - g.nab + 1;
    return v > 0 ? v : 0;
}
__host__ __device__ inline int64_t mx_hi(const MxGeom& g, int64_t r) {
    int64_t v = MX_KW * r + MX_KW;
    return v < g.nJ ? v : g.nJ;
}
// Groups before range kr: sum over r < kr of (hi(r) - lo(r)) / 8, in closed
// form (hi is linear until it reaches nJ, lo is zero until 64r reaches nab).
__host__ __device__ inline int64_t mx_prefix(const MxGeom& g, int64_t kr) {
    const int64_t r1 = g.nJ / MX_KW;
    const int64_t m = kr < r1 ? kr : r1;
    const int64_t sh = (int64_t)(MX_KW / 2) * m * (m + 1) + (kr - m) * g.nJ;
    const int64_t r0 = (g.nab + MX_KW - 1) / MX_KW;
    int64_t sl = 0;
    if (kr > r0) {
        const int64_t c = kr - r0;
        sl = (int64_t)MX_KW * ((r0 + kr - 1) * c / 2) + (1 - g.nab) * c;
    }
    return (sh - sl) / MX_GRP;
}
__host__ __device__ inline int64_t mx_groups(const MxGeom& g, int64_t kr) {
    return (mx_hi(g, kr) - mx_lo(g, kr)) / MX_GRP;
}
// The range holding group x (0 <= x < itot).
__host__ __device__ inline int64_t mx_range_of(const MxGeom& g, int64_t x) {
    int64_t lo = 0, hi = g.nkr - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (mx_prefix(g, mid) <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}
__host__ __device__ inline int64_t mx_share_begin(const MxGeom& g, int64_t w) { return w * g.itot / g.G; }
// The work-group whose share holds group x.
__host__ __device__ inline int64_t mx_group_of(const MxGeom& g, int64_t x) {
    return ((x + 1) * g.G + g.itot - 1) / g.itot - 1;
}

namespace {

struct MxArgs {
    const uint32_t* a;
    const uint32_t* b;
    MxGeom g;
    uint32_t* part;       // G * maxseg * 2048 partial residues
    uint32_t* flags;      // G range-check flags
    uint32_t* f;
    int64_t nf;
    const uint32_t* sub;  // when set, f[k] = sub[k] - (a b)[k] for k < nf
    int64_t* out_len;
    int32_t* out_status;
    Field F;
    uint32_t w[7];        // 256^e mod p
    uint32_t c63;         // 2^63 mod p
    int a_vec;            // a is 16-byte aligned
    int b_vec;            // b is 16-byte aligned
};

__device__ __forceinline__ uint32_t digits(uint32_t x) { return (x + 0x808080u) ^ 0x808080u; }

// 4x4 byte transpose: byte m of out[j] = byte j of in[m].
__device__ __forceinline__ void transpose4(const uint32_t in[4], uint32_t out[4]) {
    uint32_t t0 = __builtin_amdgcn_perm(in[1], in[0], 0x05010400u);  // in0.b0 in1.b0 in0.b1 in1.b1
    uint32_t t1 = __builtin_amdgcn_perm(in[3], in[2], 0x05010400u);  // in2.b0 in3.b0 in2.b1 in3.b1
    uint32_t t2 = __builtin_amdgcn_perm(in[1], in[0], 0x07030602u);  // in0.b2 in1.b2 in0.b3 in1.b3
    uint32_t t3 = __builtin_amdgcn_perm(in[3], in[2], 0x07030602u);  // in2.b2 in3.b2 in2.b3 in3.b3
    out[0] = __builtin_amdgcn_perm(t1, t0, 0x05040100u);
    out[1] = __builtin_amdgcn_perm(t1, t0, 0x07060302u);
    out[2] = __builtin_amdgcn_perm(t3, t2, 0x05040100u);
    out[3] = __builtin_amdgcn_perm(t3, t2, 0x07060302u);
}

// Four consecutive coefficients p[idx .. idx+3] (idx a multiple of 4),
// zero outside [0, n); one 16-byte load when the quad is whole and p is
// 16-byte aligned.
__device__ __forceinline__ uint4 load_quad(const uint32_t* p, int64_t idx, int64_t n, int vec) {
    if (vec && idx >= 0 && idx + 3 < n) return *(const uint4*)(p + idx);
    uint4 v;
    v.x = (idx >= 0 && idx < n) ? p[idx] : 0u;
    v.y = (idx + 1 >= 0 && idx + 1 < n) ? p[idx + 1] : 0u;
    v.z = (idx + 2 >= 0 && idx + 2 < n) ? p[idx + 2] : 0u;
    v.w = (idx + 3 >= 0 && idx + 3 < n) ? p[idx + 3] : 0u;
    return v;
}

constexpr int MX_AQ = MX_ANEED / 4;                          // a quads per stage
constexpr int MX_BQ = MX_RAW / 4;                            // b quads per stage
constexpr int MX_AQT = (MX_AQ + MX_THREADS - 1) / MX_THREADS;  // per thread
constexpr int MX_BQT = (MX_BQ + MX_THREADS - 1) / MX_THREADS;
static_assert(MX_RAW % 16 == 0, "b window in whole aligned quads");

// Stage the digits of one (range, J-chunk) into LDS. a window: positions
// a0 .. a0 + (KW+JC-1)*64 of a, a0 = 64*(K0 - Js - JC + 1); b window: the
// positions 64*J1 - 1 - t, t in [0, MX_RAW), J1 = Js + JC, reversed. All
// global loads are issued before any is used.
__device__ __forceinline__ uint32_t mx_stage(const MxArgs& A, uint8_t* lds, int64_t K0, int64_t Js) {
    const int tid = threadIdx.x;
    const uint32_t p = A.F.p;
    uint32_t bad = 0;
    const int64_t a0 = (K0 - Js - MX_JC + 1) * MX_T;
    const int64_t b0 = (Js + MX_JC) * MX_T - MX_RAW;   // lowest b position of the window
    uint4 va[MX_AQT], vb[MX_BQT];
#pragma unroll
    for (int k = 0; k < MX_AQT; k++) {
        const int it = tid + k * MX_THREADS;
        va[k] = it < MX_AQ ? load_quad(A.a, a0 + 4 * it, A.g.na, A.a_vec) : uint4{0, 0, 0, 0};
    }
#pragma unroll
    for (int k = 0; k < MX_BQT; k++) {
        const int c = tid + k * MX_THREADS;
        vb[k] = c < MX_BQ ? load_quad(A.b, b0 + 4 * c, A.g.nb, A.b_vec) : uint4{0, 0, 0, 0};
    }
#pragma unroll
    for (int k = 0; k < MX_AQT; k++) {
        const int it = tid + k * MX_THREADS;
        if (it < MX_AQ) {
            const uint32_t c[4] = {va[k].x, va[k].y, va[k].z, va[k].w};
            uint32_t d[4], q[4];
#pragma unroll
            for (int m = 0; m < 4; m++) {
                bad |= c[m] >= p;
                d[m] = digits(c[m]);
            }
            transpose4(d, q);
#pragma unroll
            for (int j = 0; j < 4; j++) *(uint32_t*)(lds + MX_LDS_A + j * MX_APL + 4 * it) = q[j];
        }
    }
    // raw[t] = digits of b[64*J1 - 1 - t]: quad c (positions b0 + 4c ..) lands
    // reversed at raw[MX_RAW - 4 - 4c ..]
    uint32_t* raw = (uint32_t*)(lds + MX_LDS_RAW);
#pragma unroll
    for (int k = 0; k < MX_BQT; k++) {
        const int c = tid + k * MX_THREADS;
        if (c < MX_BQ) {
            bad |= (vb[k].x >= p) | (vb[k].y >= p) | (vb[k].z >= p) | (vb[k].w >= p);
            *(uint4*)(raw + MX_RAW - 4 - 4 * c) =
                uint4{digits(vb[k].w), digits(vb[k].z), digits(vb[k].y), digits(vb[k].x)};
        }
    }
    __syncthreads();
    // copy o (0..3) of digit plane j: byte y = digit j of raw[y + o]
    for (int y4 = tid; y4 < MX_BWORDS; y4 += MX_THREADS) {
        const uint4 lo = *(const uint4*)(raw + 4 * y4);
        const uint4 hi = *(const uint4*)(raw + 4 * y4 + 4);
        const uint32_t W[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
        for (int o = 0; o < 4; o++) {
            uint32_t d[4], q[4];
#pragma unroll
            for (int m = 0; m < 4; m++) d[m] = W[o + m];
            transpose4(d, q);
#pragma unroll
            for (int j = 0; j < 4; j++) *(uint32_t*)(lds + MX_LDS_B + (4 * o + j) * MX_BPL + 4 * y4) = q[j];
        }
    }
    return bad;
}

__device__ __forceinline__ v4i ld_b128(const uint8_t* lds, int off) { return *(const v4i*)(lds + off); }
__device__ __forceinline__ v4i ld_2b64(const uint8_t* lds, int off) {
    const int2* q = (const int2*)(lds + off);
    int2 lo = q[0], hi = q[1];
    return v4i{lo.x, lo.y, hi.x, hi.y};
}

// The value of the lane i ^ 1 (resp. i ^ 2) of the same quad.
__device__ __forceinline__ int64_t quad_xor1(int64_t v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, 0xb1 /* quad_perm 1,0,3,2 */, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0xb1, 0xf, 0xf, false);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int64_t quad_xor2(int64_t v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, 0x4e /* quad_perm 2,3,0,1 */, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0x4e, 0xf, 0xf, false);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// x mod p for a signed 64-bit x with |x| < 2^63.
__device__ __forceinline__ uint32_t smod(int64_t x, const MxArgs& A) {
    uint32_t r = reduce64((uint64_t)x ^ (UINT64_C(1) << 63), A.F);
    return r >= A.c63 ? r - A.c63 : r + A.F.p - A.c63;
}

// The LDS addresses of a lane: bwin, its Toeplitz window (copy o = 3 - ul
// of digit plane j; at offset jj the 32 bytes from bwin + (JC - jj)*64 hold
// row tile t in dwords 3-t .. 6-t), and acol, its a columns (plane i, block
// 32wk + m + 8q + JC - 1 - jj, k-slot group g).
struct MxLane {
    int bwin, acol, q;
};
__device__ __forceinline__ MxLane mx_lane() {
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wu = wave & 3, wk = wave >> 2;  // u slice [16wu, +16), block half [32wk, +32)
    const int g = lane >> 4;            // k-slot group: v in [16g, 16g+16)
    const int rl = lane & 15;           // row (A side) / column (B side) of the 16x16 tile
    const int ul = rl >> 2, dj = rl & 3;   // A side: output u = 16*wu + 4t + ul, digit j of b
    const int q = rl >> 2, di = rl & 3;    // B side: block K = K0 + 32*wk + m + 8q, digit i of a
    return MxLane{MX_LDS_B + (4 * (3 - ul) + dj) * MX_BPL - 16 - 16 * wu + 16 * g,
                  MX_LDS_A + di * MX_APL + 16 * g + 32 * wk * MX_T, q};
}

// Accumulates the digit sums of output range K0 (= 64 kr) over the block
// offsets [Ja, Jend) (whole groups of 8) into acc, staging a and b a
// JC-offset chunk at a time. Called by the whole work-group; returns the
// range-check bits of the staged coefficients.
__device__ __forceinline__ uint32_t mx_range(const MxArgs& A, uint8_t* lds, const MxLane& L, int64_t K0, int64_t Ja,
                                             int64_t Jend, v4i (&acc)[4][8]) {
    const int bwin = L.bwin, acol = L.acol, q = L.q;
    uint32_t bad = 0;
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
        for (int m = 0; m < 8; m++) acc[t][m] = v4i{0, 0, 0, 0};

    // block offsets fit in 32 bits (at most nb / 64 + 1); 32-bit loop
    // bounds keep their compares on the scalar unit
    const int ja = (int)Ja, jend = (int)Jend;
    for (int js = ja; js < jend; js += MX_JC) {
        const int64_t Js = js;
        const int ngrp = (jend - js < MX_JC ? jend - js : MX_JC) / MX_GRP;
        const int last = ngrp * MX_GRP - 1;
        __syncthreads();  // the previous stage is no longer read
        bad |= mx_stage(A, lds, K0, Js);
        __syncthreads();
        v4i B[8];
#pragma unroll
        for (int m = 0; m < 8; m++) B[m] = ld_b128(lds, acol + (m + 8 * q + MX_JC - 1) * MX_T);
        // two Toeplitz windows, used alternately: offset jj reads window
        // jj mod 2 while the next offset's window loads into the other
        v4i Wa0 = ld_b128(lds, bwin + MX_JC * MX_T), Wa1 = ld_b128(lds, bwin + MX_JC * MX_T + 16);
        v4i Wb0 = Wa0, Wb1 = Wa1;

        for (int grp = 0; grp < ngrp; grp++) {
#pragma unroll
            for (int ph = 0; ph < MX_GRP; ph++) {
                const int jj = grp * MX_GRP + ph;
                const int jn = jj < last ? jj + 1 : last;  // next offset (clamped, stays in the stage)
                // new column for tile 0 at the next offset (only the q = 0
                // lanes keep it; the others take tile 7's q - 1 part)
                const v4i fresh = ld_b128(lds, acol + (MX_JC - 1 - jn) * MX_T);
                const v4i C0 = (ph & 1) ? Wb0 : Wa0, C1 = (ph & 1) ? Wb1 : Wa1;
                if (ph & 1) {
                    Wa0 = ld_b128(lds, bwin + (MX_JC - jn) * MX_T);
                    Wa1 = ld_b128(lds, bwin + (MX_JC - jn) * MX_T + 16);
                } else {
                    Wb0 = ld_b128(lds, bwin + (MX_JC - jn) * MX_T);
                    Wb1 = ld_b128(lds, bwin + (MX_JC - jn) * MX_T + 16);
                }
                // the three reads above stay ahead of this offset's MFMAs: they
                // are used one step later (window) or after all 32 (fresh)
                __builtin_amdgcn_sched_barrier(0);
                const v4i At[4] = {v4i{C0[3], C1[0], C1[1], C1[2]}, v4i{C0[2], C0[3], C1[0], C1[1]},
                                   v4i{C0[1], C0[2], C0[3], C1[0]}, C0};
#pragma unroll
                for (int t = 0; t < 4; t++)
#pragma unroll
                    for (int m = 0; m < 8; m++)
                        acc[t][m] = __builtin_amdgcn_mfma_i32_16x16x64_i8(At[t], B[(m - ph) & 7], acc[t][m], 0, 0, 0);
                const int slot = (7 - ph) & 7;
#pragma unroll
                for (int c = 0; c < 4; c++)
                    B[slot][c] = __builtin_amdgcn_update_dpp(fresh[c], B[slot][c], 0x114 /* row_shr:4 */, 0xf, 0xf,
                                                             false);
                // keep each offset's tile assembly after the previous
                // offset's MFMAs, so its LDS reads have a whole step to land
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    return bad;
}

// Epilogue: f[64K + u] = sum_{i,j} 256^(i+j) C_ij. Lane (u, K, i) holds C_ij
// for j = 0..3 of every column tile; the four lanes i of a quad share (u,
// K). Through a wave-private LDS exchange, lane i of a quad collects the
// 16 C_ij of column tile m0 + i, forms the 7 diagonal sums S_s = sum over
// i + j = s of C_ij in int32 (|S_s| <= 4 * 2^29), and then sum_s w_s S_s in
// int64 (16 products below 2^59: below 2^63), reduced modulo p once. The
// residues of the range go to LDS and leave in coalesced 16-byte stores:
// out[x] for x < nlim, x = (K - K0)*64 + u. Called by the whole work-group
// after its last MFMA; reuses the staging LDS.
constexpr int MX_EX_STRIDE = 20;  // words per lane in the exchange (16, padded)
constexpr int MX_EPI_EX = 0;
constexpr int MX_EPI_RES = MX_EPI_EX + (MX_THREADS / 64) * 64 * MX_EX_STRIDE * 4;
static_assert(MX_EPI_RES + MX_RANGE * 4 <= MX_LDS_BYTES, "epilogue LDS");

__device__ __forceinline__ void mx_epilogue(const MxArgs& A, const v4i (&acc)[4][8], uint8_t* lds, uint32_t* out,
                                            int64_t nlim) {
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wu = wave & 3, wk = wave >> 2;
    const int rl = lane & 15;
    const int q = rl >> 2, di = rl & 3;
    uint32_t* ex = (uint32_t*)(lds + MX_EPI_EX) + wave * 64 * MX_EX_STRIDE;
    uint32_t* res = (uint32_t*)(lds + MX_EPI_RES);
    const int qbase = lane & ~3;
    __syncthreads();  // every wave is done with the staged operands
#pragma unroll
    for (int t = 0; t < 4; t++) {
#pragma unroll
        for (int m0 = 0; m0 < 8; m0 += 4) {
#pragma unroll
            for (int dm = 0; dm < 4; dm++) *(v4i*)(ex + lane * MX_EX_STRIDE + 4 * dm) = acc[t][m0 + dm];
            __builtin_amdgcn_wave_barrier();
            v4i C[4];
#pragma unroll
            for (int i = 0; i < 4; i++) C[i] = *(const v4i*)(ex + (qbase + i) * MX_EX_STRIDE + 4 * di);
            __builtin_amdgcn_wave_barrier();
            const int32_t S[7] = {C[0][0],
                                  C[0][1] + C[1][0],
                                  C[0][2] + C[1][1] + C[2][0],
                                  C[0][3] + C[1][2] + C[2][1] + C[3][0],
                                  C[1][3] + C[2][2] + C[3][1],
                                  C[2][3] + C[3][2],
                                  C[3][3]};
            int64_t v = 0;
#pragma unroll
            for (int e = 0; e < 7; e++) v += (int64_t)A.w[e] * S[e];
            res[(32 * wk + m0 + di + 8 * q) * MX_T + 16 * wu + 4 * t + (lane >> 4)] = smod(v, A);
        }
    }
    __syncthreads();
    const bool vec = ((uintptr_t)out & 15) == 0;
    for (int x = 4 * tid; x < MX_RANGE; x += 4 * MX_THREADS) {
        const uint4 r = *(const uint4*)(res + x);
        if (vec && x + 3 < nlim) {
            *(uint4*)(out + x) = r;
        } else {
            if (x < nlim) out[x] = r.x;
            if (x + 1 < nlim) out[x + 1] = r.y;
            if (x + 2 < nlim) out[x + 2] = r.z;
            if (x + 3 < nlim) out[x + 3] = r.w;
        }
    }
}

__global__ __launch_bounds__(MX_THREADS, 1) void mulx_kernel(MxArgs A) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[MX_LDS_BYTES];
    const int tid = threadIdx.x;
    const MxGeom& G = A.g;
    const MxLane L = mx_lane();
    const int64_t w = blockIdx.x;
    const int64_t Ia = mx_share_begin(G, w), Ib = mx_share_begin(G, w + 1);
    uint32_t bad = 0;
    // the share's groups counted from Ia (at most MX_MAXGRP: 32-bit counts
    // keep the loop's compares on the scalar unit)
    const int nshare = (int)(Ib - Ia);
    int64_t kr = Ia < Ib ? mx_range_of(G, Ia) : 0;
    int seg = 0;
    for (int done = 0; done < nshare; seg++, kr++) {
        const int64_t I = Ia + done;
        const int64_t S0 = mx_prefix(G, kr);
        const int64_t left = S0 + mx_groups(G, kr) - I;  // groups of range kr from I on
        const int take = left < nshare - done ? (int)left : nshare - done;
        const int64_t Ja = mx_lo(G, kr) + MX_GRP * (I - S0);
        v4i acc[4][8];
        bad |= mx_range(A, lds, L, kr * MX_KW, Ja, Ja + MX_GRP * take, acc);
        // this share's partial sums of range kr (canonical residues)
        mx_epilogue(A, acc, lds, A.part + ((w * G.maxseg + seg) * MX_RANGE), MX_RANGE);
        done += take;
    }
    bad = __syncthreads_or(bad);
    if (tid == 0) A.flags[w] = bad;
}

// ------------------------------------------------------------------ batched
// Persistent matrix-core product of many independent pairs (one launch):
// each task is one output range of 4096 outputs of one product, summed over
// every block offset of b that meets it (at most 512: b is the shorter
// operand and holds at most 32704 coefficients, so the int32 digit sums stay
// exact), and reduced straight into f. The host sorts the tasks longest
// first; work-group w takes tasks w, 2G - 1 - w, 2G + w, ... (rounds of G
// in alternating directions, which evens out the sums), and loads each
// next task's descriptor while it works on the current one. No counters:
// the launch can be replayed (e.g. from a hipGraph) as it is.
__device__ __forceinline__ int mx_batch_task_at(int round) {
    const int G = (int)gridDim.x, w = (int)blockIdx.x;
    return round * G + ((round & 1) ? G - 1 - w : w);
}

__global__ __launch_bounds__(MX_THREADS, 1) void mulx_batch_kernel(const MxItem* __restrict__ items,
                                                                   const MxTask* __restrict__ tasks, int ntasks) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[MX_LDS_BYTES];
    int round = 0;
    int t = mx_batch_task_at(0);
    if (t >= ntasks) return;
    MxTask tk = tasks[t];
    while (t < ntasks) {
        const int tn = mx_batch_task_at(round + 1);
        const MxTask tkn = tasks[tn < ntasks ? tn : t];  // the next task's descriptor, in flight meanwhile
        const MxItem& it = items[tk.item];
        MxArgs A{};
        A.a = it.a;
        A.b = it.b;
        A.g.na = it.na;
        A.g.nb = it.nb;
        A.g.nab = it.nab;
        A.g.nJ = it.nJ;
        A.F = it.F;
#pragma unroll
        for (int e = 0; e < 7; e++) A.w[e] = it.w[e];
        A.c63 = it.c63;
        A.a_vec = ((uintptr_t)it.a & 15) == 0;
        A.b_vec = ((uintptr_t)it.b & 15) == 0;
        const int64_t kr = tk.kr;
        v4i acc[4][8];
        (void)mx_range(A, lds, mx_lane(), kr * MX_KW, mx_lo(A.g, kr), mx_hi(A.g, kr), acc);
        const int64_t k0 = kr * MX_RANGE;
        mx_epilogue(A, acc, lds, it.f + k0, it.na + it.nb - 1 - k0);
        tk = tkn;
        t = tn;
        round++;
    }
}

// Addition phase: work-group (kr, c), one wave, adds for outputs
// 256c .. 256c+255 of range kr (four consecutive outputs per lane, 16-byte
// loads) the partial sums of the work-groups whose shares touched kr. The
// phase moves a few MB and is bound by the latency of its loads, not by
// bandwidth: every lane issues the loads of up to MX_RED_BATCH rows before
// its first add, and the small work-groups spread the ranges over the CUs.
// The last work-group checks the flags and the degrees.
constexpr int MX_RED_OUT = 256;                       // outputs per work-group
constexpr int MX_RED_THREADS = MX_RED_OUT / 4;        // one wave
constexpr int MX_RED_BLOCKS = MX_RANGE / MX_RED_OUT;  // work-groups per range
constexpr int MX_RED_BATCH = 16;                      // rows in flight per lane
static_assert(MX_RED_THREADS == 64, "the addition phase's work-groups are single waves");

__device__ __forceinline__ void add4(uint64_t s[4], const uint4 v) {
    s[0] += v.x; s[1] += v.y; s[2] += v.z; s[3] += v.w;
}

__global__ __launch_bounds__(MX_RED_THREADS) void mulx_reduce_kernel(MxArgs A) {
    const MxGeom& G = A.g;
    const int tid = threadIdx.x;
    if ((int64_t)blockIdx.x == G.nkr * MX_RED_BLOCKS) {
        if (!A.out_len && !A.out_status) return;
        uint32_t bad = 0;
        for (int64_t w = tid; w < G.G; w += MX_RED_THREADS) bad |= A.flags[w];
        const bool any_bad = __ballot(bad != 0) != 0;
        const int64_t da = top_nonzero_wave(A.a, G.na);
        const int64_t db = top_nonzero_wave(A.b, G.nb);
        if (tid == 0) {
            if (A.out_len) *A.out_len = (da >= 0 && db >= 0) ? da + db + 1 : 0;
            if (A.out_status) *A.out_status = any_bad ? -3 /* PM_ERANGE */ : 0;
        }
        return;
    }
    const int64_t kr = blockIdx.x / MX_RED_BLOCKS;
    const int x = (int)(blockIdx.x % MX_RED_BLOCKS) * MX_RED_OUT + 4 * tid;
    const int64_t k = kr * MX_RANGE + x;
    if (k >= A.nf) return;
    const int64_t S0 = mx_prefix(G, kr), S1 = S0 + mx_groups(G, kr);
    const int64_t wf = mx_group_of(G, S0), wl = mx_group_of(G, S1 - 1);
    const int64_t seg0 = kr - mx_range_of(G, mx_share_begin(G, wf));
    const int64_t nrow = wl - wf + 1;
    // row 0 is segment seg0 of share wf; row r > 0 is the first segment of
    // share wf + r, which starts inside range kr
    const uint32_t* part = A.part + x;
    const int64_t stride = G.maxseg * MX_RANGE;   // one work-group's rows
    const uint32_t* row0 = part + (wf * G.maxseg + seg0) * MX_RANGE;
    uint64_t s[4] = {0, 0, 0, 0};
    for (int64_t r0 = 0; r0 < nrow; r0 += MX_RED_BATCH) {
        uint4 v[MX_RED_BATCH];
#pragma unroll
        for (int i = 0; i < MX_RED_BATCH; i++) {
            const int64_t r = r0 + i < nrow ? r0 + i : nrow - 1;  // past the end: a valid row, not added
            v[i] = *(const uint4*)(r == 0 ? row0 : part + (wf + r) * stride);
        }
#pragma unroll
        for (int i = 0; i < MX_RED_BATCH; i++)
            if (r0 + i < nrow) add4(s, v[i]);
    }
    uint32_t r[4] = {reduce64(s[0], A.F), reduce64(s[1], A.F), reduce64(s[2], A.F), reduce64(s[3], A.F)};
    if (A.sub) {
#pragma unroll
        for (int e = 0; e < 4; e++)
            if (k + e < A.nf) r[e] = submod(A.sub[k + e], r[e], A.F.p);
    }
    if (k + 3 < A.nf && ((uintptr_t)(A.f + k) & 15) == 0) {
        *(uint4*)(A.f + k) = uint4{r[0], r[1], r[2], r[3]};
    } else {
#pragma unroll
        for (int e = 0; e < 4; e++)
            if (k + e < A.nf) A.f[k + e] = r[e];
    }
}

uint64_t host_powmod(uint64_t x, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    x %= p;
    while (e) {
        if (e & 1) r = (unsigned __int128)r * x % p;
        x = (unsigned __int128)x * x % p;
        e >>= 1;
    }
    return r;
}

int mx_blocks_per_cu() {
    static int n = 0;
    if (!n) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, (const void*)mulx_kernel, MX_THREADS, 0) != hipSuccess ||
            v < 1)
            v = 1;
        n = v;
    }
    return n;
}

}  // namespace

namespace {
MxGeom mx_plan(int64_t na, int64_t nb, int num_cus, int64_t nout);
}

// Plans are cached per shape: planning walks every share (binary searches),
// which would otherwise cost more host time per call than a small product.
MxGeom mx_geometry(int64_t na, int64_t nb, int num_cus, int64_t nout) {
    static std::mutex mu;
    static std::map<std::tuple<int64_t, int64_t, int, int64_t>, MxGeom> cache;
    const auto key = std::make_tuple(na, nb, num_cus, nout);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const MxGeom g = mx_plan(na, nb, num_cus, nout);
    std::lock_guard<std::mutex> lk(mu);
    if (cache.size() > 4096) cache.clear();
    cache[key] = g;
    return g;
}

namespace {
MxGeom mx_plan(int64_t na, int64_t nb, int num_cus, int64_t nout) {
    MxGeom g{};
    g.na = na;
    g.nb = nb;
    const int64_t nab = (na + MX_T - 1) / MX_T;   // blocks of a
    const int64_t nJ = (nb + 62) / MX_T + 1;      // offsets J with 64J - 63 <= nb - 1
    g.nkr = (nJ + nab - 1 + MX_KW - 1) / MX_KW;
    if (nout > 0 && (nout + MX_RANGE - 1) / MX_RANGE < g.nkr)
        g.nkr = (nout + MX_RANGE - 1) / MX_RANGE;  // only the ranges below nout
    // rounded to whole groups: lo rounded down, hi rounded up
    const int64_t c = (1 - nab) >= 0 ? (1 - nab) / MX_GRP * MX_GRP : -((nab - 1 + MX_GRP - 1) / MX_GRP * MX_GRP);
    g.nab = 1 - c;
    g.nJ = (nJ + MX_GRP - 1) / MX_GRP * MX_GRP;
    g.itot = mx_prefix(g, g.nkr);
    // one share per resident work-group, or whole rounds of them when the
    // shares would exceed MX_MAXGRP groups (equal shares, no straggler round)
    const int64_t round_size = (int64_t)mx_blocks_per_cu() * num_cus;
    const int64_t need = (g.itot + MX_MAXGRP - 1) / MX_MAXGRP;
    int64_t G = (need + round_size - 1) / round_size * round_size;
    if (G > g.itot) G = g.itot;
    if (G > (INT64_C(1) << 20)) G = INT64_C(1) << 20;
    g.G = G;
    int64_t ms = 1, mg = 0;
    for (int64_t w = 0; w < G; w++) {
        const int64_t a = mx_share_begin(g, w), b = mx_share_begin(g, w + 1);
        if (a >= b) continue;
        const int64_t s = mx_range_of(g, b - 1) - mx_range_of(g, a) + 1;
        if (s > ms) ms = s;
        if (b - a > mg) mg = b - a;
    }
    g.maxseg = ms;
    g.maxgrp = mg;
    return g;
}
}  // namespace

bool mx_exact(const MxGeom& g) { return g.maxgrp <= MX_MAXGRP; }

int64_t mulx_scratch_words(const MxGeom& g) { return g.G * g.maxseg * MX_RANGE + g.G; }

int64_t mx_batch_item(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t* f, const Field& F,
                      MxItem* out) {
    MxItem it{};
    it.a = a;
    it.b = b;
    it.f = f;
    it.na = na;
    it.nb = nb;
    const int64_t nab = (na + MX_T - 1) / MX_T;
    const int64_t nJ = (nb + 62) / MX_T + 1;
    const int64_t c = (1 - nab) >= 0 ? (1 - nab) / MX_GRP * MX_GRP : -((nab - 1 + MX_GRP - 1) / MX_GRP * MX_GRP);
    it.nab = 1 - c;
    it.nJ = (nJ + MX_GRP - 1) / MX_GRP * MX_GRP;
    it.F = F;
    for (int e = 0; e < 7; e++) it.w[e] = (uint32_t)host_powmod(256, e, F.p);
    it.c63 = (uint32_t)host_powmod(2, 63, F.p);
    *out = it;
    return (nJ + nab - 1 + MX_KW - 1) / MX_KW;
}

int64_t mx_batch_offsets(const MxItem& it, int64_t kr) {
    MxGeom g{};
    g.nab = it.nab;
    g.nJ = it.nJ;
    return mx_hi(g, kr) - mx_lo(g, kr);
}

hipError_t mulx_batch_launch(const MxItem* d_items, const MxTask* d_tasks, int ntasks, int num_cus,
                             hipStream_t stream) {
    if (ntasks <= 0) return hipSuccess;
    int grid = mx_blocks_per_cu() * num_cus;
    if (grid > ntasks) grid = ntasks;
    TimingScope ts("mulx_batch_kernel", stream);
    hipLaunchKernelGGL(mulx_batch_kernel, dim3((unsigned)grid), dim3(MX_THREADS), 0, stream, d_items, d_tasks, ntasks);
    return hipGetLastError();
}

hipError_t mulx_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, const Field& F, uint32_t* f,
                       const MxGeom& g, uint32_t* scratch, int64_t* out_len, int32_t* out_status,
                       hipStream_t stream, const uint32_t* sub_from, int64_t nout) {
    if (!mx_exact(g)) return hipErrorInvalidValue;  // the int32 digit sums could overflow
    MxArgs A{};
    A.a = a;
    A.b = b;
    A.g = g;
    A.part = scratch;
    A.flags = scratch + g.G * g.maxseg * MX_RANGE;
    A.f = f;
    A.nf = nout > 0 && nout < na + nb - 1 ? nout : na + nb - 1;
    A.sub = sub_from;
    A.out_len = out_len;
    A.out_status = out_status;
    A.F = F;
    for (int e = 0; e < 7; e++) A.w[e] = (uint32_t)host_powmod(256, e, F.p);
    A.c63 = (uint32_t)host_powmod(2, 63, F.p);
    A.a_vec = ((uintptr_t)a & 15) == 0;
    A.b_vec = ((uintptr_t)b & 15) == 0;
    {
        // timed by the launch's own events (hipExtLaunchKernel): separate
        // event records around the kernel cost about 2 us per product
        TimedLaunchEvents te("mulx_kernel");
        if (te.start()) {
            void* args[] = {&A};
            hipError_t e = hipExtLaunchKernel((const void*)mulx_kernel, dim3((unsigned)g.G), dim3(MX_THREADS), args, 0,
                                              stream, te.start(), te.stop(), 0);
            if (e != hipSuccess) return e;
        } else {
            hipLaunchKernelGGL(mulx_kernel, dim3((unsigned)g.G), dim3(MX_THREADS), 0, stream, A);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        te.launched();
    }
    // no timing events around the addition phase: events between the two
    // kernels put a gap of several microseconds into every product
    hipLaunchKernelGGL(mulx_reduce_kernel, dim3((unsigned)(g.nkr * MX_RED_BLOCKS + 1)), dim3(MX_RED_THREADS), 0, stream,
                       A);
    return hipGetLastError();
}

}  // namespace pm
