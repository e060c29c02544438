// radix.hip -- the radix-sort case study (Sec. 4) on gfx950: a stable
// least-significant-digit sort of uint32 keys with s-bit digits, ceil(c/s)
// passes. Each pass is the paper's three parallel steps:
//
//  * radix_hist_kernel: each thread-block counts the digit values of its
//    tile (2^s bins) and writes them digit-major, hist[d * tiles + tile];
//  * an exclusive prefix sum over that array (scan_* kernels), after which
//    hist[d * tiles + tile] is where the tile's run of digit d starts in the
//    output;
//  * radix_scatter_kernel: each block ranks its tile stably by digit, sorts
//    the tile in LDS by digit, and writes every digit's run contiguously.
//
// The paper's blocks sort their tile with s iterations of a 1-bit split.
// Here a wave ranks 64 keys at once: s ballots give each lane the mask of
// lanes holding the same digit, and a per-wave counter per digit value
// carries the count across the tile's items, which keeps equal digits in
// input order.
#include "internal.hpp"

namespace pm {
namespace {

constexpr int RS_NT = 256;                     // threads per block (the paper's l)
constexpr int RS_IPT = 16;                     // keys per thread
constexpr int RS_TILE = RS_NT * RS_IPT;        // keys per tile
constexpr int RS_WAVES = RS_NT / 64;
constexpr int SCAN_CHUNK = 4096;               // entries per block of the scan

// Position in the tile of item j of a lane: wave-striped, so that item j of
// the 64 lanes of a wave are 64 consecutive keys.
__device__ __forceinline__ int tile_pos(int wave, int j, int lane) { return wave * 64 * RS_IPT + j * 64 + lane; }

// Mask of the lanes whose digit equals this lane's (valid lanes only).
template <int S>
__device__ __forceinline__ unsigned long long match_digit(uint32_t d, bool valid) {
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < S; b++) {
        const bool bit = (d >> b) & 1u;
        const unsigned long long bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

// Exclusive prefix sum over the block's 256 threads of v; *total gets the
// sum. Uses s_tmp[RS_WAVES].
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_tmp[wave] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; w++) {
        const uint32_t t = s_tmp[w];
        before += w < wave ? t : 0u;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// The histogram needs no order: with few digit values each wave counts
// them with one ballot per value; with many, each lane adds to its wave's
// own copy of the bins in LDS, reading four keys per 16-byte load.
template <int S>
__global__ __launch_bounds__(RS_NT) void radix_hist_kernel(const uint32_t* keys, int64_t n, int shift, uint32_t mask,
                                                           uint32_t* hist, int64_t tiles) {
    constexpr int R = 1 << S;
    __shared__ uint32_t cnt[RS_WAVES][R];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < RS_WAVES * R; i += RS_NT) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    if constexpr (S <= 3) {
        uint32_t mine[R];
#pragma unroll
        for (int v = 0; v < R; v++) mine[v] = 0;
#pragma unroll 4
        for (int j = 0; j < RS_IPT; j++) {
            const int64_t pos = base + tile_pos(wave, j, lane);
            const bool valid = pos < n;
            const uint32_t d = valid ? (keys[pos] >> shift) & mask : 0u;
#pragma unroll
            for (int v = 0; v < R; v++) mine[v] += (uint32_t)__popcll(__ballot(valid && d == (uint32_t)v));
        }
        if (lane == 0) {
#pragma unroll
            for (int v = 0; v < R; v++) cnt[wave][v] = mine[v];
        }
    } else {
        const bool vec = (((uintptr_t)keys) & 15u) == 0;
#pragma unroll 2
        for (int j = 0; j < RS_IPT / 4; j++) {
            const int64_t pos = base + 4 * ((int64_t)j * RS_NT + tid);
            uint32_t x[4];
            if (vec && pos + 3 < n) {
                const uint4 q = *(const uint4*)(keys + pos);
                x[0] = q.x; x[1] = q.y; x[2] = q.z; x[3] = q.w;
#pragma unroll
                for (int e = 0; e < 4; e++) atomicAdd(&cnt[wave][(x[e] >> shift) & mask], 1u);
            } else {
#pragma unroll
                for (int e = 0; e < 4; e++)
                    if (pos + e < n) atomicAdd(&cnt[wave][(keys[pos + e] >> shift) & mask], 1u);
            }
        }
    }
    __syncthreads();
    for (int d = tid; d < R; d += RS_NT) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < RS_WAVES; w++) c += cnt[w][d];
        hist[(int64_t)d * tiles + blockIdx.x] = c;
    }
}

template <int S>
__global__ __launch_bounds__(RS_NT) void radix_scatter_kernel(const uint32_t* kin, const uint32_t* vin,
                                                              uint32_t* kout, uint32_t* vout, int64_t n, int shift,
                                                              uint32_t mask, const uint32_t* offs, int64_t tiles) {
    constexpr int R = 1 << S;
    __shared__ uint32_t s_key[RS_TILE];
    __shared__ uint32_t s_val[RS_TILE];
    __shared__ uint32_t s_wcnt[RS_WAVES][R];  // per wave: running count, then the wave's base
    __shared__ uint32_t s_dbase[R];           // start of digit d in the locally sorted tile
    __shared__ uint32_t s_gofs[R];            // start of this tile's run of digit d in the output
    __shared__ uint32_t s_tmp[RS_WAVES];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const int count = (int)(n - base < RS_TILE ? n - base : RS_TILE);
    for (int i = tid; i < RS_WAVES * R; i += RS_NT) (&s_wcnt[0][0])[i] = 0;
    uint32_t k[RS_IPT], v[RS_IPT], rank[RS_IPT];
#pragma unroll
    for (int j = 0; j < RS_IPT; j++) {
        const int t = tile_pos(wave, j, lane);
        const bool valid = t < count;
        k[j] = valid ? kin[base + t] : 0u;
        v[j] = (valid && vin) ? vin[base + t] : 0u;
    }
    __syncthreads();
    // stable rank of each key among the keys of its wave with the same digit
    const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int j = 0; j < RS_IPT; j++) {
        const bool valid = tile_pos(wave, j, lane) < count;
        const uint32_t d = (k[j] >> shift) & mask;
        const unsigned long long m = match_digit<S>(d, valid);
        const uint32_t lower = (uint32_t)__popcll(m & lt);
        uint32_t r = 0;
        if (valid) {
            const uint32_t c = s_wcnt[wave][d];
            r = c + lower;
            if (lower == 0) s_wcnt[wave][d] = c + (uint32_t)__popcll(m);
        }
        rank[j] = r;
    }
    __syncthreads();
    // waves before this one, and digits before this one, in the tile (each
    // thread takes DPT consecutive digit values)
    constexpr int DPT = R > RS_NT ? R / RS_NT : 1;
    uint32_t tots[DPT];
    uint32_t mine = 0;
#pragma unroll
    for (int e = 0; e < DPT; e++) {
        const int d = tid * DPT + e;
        uint32_t tot = 0;
        if (d < R) {
#pragma unroll
            for (int w = 0; w < RS_WAVES; w++) {
                const uint32_t c = s_wcnt[w][d];
                s_wcnt[w][d] = tot;
                tot += c;
            }
        }
        tots[e] = tot;
        mine += tot;
    }
    uint32_t all;
    uint32_t run = block_exclusive_scan(mine, s_tmp, &all);
#pragma unroll
    for (int e = 0; e < DPT; e++) {
        const int d = tid * DPT + e;
        if (d < R) {
            s_dbase[d] = run;
            s_gofs[d] = offs[(int64_t)d * tiles + blockIdx.x];
        }
        run += tots[e];
    }
    __syncthreads();
    // the tile sorted by digit in LDS
#pragma unroll
    for (int j = 0; j < RS_IPT; j++) {
        if (tile_pos(wave, j, lane) < count) {
            const uint32_t d = (k[j] >> shift) & mask;
            const uint32_t at = s_dbase[d] + s_wcnt[wave][d] + rank[j];
            if (at < (uint32_t)RS_TILE) {  // always (the ranks are a permutation of the tile)
                s_key[at] = k[j];
                s_val[at] = v[j];
            }
        }
    }
    __syncthreads();
    // each digit's run goes out contiguously
    for (int i = tid; i < count; i += RS_NT) {
        const uint32_t key = s_key[i];
        const uint32_t d = (key >> shift) & mask;
        const int64_t at = (int64_t)s_gofs[d] + (i - (int64_t)s_dbase[d]);
        if (at < n) {  // always (the histogram and the ranks count the same keys)
            kout[at] = key;
            if (vout) vout[at] = s_val[i];
        }
    }
}

// ---------------------------------------------------------- exclusive scan
// sums[b] = sum of x[b * SCAN_CHUNK .. +SCAN_CHUNK)
__global__ __launch_bounds__(RS_NT) void scan_reduce_kernel(const uint32_t* x, int64_t m, uint32_t* sums) {
    __shared__ uint32_t s_tmp[RS_WAVES];
    const int64_t lo = (int64_t)blockIdx.x * SCAN_CHUNK;
    uint32_t acc = 0;
    for (int i = threadIdx.x; i < SCAN_CHUNK; i += RS_NT)
        if (lo + i < m) acc += x[lo + i];
    uint32_t all;
    block_exclusive_scan(acc, s_tmp, &all);
    if (threadIdx.x == 0) sums[blockIdx.x] = all;
}

// sums becomes its exclusive prefix sum (one block, pieces of 256).
__global__ __launch_bounds__(RS_NT) void scan_top_kernel(uint32_t* sums, int64_t nsums) {
    __shared__ uint32_t s_tmp[RS_WAVES];
    uint32_t carry = 0;
    for (int64_t lo = 0; lo < nsums; lo += RS_NT) {
        const int64_t i = lo + threadIdx.x;
        const uint32_t v = i < nsums ? sums[i] : 0u;
        uint32_t all;
        const uint32_t ex = block_exclusive_scan(v, s_tmp, &all);
        if (i < nsums) sums[i] = carry + ex;
        carry += all;
    }
}

// x becomes its exclusive prefix sum, chunk b starting from sums[b].
__global__ __launch_bounds__(RS_NT) void scan_down_kernel(uint32_t* x, int64_t m, const uint32_t* sums) {
    __shared__ uint32_t s_tmp[RS_WAVES];
    constexpr int PER = SCAN_CHUNK / RS_NT;  // consecutive entries per thread
    const int64_t lo = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * PER;
    uint32_t v[PER];
    uint32_t acc = 0;
#pragma unroll
    for (int e = 0; e < PER; e++) {
        v[e] = lo + e < m ? x[lo + e] : 0u;
        acc += v[e];
    }
    uint32_t all;
    uint32_t run = sums[blockIdx.x] + block_exclusive_scan(acc, s_tmp, &all);
#pragma unroll
    for (int e = 0; e < PER; e++) {
        if (lo + e < m) x[lo + e] = run;
        run += v[e];
    }
}

template <int S>
hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, int64_t n,
                      int shift, int bits, uint32_t* hist, uint32_t* sums, hipStream_t stream) {
    const int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    const int64_t m = ((int64_t)1 << S) * tiles;
    const int64_t chunks = (m + SCAN_CHUNK - 1) / SCAN_CHUNK;
    const uint32_t mask = (uint32_t)((1ull << bits) - 1);
    {
        TimingScope ts("radix_hist_kernel", stream);
        hipLaunchKernelGGL((radix_hist_kernel<S>), dim3((unsigned)tiles), dim3(RS_NT), 0, stream, kin, n, shift,
                           mask, hist, tiles);
    }
    {
        TimingScope ts("radix_scan", stream);
        hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)chunks), dim3(RS_NT), 0, stream, hist, m, sums);
        hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(RS_NT), 0, stream, sums, chunks);
        hipLaunchKernelGGL(scan_down_kernel, dim3((unsigned)chunks), dim3(RS_NT), 0, stream, hist, m, sums);
    }
    {
        TimingScope ts("radix_scatter_kernel", stream);
        hipLaunchKernelGGL((radix_scatter_kernel<S>), dim3((unsigned)tiles), dim3(RS_NT), 0, stream, kin, vin, kout,
                           vout, n, shift, mask, hist, tiles);
    }
    return hipGetLastError();
}

}  // namespace

int64_t radix_scratch_words(int64_t n, int s, bool with_vals) {
    const int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    const int64_t m = ((int64_t)1 << s) * tiles;
    const int64_t chunks = (m + SCAN_CHUNK - 1) / SCAN_CHUNK;
    return (with_vals ? 2 : 1) * ((n + 63) & ~63LL) + ((m + 63) & ~63LL) + chunks + 64;
}

hipError_t radix_sort_launch(const uint32_t* keys, const uint32_t* vals, int64_t n, int key_bits, int s,
                             uint32_t* keys_out, uint32_t* vals_out, uint32_t* scratch, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int passes = (key_bits + s - 1) / s;
    const int64_t nr = (n + 63) & ~63LL;
    uint32_t* tk = scratch;
    uint32_t* tv = vals ? scratch + nr : nullptr;
    uint32_t* hist = scratch + (vals ? 2 : 1) * nr;
    const int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    const int64_t m = ((int64_t)1 << s) * tiles;
    uint32_t* sums = hist + ((m + 63) & ~63LL);
    // the last pass writes keys_out: pass i writes buffer i % 2
    uint32_t* kb[2];
    uint32_t* vb[2];
    kb[(passes - 1) % 2] = keys_out;
    kb[passes % 2] = tk;
    vb[(passes - 1) % 2] = vals ? vals_out : nullptr;
    vb[passes % 2] = tv;
    for (int i = 0; i < passes; i++) {
        const int shift = i * s;
        const int bits = key_bits - shift < s ? key_bits - shift : s;
        const uint32_t* kin = i == 0 ? keys : kb[(i - 1) % 2];
        const uint32_t* vin = vals ? (i == 0 ? vals : vb[(i - 1) % 2]) : nullptr;
        uint32_t* ko = kb[i % 2];
        uint32_t* vo = vals ? vb[i % 2] : nullptr;
        hipError_t e;
        switch (s) {
            case 1: e = radix_pass<1>(kin, vin, ko, vo, n, shift, bits, hist, sums, stream); break;
            case 2: e = radix_pass<2>(kin, vin, ko, vo, n, shift, bits, hist, sums, stream); break;
            case 3: e = radix_pass<3>(kin, vin, ko, vo, n, shift, bits, hist, sums, stream); break;
            case 4: e = radix_pass<4>(kin, vin, ko, vo, n, shift, bits, hist, sums, stream); break;
            case 5: e = radix_pass<5>(kin, vin, ko, vo, n, shift, bits, hist, sums, stream); break;
            case 6: e = radix_pass<6>(kin, vin, ko, vo, n, shift, bits, hist, sums, stream); break;
            case 7: e = radix_pass<7>(kin, vin, ko, vo, n, shift, bits, hist, sums, stream); break;
            case 8: e = radix_pass<8>(kin, vin, ko, vo, n, shift, bits, hist, sums, stream); break;
            case 9: e = radix_pass<9>(kin, vin, ko, vo, n, shift, bits, hist, sums, stream); break;
            case 10: e = radix_pass<10>(kin, vin, ko, vo, n, shift, bits, hist, sums, stream); break;
            default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pm
