// mul.hip -- plain (schoolbook) product of dense polynomials over Z/pZ on
// gfx950 (Sec. 5: multiplication phase and addition phase).
//
// f_k = sum_i a_i * b_{k-i}. The paper's long multiplication cuts b into
// chunks of s coefficients; each thread-block multiplies one chunk of b by a
// window of a and writes partial sums into rows of an array M, and an
// addition phase adds the rows. Here:
//
//  * a thread-block owns T = 256*R consecutive outputs of one b-chunk of kc
//    coefficients (kc is the paper's s); each thread owns R consecutive
//    outputs and keeps R exact 64-bit sums in registers;
//  * the a window (T + kc - 1 words, the paper's s*l + s - 1) is staged once
//    from HBM into LDS with a padded layout, so that at every step the 64
//    lanes of a wave read 64 distinct banks;
//  * at step j each thread needs one new a value (its window slides by one)
//    and the uniform b_j, which the compiler keeps in scalar registers, so a
//    step is one LDS read plus R v_mad_u64_u32 multiply-adds;
//  * sums are folded every FOLD steps (fold(), one more multiply-add) and
//    reduced to canonical residues once at the end;
//  * with more than one chunk, residues go to row c of M (length
//    n_a + kc - 1, output k = c*kc + x) and mul_reduce_kernel adds the rows,
//    one output per thread, reading M coalesced.
#include "internal.hpp"

namespace pm {
namespace {

struct MulArgs {
    const uint32_t* a;
    const uint32_t* b;
    uint32_t* out;             // f (one chunk) or M (several chunks)
    const uint32_t* sub_from;  // optional: out = sub_from - a*b
    int64_t na, nb;
    int64_t kc;                // b-coefficients per chunk
    int64_t nchunks;
    int64_t rowlen;            // na + kc - 1
    int64_t tiles;             // thread-blocks per chunk
    int64_t out_limit;         // outputs k < out_limit are written (one chunk)
    Field F;
    int64_t* out_len;          // optional: normalised length of f
    int32_t* out_status;       // optional: validation status
};

// Padded LDS address of window index x >= 0: lanes reading x = t*R + c
// (fixed c) are R+1 words apart, an odd stride, so no two share a bank.
template <int R>
__host__ __device__ __forceinline__ int lds_addr(int x) {
    return R > 1 ? x + x / R : x;
}

// Validation block: range check of every coefficient and the normalised
// length of the product.
__device__ void mul_aux_block(const MulArgs& A) {
    __shared__ int64_t s_deg[2];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    int bad = 0;
    for (int64_t i = threadIdx.x; i < A.na; i += blockDim.x) bad |= A.a[i] >= A.F.p;
    for (int64_t i = threadIdx.x; i < A.nb; i += blockDim.x) bad |= A.b[i] >= A.F.p;
    if (bad) atomicOr(&s_bad, 1);
    const int wave = threadIdx.x >> 6;
    if (wave < 2) {
        int64_t d = top_nonzero_wave(wave == 0 ? A.a : A.b, wave == 0 ? A.na : A.nb);
        if ((threadIdx.x & 63) == 0) s_deg[wave] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t da = s_deg[0], db = s_deg[1];
        if (A.out_len) *A.out_len = (da >= 0 && db >= 0) ? da + db + 1 : 0;
        if (A.out_status) *A.out_status = s_bad ? -3 /* PM_ERANGE */ : 0;
    }
}

// One b-chunk of one output tile, accumulated into acc[] (exact 64-bit sums,
// folded every FOLD products). Tile outputs: x0 + tid*R + r relative to the
// chunk start j0 (output k = j0 + x); the chunk is b[j0 .. j0 + kc) with
// b beyond nb read as zero; `lds` holds at least tile_lds_bytes(R, kc).
// Returns with acc folded (below 2^32 p); the caller syncs before reusing
// the LDS.
template <int R, int FOLD>
__device__ __forceinline__ void tile_chunk(const uint32_t* __restrict__ a, int64_t na, const uint32_t* __restrict__ b,
                                           int64_t nb, int64_t x0, int64_t j0, int64_t kc, uint32_t c32,
                                           uint32_t* lds, uint64_t (&acc)[R]) {
    const int tid = threadIdx.x;
    constexpr int T = MUL_THREADS * R;
    constexpr int PAD = R > 1 ? R + 1 : 1;  // padded words per group of R
    // steps of this chunk, rounded up to whole blocks of R (b reads as 0 past nb)
    const int64_t left = nb - j0;
    const int steps = (int)(((left < kc ? left : kc) + R - 1) / R * R);

    // Stage the a window: index w <-> a[x0 - steps + w], w = 0 .. T + steps - 1
    // (w = 0 is one spare word below the window so the last prefetch stays in
    // bounds), then the b chunk (zero past nb).
    const int W = T + steps;
    const int64_t abase = x0 - steps;
    for (int w = tid; w < W; w += MUL_THREADS) {
        int64_t i = abase + w;
        uint32_t v = (i >= 0 && i < na) ? a[i] : 0u;
        lds[lds_addr<R>(w)] = v;
    }
    const int lb = (lds_addr<R>(W) + 7) & ~3;  // b chunk, 16-byte aligned
    for (int j = tid; j < steps; j += MUL_THREADS) lds[lb + j] = j < left ? b[j0 + j] : 0u;
    __syncthreads();

    // Thread window at step jj: w = tid*R + steps + u with u = r - jj; the
    // value of offset u lives in ring[u mod R]. For w = R*g + e (0 <= e < R)
    // the padded address is PAD*g + e, so the load of step v of a block is a
    // constant offset from one address per block.
    uint32_t ring[R];
    {
        const int g0 = PAD * (tid + steps / R);
#pragma unroll
        for (int r = 0; r < R; r++) ring[r] = lds[g0 + r];
    }
    const int nblk = steps / R;
    constexpr int BPF = FOLD >= R ? FOLD / R : 1;  // blocks between folds
    int blk = 0;
    while (blk < nblk) {
        const int stop = blk + BPF < nblk ? blk + BPF : nblk;
        for (; blk < stop; blk++) {
            uint32_t bv[R];
#pragma unroll
            for (int v = 0; v < R; v++) bv[v] = lds[lb + blk * R + v];
            const int gb = PAD * (tid + (nblk - blk - 1));
#pragma unroll
            for (int v = 0; v < R; v++) {
                // next window value (offset u = -(blk*R+v) - 1) replaces the
                // slot that acc[R-1] consumes in this step
                const uint32_t nxt = lds[gb + (R - 1 - v)];
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const int slot = ((r - v) % R + R) % R;
                    acc[r] = (uint64_t)ring[slot] * bv[v] + acc[r];
                }
                ring[(R - 1 - v) % R] = nxt;
                if (FOLD < R && (v + 1) % FOLD == 0) {
#pragma unroll
                    for (int r = 0; r < R; r++) acc[r] = fold(acc[r], c32);
                }
            }
        }
        if (FOLD >= R) {
#pragma unroll
            for (int r = 0; r < R; r++) acc[r] = fold(acc[r], c32);
        }
    }
}

template <int R, int FOLD>
__global__ __launch_bounds__(MUL_THREADS) void mul_tile_kernel(MulArgs A) {
    extern __shared__ uint32_t lds[];
    const int64_t work = A.nchunks * A.tiles;
    // the last block validates (when asked); the others stride over the
    // (chunk, tile) work units
    const int64_t workers = A.out_len || A.out_status ? (int64_t)gridDim.x - 1 : (int64_t)gridDim.x;
    if ((int64_t)blockIdx.x >= workers) {
        mul_aux_block(A);
        return;
    }
    const int tid = threadIdx.x;
    constexpr int T = MUL_THREADS * R;
    for (int64_t w = blockIdx.x; w < work; w += workers) {
        const int64_t c = w / A.tiles;
        const int64_t tile = w - c * A.tiles;
        const int64_t j0 = c * A.kc;
        const int64_t x0 = tile * T;  // first row offset of the tile (output k = j0 + x)
        uint64_t acc[R];
#pragma unroll
        for (int r = 0; r < R; r++) acc[r] = 0;
        tile_chunk<R, FOLD>(A.a, A.na, A.b, A.nb, x0, j0, A.kc, A.F.c32, lds, acc);

        // Epilogue: canonical residues, then either a row of M or f itself.
        const int64_t xt = x0 + (int64_t)tid * R;
        if (A.nchunks > 1) {
            uint32_t* row = A.out + c * A.rowlen;
#pragma unroll
            for (int r = 0; r < R; r++) {
                int64_t x = xt + r;
                if (x < A.rowlen) row[x] = reduce64(acc[r], A.F);
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; r++) {
                int64_t k = xt + r;
                if (k < A.out_limit) {
                    uint32_t v = reduce64(acc[r], A.F);
                    A.out[k] = A.sub_from ? submod(A.sub_from[k], v, A.F.p) : v;
                }
            }
        }
        __syncthreads();  // the next unit restages the LDS
    }
}

// Addition phase: f_k = sum over chunks c of M[c][k - c*kc].
__global__ __launch_bounds__(256) void mul_reduce_kernel(const uint32_t* M, int64_t rowlen, int64_t kc,
                                                         int64_t nchunks, uint32_t* f, int64_t out_limit,
                                                         const uint32_t* sub_from, Field F) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= out_limit) return;
    int64_t c_hi = k / kc;
    if (c_hi > nchunks - 1) c_hi = nchunks - 1;
    int64_t c_lo = k - rowlen + 1;
    c_lo = c_lo <= 0 ? 0 : (c_lo + kc - 1) / kc;
    uint64_t s = 0;
    for (int64_t c = c_lo; c <= c_hi; c++) s += M[c * rowlen + (k - c * kc)];
    uint32_t v = reduce64(s, F);
    f[k] = sub_from ? submod(sub_from[k], v, F.p) : v;
}

// LDS bytes of one thread-block for R outputs per thread and kc steps.
int64_t tile_lds_bytes(int R, int64_t kc) {
    int64_t W = (int64_t)MUL_THREADS * R + kc;
    int64_t padded = R > 1 ? W + W / R : W;
    return (padded + 8 + kc) * (int64_t)sizeof(uint32_t);
}

// Chunk length actually used: a multiple of R, at most nb rounded up, and
// small enough for the tile to fit in LDS.
int64_t effective_kc(const MulPlan& plan, int64_t nb) {
    const int R = plan.r;
    int64_t kc = (plan.kc + R - 1) / R * R;
    const int64_t full = (nb + R - 1) / R * R;
    if (kc >= full) kc = full;
    while (kc > R && tile_lds_bytes(R, kc) > 160 * 1024) kc = (kc / 2 + R - 1) / R * R;
    return kc;
}

// ------------------------------------------------------------------ batched
// Persistent product of many independent pairs (one launch): each task is
// one output tile of T = 256*R outputs of one product, summed over all of b
// in chunks of kc coefficients with the sums kept in registers (no partial
// rows). The host sorts the tasks longest first; thread-block w takes tasks
// w, 2G - 1 - w, 2G + w, ... (rounds of G in alternating directions) and
// loads each next task's descriptor while it works on the current one. No
// counters: the launch can be replayed (e.g. from a hipGraph) as it is.
template <int R, int FOLD>
__global__ __launch_bounds__(MUL_THREADS) void mul_batch_kernel(const MulItem* __restrict__ items,
                                                                const MulTask* __restrict__ tasks, int ntasks,
                                                                int64_t kc) {
    extern __shared__ uint32_t lds[];
    constexpr int T = MUL_THREADS * R;
    const int tid = threadIdx.x;
    const int G = (int)gridDim.x, w = (int)blockIdx.x;
    int round = 0;
    int t = w;
    if (t >= ntasks) return;
    MulTask tk = tasks[t];
    while (t < ntasks) {
        const int tn = (round + 1) * G + (((round + 1) & 1) ? G - 1 - w : w);
        const MulTask tkn = tasks[tn < ntasks ? tn : t];  // the next task's descriptor, in flight meanwhile
        const MulItem it = items[tk.item];
        const int64_t K0 = (int64_t)tk.tile * T;
        const int64_t nf = it.na + it.nb - 1;
        const int64_t nchunks = (it.nb + kc - 1) / kc;
        int64_t c_lo = K0 - it.na + 1;
        c_lo = c_lo <= 0 ? 0 : c_lo / kc;
        int64_t c_hi = (K0 + T - 1) / kc;
        if (c_hi > nchunks - 1) c_hi = nchunks - 1;
        uint64_t acc[R];
#pragma unroll
        for (int r = 0; r < R; r++) acc[r] = 0;
        for (int64_t c = c_lo; c <= c_hi; c++) {
            tile_chunk<R, FOLD>(it.a, it.na, it.b, it.nb, K0 - c * kc, c * kc, kc, it.F.c32, lds, acc);
            __syncthreads();
        }
        const int64_t kt = K0 + (int64_t)tid * R;
#pragma unroll
        for (int r = 0; r < R; r++)
            if (kt + r < nf) it.f[kt + r] = reduce64(acc[r], it.F);
        tk = tkn;
        t = tn;
        round++;
    }
}

// Range check of every coefficient of every item (one block per item).
__global__ __launch_bounds__(256) void mul_batch_check_kernel(const MulItem* __restrict__ items, int32_t* status) {
    const MulItem it = items[blockIdx.x];
    int bad = 0;
    for (int64_t i = threadIdx.x; i < it.na; i += 256) bad |= it.a[i] >= it.F.p;
    for (int64_t i = threadIdx.x; i < it.nb; i += 256) bad |= it.b[i] >= it.F.p;
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) status[blockIdx.x] = bad ? -3 /* PM_ERANGE */ : 0;
}

template <int R, int FOLD>
hipError_t launch_batch(const MulItem* items, const MulTask* tasks, int ntasks, int64_t kc, int grid,
                        hipStream_t stream) {
    size_t lds = (size_t)tile_lds_bytes(R, kc);
    hipLaunchKernelGGL((mul_batch_kernel<R, FOLD>), dim3(grid), dim3(MUL_THREADS), lds, stream, items, tasks, ntasks,
                       kc);
    return hipGetLastError();
}

template <int R>
hipError_t launch_batch_fold(uint32_t fold_min, const MulItem* items, const MulTask* tasks, int ntasks, int64_t kc,
                             int grid, hipStream_t stream) {
    if (fold_min >= 128) return launch_batch<R, 128>(items, tasks, ntasks, kc, grid, stream);
    if (fold_min >= 64) return launch_batch<R, 64>(items, tasks, ntasks, kc, grid, stream);
    if (fold_min >= 32) return launch_batch<R, 32>(items, tasks, ntasks, kc, grid, stream);
    if (fold_min >= 16) return launch_batch<R, 16>(items, tasks, ntasks, kc, grid, stream);
    return launch_batch<R, 8>(items, tasks, ntasks, kc, grid, stream);
}

template <int R>
int batch_blocks_per_cu(int64_t kc) {
    int nb = 0;
    size_t lds = (size_t)tile_lds_bytes(R, kc);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)mul_batch_kernel<R, 64>, MUL_THREADS, lds) !=
            hipSuccess || nb < 1)
        nb = 1;
    return nb;
}

template <int R, int FOLD>
hipError_t launch_tile(const MulArgs& A, int64_t grid, hipStream_t stream) {
    size_t lds = (size_t)tile_lds_bytes(R, A.kc);
    hipLaunchKernelGGL((mul_tile_kernel<R, FOLD>), dim3((unsigned)grid), dim3(MUL_THREADS), lds, stream, A);
    return hipGetLastError();
}

template <int R>
hipError_t launch_fold(const MulArgs& A, int64_t grid, hipStream_t stream) {
    uint32_t fe = A.F.fold_every;
    if (fe >= 128) return launch_tile<R, 128>(A, grid, stream);
    if (fe >= 64) return launch_tile<R, 64>(A, grid, stream);
    if (fe >= 32) return launch_tile<R, 32>(A, grid, stream);
    if (fe >= 16) return launch_tile<R, 16>(A, grid, stream);
    return launch_tile<R, 8>(A, grid, stream);
}

}  // namespace

int64_t mul_batch_tile(int r) { return (int64_t)MUL_THREADS * r; }

int64_t mul_batch_kc(int r, int64_t kc) {
    MulPlan p{r, kc};
    return effective_kc(p, INT64_C(1) << 40);
}

hipError_t mul_batch_launch(const MulItem* d_items, const MulTask* d_tasks, int ntasks, int r, int64_t kc,
                            uint32_t fold_min, int num_cus, hipStream_t stream, int blocks_per_cu) {
    if (ntasks <= 0) return hipSuccess;
    kc = mul_batch_kc(r, kc);
    int per_cu = 1, grid;
    switch (r) {
        case 4: per_cu = batch_blocks_per_cu<4>(kc); break;
        case 8: per_cu = batch_blocks_per_cu<8>(kc); break;
        case 16: per_cu = batch_blocks_per_cu<16>(kc); break;
        default: return hipErrorInvalidValue;
    }
    if (blocks_per_cu > 0 && per_cu > blocks_per_cu) per_cu = blocks_per_cu;
    grid = per_cu * num_cus;
    if (grid > ntasks) grid = ntasks;
    TimingScope ts("mul_batch_kernel", stream);
    switch (r) {
        case 4: return launch_batch_fold<4>(fold_min, d_items, d_tasks, ntasks, kc, grid, stream);
        case 8: return launch_batch_fold<8>(fold_min, d_items, d_tasks, ntasks, kc, grid, stream);
        default: return launch_batch_fold<16>(fold_min, d_items, d_tasks, ntasks, kc, grid, stream);
    }
}

hipError_t mul_batch_check_launch(const MulItem* d_items, int count, int32_t* d_status, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    TimingScope ts("mul_batch_check_kernel", stream);
    hipLaunchKernelGGL(mul_batch_check_kernel, dim3(count), dim3(256), 0, stream, d_items, d_status);
    return hipGetLastError();
}

int64_t mul_scratch_words(int64_t na, int64_t nb, const MulPlan& plan) {
    if (na <= 0 || nb <= 0) return 0;
    int64_t kc = effective_kc(plan, nb);
    if (kc >= nb) return 0;
    int64_t nchunks = (nb + kc - 1) / kc;
    return nchunks * (na + kc - 1);
}

MulPlan mul_default_plan(int64_t na, int64_t nb, int num_cus) {
    MulPlan best{1, 64};
    if (na <= 0 || nb <= 0) return best;
    // products the matrix cores do not take (below about 40M coefficient
    // products): 4 outputs per thread and short b-chunks, as measured on
    // graph-replayed square products of 256 to 6144 terms
    const int64_t lo = na < nb ? na : nb;
    if ((double)na * (double)nb < 40.0e6) {
        if (lo <= 256) return MulPlan{2, 64};
        if (lo <= 512) return MulPlan{4, 64};
        if (lo <= 3072) return MulPlan{4, 128};
        return MulPlan{4, 256};
    }
    const int64_t target = 4LL * num_cus;
    static const int Rs[] = {16, 8, 4, 2, 1};
    static const int64_t KCs[] = {2048, 1024, 512, 256, 128, 64, 32};
    for (int R : Rs) {
        if ((int64_t)MUL_THREADS * R > 2 * (na + nb)) continue;
        for (int64_t kc : KCs) {
            if (kc % R) continue;
            int64_t k = kc < nb ? kc : (nb + R - 1) / R * R;
            int64_t nch = (nb + k - 1) / k;
            int64_t tiles = (na + k - 1 + MUL_THREADS * R - 1) / (MUL_THREADS * R);
            if (nch * tiles >= target) return MulPlan{R, kc};
        }
    }
    // small products: as much parallelism as the sizes allow
    return MulPlan{1, 32};
}

hipError_t mul_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, const Field& F,
                      uint32_t* f, const MulPlan& plan, uint32_t* M, int64_t* out_len, int32_t* out_status,
                      const uint32_t* sub_from, int64_t out_limit, hipStream_t stream) {
    MulArgs A{};
    A.a = a; A.b = b; A.F = F; A.na = na; A.nb = nb; A.sub_from = sub_from;
    A.out_len = out_len; A.out_status = out_status;
    const bool aux = out_len || out_status;
    const int R = plan.r;
    int64_t nf = (na > 0 && nb > 0) ? na + nb - 1 : 0;
    if (out_limit >= 0 && out_limit < nf) nf = out_limit;
    A.out_limit = nf;
    if (nf == 0) {
        if (!aux) return hipSuccess;
        A.nchunks = 0; A.tiles = 0; A.kc = R; A.rowlen = 0; A.out = f;
        TimingScope ts("mul_tile_kernel", stream);
        hipLaunchKernelGGL((mul_tile_kernel<1, 8>), dim3(1), dim3(MUL_THREADS), 8, stream, A);
        return hipGetLastError();
    }
    const int64_t kc = effective_kc(plan, nb);
    A.kc = kc;
    A.nchunks = (nb + kc - 1) / kc;
    A.rowlen = na + kc - 1;
    A.tiles = (A.rowlen + MUL_THREADS * R - 1) / (MUL_THREADS * R);
    A.out = A.nchunks > 1 ? M : f;
    // at most 2^20 blocks (the runtime counts grid*block work-items in 32
    // bits); blocks stride over the remaining (chunk, tile) units
    int64_t units = A.nchunks * A.tiles;
    if (units > (INT64_C(1) << 20)) units = INT64_C(1) << 20;
    int64_t grid = units + (aux ? 1 : 0);
    hipError_t e;
    {
    TimingScope ts("mul_tile_kernel", stream);
    switch (R) {
        case 1: e = launch_fold<1>(A, grid, stream); break;
        case 2: e = launch_fold<2>(A, grid, stream); break;
        case 4: e = launch_fold<4>(A, grid, stream); break;
        case 8: e = launch_fold<8>(A, grid, stream); break;
        case 16: e = launch_fold<16>(A, grid, stream); break;
        case 32: e = launch_fold<32>(A, grid, stream); break;
        default: return hipErrorInvalidValue;
    }
    }
    if (e != hipSuccess || A.nchunks == 1) return e;
    int64_t blocks = (nf + 255) / 256;
    TimingScope ts("mul_reduce_kernel", stream);
    hipLaunchKernelGGL(mul_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, M, A.rowlen, kc,
                       A.nchunks, f, nf, sub_from, F);
    return hipGetLastError();
}

}  // namespace pm
