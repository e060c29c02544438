// divrem.hip -- Euclidean division of dense polynomials over Z/pZ on gfx950
// (Sec. 3: naive and optimized division).
//
// The quotient q depends only on the top deg a - deg b + 1 coefficients of a
// (the head) and on the top coefficients of b: step i of the long division
// takes the current leading coefficient of the head, multiplies it by
// lc(b)^{-1} to get one quotient coefficient, and subtracts that multiple of
// the shifted b. As in the paper's optimized division, the steps are fused s
// at a time: one wave runs s consecutive steps on the s-head (the top s
// coefficients still pending, one per lane, no barrier between steps); then
// the whole thread-block applies those s quotient coefficients to the rest
// of the head at once, each coefficient summing its s products lazily in 64
// bits and reducing once. The inverse of lc(b) is computed once (Fermat).
//
// The part of a below deg b only ever receives updates, never feeds a
// decision, so it is done afterwards in one fully parallel launch:
// r_k = a_k - sum_t q_t b_{k-t} for k < deg b, a product with a subtracting
// epilogue (mul.hip).
#include "internal.hpp"

namespace pm {
namespace {

// Degrees (largest non-zero index) of a and b by two waves, range check by
// all threads. Results in the block's shared variables.
__device__ void block_degrees(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb,
                              uint32_t p, int64_t* s_deg, int* s_bad) {
    if (threadIdx.x == 0) *s_bad = 0;
    __syncthreads();
    int bad = 0;
    for (int64_t i = threadIdx.x; i < na; i += blockDim.x) bad |= a[i] >= p;
    for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) bad |= b[i] >= p;
    if (bad) atomicOr(s_bad, 1);
    const int wave = threadIdx.x >> 6;
    if (wave < 2) {
        int64_t d = top_nonzero_wave(wave == 0 ? a : b, wave == 0 ? na : nb);
        if ((threadIdx.x & 63) == 0) s_deg[wave] = d;
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void degrees_kernel(const uint32_t* a, int64_t na, const uint32_t* b,
                                                      int64_t nb, Field F, CallInfo* info) {
    __shared__ int64_t s_deg[2];
    __shared__ int s_bad;
    block_degrees(a, na, b, nb, F.p, s_deg, &s_bad);
    if (threadIdx.x == 0) {
        info->deg_a = s_deg[0];
        info->deg_b = s_deg[1];
        info->status = s_bad ? -3 /* PM_ERANGE */ : 0;
        info->n0 = info->n1 = 0;
        info->steps = info->chunks = info->updates = 0;
    }
}

__global__ __launch_bounds__(DIV_THREADS) void divrem_head_kernel(const uint32_t* a, int64_t na,
                                                                  const uint32_t* b, int64_t nb, Field F,
                                                                  uint32_t* q, int64_t q_cap, int64_t r_cap,
                                                                  uint32_t* h, CallInfo* info, int S) {
    __shared__ int64_t s_deg[2];
    __shared__ int s_bad;
    __shared__ uint32_t s_q[64];
    block_degrees(a, na, b, nb, F.p, s_deg, &s_bad);
    const int64_t da = s_deg[0], db = s_deg[1];
    const int tid = threadIdx.x;
    int status = 0;
    if (s_bad) status = -3;                         // PM_ERANGE
    else if (db < 0) status = -4;                   // PM_EDIVZERO
    const int64_t mu = (status == 0 && da >= db) ? da - db + 1 : 0;
    const int64_t nr_max = (da < db) ? da + 1 : db; // room the remainder may need
    if (status == 0 && (mu > q_cap || nr_max > r_cap)) status = -1;  // PM_EINVAL
    if (tid == 0) {
        info->deg_a = da;
        info->deg_b = db;
        info->status = status;
        info->n0 = status == 0 ? mu : 0;
        info->n1 = 0;
        info->chunks = (mu + S - 1) / S;
        info->steps = mu;
        info->updates = mu * (db + 1);
    }
    if (status != 0 || mu == 0) return;

    // head of a: h[x] = a[db + x], x = 0 .. mu-1
    for (int64_t x = tid; x < mu; x += DIV_THREADS) h[x] = a[db + x];
    const uint32_t inv = invmod(b[db], F);
    __syncthreads();
    const int lane = tid & 63;
    for (int64_t c0 = 0; c0 < mu; c0 += S) {
        const int cs = (int)(mu - c0 < S ? mu - c0 : S);
        const int64_t top = mu - 1 - c0;  // head index of this chunk's first step
        if (tid < 64) {
            // s-head: lane l holds the pending coefficient at head index top - l
            uint32_t val = lane < cs ? h[top - lane] : 0u;
            for (int kk = 0; kk < cs; kk++) {
                uint32_t lead = __builtin_amdgcn_readlane(val, kk);
                uint32_t qk = mulmod(lead, inv, F);
                int64_t d = lane - kk;  // distance below the step's position
                if (lane > kk && lane < cs && d <= db)
                    val = submod(val, mulmod(qk, b[db - d], F), F.p);
                if (lane == 0) {
                    s_q[kk] = qk;
                    q[top - kk] = qk;
                }
            }
        }
        __syncthreads();
        // rest of the head: positions x <= top - cs that these cs steps reach
        const int64_t xhi = top - cs;
        int64_t xlo = top - cs + 1 - db;
        if (xlo < 0) xlo = 0;
        for (int64_t x = xlo + tid; x <= xhi; x += DIV_THREADS) {
            uint64_t acc = 0;
            uint32_t cnt = 0;
            for (int kk = 0; kk < cs; kk++) {
                int64_t d = (top - kk) - x;
                if (d <= db) {
                    acc += (uint64_t)s_q[kk] * b[db - d];
                    if (++cnt == F.fold_every) { acc = fold(acc, F.c32); cnt = 0; }
                }
            }
            h[x] = submod(h[x], reduce64(acc, F), F.p);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void trim_kernel(const uint32_t* r, int64_t n, CallInfo* info) {
    if (threadIdx.x < 64) {
        int64_t d = top_nonzero_wave(r, n);
        if (threadIdx.x == 0) info->n1 = d + 1;
    }
}

}  // namespace

hipError_t degrees_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, const Field& F,
                          CallInfo* info, hipStream_t stream) {
    TimingScope ts("degrees_kernel", stream);
    hipLaunchKernelGGL(degrees_kernel, dim3(1), dim3(256), 0, stream, a, na, b, nb, F, info);
    return hipGetLastError();
}

hipError_t divrem_head_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, const Field& F,
                              uint32_t* q, int64_t q_cap, int64_t r_cap, uint32_t* head, CallInfo* info,
                              int s, hipStream_t stream) {
    if (s < 1) s = 1;
    if (s > 64) s = 64;
    TimingScope ts("divrem_head_kernel", stream);
    hipLaunchKernelGGL(divrem_head_kernel, dim3(1), dim3(DIV_THREADS), 0, stream, a, na, b, nb, F, q, q_cap,
                       r_cap, head, info, s);
    return hipGetLastError();
}

hipError_t trim_launch(const uint32_t* r, int64_t n, CallInfo* info, hipStream_t stream) {
    TimingScope ts("trim_kernel", stream);
    hipLaunchKernelGGL(trim_kernel, dim3(1), dim3(64), 0, stream, r, n, info);
    return hipGetLastError();
}

}  // namespace pm
