// naive.hip -- the naive division and gcd of Sec. 3 and Sec. 6 (Alg. 1/2 and
// Alg. 8/9): one division step per kernel launch, each launch a global
// synchronisation of the whole grid. They are the s = 1 end of the sweeps
// over the program parameter s; the fused kernels (divrem.hip, gcd.hip) are
// the optimized algorithms.
//
// A step's multiplier is formed apart from its update, by the launch before
// it: the division's next quotient term by the thread that updates the next
// leading position, the gcd's next multiplier by the one-wave rescan that
// finds the new degree. A step launch then only subtracts a multiple of the
// divisor, grid-striding over its coefficients; every position it writes is
// written by one thread and read by no other.
#include "internal.hpp"

namespace pm {
namespace {

// deg a, deg b (two waves scanning from the top) and the range check
// (info->flags = 1 when a coefficient is not a residue); resets the call's
// results.
__global__ __launch_bounds__(256) void naive_prep_kernel(const uint32_t* a, int64_t na, const uint32_t* b,
                                                         int64_t nb, uint32_t p, CallInfo* info) {
    __shared__ int s_bad;
    __shared__ int64_t s_deg[2];
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    int bad = 0;
    for (int64_t i = threadIdx.x; i < na; i += 256) bad |= a[i] >= p;
    for (int64_t i = threadIdx.x; i < nb; i += 256) bad |= b[i] >= p;
    if (bad) atomicOr(&s_bad, 1);
    const int wave = threadIdx.x >> 6;
    if (wave < 2) {
        const int64_t d = top_nonzero_wave(wave == 0 ? a : b, wave == 0 ? na : nb);
        if ((threadIdx.x & 63) == 0) s_deg[wave] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        info->deg_a = s_deg[0];
        info->deg_b = s_deg[1];
        info->flags = s_bad;
        info->status = s_bad ? -3 /* PM_ERANGE */ : 0;
        info->n0 = info->n1 = 0;
        info->steps = info->chunks = info->updates = 0;
    }
}

// Division step at head position i (Alg. 1/2): with c = q[i - db], the
// quotient term of position i (formed by the launch before), the positions
// i - db + j, j < db, lose c b[j]; the thread that updates position i - 1,
// the next step's leading position, also forms its term q[i - 1 - db] =
// w[i - 1] lc(b)^-1 from its own new value. For db = 0 nothing is updated
// and the next term is w[i - 1] lc(b)^-1 as it stands.
__global__ __launch_bounds__(256) void naive_div_step_kernel(uint32_t* w, const uint32_t* b, int64_t db, int64_t i,
                                                             uint32_t inv, uint32_t* q, Field F) {
    const uint32_t c = q[i - db];
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < db; j += stride) {
        const int64_t x = i - db + j;
        const uint32_t v = submod(w[x], mulmod(c, b[j], F), F.p);
        w[x] = v;
        if (j == db - 1 && i - 1 >= db) q[i - 1 - db] = mulmod(v, inv, F);
    }
    if (db == 0 && i >= 1 && blockIdx.x == 0 && threadIdx.x == 0) q[i - 1] = mulmod(w[i - 1], inv, F);
}

// The first quotient term, q[da - db] = w[da] lc(b)^-1. One thread.
__global__ __launch_bounds__(64) void naive_div_first_kernel(const uint32_t* w, int64_t da, int64_t db, uint32_t inv,
                                                             uint32_t* q, Field F) {
    if (threadIdx.x == 0) q[da - db] = mulmod(w[da], inv, F);
}

// The multiplier of the next gcd step (Alg. 9), lc(X) lc(Y)^-1 with X the
// operand of higher degree (A on a tie), into info->mult. One thread.
__device__ __forceinline__ void naive_gcd_next_mult(const uint32_t* A, const uint32_t* B, int64_t dA, int64_t dB,
                                                    const Field& F, CallInfo* info) {
    if (dA < 0 || dB < 0) return;
    const bool redA = dA >= dB;
    const uint32_t lx = redA ? A[dA] : B[dB];
    const uint32_t ly = redA ? B[dB] : A[dA];
    info->mult = mulmod(lx, invmod(ly, F), F);
}

__global__ __launch_bounds__(64) void naive_gcd_mult_kernel(const uint32_t* A, const uint32_t* B, Field F,
                                                            CallInfo* info) {
    if (threadIdx.x == 0) naive_gcd_next_mult(A, B, info->deg_a, info->deg_b, F, info);
}

// One step of the naive gcd (Alg. 9) on the working copies A, B with the
// degrees in info: X, the operand of higher degree (A on a tie), loses
// c x^d Y, c = info->mult, d = deg X - deg Y (grid-stride over the
// coefficients of Y below its leading one). Position deg X cancels and is
// left for naive_gcd_rescan_kernel.
__global__ __launch_bounds__(256) void naive_gcd_step_kernel(uint32_t* A, uint32_t* B, Field F, CallInfo* info) {
    const int64_t dA = info->deg_a, dB = info->deg_b;
    if (dA < 0 || dB < 0) return;
    const bool redA = dA >= dB;
    uint32_t* X = redA ? A : B;
    const uint32_t* Y = redA ? B : A;
    const int64_t d = redA ? dA - dB : dB - dA, dY = redA ? dB : dA;
    const uint32_t c = info->mult;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < dY; j += stride)
        X[j + d] = submod(X[j + d], mulmod(c, Y[j], F), F.p);
}

// After a step: clears X's cancelled leading coefficient, finds X's new
// degree below it, counts the step and its updates (deg Y + 1), and forms
// the next step's multiplier. The positions between the old and the new
// leading coefficient that are still at or above deg Y are steps too, each
// with a zero multiplier (the long division visits every position, Alg.
// 1/2): they are counted, not run. One wave.
__global__ __launch_bounds__(64) void naive_gcd_rescan_kernel(uint32_t* A, uint32_t* B, Field F, CallInfo* info) {
    const int64_t dA = info->deg_a, dB = info->deg_b;
    if (dA < 0 || dB < 0) return;
    const bool redA = dA >= dB;
    uint32_t* X = redA ? A : B;
    const int64_t dX = redA ? dA : dB, dY = redA ? dB : dA;
    const int64_t nd = top_nonzero_wave(X, dX);  // indices below dX
    if (threadIdx.x == 0) {
        X[dX] = 0;
        if (redA) info->deg_a = nd;
        else info->deg_b = nd;
        const int64_t floor_ = nd > dY - 1 ? nd : dY - 1;
        const int64_t zero = dX - 1 - floor_ > 0 ? dX - 1 - floor_ : 0;
        info->steps += 1 + zero;
        info->updates += (1 + zero) * (dY + 1);
        naive_gcd_next_mult(A, B, redA ? nd : dA, redA ? dB : nd, F, info);
    }
}

// g = R / lc(R) for R = the non-zero one of A, B (degree dR from info).
__global__ __launch_bounds__(256) void naive_monic_kernel(const uint32_t* A, const uint32_t* B, uint32_t* g,
                                                          int64_t g_cap, Field F, CallInfo* info) {
    const int64_t dA = info->deg_a, dB = info->deg_b;
    const uint32_t* R = dA >= 0 ? A : B;
    const int64_t dR = dA >= 0 ? dA : dB;
    if (dR < 0 || dR + 1 > g_cap) return;
    const uint32_t inv = invmod(R[dR], F);
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k <= dR; k += (int64_t)gridDim.x * 256)
        g[k] = mulmod(R[k], inv, F);
}

unsigned grid_for(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t naive_prep_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, const Field& F,
                             CallInfo* info, hipStream_t stream) {
    TimingScope ts("naive_prep_kernel", stream);
    hipLaunchKernelGGL(naive_prep_kernel, dim3(1), dim3(256), 0, stream, a, na, b, nb, F.p, info);
    return hipGetLastError();
}

hipError_t naive_divrem_launch(uint32_t* w, const uint32_t* b, int64_t da, int64_t db, uint32_t inv, uint32_t* q,
                               const Field& F, hipStream_t stream) {
    unsigned grid = grid_for(db);
    if (grid > 1024) grid = 1024;
    TimingScope ts("naive_div_step_kernel", stream);
    hipLaunchKernelGGL(naive_div_first_kernel, dim3(1), dim3(64), 0, stream, w, da, db, inv, q, F);
    for (int64_t i = da; i >= db; i--) {
        hipLaunchKernelGGL(naive_div_step_kernel, dim3(grid), dim3(256), 0, stream, w, b, db, i, inv, q, F);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t naive_gcd_steps_launch(uint32_t* A, uint32_t* B, int64_t n, int64_t count, const Field& F,
                                  CallInfo* info, hipStream_t stream) {
    unsigned grid = grid_for(n);
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(naive_gcd_mult_kernel, dim3(1), dim3(64), 0, stream, A, B, F, info);
    for (int64_t k = 0; k < count; k++) {
        hipLaunchKernelGGL(naive_gcd_step_kernel, dim3(grid), dim3(256), 0, stream, A, B, F, info);
        hipLaunchKernelGGL(naive_gcd_rescan_kernel, dim3(1), dim3(64), 0, stream, A, B, F, info);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t naive_monic_launch(const uint32_t* A, const uint32_t* B, uint32_t* g, int64_t g_cap, int64_t n,
                              const Field& F, CallInfo* info, hipStream_t stream) {
    unsigned grid = grid_for(n);
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(naive_monic_kernel, dim3(grid), dim3(256), 0, stream, A, B, g, g_cap, F, info);
    return hipGetLastError();
}

}  // namespace pm
