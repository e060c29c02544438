// valu_peak.hip -- calibration kernels for the rooflines and the model's U
// (libpolymodp_calib.so, driven by paper_1402_0264_amd/calib.py; not part of
// the library's interface).
//
//  * mad_kernel: the exact 32x32->64-bit multiply-add (v_mad_u64_u32) that
//    every coefficient product of the VALU kernels costs, 8 independent
//    accumulators per lane so that issue, not latency, bounds it;
//  * mulmod_kernel: the same products with the kernels' lazy reduction (a
//    fold of the high word every `fold` products, one Barrett reduction at
//    the end): the rate of complete exact mulmods;
//  * chase_kernel: one lane follows a random cycle of indices through a
//    buffer far larger than the caches, so every load is a trip to HBM:
//    cycles per load (the model's U in its latency view).
#include <hip/hip_runtime.h>
#include <stdint.h>

extern "C" {

__global__ __launch_bounds__(256) void mad_kernel(const uint32_t* in, uint64_t* out, int iters) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    uint32_t a[8];
    uint64_t acc[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
        a[j] = in[(t * 8 + j) & 1023];
        acc[j] = j;
    }
    uint32_t b = in[t & 1023] | 1u;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int j = 0; j < 8; j++) acc[j] += (uint64_t)a[j] * b;
        b += 0x9E3779B9u;
    }
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) s ^= acc[j];
    out[t] = s;
}

__global__ __launch_bounds__(256) void mulmod_kernel(const uint32_t* in, uint64_t* out, int iters, uint32_t p,
                                                     uint32_t c32, uint64_t mu, int fold) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    uint32_t a[8];
    uint64_t acc[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
        a[j] = in[(t * 8 + j) & 1023] % p;
        acc[j] = 0;
    }
    uint32_t b = in[t & 1023] % p;
    int cnt = 0;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int j = 0; j < 8; j++) acc[j] += (uint64_t)a[j] * b;
        b += 12345u;  // the next residue (p > 12345)
        b = b >= p ? b - p : b;
        if (++cnt == fold) {
#pragma unroll
            for (int j = 0; j < 8; j++) acc[j] = (uint64_t)(uint32_t)(acc[j] >> 32) * c32 + (uint32_t)acc[j];
            cnt = 0;
        }
    }
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const uint64_t q = __umul64hi(acc[j], mu);
        uint64_t r = acc[j] - q * p;
        if (r >= p) r -= p;
        if (r >= p) r -= p;
        s += r;
    }
    out[t] = s;
}

__global__ void chase_kernel(const uint32_t* next, int64_t steps, uint64_t* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t i = 0;
    const uint64_t t0 = wall_clock64();
    const uint64_t c0 = clock64();
    for (int64_t k = 0; k < steps; k++) i = __builtin_nontemporal_load(next + i);
    const uint64_t c1 = clock64();
    const uint64_t t1 = wall_clock64();
    out[0] = c1 - c0;
    out[1] = t1 - t0;
    out[2] = i;
}

// Host wrappers (plain pointers; the caller owns device memory).
int calib_mad(const uint32_t* in, uint64_t* out, int blocks, int iters, void* stream) {
    hipLaunchKernelGGL(mad_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, in, out, iters);
    return (int)hipGetLastError();
}

int calib_mulmod(const uint32_t* in, uint64_t* out, int blocks, int iters, uint32_t p, uint32_t c32, uint64_t mu,
                 int fold, void* stream) {
    hipLaunchKernelGGL(mulmod_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, in, out, iters, p, c32, mu,
                       fold);
    return (int)hipGetLastError();
}

int calib_chase(const uint32_t* next, int64_t steps, uint64_t* out, void* stream) {
    hipLaunchKernelGGL(chase_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, next, steps, out);
    return (int)hipGetLastError();
}

int calib_wall_khz(int* khz) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(khz, hipDeviceAttributeWallClockRate, dev);
    return (int)e;
}

}  // extern "C"
