// internal.hpp -- host-side interfaces between the C ABI (capi.cpp) and the
// kernel launchers (mul.hip, divrem.hip, gcd.hip, batch.hip, serve.cpp).
// Not installed; the public interface is include/polymodp.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "common.hpp"

#include <new>

namespace pm {
// The status a function of the C interface returns for a C++ exception that
// reached it (sets the message of pm_last_error): PM_ENOMEM for host memory
// exhaustion, PM_EDEVICE for anything else.
int32_t api_exception(bool out_of_memory);
}  // namespace pm

// Every function of the C interface runs its body between PM_API_BEGIN and
// PM_API_END (PM_API_END_VOID for those that return nothing), so that no
// C++ exception crosses the interface.
#define PM_API_BEGIN try {
#define PM_API_END                                   \
    }                                                \
    catch (const std::bad_alloc&) {                  \
        return pm::api_exception(true);              \
    }                                                \
    catch (...) {                                    \
        return pm::api_exception(false);             \
    }
#define PM_API_END_VOID \
    }                   \
    catch (...) {       \
    }

namespace pm {

// Kernel timing for diagnostics (pm_timing_enable in the C ABI): when on,
// each launch wrapped in a TimingScope is bracketed by two HIP events on its
// stream; pm_timing_read sums the elapsed times per kernel name.
class TimingScope {
public:
    TimingScope(const char* kernel, hipStream_t stream);
    ~TimingScope();
    TimingScope(const TimingScope&) = delete;
    TimingScope& operator=(const TimingScope&) = delete;

private:
    const char* kernel_;
    hipStream_t stream_;
    hipEvent_t start_ = nullptr;
};

// The same timing carried by the launch itself: start() and stop() go to
// hipExtLaunchKernel, which sets them from the dispatch's own start and end,
// with no marker packets on the stream around it. Both are null when timing
// is off (then launch as usual). After a successful launch, launched()
// registers the pair for pm_timing_read; otherwise the events are returned.
class TimedLaunchEvents {
public:
    explicit TimedLaunchEvents(const char* kernel);
    ~TimedLaunchEvents();
    hipEvent_t start() const { return start_; }
    hipEvent_t stop() const { return stop_; }
    void launched() { ok_ = true; }
    TimedLaunchEvents(const TimedLaunchEvents&) = delete;
    TimedLaunchEvents& operator=(const TimedLaunchEvents&) = delete;

private:
    const char* kernel_;
    hipEvent_t start_ = nullptr, stop_ = nullptr;
    bool ok_ = false;
};

// ------------------------------------------------------------------ product
// Tiling of one product f = a*b (Sec. 5). The b operand is cut into chunks
// of `kc` coefficients (the paper's s: b-coefficients handled per
// thread-block); each thread-block owns `r` * 256 consecutive outputs of one
// chunk and each thread `r` consecutive outputs. With more than one chunk the
// per-chunk partial sums go to the array M (one row of n_a + kc - 1 residues
// per chunk, as in the paper's multiplication phase) and a second kernel adds
// the rows (the addition phase).
struct MulPlan {
    int r;        // outputs per thread: 1, 2, 4, 8, 16 or 32
    int64_t kc;   // b-coefficients per chunk (multiple of r)
};

constexpr int MUL_THREADS = 256;

// Scratch words (uint32) needed for the partial-sum rows of a plan.
int64_t mul_scratch_words(int64_t na, int64_t nb, const MulPlan& plan);

// Default plan for a product of the given sizes on this device.
MulPlan mul_default_plan(int64_t na, int64_t nb, int num_cus);

// Enqueue f = a*b (f has room for na+nb-1 words). When out_len or
// out_status is non-null one extra thread-block validates the inputs and
// writes the normalised length of f and the status there. `M` is scratch of mul_scratch_words words
// (may be null when the plan has one chunk). `sub_from` (optional, for the
// division remainder) switches the epilogue to f[k] = sub_from[k] - (a*b)[k]
// for k < out_limit, and limits the outputs to k < out_limit.
hipError_t mul_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb,
                      const Field& F, uint32_t* f, const MulPlan& plan, uint32_t* M,
                      int64_t* out_len, int32_t* out_status, const uint32_t* sub_from,
                      int64_t out_limit, hipStream_t stream);

// Batched product: one item per independent product (a is the longer
// operand), one task per output tile of 256*r outputs.
struct MulItem {
    const uint32_t* a;
    const uint32_t* b;
    uint32_t* f;
    int64_t na, nb;
    Field F;
};
struct MulTask {
    int32_t item;
    int32_t tile;
};
int64_t mul_batch_tile(int r);
// Chunk length the batched kernel uses for a requested kc.
int64_t mul_batch_kc(int r, int64_t kc);
// Tasks sorted longest first (a static assignment, no counters).
// fold_min: the smallest Field::fold_every over the items.
// blocks_per_cu > 0 caps the persistent grid (e.g. one block per CU beside
// other work); 0 fills the device.
hipError_t mul_batch_launch(const MulItem* d_items, const MulTask* d_tasks, int ntasks, int r, int64_t kc,
                            uint32_t fold_min, int num_cus, hipStream_t stream, int blocks_per_cu = 0);
hipError_t mul_batch_check_launch(const MulItem* d_items, int count, int32_t* d_status, hipStream_t stream);

// Product on the matrix cores (mul_mfma.hip): int8 digit products of the
// Toeplitz form of the schoolbook product, split stream-K over equal shares
// of (output range, b block offset) iterations. mx_geometry plans one
// product; the scratch holds the partial sums of every share.
struct MxGeom {
    int64_t na, nb;   // a: the plain side, b: the Toeplitz side
    int64_t nab;      // 64-coefficient blocks of a, rounded so that offset ranges start on groups of 8
    int64_t nJ;       // block offsets of b, rounded up to a multiple of 8
    int64_t nkr;      // output ranges of 4096
    int64_t itot;     // (range, group of 8 offsets) iterations
    int64_t G;        // work-groups (one share each)
    int64_t maxseg;   // most ranges one share touches
    int64_t maxgrp;   // most groups one share sums
};
// nout > 0: only the ranges holding outputs below nout are planned.
MxGeom mx_geometry(int64_t na, int64_t nb, int num_cus, int64_t nout = -1);
// The int32 digit sums of a plan are exact: no share sums more than 64
// groups of 8 block offsets (|sum| < 512 * 64 * 2^14 = 2^29). Products too
// large for the planner's cap on work-groups fail this and go to the VALU
// tiles; mulx_launch refuses them.
bool mx_exact(const MxGeom& g);

// Batched matrix-core product: one item per product whose shorter operand
// (b) holds at most MX_BATCH_MAXB coefficients, one task per output range
// of 4096 outputs; a task sums every block offset of its range (at most
// 512, which keeps the int32 digit sums exact) and writes f directly.
constexpr int64_t MX_BATCH_MAXB = 512 * 64 - 64;
struct MxItem {
    const uint32_t* a;  // the longer operand
    const uint32_t* b;
    uint32_t* f;
    int64_t na, nb;
    int64_t nab, nJ;    // MxGeom's rounded block counts
    Field F;
    uint32_t w[7];      // 256^e mod p
    uint32_t c63;       // 2^63 mod p
};
struct MxTask {
    int32_t item;
    int32_t kr;
};
// Fills an item (na >= nb >= 1, nb <= MX_BATCH_MAXB); returns its ranges.
int64_t mx_batch_item(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t* f, const Field& F,
                      MxItem* out);
// Block offsets range kr of an item sums (its share of the work).
int64_t mx_batch_offsets(const MxItem& it, int64_t kr);
// Tasks sorted longest first; no counters (a static assignment).
hipError_t mulx_batch_launch(const MxItem* d_items, const MxTask* d_tasks, int ntasks, int num_cus,
                             hipStream_t stream);
int64_t mulx_scratch_words(const MxGeom& g);
// f = a*b for na, nb >= 1 and p < 2^30; out_len/out_status as mul_launch.
// With sub_from, f[k] = sub_from[k] - (a*b)[k]; with nout > 0 only f[k] for
// k < nout is written (g planned with the same nout).
hipError_t mulx_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, const Field& F, uint32_t* f,
                       const MxGeom& g, uint32_t* scratch, int64_t* out_len, int32_t* out_status,
                       hipStream_t stream, const uint32_t* sub_from = nullptr, int64_t nout = -1);

// ----------------------------------------------------------------- division
// Euclidean division (Sec. 3) runs in two steps around one host read of the
// degrees: divrem_head_launch validates the inputs, finds deg a and deg b,
// and computes the whole quotient from the head of a and b (the division
// steps, s at a time, on up to num_cus cooperating blocks); the remainder
// r = a - q*b restricted to exponents below deg b is then one product launch
// with a subtracting epilogue (mulx_launch or mul_launch with sub_from = a),
// and trim_launch finds its length.
constexpr int DIV_THREADS = 256;
// Scratch words: the head of a (deg a - deg b + 1 <= na words) and one
// 64-bit published word per quotient term.
inline int64_t divrem_head_words(int64_t na) {
    const int64_t w = na > 0 ? na : 1;
    return ((w + 1) & ~1LL) + 2 * w;
}
hipError_t divrem_head_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb,
                              const Field& F, uint32_t* q, int64_t q_cap, int64_t r_cap,
                              uint32_t* head, CallInfo* info, int s, int num_cus, hipStream_t stream);
// Asynchronous division, between the quotient and the remainder product:
// q[i] = 0 for info->n0 <= i < q_plan, and PM_EINVAL in info->status when
// b[nb - 1] == 0.
hipError_t divrem_async_fix_launch(uint32_t* q, int64_t q_plan, const uint32_t* b, int64_t nb, CallInfo* info,
                                   hipStream_t stream);
// *d_status = info->status, *d_n0 = info->n0, *d_n1 = info->n1 (lengths 0
// on error); null pointers are skipped.
hipError_t info_export_launch(const CallInfo* info, int64_t* d_n0, int64_t* d_n1, int32_t* d_status,
                              hipStream_t stream);
// info->n1 = 1 + (largest k < n with r[k] != 0), or 0.
hipError_t trim_launch(const uint32_t* r, int64_t n, CallInfo* info, hipStream_t stream);
// out[i] = -x[i] for i < n (out[0] = 0 when drop0)
hipError_t negate_launch(const uint32_t* x, int64_t n, uint32_t* out, uint32_t p, bool drop0,
                         hipStream_t stream);
// out[i] = x[i] - y[i] for i < n (x read as zero past nx, y past ny)
hipError_t sub_launch(const uint32_t* x, int64_t nx, const uint32_t* y, int64_t ny, int64_t n, uint32_t* out,
                      uint32_t p, hipStream_t stream);
// out[i] = r[i] + q[0] y[i] for i < n (r read as zero past nr)
hipError_t fold_q0_launch(const uint32_t* r, int64_t nr, const uint32_t* q, const uint32_t* y, int64_t n,
                          uint32_t* out, const Field& F, hipStream_t stream);

// ------------------------------------------------- naive division and gcd
// One division step per launch (Sec. 3 Alg. 1/2, Sec. 6 Alg. 8/9).
// Degrees, range check (info->flags) and reset of the call's results.
hipError_t naive_prep_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, const Field& F,
                             CallInfo* info, hipStream_t stream);
// The steps at head positions da .. db of the working copy w of a, one
// launch each; q[i - db] for every step i.
hipError_t naive_divrem_launch(uint32_t* w, const uint32_t* b, int64_t da, int64_t db, uint32_t inv, uint32_t* q,
                               const Field& F, hipStream_t stream);
// count gcd steps (two launches each) on the working copies A, B of n
// words, degrees in info (no-ops once one operand is zero).
hipError_t naive_gcd_steps_launch(uint32_t* A, uint32_t* B, int64_t n, int64_t count, const Field& F,
                                  CallInfo* info, hipStream_t stream);
// g = the non-zero one of A, B made monic (nothing when g_cap is too small).
hipError_t naive_monic_launch(const uint32_t* A, const uint32_t* B, uint32_t* g, int64_t g_cap, int64_t n,
                              const Field& F, CallInfo* info, hipStream_t stream);

// ---------------------------------------------------------------------- gcd
struct GcdPlan {
    int groups;      // cooperating thread-blocks (1 = single block)
    int slice;       // coefficient positions owned by each block
    int head;        // head length (128 or 256)
    int s;           // max Euclidean division steps per fused chunk
};

// Per-instance results of the batched gcd kernel (device or host-mapped
// memory). `done` is set last, with release order, when the instance ends.
struct GcdResult {
    int64_t ng;       // gcd: length of g; division: length of q
    int64_t steps;
    int64_t updates;
    int64_t chunks;
    int32_t status;
    int32_t done;
    int64_t nr;       // division: length of r
};

// One instance of the batched gcd (or, for the server, one division):
// inputs, outputs and where to report.
struct GcdJob {
    const uint32_t* a;
    const uint32_t* b;
    int64_t na, nb;
    uint32_t* g;      // gcd: g; division: q
    int64_t g_cap;
    GcdResult* out;
    Field F;
    // 1 when a and b were written by another agent (a copy engine) after
    // the running kernel started: they are then read past the caches
    int32_t fresh;
    int32_t op;       // JOB_GCD or JOB_DIVREM
    uint32_t* r;      // division: the remainder
    int64_t r_cap;
};
enum { JOB_GCD = 0, JOB_DIVREM = 1 };

// Capacity (max(na, nb)) of the two batched kernel shapes: kind 0 = 256
// threads, kind 1 = 1024 threads.
int64_t gcd_batch_cap(int kind);
// One block for each of the first njobs entries of `order` (job indices
// into d_jobs; when order is null, block i runs job i). Jobs must fit the
// capacity of `kind`.
hipError_t gcd_batch_launch(const GcdJob* d_jobs, const int32_t* d_order, int njobs, int kind, int s,
                            hipStream_t stream);
// Persistent worker of the server, of block shape `kind` (as
// gcd_batch_cap): blocks claim sequence numbers h < *tail from *head and
// run jobs[order[h % order_cap]] (order_cap a power of two), a gcd or a
// division (GcdJob::op). tail, stop, order, jobs and started live in pinned
// host memory written by the host; head in device memory, zero at first.
// Every block adds 1 to *started when it begins. Exits when stop is raised
// with nothing left, or after idle_seconds without work.
hipError_t gcd_worker_launch(int kind, const GcdJob* jobs, const uint32_t* order, uint32_t order_cap,
                             const uint32_t* tail, const uint32_t* stop, uint32_t* head, uint32_t* started, int s,
                             int blocks, double idle_seconds, hipStream_t stream);
// Blocks of one worker shape that fit a CU beside nothing else.
int gcd_worker_blocks_per_cu(int kind);
constexpr int GCD_THREADS = 256;
GcdPlan gcd_default_plan(int64_t n, int num_cus, int s);
// The extended gcd's cofactor tracking: the cofactor of the caller's a in
// the kernel's two operands starts as sa0 / sb0 (device, nsa / nsb words)
// and takes every chunk's M; s_res (gcd_positions(plan) words) receives
// the cofactor of the last non-zero remainder, scaled as g is. deg_cap
// (deg of the caller's b) bounds every cofactor's degree.
struct GcdCofactors {
    const uint32_t* sa0;
    int64_t nsa;
    const uint32_t* sb0;
    int64_t nsb;
    int64_t deg_cap;
    uint32_t* s_res;
};
// ---- radix sort (radix.hip): stable LSD sort of uint32 keys on their low
// key_bits bits, s-bit digits (1..10), vals (may be null) moving along;
// scratch: radix_scratch_words(n, s, vals != null) words
int64_t radix_scratch_words(int64_t n, int s, bool with_vals);
hipError_t radix_sort_launch(const uint32_t* keys, const uint32_t* vals, int64_t n, int key_bits, int s,
                             uint32_t* keys_out, uint32_t* vals_out, uint32_t* scratch, hipStream_t stream);

// Diagnostics of one gcd_launch (plain variant only):
//  * log (optional): the steps of every chunk, written by block 0 once a
//    chunk's head run is over. int32 words: a header {chunks, steps,
//    overflow, 0}, then chunk_cap records {deg A, deg B at the chunk's
//    start, index of its first step, its step count} (the last record, with
//    no steps, holds the final degrees), then step_cap records {shift,
//    which: 0 = A was reduced, 1 = B}. Steps with a zero multiplier are not
//    run and not recorded.
//  * max_steps >= 0: the kernel stops after that many run steps and writes
//    both operands made monic, A to g (info->n0 = its length) and B to
//    b_out (info->n1), instead of the gcd.
struct GcdTrace {
    int32_t* log;
    int64_t chunk_cap;
    int64_t step_cap;
    int64_t max_steps;
    uint32_t* b_out;
    int64_t b_cap;
};
constexpr int GCD_TRACE_HDR = 4;
inline int64_t gcd_trace_words(int64_t chunk_cap, int64_t step_cap) {
    return GCD_TRACE_HDR + 4 * chunk_cap + 2 * step_cap;
}

// coefficient positions of the plan's grid (>= n)
int64_t gcd_positions(const GcdPlan& plan);
int64_t gcd_scratch_words(int64_t n, const GcdPlan& plan, bool cofactors = false);
hipError_t gcd_launch(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb,
                      const Field& F, uint32_t* g, int64_t g_cap, uint32_t* scratch,
                      CallInfo* info, const GcdPlan& plan, hipStream_t stream,
                      const GcdCofactors* xg = nullptr, const GcdTrace* tr = nullptr);

}  // namespace pm
