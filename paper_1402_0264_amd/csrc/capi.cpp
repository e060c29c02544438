// capi.cpp -- the extern "C" entry points of libpolymodp (include/polymodp.h):
// argument checks, per-prime constants, the scratch pool and the sequencing
// of the kernel launches in mul.hip, divrem.hip and gcd.hip.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/polymodp.h"
#include "internal.hpp"

#include <algorithm>

struct pm_gcd_batch {
    int device = 0;
    int32_t count = 0;
    int32_t n_large = 0, n_small = 0;
    int s = 128;
    pm::GcdJob* d_jobs = nullptr;
    int32_t* d_order = nullptr;
    pm::GcdResult* d_res = nullptr;
    // With both shapes, the 256-thread blocks run on a second stream beside
    // the 1024-thread ones, so that they take each CU a large instance
    // leaves instead of waiting for the longest one; side joins the
    // caller's stream through the two events, so a capture takes both.
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

struct pm_mul_batch {
    int device = 0;
    int count = 0;
    int ntasks = 0;
    int r = 8;
    int64_t kc = 1024;
    uint32_t fold_min = 1u << 30;
    pm::MulItem* d_items = nullptr;
    pm::MulTask* d_tasks = nullptr;
    int n_mx_tasks = 0;               // items on the matrix cores: one task per output range
    pm::MxItem* d_mx_items = nullptr;
    pm::MxTask* d_mx_tasks = nullptr;
    // With both kinds of tasks and r = 4, the VALU tiles run on a second
    // stream beside the matrix cores, one work-group per CU (it fits beside
    // the matrix-core work-group: VGPRs, LDS and waves); side joins the
    // caller's stream through the two events, so a capture takes both.
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace {

thread_local char g_err[512] = "";
thread_local pm_gcd_stats g_gcd_stats = {0, 0, 0};

pm_status fail(pm_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

pm_status hip_fail(hipError_t e, const char* what) {
    return fail(PM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// ------------------------------------------------------------ prime field
uint64_t mulmod_host(uint64_t a, uint64_t b, uint64_t m) { return (unsigned __int128)a * b % m; }

uint64_t powmod_host(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod_host(r, a, m);
        a = mulmod_host(a, a, m);
        e >>= 1;
    }
    return r;
}

// Deterministic Miller-Rabin for 32-bit n (bases 2, 7, 61 suffice).
bool is_prime_u32(uint32_t n) {
    if (n < 2) return false;
    for (uint32_t sp : {2u, 3u, 5u, 7u, 11u, 13u, 61u})
        if (n % sp == 0) return n == sp;
    uint32_t d = n - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; r++; }
    for (uint32_t a : {2u, 7u, 61u}) {
        uint64_t x = powmod_host(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < r; i++) {
            x = mulmod_host(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

std::mutex g_field_mu;
std::map<uint32_t, pm::Field> g_fields;

pm_status field_for(uint32_t p, pm::Field* out) {
    if (p < 2 || p >= (1u << 30)) return fail(PM_EMODULUS, "modulus %u is outside [2, 2^30)", p);
    std::lock_guard<std::mutex> lk(g_field_mu);
    auto it = g_fields.find(p);
    if (it != g_fields.end()) { *out = it->second; return PM_OK; }
    if (!is_prime_u32(p)) return fail(PM_EMODULUS, "modulus %u is not prime", p);
    pm::Field F{};
    F.p = p;
    F.c32 = (uint32_t)((1ULL << 32) % p);
    // -p^{-1} mod 2^32 by Newton iteration (p odd). For p = 2 there is no
    // such inverse; 2^31 makes the same REDC sequence return x mod 2 for any
    // x < 2^32 (t = (x mod 2) 2^31, so (x + 2t) >> 32 = x mod 2), which
    // covers every REDC input of the gcd at p = 2: sums of two products of
    // residues below 2
    uint32_t inv = 1;
    if (p & 1) {
        inv = p;
        for (int i = 0; i < 5; i++) inv *= 2u - p * inv;
        F.pinv_neg = (uint32_t)(0u - inv);
    } else {
        F.pinv_neg = 0x80000000u;
    }
    F.mu = ~0ULL / p;
    // after a fold the accumulator is below (2^32-1)*c32 + 2^32; each further
    // product is at most (p-1)^2
    unsigned __int128 after = (unsigned __int128)0xFFFFFFFFull * F.c32 + 0xFFFFFFFFull;
    unsigned __int128 room = ((unsigned __int128)1 << 64) - 1 - after;
    unsigned __int128 sq = (unsigned __int128)(p - 1) * (p - 1);
    unsigned __int128 fe = sq ? room / sq : ((unsigned __int128)1 << 30);
    F.fold_every = fe > (1u << 30) ? (1u << 30) : (uint32_t)fe;
    g_fields[p] = F;
    *out = F;
    return PM_OK;
}

// ------------------------------------------------------------ parameters
std::mutex g_param_mu;
pm_params g_params = {0, 0, 0, 0, 0};

pm_params params_now() {
    std::lock_guard<std::mutex> lk(g_param_mu);
    return g_params;
}

// ------------------------------------------------------------ scratch pool
// Scratch of a call: the library's pool for its device and stream, or the
// caller's workspace when one is set for the stream (pm_set_workspace). A
// pool buffer that a larger call outgrows is retired, not freed: a graph
// captured earlier may still hold its address, so retired buffers are freed
// only by pm_release.
constexpr int64_t INFO_WORDS = 64;  // the device CallInfo, rounded up to 256 bytes
static_assert(sizeof(pm::CallInfo) <= INFO_WORDS * sizeof(uint32_t), "CallInfo too large");

struct Pool {
    pm::CallInfo* d_info = nullptr;  // device: the call's results and barrier words
    pm::CallInfo* h_info = nullptr;  // pinned host copy (synchronous calls)
    uint32_t* words = nullptr;       // device scratch
    int64_t cap = 0;
};

struct StreamState {
    Pool own;                 // the library's buffers
    Pool view;                // onto the caller's workspace
    uint32_t* ws = nullptr;   // the caller's workspace (device), if set
    int64_t ws_words = 0;
};

std::mutex g_pool_mu;
std::map<std::pair<int, hipStream_t>, StreamState> g_pools;
std::vector<void*> g_retired;  // outgrown device buffers, guarded by g_pool_mu

pm_status pool_get(hipStream_t stream, int64_t words, Pool** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_pool_mu);
    StreamState& S = g_pools[{dev, stream}];
    if (S.ws) {
        if (words > S.ws_words - INFO_WORDS)
            return fail(PM_ENOMEM, "the stream's workspace holds %lld words; the call needs %lld",
                        (long long)S.ws_words, (long long)(words + INFO_WORDS));
        *out = &S.view;
        return PM_OK;
    }
    Pool& P = S.own;
    if (!P.d_info) {
        HIP_TRY(hipMalloc((void**)&P.d_info, INFO_WORDS * sizeof(uint32_t)), "hipMalloc(info)");
        HIP_TRY(hipMemset(P.d_info, 0, INFO_WORDS * sizeof(uint32_t)), "hipMemset(info)");
        HIP_TRY(hipHostMalloc((void**)&P.h_info, sizeof(pm::CallInfo), hipHostMallocDefault), "hipHostMalloc");
    }
    if (words > P.cap) {
        if (P.words) g_retired.push_back(P.words);
        P.words = nullptr;
        P.cap = 0;
        int64_t want = words + words / 4 + 1024;
        if (hipMalloc((void**)&P.words, (size_t)want * sizeof(uint32_t)) != hipSuccess) {
            P.words = nullptr;
            return fail(PM_ENOMEM, "cannot allocate %lld scratch words", (long long)want);
        }
        P.cap = want;
    }
    *out = &P;
    return PM_OK;
}

// Scratch apart from the pool that the division and the gcd use, one per
// purpose: the gcd's leading division (quotient, remainder, folded operand;
// AUX_LEAD) and the gcd's step log (AUX_TRACE).
struct Aux {
    uint32_t* w = nullptr;
    int64_t cap = 0;
};
enum { AUX_LEAD = 0, AUX_TRACE = 1 };
std::map<std::tuple<int, hipStream_t, int>, Aux> g_aux;  // guarded by g_pool_mu

pm_status aux_get(hipStream_t stream, int64_t words, uint32_t** out, int key = AUX_LEAD) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_pool_mu);
    Aux& X = g_aux[{dev, stream, key}];
    if (words > X.cap) {
        if (X.w) g_retired.push_back(X.w);
        X.w = nullptr;
        X.cap = 0;
        const int64_t want = words + words / 4 + 1024;
        if (hipMalloc((void**)&X.w, (size_t)want * sizeof(uint32_t)) != hipSuccess) {
            X.w = nullptr;
            return fail(PM_ENOMEM, "cannot allocate %lld scratch words", (long long)want);
        }
        X.cap = want;
    }
    *out = X.w;
    return PM_OK;
}

pm_status read_info(Pool* P, hipStream_t stream) {
    HIP_TRY(hipMemcpyAsync(P->h_info, P->d_info, sizeof(pm::CallInfo), hipMemcpyDeviceToHost, stream),
            "hipMemcpyAsync(info)");
    HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    return PM_OK;
}

int num_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t pr;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&pr, dev) == hipSuccess)
            cus = pr.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

pm::MulPlan mul_plan(int64_t na, int64_t nb) {
    pm::MulPlan plan = pm::mul_default_plan(na, nb, num_cus());
    pm_params pp = params_now();
    if (pp.mul_r > 0) plan.r = pp.mul_r;
    if (pp.mul_s > 0) plan.kc = pp.mul_s;
    if (plan.kc < plan.r) plan.kc = plan.r;
    return plan;
}

const char* status_text(pm_status st) {
    switch (st) {
        case PM_ERANGE: return "an input coefficient is not below p";
        case PM_EDIVZERO: return "division by the zero polynomial";
        case PM_EINVAL: return "output capacity below what the result needs";
        case PM_EDEVICE: return "device invariant broken";
        default: return "error";
    }
}

bool bad_len(const void* ptr, int64_t n) { return n < 0 || (n > 0 && ptr == nullptr); }

// The words an argument covers: an input's length, an output's capacity.
struct Span {
    const void* p;
    int64_t n;
};

bool spans_overlap(const Span& x, const Span& y) {
    if (!x.p || !y.p || x.n <= 0 || y.n <= 0) return false;
    const uintptr_t a = (uintptr_t)x.p, b = (uintptr_t)y.p;
    return a < b + (uintptr_t)y.n * sizeof(uint32_t) && b < a + (uintptr_t)x.n * sizeof(uint32_t);
}

// Outputs may overlap neither the inputs nor each other (PM_EINVAL).
pm_status check_aliasing(std::initializer_list<Span> outs, std::initializer_list<Span> ins) {
    for (auto o = outs.begin(); o != outs.end(); ++o) {
        for (const Span& i : ins)
            if (spans_overlap(*o, i)) return fail(PM_EINVAL, "an output overlaps an input");
        for (auto o2 = o + 1; o2 != outs.end(); ++o2)
            if (spans_overlap(*o, *o2)) return fail(PM_EINVAL, "two outputs overlap");
    }
    return PM_OK;
}

// Ordered larger-first for the product kernel: the longer operand is staged
// in LDS windows, the shorter one is walked step by step.
void order_operands(const uint32_t*& a, int64_t& na, const uint32_t*& b, int64_t& nb) {
    if (nb > na) {
        std::swap(a, b);
        std::swap(na, nb);
    }
}

// The matrix-core product for large operands: it needs both operands
// non-empty; below a few million coefficient products its fixed costs
// (staging, the addition phase) outweigh the VALU tiles.
bool use_mfma(int64_t na, int64_t nb) {
    if (na <= 0 || nb <= 0) return false;
    const pm_params pp = params_now();
    if (pp.mul_engine == 1) return false;
    if (pp.mul_engine == 2) return true;
    if (pp.mul_s > 0 || pp.mul_r > 0) return false;
    // measured on graph-replayed products: below about 6400 x 6400 the VALU
    // tiles finish first (the matrix-core engine has a fixed cost of about
    // 15 us: staging, stream-K shares, the addition phase)
    const int64_t lo = na < nb ? na : nb;
    return lo >= 256 && (double)na * (double)nb >= 40.0e6;
}

// The matrix-core plan of a product (ordered operands) when that engine
// takes it: use_mfma's choice, and only a plan whose int32 digit sums stay
// exact (larger products go to the VALU tiles).
bool mfma_plan(int64_t na, int64_t nb, int64_t nout, pm::MxGeom* g) {
    if (!use_mfma(na, nb)) return false;
    *g = pm::mx_geometry(na, nb, num_cus(), nout);
    return pm::mx_exact(*g);
}

pm_status mul_enqueue(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, const pm::Field& F,
                      uint32_t* f, int64_t* d_nf, int32_t* d_status, hipStream_t stream) {
    order_operands(a, na, b, nb);
    pm::MxGeom g;
    if (mfma_plan(na, nb, -1, &g)) {
        Pool* P = nullptr;
        pm_status st = pool_get(stream, pm::mulx_scratch_words(g), &P);
        if (st) return st;
        HIP_TRY(pm::mulx_launch(a, na, b, nb, F, f, g, P->words, d_nf, d_status, stream), "mul launch");
        return PM_OK;
    }
    pm::MulPlan plan = mul_plan(na, nb);
    int64_t words = pm::mul_scratch_words(na, nb, plan);
    Pool* P = nullptr;
    uint32_t* M = nullptr;
    if (words > 0) {
        pm_status st = pool_get(stream, words, &P);
        if (st) return st;
        M = P->words;
    }
    HIP_TRY(pm::mul_launch(a, na, b, nb, F, f, plan, M, d_nf, d_status, nullptr, -1, stream), "mul launch");
    return PM_OK;
}

// ------------------------------------------------------------ kernel timing
std::atomic<int> g_timing_on{0};
std::mutex g_timing_mu;
struct TimedLaunch {
    std::string kernel;
    hipEvent_t start, stop;
};
std::vector<TimedLaunch> g_timed;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event() {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    // no system-scope fence: the events only timestamp the stream, and a
    // fence (an L2 write-back) at every record would slow the timed launches
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

namespace pm {

int32_t api_exception(bool out_of_memory) {
    return out_of_memory ? fail(PM_ENOMEM, "out of host memory") : fail(PM_EDEVICE, "internal error (exception)");
}
pm_status server_field(uint32_t p, Field* out) { return field_for(p, out); }
pm_status server_fail(pm_status st, const char* msg) { return fail(st, "%s", msg); }
int server_num_cus() { return num_cus(); }

TimingScope::TimingScope(const char* kernel, hipStream_t stream) : kernel_(kernel), stream_(stream) {
    if (!g_timing_on.load(std::memory_order_relaxed)) return;
    start_ = take_event();
    if (start_ && hipEventRecord(start_, stream_) != hipSuccess) start_ = nullptr;
}

TimingScope::~TimingScope() {
    if (!start_) return;
    hipEvent_t stop = take_event();
    if (!stop || hipEventRecord(stop, stream_) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timed.push_back(TimedLaunch{kernel_, start_, stop});
}

TimedLaunchEvents::TimedLaunchEvents(const char* kernel) : kernel_(kernel) {
    if (!g_timing_on.load(std::memory_order_relaxed)) return;
    start_ = take_event();
    stop_ = take_event();
    if (!start_ || !stop_) {
        std::lock_guard<std::mutex> lk(g_timing_mu);
        if (start_) g_event_pool.push_back(start_);
        if (stop_) g_event_pool.push_back(stop_);
        start_ = stop_ = nullptr;
    }
}

TimedLaunchEvents::~TimedLaunchEvents() {
    if (!start_) return;
    std::lock_guard<std::mutex> lk(g_timing_mu);
    if (ok_) {
        g_timed.push_back(TimedLaunch{kernel_, start_, stop_});
    } else {
        g_event_pool.push_back(start_);
        g_event_pool.push_back(stop_);
    }
}

}  // namespace pm

extern "C" {

void pm_timing_enable(int on) { PM_API_BEGIN g_timing_on.store(on ? 1 : 0); PM_API_END_VOID }

void pm_timing_reset(void) {
    PM_API_BEGIN
    std::lock_guard<std::mutex> lk(g_timing_mu);
    for (auto& t : g_timed) {
        (void)hipEventSynchronize(t.stop);
        g_event_pool.push_back(t.start);
        g_event_pool.push_back(t.stop);
    }
    g_timed.clear();
    PM_API_END_VOID
}

pm_status pm_timing_read(const char* kernel, int64_t* launches, double* total_ms) {
    PM_API_BEGIN
    if (!kernel || !launches || !total_ms) return fail(PM_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(g_timing_mu);
    int64_t n = 0;
    double ms = 0;
    for (auto& t : g_timed) {
        if (t.kernel != kernel) continue;
        HIP_TRY(hipEventSynchronize(t.stop), "hipEventSynchronize");
        float x = 0;
        HIP_TRY(hipEventElapsedTime(&x, t.start, t.stop), "hipEventElapsedTime");
        n++;
        ms += x;
    }
    *launches = n;
    *total_ms = ms;
    return PM_OK;
    PM_API_END
}


const char* pm_last_error(void) { return g_err; }

void pm_last_gcd_stats(pm_gcd_stats* out) {
    PM_API_BEGIN
    if (out) *out = g_gcd_stats;
    PM_API_END_VOID
}

pm_status pm_set_params(const pm_params* params) {
    PM_API_BEGIN
    if (!params) return fail(PM_EINVAL, "null params");
    const pm_params& q = *params;
    if (q.mul_r != 0 && q.mul_r != 1 && q.mul_r != 2 && q.mul_r != 4 && q.mul_r != 8 && q.mul_r != 16 &&
        q.mul_r != 32)
        return fail(PM_EINVAL, "mul_r must be 0, 1, 2, 4, 8, 16 or 32");
    if (q.mul_s < 0 || q.mul_s > 16384) return fail(PM_EINVAL, "mul_s must be in [0, 16384]");
    if (q.div_s < 0 || q.div_s > 64) return fail(PM_EINVAL, "div_s must be in [0, 64]");
    if (q.gcd_s < 0 || q.gcd_s > 256) return fail(PM_EINVAL, "gcd_s must be in [0, 256]");
    if (q.mul_engine < 0 || q.mul_engine > 2) return fail(PM_EINVAL, "mul_engine must be 0, 1 or 2");
    std::lock_guard<std::mutex> lk(g_param_mu);
    g_params = q;
    return PM_OK;
    PM_API_END
}

void pm_get_params(pm_params* params) {
    PM_API_BEGIN
    if (params) *params = params_now();
    PM_API_END_VOID
}

void pm_release(void) {
    PM_API_BEGIN
    std::lock_guard<std::mutex> lk(g_pool_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_pools) {
        (void)hipSetDevice(kv.first.first);
        (void)hipStreamSynchronize(kv.first.second);
        Pool& P = kv.second.own;
        if (P.words) (void)hipFree(P.words);
        if (P.d_info) (void)hipFree(P.d_info);
        if (P.h_info) (void)hipHostFree(P.h_info);
        if (kv.second.view.h_info) (void)hipHostFree(kv.second.view.h_info);
    }
    (void)hipDeviceSynchronize();
    for (void* w : g_retired) (void)hipFree(w);
    g_retired.clear();
    for (auto& kv : g_aux)
        if (kv.second.w) (void)hipFree(kv.second.w);
    g_aux.clear();
    (void)hipSetDevice(cur);
    g_pools.clear();
    PM_API_END_VOID
}

pm_status pm_set_workspace(void* stream, void* d_words, int64_t words) {
    PM_API_BEGIN
    if (words < 0 || (words > 0 && !d_words)) return fail(PM_EINVAL, "null workspace or negative size");
    if (words > 0 && words < INFO_WORDS)
        return fail(PM_EINVAL, "a workspace needs at least %lld words", (long long)INFO_WORDS);
    if (((uintptr_t)d_words & 255) != 0) return fail(PM_EINVAL, "the workspace must be 256-byte aligned");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    StreamState& S = g_pools[{dev, s}];
    // calls already enqueued on the stream may still use the old scratch
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (words == 0) {
        S.ws = nullptr;
        S.ws_words = 0;
        return PM_OK;
    }
    if (!S.view.h_info)
        HIP_TRY(hipHostMalloc((void**)&S.view.h_info, sizeof(pm::CallInfo), hipHostMallocDefault), "hipHostMalloc");
    // the call results and the grid barrier words start at zero
    HIP_TRY(hipMemsetAsync(d_words, 0, INFO_WORDS * sizeof(uint32_t), s), "hipMemsetAsync(workspace)");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    S.ws = (uint32_t*)d_words;
    S.ws_words = words;
    S.view.d_info = (pm::CallInfo*)d_words;
    S.view.words = (uint32_t*)d_words + INFO_WORDS;
    S.view.cap = words - INFO_WORDS;
    return PM_OK;
    PM_API_END
}

pm_status poly_mul_modp_async(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p,
                              uint32_t* f, int64_t f_cap, int64_t* d_nf, int32_t* d_status, void* stream) {
    PM_API_BEGIN
    if (bad_len(a, na) || bad_len(b, nb)) return fail(PM_EINVAL, "null input or negative length");
    int64_t need = (na > 0 && nb > 0) ? na + nb - 1 : 0;
    if (need > 0 && (f == nullptr || f_cap < need))
        return fail(PM_EINVAL, "f_cap %lld < na + nb - 1 = %lld", (long long)f_cap, (long long)need);
    if (check_aliasing({{f, need}}, {{a, na}, {b, nb}})) return PM_EINVAL;
    pm::Field F;
    pm_status st = field_for(p, &F);
    if (st) return st;
    return mul_enqueue(a, na, b, nb, F, f, d_nf, d_status, (hipStream_t)stream);
    PM_API_END
}

}  // extern "C"

namespace {

// ------------------------------------------- static scratch (no allocation)
// The scratch of poly_mul_modp_noalloc: a fixed array in every device's
// copy of the code object, held until the process ends. Host code never
// passes `scratch` itself (on the host it is only a stand-in for the symbol)
// but the device address hipGetSymbolAddress gives for the current device.
static __device__ __align__(256) uint32_t scratch[PM_NOALLOC_SCRATCH_WORDS];

std::mutex g_static_mu;
std::map<int, uint32_t*> g_static_ptr;  // device -> address of its scratch

pm_status static_scratch(uint32_t** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_static_mu);
    auto it = g_static_ptr.find(dev);
    if (it == g_static_ptr.end()) {
        uint32_t* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(PM_EDEVICE, "no device address for the static scratch");
        it = g_static_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return PM_OK;
}

}  // namespace

extern "C" {

pm_status poly_mul_modp_noalloc(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p,
                                uint32_t* f, int64_t f_cap, int64_t* d_nf, int32_t* d_status, void* stream) {
    PM_API_BEGIN
    if (bad_len(a, na) || bad_len(b, nb)) return fail(PM_EINVAL, "null input or negative length");
    int64_t need = (na > 0 && nb > 0) ? na + nb - 1 : 0;
    if (need > 0 && (f == nullptr || f_cap < need))
        return fail(PM_EINVAL, "f_cap %lld < na + nb - 1 = %lld", (long long)f_cap, (long long)need);
    if (check_aliasing({{f, need}}, {{a, na}, {b, nb}})) return PM_EINVAL;
    pm::Field F;
    pm_status st = field_for(p, &F);
    if (st) return st;
    uint32_t* ws = nullptr;
    if ((st = static_scratch(&ws))) return st;
    hipStream_t s = (hipStream_t)stream;
    order_operands(a, na, b, nb);
    // the engine poly_mul_modp_async picks, else the VALU tiles, whichever
    // plan's scratch fits the static array (the results are identical)
    pm::MxGeom g;
    if (mfma_plan(na, nb, -1, &g)) {
        if (pm::mulx_scratch_words(g) <= PM_NOALLOC_SCRATCH_WORDS) {
            HIP_TRY(pm::mulx_launch(a, na, b, nb, F, f, g, ws, d_nf, d_status, s), "mul launch");
            return PM_OK;
        }
    }
    const pm::MulPlan plan = mul_plan(na, nb);
    const int64_t words = pm::mul_scratch_words(na, nb, plan);
    if (words > PM_NOALLOC_SCRATCH_WORDS)
        return fail(PM_EINVAL, "the product of %lld x %lld terms needs %lld scratch words, above the static %lld",
                    (long long)na, (long long)nb, (long long)words, (long long)PM_NOALLOC_SCRATCH_WORDS);
    HIP_TRY(pm::mul_launch(a, na, b, nb, F, f, plan, words > 0 ? ws : nullptr, d_nf, d_status, nullptr, -1, s),
            "mul launch");
    return PM_OK;
    PM_API_END
}

void pm_mul_batch_destroy(pm_mul_batch* B) {
    PM_API_BEGIN
    if (!B) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(B->device);
    (void)hipDeviceSynchronize();
    if (B->d_items) (void)hipFree(B->d_items);
    if (B->d_tasks) (void)hipFree(B->d_tasks);
    if (B->d_mx_items) (void)hipFree(B->d_mx_items);
    if (B->d_mx_tasks) (void)hipFree(B->d_mx_tasks);
    if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
    if (B->ev_join) (void)hipEventDestroy(B->ev_join);
    if (B->side) (void)hipStreamDestroy(B->side);
    (void)hipSetDevice(cur);
    delete B;
    PM_API_END_VOID
}

// Which engine a batch item goes to: the matrix cores when the estimated
// cycles of its range tasks on one CU (block offsets at about 2048 cycles
// each, half the MFMA peak, plus staging and epilogue per task) undercut
// the VALU tiles' (about 25 multiply-adds per cycle per CU, measured on the
// batch), or always under PM_MUL_MFMA; never past the exactness bound.
bool batch_on_matrix_cores(const pm::MxItem& it, int64_t nkr, int engine) {
    if (engine == PM_MUL_VALU || it.nb > pm::MX_BATCH_MAXB) return false;
    if (engine == PM_MUL_MFMA) return true;
    double mx = 0;
    for (int64_t kr = 0; kr < nkr; kr++) mx += 2048.0 * (double)pm::mx_batch_offsets(it, kr) + 4000.0;
    return mx < (double)it.na * (double)it.nb / 25.0;
}

pm_status pm_mul_batch_create(const pm_mul_item* items, int32_t count, int32_t r, int32_t kc, pm_mul_batch** out) {
    PM_API_BEGIN
    if (!out || count < 0 || (count > 0 && !items)) return fail(PM_EINVAL, "bad arguments");
    if (r == 0) r = 8;
    if (r != 4 && r != 8 && r != 16) return fail(PM_EINVAL, "r must be 4, 8 or 16");
    if (kc == 0) kc = 1024;
    if (kc < r) return fail(PM_EINVAL, "kc must be at least r");
    std::vector<pm::MulItem> host((size_t)count);
    std::vector<std::pair<int64_t, pm::MulTask>> tasks;
    std::vector<pm::MxItem> mx_items;
    std::vector<std::pair<int64_t, pm::MxTask>> mx_tasks;
    uint32_t fold_min = 1u << 30;
    const int64_t T = pm::mul_batch_tile(r);
    const int engine = params_now().mul_engine;
    for (int32_t i = 0; i < count; i++) {
        const pm_mul_item& it = items[i];
        if (bad_len(it.a, it.na) || bad_len(it.b, it.nb)) return fail(PM_EINVAL, "item %d: bad input", i);
        const int64_t need = (it.na > 0 && it.nb > 0) ? it.na + it.nb - 1 : 0;
        if (need > 0 && (!it.f || it.f_cap < need)) return fail(PM_EINVAL, "item %d: f_cap < na + nb - 1", i);
        if (check_aliasing({{it.f, need}}, {{it.a, it.na}, {it.b, it.nb}}))
            return fail(PM_EINVAL, "item %d: the output overlaps an input", i);
        pm::Field F;
        pm_status st = field_for(it.p, &F);
        if (st) return st;
        fold_min = std::min(fold_min, F.fold_every);
        const uint32_t *x = it.a, *y = it.b;
        int64_t nx = it.na, ny = it.nb;
        order_operands(x, nx, y, ny);
        host[i] = pm::MulItem{x, y, it.f, nx, ny, F};
        if (need == 0) continue;
        if (ny <= pm::MX_BATCH_MAXB) {
            pm::MxItem mi;
            const int64_t nkr = pm::mx_batch_item(x, nx, y, ny, it.f, F, &mi);
            if (batch_on_matrix_cores(mi, nkr, engine)) {
                const int32_t idx = (int32_t)mx_items.size();
                mx_items.push_back(mi);
                for (int64_t kr = 0; kr < nkr; kr++)
                    mx_tasks.push_back({pm::mx_batch_offsets(mi, kr), pm::MxTask{idx, (int32_t)kr}});
                continue;
            }
        }
        const int64_t tiles = (need + T - 1) / T;
        if (tiles > INT32_MAX) return fail(PM_EINVAL, "item %d too large", i);
        for (int64_t t = 0; t < tiles; t++) tasks.push_back({T * ny, pm::MulTask{i, (int32_t)t}});
    }
    if (tasks.size() > (size_t)INT32_MAX || mx_tasks.size() > (size_t)INT32_MAX)
        return fail(PM_EINVAL, "too many tasks");
    std::stable_sort(mx_tasks.begin(), mx_tasks.end(),
                     [](const std::pair<int64_t, pm::MxTask>& u, const std::pair<int64_t, pm::MxTask>& v) {
                         return u.first > v.first;
                     });
    std::vector<pm::MxTask> mtv(mx_tasks.size());
    for (size_t i = 0; i < mx_tasks.size(); i++) mtv[i] = mx_tasks[i].second;
    // longest first: a greedy queue then ends with the short tasks
    std::stable_sort(tasks.begin(), tasks.end(),
                     [](const std::pair<int64_t, pm::MulTask>& u, const std::pair<int64_t, pm::MulTask>& v) {
                         return u.first > v.first;
                     });
    std::vector<pm::MulTask> tv(tasks.size());
    for (size_t i = 0; i < tasks.size(); i++) tv[i] = tasks[i].second;
    pm_mul_batch* B = new pm_mul_batch();
    (void)hipGetDevice(&B->device);
    B->count = count;
    B->ntasks = (int)tv.size();
    B->r = r;
    B->kc = pm::mul_batch_kc(r, kc);
    B->fold_min = fold_min;
    hipError_t e = hipSuccess;
    if (count > 0) e = hipMalloc((void**)&B->d_items, host.size() * sizeof(pm::MulItem));
    if (e == hipSuccess && !tv.empty()) e = hipMalloc((void**)&B->d_tasks, tv.size() * sizeof(pm::MulTask));
    B->n_mx_tasks = (int)mtv.size();
    if (e == hipSuccess && !mx_items.empty())
        e = hipMalloc((void**)&B->d_mx_items, mx_items.size() * sizeof(pm::MxItem));
    if (e == hipSuccess && !mtv.empty()) e = hipMalloc((void**)&B->d_mx_tasks, mtv.size() * sizeof(pm::MxTask));
    if (e != hipSuccess) {
        pm_mul_batch_destroy(B);
        return fail(PM_ENOMEM, "batch tables: %s", hipGetErrorString(e));
    }
    if (count > 0) e = hipMemcpy(B->d_items, host.data(), host.size() * sizeof(pm::MulItem), hipMemcpyHostToDevice);
    if (e == hipSuccess && !tv.empty())
        e = hipMemcpy(B->d_tasks, tv.data(), tv.size() * sizeof(pm::MulTask), hipMemcpyHostToDevice);
    if (e == hipSuccess && !mx_items.empty())
        e = hipMemcpy(B->d_mx_items, mx_items.data(), mx_items.size() * sizeof(pm::MxItem), hipMemcpyHostToDevice);
    if (e == hipSuccess && !mtv.empty())
        e = hipMemcpy(B->d_mx_tasks, mtv.data(), mtv.size() * sizeof(pm::MxTask), hipMemcpyHostToDevice);
    if (e == hipSuccess && B->r == 4 && B->ntasks > 0 && B->n_mx_tasks > 0) {
        e = hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        pm_mul_batch_destroy(B);
        return hip_fail(e, "batch upload");
    }
    *out = B;
    return PM_OK;
    PM_API_END
}

pm_status pm_mul_batch_run(pm_mul_batch* B, int32_t* d_status, void* stream) {
    PM_API_BEGIN
    if (!B) return fail(PM_EINVAL, "null batch");
    hipStream_t s = (hipStream_t)stream;
    if (d_status) HIP_TRY(pm::mul_batch_check_launch(B->d_items, B->count, d_status, s), "batch check launch");
    if (B->side) {
        HIP_TRY(hipEventRecord(B->ev_fork, s), "batch fork");
        HIP_TRY(hipStreamWaitEvent(B->side, B->ev_fork, 0), "batch fork");
        HIP_TRY(pm::mulx_batch_launch(B->d_mx_items, B->d_mx_tasks, B->n_mx_tasks, num_cus(), s),
                "batch launch (matrix cores)");
        HIP_TRY(pm::mul_batch_launch(B->d_items, B->d_tasks, B->ntasks, B->r, B->kc, B->fold_min, num_cus(),
                                     B->side, 1),
                "batch launch");
        HIP_TRY(hipEventRecord(B->ev_join, B->side), "batch join");
        HIP_TRY(hipStreamWaitEvent(s, B->ev_join, 0), "batch join");
        return PM_OK;
    }
    HIP_TRY(pm::mulx_batch_launch(B->d_mx_items, B->d_mx_tasks, B->n_mx_tasks, num_cus(), s),
            "batch launch (matrix cores)");
    HIP_TRY(pm::mul_batch_launch(B->d_items, B->d_tasks, B->ntasks, B->r, B->kc, B->fold_min, num_cus(), s),
            "batch launch");
    return PM_OK;
    PM_API_END
}

pm_status poly_mul_modp_batch(const pm_mul_item* items, int32_t count, int32_t* d_status, void* stream) {
    PM_API_BEGIN
    pm_mul_batch* B = nullptr;
    pm_params pp = params_now();
    int r = pp.mul_r == 4 || pp.mul_r == 8 || pp.mul_r == 16 ? pp.mul_r : 0;
    pm_status st = pm_mul_batch_create(items, count, r, pp.mul_s, &B);
    if (st) return st;
    st = pm_mul_batch_run(B, d_status, stream);
    if (st == PM_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) st = fail(PM_EDEVICE, "sync");
    pm_mul_batch_destroy(B);
    return st;
    PM_API_END
}

pm_status poly_mul_modp(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p, uint32_t* f,
                        int64_t f_cap, int64_t* nf, void* stream) {
    PM_API_BEGIN
    if (!nf) return fail(PM_EINVAL, "null nf");
    if (bad_len(a, na) || bad_len(b, nb)) return fail(PM_EINVAL, "null input or negative length");
    int64_t need = (na > 0 && nb > 0) ? na + nb - 1 : 0;
    if (need > 0 && (f == nullptr || f_cap < need))
        return fail(PM_EINVAL, "f_cap %lld < na + nb - 1 = %lld", (long long)f_cap, (long long)need);
    if (check_aliasing({{f, need}}, {{a, na}, {b, nb}})) return PM_EINVAL;
    pm::Field F;
    pm_status st = field_for(p, &F);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    Pool* P = nullptr;
    if ((st = pool_get(s, 0, &P))) return st;
    if ((st = mul_enqueue(a, na, b, nb, F, f, &P->d_info->n0, &P->d_info->status, s))) return st;
    if ((st = read_info(P, s))) return st;
    *nf = P->h_info->n0;
    if (P->h_info->status) return fail(P->h_info->status, "%s", status_text(P->h_info->status));
    return PM_OK;
    PM_API_END
}

}  // extern "C"

namespace {

// The remainder of a division once q is known: r_k = a_k - (q*b)_k for
// k < nout (nout = deg b). Only b_0 .. b_{nout-1} and q_0 .. q_{nout-1}
// reach those exponents, so the product takes nout coefficients of b and
// nq <= nout of q. Returns the pool it used in *P.
void remainder_shape(const uint32_t*& x, int64_t& nx, const uint32_t*& y, int64_t& ny, const uint32_t* b,
                     const uint32_t* q, int64_t nq, int64_t nout) {
    x = b;
    nx = nout;
    y = q;
    ny = nq;
    order_operands(x, nx, y, ny);
}

int64_t remainder_scratch_words(int64_t nq, int64_t nout) {
    if (nq <= 0 || nout <= 0) return 0;
    const uint32_t *x = nullptr, *y = nullptr;
    int64_t nx = 0, ny = 0;
    remainder_shape(x, nx, y, ny, nullptr, nullptr, nq, nout);
    pm::MxGeom g;
    if (mfma_plan(nx, ny, nout, &g)) return pm::mulx_scratch_words(g);
    return pm::mul_scratch_words(nx, ny, mul_plan(nx, ny));
}

pm_status remainder_enqueue(const uint32_t* a, const uint32_t* b, const uint32_t* q, int64_t nq, int64_t nout,
                            const pm::Field& F, uint32_t* r, hipStream_t s, Pool** P) {
    const uint32_t *x, *y;
    int64_t nx, ny;
    remainder_shape(x, nx, y, ny, b, q, nq, nout);
    pm_status st;
    pm::MxGeom g;
    if (mfma_plan(nx, ny, nout, &g)) {
        if ((st = pool_get(s, pm::mulx_scratch_words(g), P))) return st;
        HIP_TRY(pm::mulx_launch(x, nx, y, ny, F, r, g, (*P)->words, nullptr, nullptr, s, a, nout),
                "remainder launch");
    } else {
        const pm::MulPlan plan = mul_plan(nx, ny);
        if ((st = pool_get(s, pm::mul_scratch_words(nx, ny, plan), P))) return st;
        HIP_TRY(pm::mul_launch(x, nx, y, ny, F, r, plan, (*P)->words, nullptr, nullptr, a, nout, s),
                "remainder launch");
    }
    return PM_OK;
}

// The division of poly_divrem_modp; also reports deg a and deg b (degs[0],
// degs[1]) when degs is given.
pm_status divrem_impl(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p, uint32_t* q,
                      int64_t q_cap, int64_t* nq, uint32_t* r, int64_t r_cap, int64_t* nr, void* stream,
                      int64_t* degs) {
    if (!nq || !nr) return fail(PM_EINVAL, "null nq or nr");
    if (bad_len(a, na) || bad_len(b, nb)) return fail(PM_EINVAL, "null input or negative length");
    if (q_cap < 0 || r_cap < 0 || (q_cap > 0 && !q) || (r_cap > 0 && !r))
        return fail(PM_EINVAL, "bad output buffer");
    if (check_aliasing({{q, q_cap}, {r, r_cap}}, {{a, na}, {b, nb}})) return PM_EINVAL;
    if (nb == 0) return fail(PM_EDIVZERO, "division by the zero polynomial");
    if (na - nb + 1 > q_cap) return fail(PM_EINVAL, "q_cap %lld < na - nb + 1", (long long)q_cap);
    pm::Field F;
    pm_status st = field_for(p, &F);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    Pool* P = nullptr;
    if ((st = pool_get(s, pm::divrem_head_words(na), &P))) return st;
    pm_params pp = params_now();
    HIP_TRY(pm::divrem_head_launch(a, na, b, nb, F, q, q_cap, r_cap, P->words, P->d_info,
                                   pp.div_s > 0 ? pp.div_s : 64, num_cus(), s),
            "divrem head launch");
    if ((st = read_info(P, s))) return st;
    const pm::CallInfo I = *P->h_info;
    if (I.status) return fail(I.status, "%s", status_text(I.status));
    const int64_t da = I.deg_a, db = I.deg_b;
    if (degs) {
        degs[0] = da;
        degs[1] = db;
    }
    if (da < db) {  // q = 0, r = a
        if (da >= 0)
            HIP_TRY(hipMemcpyAsync(r, a, (size_t)(da + 1) * 4, hipMemcpyDeviceToDevice, s), "copy r");
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        *nq = 0;
        *nr = da + 1;
        return PM_OK;
    }
    const int64_t mu = da - db + 1;
    *nq = mu;
    if (db == 0) {
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        *nr = 0;
        return PM_OK;
    }
    if ((st = remainder_enqueue(a, b, q, mu < db ? mu : db, db, F, r, s, &P))) return st;
    HIP_TRY(pm::trim_launch(r, db, P->d_info, s), "trim launch");
    if ((st = read_info(P, s))) return st;
    *nr = P->h_info->n1;
    return PM_OK;
}

}  // namespace

extern "C" {

pm_status poly_divrem_modp(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p, uint32_t* q,
                           int64_t q_cap, int64_t* nq, uint32_t* r, int64_t r_cap, int64_t* nr, void* stream) {
    PM_API_BEGIN
    return divrem_impl(a, na, b, nb, p, q, q_cap, nq, r, r_cap, nr, stream, nullptr);
    PM_API_END
}

pm_status poly_divrem_modp_naive(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p,
                                 uint32_t* q, int64_t q_cap, int64_t* nq, uint32_t* r, int64_t r_cap, int64_t* nr,
                                 void* stream) {
    PM_API_BEGIN
    if (!nq || !nr) return fail(PM_EINVAL, "null nq or nr");
    if (bad_len(a, na) || bad_len(b, nb)) return fail(PM_EINVAL, "null input or negative length");
    if (q_cap < 0 || r_cap < 0 || (q_cap > 0 && !q) || (r_cap > 0 && !r))
        return fail(PM_EINVAL, "bad output buffer");
    if (check_aliasing({{q, q_cap}, {r, r_cap}}, {{a, na}, {b, nb}})) return PM_EINVAL;
    if (nb == 0) return fail(PM_EDIVZERO, "division by the zero polynomial");
    if (na - nb + 1 > q_cap) return fail(PM_EINVAL, "q_cap %lld < na - nb + 1", (long long)q_cap);
    pm::Field F;
    pm_status st = field_for(p, &F);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    Pool* P = nullptr;
    if ((st = pool_get(s, na > 0 ? na : 1, &P))) return st;
    HIP_TRY(pm::naive_prep_launch(a, na, b, nb, F, P->d_info, s), "naive prep launch");
    if ((st = read_info(P, s))) return st;
    const int64_t da = P->h_info->deg_a, db = P->h_info->deg_b;
    if (P->h_info->flags) return fail(PM_ERANGE, "%s", status_text(PM_ERANGE));
    if (db < 0) return fail(PM_EDIVZERO, "division by the zero polynomial");
    if (da < db) {  // q = 0, r = a
        if (da + 1 > r_cap) return fail(PM_EINVAL, "r_cap %lld < deg a + 1", (long long)r_cap);
        if (da >= 0)
            HIP_TRY(hipMemcpyAsync(r, a, (size_t)(da + 1) * 4, hipMemcpyDeviceToDevice, s), "copy r");
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        *nq = 0;
        *nr = da + 1;
        return PM_OK;
    }
    const int64_t mu = da - db + 1;
    if (mu > q_cap || db > r_cap) return fail(PM_EINVAL, "output capacity below the true degrees");
    uint32_t lc = 0;
    HIP_TRY(hipMemcpy(&lc, b + db, 4, hipMemcpyDeviceToHost), "read lc(b)");
    const uint32_t inv = (uint32_t)powmod_host(lc, p - 2, p);
    uint32_t* w = P->words;
    HIP_TRY(hipMemcpyAsync(w, a, (size_t)(da + 1) * 4, hipMemcpyDeviceToDevice, s), "copy a");
    HIP_TRY(pm::naive_divrem_launch(w, b, da, db, inv, q, F, s), "naive division launch");
    *nq = mu;
    if (db == 0) {
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        *nr = 0;
        return PM_OK;
    }
    HIP_TRY(hipMemcpyAsync(r, w, (size_t)db * 4, hipMemcpyDeviceToDevice, s), "copy r");
    HIP_TRY(pm::trim_launch(r, db, P->d_info, s), "trim launch");
    if ((st = read_info(P, s))) return st;
    *nr = P->h_info->n1;
    return PM_OK;
    PM_API_END
}

pm_status poly_gcd_modp_naive(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p, uint32_t* g,
                              int64_t g_cap, int64_t* ng, void* stream) {
    PM_API_BEGIN
    if (!ng) return fail(PM_EINVAL, "null ng");
    if (bad_len(a, na) || bad_len(b, nb)) return fail(PM_EINVAL, "null input or negative length");
    if (g_cap < 0 || (g_cap > 0 && !g)) return fail(PM_EINVAL, "bad output buffer");
    if (check_aliasing({{g, g_cap}}, {{a, na}, {b, nb}})) return PM_EINVAL;
    pm::Field F;
    pm_status st = field_for(p, &F);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    g_gcd_stats = pm_gcd_stats{0, 0, 0};
    const int64_t n = (na > nb ? na : nb) > 0 ? (na > nb ? na : nb) : 1;
    Pool* P = nullptr;
    if ((st = pool_get(s, 2 * n, &P))) return st;
    uint32_t* A = P->words;
    uint32_t* B = P->words + n;
    HIP_TRY(pm::naive_prep_launch(a, na, b, nb, F, P->d_info, s), "naive prep launch");
    HIP_TRY(hipMemsetAsync(P->words, 0, (size_t)(2 * n) * 4, s), "clear");
    if (na) HIP_TRY(hipMemcpyAsync(A, a, (size_t)na * 4, hipMemcpyDeviceToDevice, s), "copy a");
    if (nb) HIP_TRY(hipMemcpyAsync(B, b, (size_t)nb * 4, hipMemcpyDeviceToDevice, s), "copy b");
    if ((st = read_info(P, s))) return st;
    if (P->h_info->flags) return fail(PM_ERANGE, "%s", status_text(PM_ERANGE));
    // every step lowers deg a + deg b by at least one; the host checks for
    // the end every 512 steps (later launches of a finished run do nothing)
    int64_t left = (P->h_info->deg_a > 0 ? P->h_info->deg_a : 0) + (P->h_info->deg_b > 0 ? P->h_info->deg_b : 0) + 2;
    while (P->h_info->deg_a >= 0 && P->h_info->deg_b >= 0 && left > 0) {
        const int64_t k = left < 512 ? left : 512;
        HIP_TRY(pm::naive_gcd_steps_launch(A, B, n, k, F, P->d_info, s), "naive gcd launch");
        left -= k;
        if ((st = read_info(P, s))) return st;
    }
    if (P->h_info->deg_a >= 0 && P->h_info->deg_b >= 0) return fail(PM_EDEVICE, "naive gcd did not finish");
    const int64_t dR = P->h_info->deg_a >= 0 ? P->h_info->deg_a : P->h_info->deg_b;
    g_gcd_stats = pm_gcd_stats{P->h_info->steps, P->h_info->updates, P->h_info->steps};
    if (dR + 1 > g_cap) return fail(PM_EINVAL, "g_cap %lld < deg gcd + 1", (long long)g_cap);
    if (dR >= 0) HIP_TRY(pm::naive_monic_launch(A, B, g, g_cap, n, F, P->d_info, s), "monic launch");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    *ng = dR + 1;
    return PM_OK;
    PM_API_END
}

static_assert(sizeof(pm_gcd_result) == sizeof(pm::GcdResult), "result layouts differ");

}  // extern "C"

namespace {

// Checks every item of a gcd batch on the host and builds its jobs (out
// pointers left null) and the launch order: the items of the 1024-thread
// shape, then those of the 256-thread shape, each longest first (by
// na * nb; blocks start in index order, so the longest start first).
pm_status gcd_batch_jobs(const pm_gcd_item* items, int32_t count, std::vector<pm::GcdJob>& jobs,
                         std::vector<int32_t>& large, std::vector<int32_t>& small) {
    jobs.assign((size_t)count, pm::GcdJob{});
    large.clear();
    small.clear();
    for (int32_t i = 0; i < count; i++) {
        const pm_gcd_item& it = items[i];
        if (bad_len(it.a, it.na) || bad_len(it.b, it.nb) || it.g_cap < 0 || (it.g_cap > 0 && !it.g))
            return fail(PM_EINVAL, "item %d: bad pointer or length", i);
        if (check_aliasing({{it.g, it.g_cap}}, {{it.a, it.na}, {it.b, it.nb}}))
            return fail(PM_EINVAL, "item %d: the output overlaps an input", i);
        int64_t n = it.na > it.nb ? it.na : it.nb;
        if (n > PM_GCD_BATCH_MAX)
            return fail(PM_EINVAL, "item %d: %lld terms exceed the batch limit", i, (long long)n);
        pm::Field F;
        pm_status st = field_for(it.p, &F);
        if (st) return st;
        jobs[i] = pm::GcdJob{it.a, it.b, it.na, it.nb, it.g, it.g_cap, nullptr, F, 0, 0};
        (n <= pm::gcd_batch_cap(0) ? small : large).push_back(i);
    }
    auto longest_first = [items](int32_t x, int32_t y) {
        return (double)items[x].na * (double)items[x].nb > (double)items[y].na * (double)items[y].nb;
    };
    std::stable_sort(large.begin(), large.end(), longest_first);
    std::stable_sort(small.begin(), small.end(), longest_first);
    return PM_OK;
}

}  // namespace

extern "C" {

pm_status poly_gcd_modp_batch(const pm_gcd_item* items, int32_t count, pm_gcd_result* results, void* stream) {
    PM_API_BEGIN
    if (count < 0 || (count > 0 && (!items || !results))) return fail(PM_EINVAL, "bad item or result array");
    if (count == 0) return PM_OK;
    hipStream_t s = (hipStream_t)stream;
    std::vector<pm::GcdJob> jobs;
    std::vector<int32_t> small, large;
    {
        pm_status st0 = gcd_batch_jobs(items, count, jobs, large, small);
        if (st0) return st0;
    }
    // scratch: jobs | order | results
    const int64_t job_words = ((int64_t)count * (int64_t)sizeof(pm::GcdJob) + 3) / 4;
    const int64_t res_off = (job_words + count + 3) & ~3LL;
    const int64_t res_words = ((int64_t)count * (int64_t)sizeof(pm::GcdResult) + 3) / 4;
    Pool* P = nullptr;
    pm_status st = pool_get(s, res_off + res_words + 16, &P);
    if (st) return st;
    pm::GcdJob* d_jobs = (pm::GcdJob*)P->words;
    int32_t* d_order = (int32_t*)(P->words + job_words);
    pm::GcdResult* d_res = (pm::GcdResult*)(P->words + res_off);
    for (int32_t i = 0; i < count; i++) jobs[i].out = d_res + i;
    std::vector<int32_t> order;
    order.insert(order.end(), large.begin(), large.end());
    order.insert(order.end(), small.begin(), small.end());
    HIP_TRY(hipMemcpyAsync(d_jobs, jobs.data(), jobs.size() * sizeof(pm::GcdJob), hipMemcpyHostToDevice, s),
            "copy jobs");
    HIP_TRY(hipMemcpyAsync(d_order, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice, s),
            "copy order");
    pm_params pp = params_now();
    const int gs = pp.gcd_s > 0 ? pp.gcd_s : 128;
    if (!large.empty())
        HIP_TRY(pm::gcd_batch_launch(d_jobs, d_order, (int)large.size(), 1, gs, s), "gcd batch launch");
    if (!small.empty())
        HIP_TRY(pm::gcd_batch_launch(d_jobs, d_order + large.size(), (int)small.size(), 0, gs, s),
                "gcd batch launch");
    HIP_TRY(hipMemcpyAsync(results, d_res, (size_t)count * sizeof(pm::GcdResult), hipMemcpyDeviceToHost, s),
            "copy results");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    return PM_OK;
    PM_API_END
}

pm_status pm_gcd_batch_create(const pm_gcd_item* items, int32_t count, int32_t s, pm_gcd_batch** out) {
    PM_API_BEGIN
    if (!out || count < 0 || (count > 0 && !items)) return fail(PM_EINVAL, "bad arguments");
    if (s < 0 || s > 256) return fail(PM_EINVAL, "s must be in [0, 256]");
    *out = nullptr;
    std::vector<pm::GcdJob> jobs;
    std::vector<int32_t> small, large;
    pm_status st = gcd_batch_jobs(items, count, jobs, large, small);
    if (st) return st;
    pm_gcd_batch* B = new pm_gcd_batch();
    HIP_TRY(hipGetDevice(&B->device), "hipGetDevice");
    B->count = count;
    B->n_large = (int32_t)large.size();
    B->n_small = (int32_t)small.size();
    B->s = s > 0 ? s : 128;
    const size_t n = (size_t)(count > 0 ? count : 1);
    if (hipMalloc((void**)&B->d_jobs, n * sizeof(pm::GcdJob)) != hipSuccess ||
        hipMalloc((void**)&B->d_order, n * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void**)&B->d_res, n * sizeof(pm::GcdResult)) != hipSuccess) {
        pm_gcd_batch_destroy(B);
        return fail(PM_ENOMEM, "cannot allocate the batch");
    }
    for (int32_t i = 0; i < count; i++) jobs[(size_t)i].out = B->d_res + i;
    std::vector<int32_t> order;
    order.insert(order.end(), large.begin(), large.end());
    order.insert(order.end(), small.begin(), small.end());
    if ((count > 0 && (hipMemcpy(B->d_jobs, jobs.data(), (size_t)count * sizeof(pm::GcdJob),
                                 hipMemcpyHostToDevice) != hipSuccess ||
                       hipMemcpy(B->d_order, order.data(), (size_t)count * sizeof(int32_t),
                                 hipMemcpyHostToDevice) != hipSuccess)) ||
        hipMemset(B->d_res, 0, n * sizeof(pm::GcdResult)) != hipSuccess) {
        pm_gcd_batch_destroy(B);
        return fail(PM_EDEVICE, "cannot upload the batch");
    }
    if (B->n_large > 0 && B->n_small > 0 &&
        (hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking) != hipSuccess ||
         hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming) != hipSuccess ||
         hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming) != hipSuccess)) {
        pm_gcd_batch_destroy(B);
        return fail(PM_EDEVICE, "cannot create the batch's second stream");
    }
    *out = B;
    return PM_OK;
    PM_API_END
}

pm_status pm_gcd_batch_run(pm_gcd_batch* B, void* stream) {
    PM_API_BEGIN
    if (!B) return fail(PM_EINVAL, "null batch");
    hipStream_t hs = (hipStream_t)stream;
    if (B->side) {
        HIP_TRY(hipEventRecord(B->ev_fork, hs), "gcd batch fork");
        HIP_TRY(hipStreamWaitEvent(B->side, B->ev_fork, 0), "gcd batch fork");
        HIP_TRY(pm::gcd_batch_launch(B->d_jobs, B->d_order, B->n_large, 1, B->s, hs), "gcd batch launch");
        HIP_TRY(pm::gcd_batch_launch(B->d_jobs, B->d_order + B->n_large, B->n_small, 0, B->s, B->side),
                "gcd batch launch");
        HIP_TRY(hipEventRecord(B->ev_join, B->side), "gcd batch join");
        HIP_TRY(hipStreamWaitEvent(hs, B->ev_join, 0), "gcd batch join");
        return PM_OK;
    }
    if (B->n_large > 0)
        HIP_TRY(pm::gcd_batch_launch(B->d_jobs, B->d_order, B->n_large, 1, B->s, hs), "gcd batch launch");
    if (B->n_small > 0)
        HIP_TRY(pm::gcd_batch_launch(B->d_jobs, B->d_order + B->n_large, B->n_small, 0, B->s, hs),
                "gcd batch launch");
    return PM_OK;
    PM_API_END
}

pm_status pm_gcd_batch_results(pm_gcd_batch* B, pm_gcd_result* results, void* stream) {
    PM_API_BEGIN
    if (!B || (B->count > 0 && !results)) return fail(PM_EINVAL, "null argument");
    if (B->count == 0) return PM_OK;
    hipStream_t hs = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(results, B->d_res, (size_t)B->count * sizeof(pm::GcdResult), hipMemcpyDeviceToHost, hs),
            "copy results");
    HIP_TRY(hipStreamSynchronize(hs), "hipStreamSynchronize");
    return PM_OK;
    PM_API_END
}

void pm_gcd_batch_destroy(pm_gcd_batch* B) {
    PM_API_BEGIN
    if (!B) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(B->device);
    (void)hipDeviceSynchronize();
    if (B->d_jobs) (void)hipFree(B->d_jobs);
    if (B->d_order) (void)hipFree(B->d_order);
    if (B->d_res) (void)hipFree(B->d_res);
    if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
    if (B->ev_join) (void)hipEventDestroy(B->ev_join);
    if (B->side) (void)hipStreamDestroy(B->side);
    (void)hipSetDevice(cur);
    delete B;
    PM_API_END_VOID
}

}  // extern "C"

namespace {

// A degree gap of at least this many positions starts the gcd with one
// Euclidean division: the chunked steps would take each step of a long
// quotient alone (its shift is beyond what a chunk's matrix holds).
constexpr int64_t GCD_LEAD_GAP = 128;

// The gcd of validated operands on the cooperative kernel, at every size:
// one call's latency is its step chain, and slices of 512 positions per
// block keep the apply short (one block below 513 terms). The one-block
// instance of the batch, which holds the pair in LDS, is for throughput
// over many instances. Sets the call's counts.
// The divisor degree of every step in a gcd step log (the layout of
// pm::GcdTrace), appended to divs in step order. Each step's operand
// degrees are rebuilt from the chunk's starting degrees and the shifts, and
// checked: the reduced operand is the one of higher degree (a on a tie),
// its degree falls, and every chunk ends at the next one's start. Returns
// false when the log is incomplete or inconsistent.
bool trace_divisor_degrees(const std::vector<int32_t>& log, int64_t chunk_cap, std::vector<int64_t>& divs) {
    const int32_t nrec = log[0], nst = log[1];
    if (log[2] != 0 || nrec < 1 || nrec > chunk_cap) return false;
    const int32_t* rec = log.data() + pm::GCD_TRACE_HDR;
    const int32_t* stp = rec + 4 * chunk_cap;
    for (int32_t c = 0; c + 1 < nrec; c++) {
        int64_t dA = rec[4 * c], dB = rec[4 * c + 1];
        const int32_t first = rec[4 * c + 2], n = rec[4 * c + 3];
        const int64_t eA = rec[4 * (c + 1)], eB = rec[4 * (c + 1) + 1];
        if (first < 0 || n < 1 || first + n > nst) return false;
        for (int32_t j = 0; j < n; j++) {
            const int32_t d = stp[2 * (first + j)], which = stp[2 * (first + j) + 1];
            const int64_t dX = which ? dB : dA, dY = which ? dA : dB;
            const bool rule = which ? dB > dA : dA >= dB;
            if (dY < 0 || !rule || dX - dY != d) return false;
            divs.push_back(dY);
            int64_t nd;
            if (j + 1 < n) {
                const int32_t d2 = stp[2 * (first + j + 1)], w2 = stp[2 * (first + j + 1) + 1];
                nd = w2 == which ? dY + d2 : dY - d2;
            } else {
                nd = which ? eB : eA;
            }
            if (nd >= dX) return false;
            (which ? dB : dA) = nd;
        }
        if (dA != eA || dB != eB) return false;
    }
    return true;
}

// The gcd of validated operands on the cooperative kernel, at every size:
// one call's latency is its step chain, and slices of 512 positions per
// block keep the apply short (one block below 513 terms). The one-block
// instance of the batch, which holds the pair in LDS, is for throughput
// over many instances. Sets the call's counts. With divs, the kernel also
// logs its steps and the divisor degree of each is appended to divs.
pm_status gcd_run(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, const pm::Field& F, uint32_t* g,
                  int64_t g_cap, int64_t* ng, hipStream_t s, std::vector<int64_t>* divs = nullptr) {
    const int64_t n = na > nb ? na : nb;
    pm_params pp = params_now();
    pm::GcdPlan plan = pm::gcd_default_plan(n > 0 ? n : 1, num_cus(), pp.gcd_s);
    Pool* P = nullptr;
    pm_status st;
    pm::GcdTrace tr{};
    std::vector<int32_t> log;
    if (divs) {
        if (na + nb + 8 > INT32_MAX / 8) return fail(PM_EINVAL, "operands too long for the step log");
        tr.chunk_cap = tr.step_cap = na + nb + 8;  // every chunk but the last runs a step
        tr.max_steps = -1;
        const int64_t words = pm::gcd_trace_words(tr.chunk_cap, tr.step_cap);
        uint32_t* w = nullptr;
        if ((st = aux_get(s, words, &w, AUX_TRACE))) return st;
        tr.log = (int32_t*)w;
        HIP_TRY(hipMemsetAsync(w, 0, pm::GCD_TRACE_HDR * sizeof(int32_t), s), "clear log");
        log.resize((size_t)words);
    }
    if ((st = pool_get(s, pm::gcd_scratch_words(n, plan), &P))) return st;
    HIP_TRY(pm::gcd_launch(a, na, b, nb, F, g, g_cap, P->words, P->d_info, plan, s, nullptr, divs ? &tr : nullptr),
            "gcd launch");
    if (divs)
        HIP_TRY(hipMemcpyAsync(log.data(), tr.log, log.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s),
                "copy log");
    if ((st = read_info(P, s))) return st;
    const pm::CallInfo I = *P->h_info;
    g_gcd_stats = pm_gcd_stats{I.steps, I.updates, I.chunks};
    if (I.status) return fail(I.status, "%s", status_text(I.status));
    if (divs && !trace_divisor_degrees(log, tr.chunk_cap, *divs))
        return fail(PM_EDEVICE, "the gcd's step log is inconsistent");
    *ng = I.n0;
    return PM_OK;
}

// The first division of the remainder sequence (Sec. 6) as one Euclidean
// division (Sec. 3), then the chunked gcd on what remains. The operand of
// higher degree, X, loses steps at every position from deg X down to deg Y,
// except that on a tie the paper reduces a: when X = b, the steps stop
// above deg a, so b becomes r + q_0 a rather than r. The steps and updates
// the division stands for are counted as the steps would be: one per
// position, deg Y + 1 updates each.
pm_status gcd_lead_division(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p,
                            const pm::Field& F, uint32_t* g, int64_t g_cap, int64_t* ng, hipStream_t s,
                            std::vector<int64_t>* divs = nullptr) {
    Pool* P = nullptr;
    pm_status st;
    if ((st = pool_get(s, 0, &P))) return st;
    HIP_TRY(pm::naive_prep_launch(a, na, b, nb, F, P->d_info, s), "degree scan");
    if ((st = read_info(P, s))) return st;
    if (P->h_info->flags) return fail(PM_ERANGE, "%s", status_text(PM_ERANGE));
    const int64_t dA = P->h_info->deg_a, dB = P->h_info->deg_b;
    const int64_t gap = dA > dB ? dA - dB : dB - dA;
    if (dA < 0 || dB < 0 || gap < GCD_LEAD_GAP) return gcd_run(a, na, b, nb, F, g, g_cap, ng, s, divs);
    const bool redA = dA > dB;
    const uint32_t* X = redA ? a : b;
    const uint32_t* Y = redA ? b : a;
    const int64_t dX = redA ? dA : dB, dY = redA ? dB : dA;
    const int64_t mu = dX - dY + 1;
    uint32_t* w = nullptr;
    const int64_t qw = (mu + 63) & ~63LL, rw = (dY + 1 + 63) & ~63LL;
    if ((st = aux_get(s, qw + 2 * rw, &w))) return st;
    uint32_t* q = w;
    uint32_t* r = w + qw;
    uint32_t* fold = r + rw;
    int64_t nq = 0, nr = 0;
    if ((st = divrem_impl(X, dX + 1, Y, dY + 1, p, q, mu, &nq, r, dY + 1, &nr, s, nullptr))) return st;
    int64_t count = mu;
    if (divs) divs->push_back(dY);  // every step of the division has Y as its divisor
    if (redA) {
        st = gcd_run(r, nr, b, dB + 1, F, g, g_cap, ng, s, divs);
    } else {
        uint32_t q0 = 0;
        HIP_TRY(hipMemcpyAsync(&q0, q, sizeof(q0), hipMemcpyDeviceToHost, s), "copy q_0");
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (q0 == 0) {
            st = gcd_run(a, dA + 1, r, nr, F, g, g_cap, ng, s, divs);
        } else {
            count = mu - 1;  // position deg a is a's step (the tie)
            HIP_TRY(pm::fold_q0_launch(r, nr, q, a, dA + 1, fold, F, s), "fold launch");
            st = gcd_run(a, dA + 1, fold, dA + 1, F, g, g_cap, ng, s, divs);
        }
    }
    g_gcd_stats.steps += count;
    g_gcd_stats.updates += count * (dY + 1);
    return st;
}

}  // namespace

extern "C" {

pm_status poly_gcd_modp(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p, uint32_t* g,
                        int64_t g_cap, int64_t* ng, void* stream) {
    PM_API_BEGIN
    if (!ng) return fail(PM_EINVAL, "null ng");
    if (bad_len(a, na) || bad_len(b, nb)) return fail(PM_EINVAL, "null input or negative length");
    if (g_cap < 0 || (g_cap > 0 && !g)) return fail(PM_EINVAL, "bad output buffer");
    if (check_aliasing({{g, g_cap}}, {{a, na}, {b, nb}})) return PM_EINVAL;
    pm::Field F;
    pm_status st = field_for(p, &F);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    g_gcd_stats = pm_gcd_stats{0, 0, 0};
    const int64_t gap = na > nb ? na - nb : nb - na;
    if (na > 0 && nb > 0 && gap >= GCD_LEAD_GAP) return gcd_lead_division(a, na, b, nb, p, F, g, g_cap, ng, s);
    return gcd_run(a, na, b, nb, F, g, g_cap, ng, s);
    PM_API_END
}

pm_status poly_gcd_modp_degrees(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p,
                                uint32_t* g, int64_t g_cap, int64_t* ng, int64_t* degs, int64_t degs_cap,
                                int64_t* n_degs, void* stream) {
    PM_API_BEGIN
    if (!ng || !n_degs || degs_cap < 0 || (degs_cap > 0 && !degs)) return fail(PM_EINVAL, "null ng, n_degs or degs");
    if (bad_len(a, na) || bad_len(b, nb)) return fail(PM_EINVAL, "null input or negative length");
    if (g_cap < 0 || (g_cap > 0 && !g)) return fail(PM_EINVAL, "bad output buffer");
    if (check_aliasing({{g, g_cap}}, {{a, na}, {b, nb}})) return PM_EINVAL;
    pm::Field F;
    pm_status st = field_for(p, &F);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    g_gcd_stats = pm_gcd_stats{0, 0, 0};
    // the trimmed degrees start the sequence
    Pool* P = nullptr;
    if ((st = pool_get(s, 0, &P))) return st;
    HIP_TRY(pm::naive_prep_launch(a, na, b, nb, F, P->d_info, s), "degree scan");
    if ((st = read_info(P, s))) return st;
    if (P->h_info->flags) return fail(PM_ERANGE, "%s", status_text(PM_ERANGE));
    const int64_t dA = P->h_info->deg_a, dB = P->h_info->deg_b;
    std::vector<int64_t> divs;
    const int64_t gap = na > nb ? na - nb : nb - na;
    if (na > 0 && nb > 0 && gap >= GCD_LEAD_GAP) st = gcd_lead_division(a, na, b, nb, p, F, g, g_cap, ng, s, &divs);
    else st = gcd_run(a, na, b, nb, F, g, g_cap, ng, s, &divs);
    if (st) return st;
    // deg r0, then each divisor's degree once (the remainders, in order), then
    // the zero remainder that ends the sequence
    std::vector<int64_t> seq{dA > dB ? dA : dB};
    for (int64_t d : divs)
        if (seq.size() == 1 || seq.back() != d) seq.push_back(d);
    seq.push_back(-1);  // with a zero operand the sequence is (deg r0, -1)
    *n_degs = (int64_t)seq.size();
    for (int64_t i = 0; i < (int64_t)seq.size() && i < degs_cap; i++) degs[i] = seq[(size_t)i];
    return PM_OK;
    PM_API_END
}

pm_status poly_euclid_steps_modp(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p,
                                 int64_t k, uint32_t* x, int64_t x_cap, int64_t* nx, uint32_t* y, int64_t y_cap,
                                 int64_t* ny, int64_t* taken, void* stream) {
    PM_API_BEGIN
    if (!nx || !ny || !taken) return fail(PM_EINVAL, "null nx, ny or taken");
    if (k < 0) return fail(PM_EINVAL, "negative step count");
    if (bad_len(a, na) || bad_len(b, nb)) return fail(PM_EINVAL, "null input or negative length");
    if (x_cap < 0 || (x_cap > 0 && !x) || y_cap < 0 || (y_cap > 0 && !y)) return fail(PM_EINVAL, "bad output buffer");
    if (check_aliasing({{x, x_cap}, {y, y_cap}}, {{a, na}, {b, nb}})) return PM_EINVAL;
    pm::Field F;
    pm_status st = field_for(p, &F);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = na > nb ? na : nb;
    pm_params pp = params_now();
    const pm::GcdPlan plan = pm::gcd_default_plan(n > 0 ? n : 1, num_cus(), pp.gcd_s);
    Pool* P = nullptr;
    if ((st = pool_get(s, pm::gcd_scratch_words(n, plan), &P))) return st;
    const pm::GcdTrace tr{nullptr, 0, 0, k, y, y_cap};
    HIP_TRY(pm::gcd_launch(a, na, b, nb, F, x, x_cap, P->words, P->d_info, plan, s, nullptr, &tr), "gcd launch");
    if ((st = read_info(P, s))) return st;
    const pm::CallInfo I = *P->h_info;
    if (I.status) return fail(I.status, "%s", status_text(I.status));
    *nx = I.n0;
    *ny = I.n1;
    *taken = I.run_steps;
    return PM_OK;
    PM_API_END
}

}  // extern "C"

namespace {

// Consecutive 64-word-aligned pieces of one scratch buffer.
struct Carve {
    uint32_t* base;
    int64_t used;
    uint32_t* take(int64_t words) {
        uint32_t* p = base + used;
        used += (words + 63) & ~63LL;
        return p;
    }
};

pm_status trimmed_length(const uint32_t* x, int64_t n, hipStream_t s, int64_t* out) {
    *out = 0;
    if (n <= 0) return PM_OK;
    Pool* P = nullptr;
    pm_status st;
    if ((st = pool_get(s, 0, &P))) return st;
    HIP_TRY(pm::trim_launch(x, n, P->d_info, s), "trim launch");
    if ((st = read_info(P, s))) return st;
    *out = P->h_info->n1;
    return PM_OK;
}

}  // namespace

extern "C" {

pm_status poly_xgcd_modp(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p, uint32_t* g,
                         int64_t g_cap, int64_t* ng, uint32_t* s_out, int64_t s_cap, int64_t* ns, uint32_t* t_out,
                         int64_t t_cap, int64_t* nt, void* stream) {
    PM_API_BEGIN
    if (!ng || !ns || !nt) return fail(PM_EINVAL, "null ng, ns or nt");
    if (bad_len(a, na) || bad_len(b, nb)) return fail(PM_EINVAL, "null input or negative length");
    if (g_cap < 0 || (g_cap > 0 && !g) || s_cap < 0 || (s_cap > 0 && !s_out) || t_cap < 0 || (t_cap > 0 && !t_out))
        return fail(PM_EINVAL, "bad output buffer");
    if (check_aliasing({{g, g_cap}, {s_out, s_cap}, {t_out, t_cap}}, {{a, na}, {b, nb}})) return PM_EINVAL;
    pm::Field F;
    pm_status st = field_for(p, &F);
    if (st) return st;
    hipStream_t hs = (hipStream_t)stream;
    g_gcd_stats = pm_gcd_stats{0, 0, 0};
    *ng = *ns = *nt = 0;
    Pool* P = nullptr;
    if ((st = pool_get(hs, 0, &P))) return st;
    HIP_TRY(pm::naive_prep_launch(a, na, b, nb, F, P->d_info, hs), "degree scan");
    if ((st = read_info(P, hs))) return st;
    if (P->h_info->flags) return fail(PM_ERANGE, "%s", status_text(PM_ERANGE));
    const int64_t dA = P->h_info->deg_a, dB = P->h_info->deg_b;
    if (dA < 0 && dB < 0) return PM_OK;  // gcd(0, 0) = 0 = 0 a + 0 b
    const int64_t n = (dA > dB ? dA : dB) + 1;
    pm_params pp = params_now();
    const pm::GcdPlan plan = pm::gcd_default_plan(n, num_cus(), pp.gcd_s);
    const int64_t N = pm::gcd_positions(plan);
    uint32_t* wbase = nullptr;
    if ((st = aux_get(hs, N + 20 * (n + 64) + 64, &wbase))) return st;
    Carve W{wbase, 0};
    uint32_t* one = W.take(1);
    HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)one, 1u, 1, hs), "set 1");

    // the pair the gcd kernel starts from, and the cofactor of a in each
    const uint32_t *A1 = a, *B1 = b;
    int64_t nA1 = dA + 1, nB1 = dB + 1;
    const uint32_t* sb0 = nullptr;
    int64_t nsb = 0, count = 0, cY = 0;
    const int64_t gap = dA > dB ? dA - dB : dB - dA;
    if (dA >= 0 && dB >= 0 && gap >= GCD_LEAD_GAP) {
        // the leading division, as in poly_gcd_modp
        const bool redA = dA > dB;
        const uint32_t* X = redA ? a : b;
        const uint32_t* Y = redA ? b : a;
        const int64_t dX = redA ? dA : dB, dY = redA ? dB : dA;
        const int64_t mu = dX - dY + 1;
        uint32_t* q = W.take(mu);
        uint32_t* r = W.take(dY + 1);
        int64_t nq = 0, nr = 0;
        if ((st = divrem_impl(X, dX + 1, Y, dY + 1, p, q, mu, &nq, r, dY + 1, &nr, hs, nullptr))) return st;
        count = mu;
        cY = dY + 1;
        if (redA) {
            A1 = r;  // a - q b: cofactor 1
            nA1 = nr;
        } else {
            uint32_t q0 = 0;
            HIP_TRY(hipMemcpyAsync(&q0, q, sizeof(q0), hipMemcpyDeviceToHost, hs), "copy q_0");
            HIP_TRY(hipStreamSynchronize(hs), "hipStreamSynchronize");
            uint32_t* sneg = W.take(mu);
            HIP_TRY(pm::negate_launch(q, mu, sneg, p, q0 != 0, hs), "negate launch");
            sb0 = sneg;  // b - q a, or b - (q - q_0) a: cofactor -q or -(q - q_0)
            nsb = mu;
            if (q0 == 0) {
                B1 = r;
                nB1 = nr;
            } else {
                count = mu - 1;
                uint32_t* fold = W.take(dA + 1);
                HIP_TRY(pm::fold_q0_launch(r, nr, q, a, dA + 1, fold, F, hs), "fold launch");
                B1 = fold;
                nB1 = dA + 1;
            }
        }
    }

    // the remainder sequence with the cofactor of a carried along
    uint32_t* s_res = W.take(N);
    if ((st = pool_get(hs, pm::gcd_scratch_words(n, plan, true), &P))) return st;
    const pm::GcdCofactors xg{one, 1, sb0, nsb, dB > 0 ? dB : 0, s_res};
    HIP_TRY(pm::gcd_launch(A1, nA1, B1, nB1, F, g, g_cap, P->words, P->d_info, plan, hs, &xg), "gcd launch");
    if ((st = read_info(P, hs))) return st;
    const pm::CallInfo I = *P->h_info;
    g_gcd_stats = pm_gcd_stats{I.steps + count, I.updates + count * cY, I.chunks};
    if (I.status) return fail(I.status, "%s", status_text(I.status));
    const int64_t n_g = I.n0, dg = n_g - 1;

    // the unique cofactors: deg s < deg b - deg g (s = 0 when g ~ b), and
    // t = (g - s a) / b exactly; t = 0 when b = 0
    int64_t ls = 0;
    if ((st = trimmed_length(s_res, dB > 0 ? dB + 1 : 1, hs, &ls))) return st;
    const uint32_t* sf = s_res;
    int64_t nsf = ls;
    const uint32_t* tf = nullptr;
    int64_t ntf = 0;
    if (dB >= 0) {
        if (dg == dB) {
            nsf = 0;
        } else if (ls - 1 >= dB - dg) {
            uint32_t* h = W.take(dB + 1);
            uint32_t* hr = W.take(dB + 1);
            int64_t nh = 0, nhr = 0;
            if ((st = divrem_impl(b, dB + 1, g, n_g, p, h, dB + 1, &nh, hr, dB + 1, &nhr, hs, nullptr))) return st;
            if (nhr != 0) return fail(PM_EDEVICE, "extended gcd: g does not divide b");
            uint32_t* sq = W.take(ls);
            uint32_t* sc = W.take(dB + 1);
            int64_t nsq = 0, nsc = 0;
            if ((st = divrem_impl(s_res, ls, h, nh, p, sq, ls, &nsq, sc, dB + 1, &nsc, hs, nullptr))) return st;
            sf = sc;
            nsf = nsc;
        }
        const uint32_t* w = g;
        int64_t nw = n_g;
        if (nsf > 0) {
            if (dA < 0) return fail(PM_EDEVICE, "extended gcd: non-zero cofactor of a = 0");
            const int64_t nprod = nsf + dA;
            uint32_t* prod = W.take(nprod);
            if ((st = mul_enqueue(sf, nsf, a, dA + 1, F, prod, nullptr, nullptr, hs))) return st;
            nw = nprod > n_g ? nprod : n_g;
            uint32_t* wd = W.take(nw);
            HIP_TRY(pm::sub_launch(g, n_g, prod, nprod, nw, wd, p, hs), "sub launch");
            w = wd;
        }
        uint32_t* tq = W.take(nw);
        uint32_t* tr = W.take(dB + 1);
        int64_t ntr = 0;
        if ((st = divrem_impl(w, nw, b, dB + 1, p, tq, nw, &ntf, tr, dB + 1, &ntr, hs, nullptr))) return st;
        if (ntr != 0) return fail(PM_EDEVICE, "extended gcd: g - s a is not a multiple of b");
        tf = tq;
    }
    if (nsf > s_cap) return fail(PM_EINVAL, "s_cap %lld < %lld", (long long)s_cap, (long long)nsf);
    if (ntf > t_cap) return fail(PM_EINVAL, "t_cap %lld < %lld", (long long)t_cap, (long long)ntf);
    if (nsf > 0) HIP_TRY(hipMemcpyAsync(s_out, sf, (size_t)nsf * 4, hipMemcpyDeviceToDevice, hs), "copy s");
    if (ntf > 0) HIP_TRY(hipMemcpyAsync(t_out, tf, (size_t)ntf * 4, hipMemcpyDeviceToDevice, hs), "copy t");
    HIP_TRY(hipStreamSynchronize(hs), "hipStreamSynchronize");
    *ng = n_g;
    *ns = nsf;
    *nt = ntf;
    return PM_OK;
    PM_API_END
}

pm_status poly_divrem_modp_async(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p,
                                 uint32_t* q, int64_t q_cap, int64_t* d_nq, uint32_t* r, int64_t r_cap,
                                 int64_t* d_nr, int32_t* d_status, void* stream) {
    PM_API_BEGIN
    if (bad_len(a, na) || bad_len(b, nb)) return fail(PM_EINVAL, "null input or negative length");
    if (q_cap < 0 || r_cap < 0 || (q_cap > 0 && !q) || (r_cap > 0 && !r))
        return fail(PM_EINVAL, "bad output buffer");
    if (nb == 0) return fail(PM_EDIVZERO, "division by the zero polynomial");
    // the launch shapes come from the given lengths: with b[nb - 1] != 0
    // (checked on the device) the quotient has at most na - nb + 1 terms and
    // the remainder at most min(na, nb - 1)
    const int64_t mu_plan = na - nb + 1 > 0 ? na - nb + 1 : 0;
    const int64_t r_need = na < nb - 1 ? na : nb - 1;
    if (q_cap < mu_plan) return fail(PM_EINVAL, "q_cap %lld < na - nb + 1", (long long)q_cap);
    if (r_cap < r_need) return fail(PM_EINVAL, "r_cap %lld < min(na, nb - 1)", (long long)r_cap);
    if (check_aliasing({{q, q_cap}, {r, r_cap}}, {{a, na}, {b, nb}})) return PM_EINVAL;
    pm::Field F;
    pm_status st = field_for(p, &F);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nq_prod = mu_plan < nb - 1 ? mu_plan : nb - 1;
    int64_t words = pm::divrem_head_words(na);
    if (mu_plan > 0) words = std::max(words, remainder_scratch_words(nq_prod, nb - 1));
    Pool* P = nullptr;
    if ((st = pool_get(s, words, &P))) return st;
    pm::CallInfo* info = P->d_info;
    const pm_params pp = params_now();
    HIP_TRY(pm::divrem_head_launch(a, na, b, nb, F, q, q_cap, r_cap, P->words, info, pp.div_s > 0 ? pp.div_s : 64,
                                   num_cus(), s),
            "divrem head launch");
    HIP_TRY(pm::divrem_async_fix_launch(q, mu_plan, b, nb, info, s), "quotient fix launch");
    if (mu_plan == 0) {
        // na < nb: deg a < deg b for every normalised b, so r = a
        if (na > 0) HIP_TRY(hipMemcpyAsync(r, a, (size_t)na * 4, hipMemcpyDeviceToDevice, s), "copy r");
        HIP_TRY(pm::trim_launch(r, na, info, s), "trim launch");
    } else {
        // stream order: the product's scratch may reuse the head's (same buffer)
        Pool* P2 = nullptr;
        if (nq_prod > 0 && (st = remainder_enqueue(a, b, q, nq_prod, nb - 1, F, r, s, &P2))) return st;
        HIP_TRY(pm::trim_launch(r, nb - 1, info, s), "trim launch");
    }
    HIP_TRY(pm::info_export_launch(info, d_nq, d_nr, d_status, s), "export launch");
    return PM_OK;
    PM_API_END
}

pm_status poly_gcd_modp_async(const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t p, uint32_t* g,
                              int64_t g_cap, int64_t* d_ng, int32_t* d_status, void* stream) {
    PM_API_BEGIN
    if (bad_len(a, na) || bad_len(b, nb)) return fail(PM_EINVAL, "null input or negative length");
    if (g_cap < 0 || (g_cap > 0 && !g)) return fail(PM_EINVAL, "bad output buffer");
    if (check_aliasing({{g, g_cap}}, {{a, na}, {b, nb}})) return PM_EINVAL;
    pm::Field F;
    pm_status st = field_for(p, &F);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = na > nb ? na : nb;
    const pm::GcdPlan plan = pm::gcd_default_plan(n > 0 ? n : 1, num_cus(), params_now().gcd_s);
    Pool* P = nullptr;
    if ((st = pool_get(s, pm::gcd_scratch_words(n, plan), &P))) return st;
    HIP_TRY(pm::gcd_launch(a, na, b, nb, F, g, g_cap, P->words, P->d_info, plan, s), "gcd launch");
    HIP_TRY(pm::info_export_launch(P->d_info, d_ng, nullptr, d_status, s), "export launch");
    return PM_OK;
    PM_API_END
}

pm_status pm_workspace_size(int32_t op, int64_t na, int64_t nb, int64_t* words) {
    PM_API_BEGIN
    if (!words || na < 0 || nb < 0) return fail(PM_EINVAL, "null words or negative length");
    int64_t w = 0;
    if (op == PM_OP_MUL) {
        const uint32_t *x = nullptr, *y = nullptr;
        int64_t nx = na, ny = nb;
        order_operands(x, nx, y, ny);
        pm::MxGeom g;
        if (nx > 0 && ny > 0)
            w = mfma_plan(nx, ny, -1, &g) ? pm::mulx_scratch_words(g) : pm::mul_scratch_words(nx, ny, mul_plan(nx, ny));
    } else if (op == PM_OP_DIVREM) {
        w = pm::divrem_head_words(na);
        const int64_t mu_plan = na - nb + 1;
        if (nb > 1 && mu_plan > 0) w = std::max(w, remainder_scratch_words(std::min(mu_plan, nb - 1), nb - 1));
    } else if (op == PM_OP_GCD) {
        const int64_t n = na > nb ? na : nb;
        w = pm::gcd_scratch_words(n, pm::gcd_default_plan(n > 0 ? n : 1, num_cus(), params_now().gcd_s));
    } else {
        return fail(PM_EINVAL, "unknown operation %d", op);
    }
    *words = INFO_WORDS + w;
    return PM_OK;
    PM_API_END
}

pm_status pm_mul_plan(int64_t na, int64_t nb, pm_mul_plan_info* out) {
    PM_API_BEGIN
    if (!out || na < 0 || nb < 0) return fail(PM_EINVAL, "null out or negative length");
    *out = pm_mul_plan_info{0, 0, 0, 0, 0, 0};
    const uint32_t *x = nullptr, *y = nullptr;
    int64_t nx = na, ny = nb;
    order_operands(x, nx, y, ny);
    if (nx <= 0 || ny <= 0) return PM_OK;
    pm::MxGeom g;
    if (mfma_plan(nx, ny, -1, &g)) {
        out->engine = PM_MUL_MFMA;
        out->s = 4096;
        out->scratch_words = pm::mulx_scratch_words(g);
        out->work_groups = g.G;
        out->max_share_groups = g.maxgrp;
        return PM_OK;
    }
    const pm::MulPlan plan = mul_plan(nx, ny);
    out->engine = PM_MUL_VALU;
    out->r = plan.r;
    out->s = plan.kc;
    out->scratch_words = pm::mul_scratch_words(nx, ny, plan);
    return PM_OK;
    PM_API_END
}

pm_status pm_autotune_load(const char* path) {
    PM_API_BEGIN
    if (!path) return fail(PM_EINVAL, "null path");
    FILE* fh = fopen(path, "r");
    if (!fh) return fail(PM_EINVAL, "cannot open %s", path);
    pm_params q = params_now();
    char line[256];
    int lineno = 0;
    pm_status st = PM_OK;
    while (st == PM_OK && fgets(line, sizeof line, fh)) {
        lineno++;
        char* c = strchr(line, '#');
        if (c) *c = 0;
        for (char* t = line; *t; t++)
            if (*t == '=' || *t == ':' || *t == ',') *t = ' ';
        char key[64];
        long long v = 0;
        const int got = sscanf(line, "%63s %lld", key, &v);
        if (got <= 0) continue;  // blank or comment
        if (got != 2) { st = fail(PM_EINVAL, "%s:%d: expected a name and an integer", path, lineno); break; }
        if (v < INT32_MIN || v > INT32_MAX) { st = fail(PM_EINVAL, "%s:%d: value out of range", path, lineno); break; }
        if (!strcmp(key, "mul_s")) q.mul_s = (int32_t)v;
        else if (!strcmp(key, "mul_r")) q.mul_r = (int32_t)v;
        else if (!strcmp(key, "div_s")) q.div_s = (int32_t)v;
        else if (!strcmp(key, "gcd_s")) q.gcd_s = (int32_t)v;
        else if (!strcmp(key, "mul_engine")) q.mul_engine = (int32_t)v;
        else st = fail(PM_EINVAL, "%s:%d: unknown parameter %s", path, lineno, key);
    }
    fclose(fh);
    if (st) return st;
    return pm_set_params(&q);  // checks every value; nothing changes on an error
    PM_API_END
}

pm_status pm_radix_sort_u32(const uint32_t* keys, const uint32_t* vals, int64_t n, int32_t key_bits, int32_t s,
                            uint32_t* keys_out, uint32_t* vals_out, void* stream) {
    PM_API_BEGIN
    if (n < 0 || n > (int64_t)0xFFFFFFFFLL) return fail(PM_EINVAL, "n must be in [0, 2^32 - 1]");
    if (key_bits < 1 || key_bits > 32) return fail(PM_EINVAL, "key_bits must be in [1, 32]");
    if (s < 0 || s > 10) return fail(PM_EINVAL, "s must be in [0, 10]");
    if (n == 0) return PM_OK;
    if (!keys || !keys_out) return fail(PM_EINVAL, "null keys");
    if (vals && !vals_out) return fail(PM_EINVAL, "vals given without vals_out");
    auto overlap = [n](const uint32_t* x, const uint32_t* y) { return x && y && x < y + n && y < x + n; };
    if (overlap(keys, keys_out) || overlap(vals, vals_out) || overlap(keys, vals_out) || overlap(vals, keys_out) ||
        overlap(keys_out, vals_out))
        return fail(PM_EINVAL, "outputs overlap the inputs or each other");
    const int sd = s > 0 ? s : 8;
    hipStream_t hs = (hipStream_t)stream;
    Pool* P = nullptr;
    pm_status st = pool_get(hs, pm::radix_scratch_words(n, sd, vals != nullptr), &P);
    if (st) return st;
    HIP_TRY(pm::radix_sort_launch(keys, vals, n, key_bits, sd, keys_out, vals ? vals_out : nullptr, P->words, hs),
            "radix sort launch");
    return PM_OK;
    PM_API_END
}

}  // extern "C"
