// serve.cpp -- continuous-batching gcd server (pm_server_* in polymodp.h).
//
// A persistent worker kernel (one 1024-thread block per CU) takes requests
// one at a time from a queue the host publishes in pinned memory: block b
// claims sequence number h (an atomic on a device counter), reads the slot
// of request h, runs the whole remainder sequence with both polynomials in
// its LDS, writes the monic gcd and the result into the slot's pinned
// buffers and raises the slot's `done` flag (system-scope release), then
// claims the next one. Requests therefore join and leave the GPU one by one:
// nothing waits for a batch or a launch to finish.
//
// The host side (pm_server_submit and pm_server_poll, called by one thread):
//  1. poll harvests finished slots (done flag, acquire) and frees them;
//  2. submit and poll admit queued requests in FIFO order (the requests of
//     one batch call longest first) while a slot and room in the
//     resident-input budget are free: the inputs go into the slot's pinned
//     staging buffer (mapped into the device's address space), and the
//     request is published at once by raising the shared tail (release);
//     the claiming block reads the inputs once, past the caches, straight
//     into its LDS (copies queued on a stream would wait behind the
//     worker's own blocks, which hold the CUs);
//  3. makes sure the worker runs (it stops by itself after an idle period).
// All device and pinned memory is allocated by pm_server_create.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "../../include/polymodp.h"
#include "internal.hpp"

namespace pm {
pm_status server_field(uint32_t p, Field* out);  // capi.cpp
pm_status server_fail(pm_status st, const char* msg);
int server_num_cus();
}  // namespace pm

namespace {

// Sequence numbers index the order ring modulo ORDER_CAP. A block reads
// order[h] right after claiming h; the host can only overwrite that entry
// after publishing h + ORDER_CAP, which needs ORDER_CAP - max_inflight
// further requests to finish in between, so the entry is always intact.
constexpr uint32_t ORDER_CAP = 1u << 16;
constexpr double IDLE_SECONDS = 0.5;

struct Pending {
    uint64_t ticket;
    uint64_t tag;
    std::vector<uint32_t> ab;  // a then b
    int64_t na, nb;
    uint32_t* g_user;
    int64_t g_cap;
    pm::Field F;
    double t_submit;
};

struct Slot {
    bool busy = false;
    uint64_t ticket = 0, tag = 0;
    int64_t arena_off = 0, arena_len = 0;
    uint32_t* g_user = nullptr;
    int64_t g_cap = 0;
    double t_submit = 0, t_start = 0;
};

// First-fit allocator over [0, cap) words with coalescing (64-word grain):
// the budget of input words resident for admitted requests.
class Arena {
public:
    explicit Arena(int64_t cap) { free_[0] = cap & ~INT64_C(63); }
    static int64_t grain(int64_t n) { return ((n > 0 ? n : 1) + 63) & ~INT64_C(63); }
    bool alloc(int64_t n, int64_t* off) {
        n = grain(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const int64_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest > 0) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(int64_t off, int64_t n) {
        n = grain(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<int64_t, int64_t> free_;
};

}  // namespace

struct pm_server {
    pm_server_opts opt{};
    int device = 0;
    int64_t cap = 0;  // words per input polynomial and per output of a slot
    hipStream_t worker_stream = nullptr;
    bool worker_launched = false;
    uint32_t* d_head = nullptr;
    Arena* arena = nullptr;
    pm::GcdJob* h_jobs = nullptr;        // pinned, one per slot
    pm::GcdResult* h_results = nullptr;  // pinned, one per slot
    uint32_t* h_in = nullptr;            // pinned, 2*cap words per slot
    uint32_t* h_g = nullptr;             // pinned, cap words per slot
    uint32_t* h_order = nullptr;         // pinned, ORDER_CAP slot ids
    uint32_t* h_ctl = nullptr;           // pinned: [0] tail, [1] stop
    uint32_t tail = 0;
    std::vector<Slot> slots;
    std::vector<int> free_slots;
    std::deque<Pending> queue;
    uint64_t next_ticket = 1;
    int64_t inflight = 0;
    std::chrono::steady_clock::time_point t0;
    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void destroy(pm_server* S) {
    if (!S) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(S->device);
    if (S->h_ctl) __atomic_store_n(&S->h_ctl[1], 1u, __ATOMIC_RELEASE);  // stop the worker
    if (S->worker_stream) (void)hipStreamSynchronize(S->worker_stream);
    if (S->worker_stream) (void)hipStreamDestroy(S->worker_stream);
    if (S->d_head) (void)hipFree(S->d_head);
    for (void* p : {(void*)S->h_jobs, (void*)S->h_results, (void*)S->h_in, (void*)S->h_g, (void*)S->h_order,
                    (void*)S->h_ctl})
        if (p) (void)hipHostFree(p);
    delete S->arena;
    (void)hipSetDevice(cur);
    delete S;
}

pm_status ensure_worker(pm_server* S) {
    if (S->worker_launched && hipStreamQuery(S->worker_stream) == hipErrorNotReady) return PM_OK;
    const int blocks = pm::server_num_cus();
    if (pm::gcd_worker_launch(S->h_jobs, S->h_order, ORDER_CAP, &S->h_ctl[0], &S->h_ctl[1], S->d_head, S->opt.s,
                              blocks, IDLE_SECONDS, S->worker_stream) != hipSuccess)
        return pm::server_fail(PM_EDEVICE, "worker launch");
    S->worker_launched = true;
    return PM_OK;
}

// Puts one request into slot si at arena offset off: inputs into the slot's
// pinned staging, the job record, and the next entry of the order ring
// (published by the caller with one store of the tail).
void place(pm_server* S, int si, int64_t off, uint64_t ticket, uint64_t tag, const uint32_t* a, int64_t na,
           const uint32_t* b, int64_t nb, uint32_t* g_user, int64_t g_cap, const pm::Field& F, double t_submit,
           double t_start) {
    Slot& sl = S->slots[si];
    sl.busy = true;
    sl.ticket = ticket;
    sl.tag = tag;
    sl.arena_off = off;
    sl.arena_len = na + nb;
    sl.g_user = g_user;
    sl.g_cap = g_cap;
    sl.t_submit = t_submit;
    sl.t_start = t_start;
    std::memset(&S->h_results[si], 0, sizeof(pm::GcdResult));
    uint32_t* stage = S->h_in + (int64_t)si * 2 * S->cap;
    if (na) std::memcpy(stage, a, (size_t)na * 4);
    if (nb) std::memcpy(stage + na, b, (size_t)nb * 4);
    S->h_jobs[si] = pm::GcdJob{stage, stage + na, na, nb, S->h_g + (int64_t)si * S->cap, S->cap,
                               &S->h_results[si], F, 1, 0};
    S->h_order[S->tail & (ORDER_CAP - 1)] = (uint32_t)si;
    S->tail++;
    S->inflight++;
}

// Admits queued requests in FIFO order while a slot and room in the budget
// are free and publishes them. With `check`, also makes sure the worker runs
// (a query of its stream); without it, only a worker never launched is
// started, and the next poll relaunches one that has left.
pm_status admit(pm_server* S, bool check) {
    bool published = __atomic_load_n(&S->h_ctl[0], __ATOMIC_RELAXED) != S->tail;  // direct placements
    const double t = S->now_ms();
    while (!S->queue.empty() && !S->free_slots.empty()) {
        Pending& P = S->queue.front();
        const int64_t len = P.na + P.nb;
        int64_t off = 0;
        if (!S->arena->alloc(len, &off)) break;  // FIFO: wait for room, no overtaking
        const int si = S->free_slots.back();
        S->free_slots.pop_back();
        place(S, si, off, P.ticket, P.tag, P.ab.data(), P.na, P.ab.data() + P.na, P.nb, P.g_user, P.g_cap, P.F,
              P.t_submit, t);
        S->queue.pop_front();
        published = true;
    }
    if (published) __atomic_store_n(&S->h_ctl[0], S->tail, __ATOMIC_RELEASE);
    // (re)launch the worker whenever published work may be waiting and the
    // previous worker has left (it leaves after an idle period)
    if (S->inflight > 0 && (check || !S->worker_launched)) return ensure_worker(S);
    return PM_OK;
}

}  // namespace

extern "C" {

pm_status pm_server_create(const pm_server_opts* opts, pm_server** out) {
    if (!out) return pm::server_fail(PM_EINVAL, "null output");
    pm_server* S = new pm_server();
    if (opts) S->opt = *opts;
    if (S->opt.max_inflight <= 0) S->opt.max_inflight = 1024;
    if (S->opt.max_inflight > (int32_t)(ORDER_CAP / 4)) S->opt.max_inflight = (int32_t)(ORDER_CAP / 4);
    if (S->opt.arena_words <= 0) S->opt.arena_words = INT64_C(32) << 20;
    if (S->opt.s < 0 || S->opt.s > 256) {
        delete S;
        return pm::server_fail(PM_EINVAL, "s must be in [0, 256]");
    }
    if (S->opt.s == 0) S->opt.s = 128;
    (void)hipGetDevice(&S->device);
    S->t0 = std::chrono::steady_clock::now();
    S->cap = pm::gcd_batch_cap(1);
    const size_t M = (size_t)S->opt.max_inflight;
    hipError_t e = hipStreamCreateWithFlags(&S->worker_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void**)&S->d_head, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(S->d_head, 0, sizeof(uint32_t));
    if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_jobs, M * sizeof(pm::GcdJob), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_results, M * sizeof(pm::GcdResult), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_in, M * 2 * S->cap * sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_g, M * S->cap * sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_order, ORDER_CAP * sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_ctl, 2 * sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        destroy(S);
        return pm::server_fail(PM_ENOMEM, "cannot allocate the server's buffers");
    }
    std::memset(S->h_results, 0, M * sizeof(pm::GcdResult));
    std::memset(S->h_order, 0, ORDER_CAP * sizeof(uint32_t));
    S->h_ctl[0] = 0;
    S->h_ctl[1] = 0;
    S->arena = new Arena(S->opt.arena_words);
    S->slots.resize(M);
    for (int i = (int)M - 1; i >= 0; i--) S->free_slots.push_back(i);
    *out = S;
    return PM_OK;
}

void pm_server_destroy(pm_server* S) { destroy(S); }

}  // extern "C"

namespace {

pm_status enqueue(pm_server* S, const pm_gcd_request* r, uint64_t* ticket) {
    if (!r) return pm::server_fail(PM_EINVAL, "null request");
    if (r->na < 0 || r->nb < 0 || (r->na > 0 && !r->a) || (r->nb > 0 && !r->b) || r->g_cap < 0 ||
        (r->g_cap > 0 && !r->g))
        return pm::server_fail(PM_EINVAL, "bad request buffers");
    const int64_t n = r->na > r->nb ? r->na : r->nb;
    if (n > S->cap) return pm::server_fail(PM_EINVAL, "request exceeds PM_GCD_BATCH_MAX terms");
    if (Arena::grain(r->na + r->nb) > S->opt.arena_words)
        return pm::server_fail(PM_ENOMEM, "request larger than the whole resident-input budget");
    pm::Field F;
    pm_status st = pm::server_field(r->p, &F);
    if (st) return st;
    if ((r->p & 1u) == 0) return pm::server_fail(PM_EMODULUS, "p = 2 is not supported by the gcd");
    int64_t off = 0;
    if (S->queue.empty() && !S->free_slots.empty() && S->arena->alloc(r->na + r->nb, &off)) {
        // nothing waits ahead of it: straight from the caller's arrays into a
        // slot (published by the caller's next admission pass)
        const int si = S->free_slots.back();
        S->free_slots.pop_back();
        const uint64_t t = S->next_ticket++;
        const double now = S->now_ms();
        place(S, si, off, t, r->tag, r->a, r->na, r->b, r->nb, r->g, r->g_cap, F, now, now);
        if (ticket) *ticket = t;
        return PM_OK;
    }
    Pending P;
    P.ticket = S->next_ticket++;
    P.tag = r->tag;
    P.na = r->na;
    P.nb = r->nb;
    P.ab.resize((size_t)(r->na + r->nb));
    if (r->na) std::memcpy(P.ab.data(), r->a, (size_t)r->na * 4);
    if (r->nb) std::memcpy(P.ab.data() + r->na, r->b, (size_t)r->nb * 4);
    P.g_user = r->g;
    P.g_cap = r->g_cap;
    P.F = F;
    P.t_submit = S->now_ms();
    if (ticket) *ticket = P.ticket;
    S->queue.push_back(std::move(P));
    return PM_OK;
}

}  // namespace

extern "C" {

pm_status pm_server_submit(pm_server* S, const pm_gcd_request* r, uint64_t* ticket) {
    if (!S || !r) return pm::server_fail(PM_EINVAL, "null argument");
    pm_status st = enqueue(S, r, ticket);
    if (st) return st;
    return admit(S, false);  // on the GPU at once when a slot is free
}

pm_status pm_server_submit_batch(pm_server* S, const pm_gcd_request* reqs, int32_t count, uint64_t* tickets) {
    if (!S || count < 0 || (count > 0 && !reqs)) return pm::server_fail(PM_EINVAL, "null argument");
    // every request is checked before any is queued: a bad one queues none
    for (int32_t i = 0; i < count; i++) {
        const pm_gcd_request* r = &reqs[i];
        const int64_t n = r->na > r->nb ? r->na : r->nb;
        if (r->na < 0 || r->nb < 0 || (r->na > 0 && !r->a) || (r->nb > 0 && !r->b) || r->g_cap < 0 ||
            (r->g_cap > 0 && !r->g) || n > S->cap || Arena::grain(r->na + r->nb) > S->opt.arena_words)
            return pm::server_fail(PM_EINVAL, "bad request in the batch");
        pm::Field F;
        pm_status st = pm::server_field(r->p, &F);
        if (st) return st;
        if ((r->p & 1u) == 0) return pm::server_fail(PM_EMODULUS, "p = 2 is not supported by the gcd");
    }
    // The requests of one call arrive together, so they may start in any
    // order: longest first (work ~ na * nb), which keeps the largest
    // remainder sequences, each bound by its own step chain on one CU, from
    // starting last and setting the span.
    std::vector<int32_t> order((size_t)count);
    for (int32_t i = 0; i < count; i++) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [reqs](int32_t x, int32_t y) {
        return (double)reqs[x].na * (double)reqs[x].nb > (double)reqs[y].na * (double)reqs[y].nb;
    });
    for (int32_t k = 0; k < count; k++) {
        const int32_t i = order[(size_t)k];
        pm_status st = enqueue(S, &reqs[i], tickets ? &tickets[i] : nullptr);
        if (st) return st;
        if ((k & 15) == 15) {  // the first requests start while the rest are copied
            st = admit(S, false);
            if (st) return st;
        }
    }
    return admit(S, false);
}

int64_t pm_server_pending(pm_server* S) { return S ? (int64_t)S->queue.size() + S->inflight : 0; }

pm_status pm_server_poll(pm_server* S, pm_completion* out, int32_t max, int32_t* n) {
    if (!S || !n || (max > 0 && !out)) return pm::server_fail(PM_EINVAL, "null argument");
    *n = 0;
    // 1. harvest
    for (int si = 0; si < S->opt.max_inflight && *n < max; si++) {
        Slot& sl = S->slots[si];
        if (!sl.busy) continue;
        pm::GcdResult* R = &S->h_results[si];
        if (__atomic_load_n(&R->done, __ATOMIC_ACQUIRE) == 0) continue;
        pm_completion& c = out[(*n)++];
        c.ticket = sl.ticket;
        c.tag = sl.tag;
        c.status = R->status;
        c.reserved = 0;
        c.ng = R->status == 0 ? R->ng : 0;
        c.steps = R->steps;
        c.updates = R->updates;
        c.t_submit_ms = sl.t_submit;
        c.t_start_ms = sl.t_start;
        c.t_done_ms = S->now_ms();
        if (c.status == 0) {
            if (c.ng > sl.g_cap) {
                c.status = PM_EINVAL;
                c.ng = 0;
            } else if (c.ng > 0) {
                std::memcpy(sl.g_user, S->h_g + (int64_t)si * S->cap, (size_t)c.ng * 4);
            }
        }
        S->arena->release(sl.arena_off, sl.arena_len);
        S->inflight--;
        sl.busy = false;
        S->free_slots.push_back(si);
    }
    return admit(S, true);
}

}  // extern "C"
