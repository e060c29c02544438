// serve.cpp -- continuous-batching server of gcd and division requests
// (pm_server_* in polymodp.h).
//
// Two persistent worker kernels take requests one at a time from rings the
// host publishes in pinned memory: the 1024-thread worker (one block per
// CU, operands up to 17408 terms) and the 256-thread worker (several blocks
// per CU, operands up to 4096 terms). A block claims sequence number h of
// its ring (an atomic on a device counter), reads the job record of h, runs
// the whole remainder sequence (or the division) with both operands in its
// LDS, writes the results into the request's pinned output buffers and
// raises the request's `done` flag (system-scope release), then claims the
// next one. Requests therefore join and leave the GPU one by one: nothing
// waits for a batch or a launch to finish.
//
// The host side (pm_server_submit and pm_server_poll, called by one thread):
//  1. poll harvests finished slots (done flag, acquire) and frees them;
//  2. submit and poll admit queued requests in FIFO order (the requests of
//     one batch call longest first) while a slot, room in the device input
//     arena and room in the pinned output arena are free: the inputs are
//     copied into the arena's pinned mirror, and one copy per contiguous
//     run of the admission pass moves them to device memory on an SDMA
//     engine, through ROCr, with one completion signal per pass. (The HIP
//     runtime's hipMemcpyAsync does such copies with blit kernels, which
//     need a CU and so wait behind the persistent workers: measured, the
//     saturated rate fell from about 60 K to 4 K requests/s.) Without an
//     SDMA engine, or with staging = 2, the workers read the pinned mirror
//     itself instead, and a pass is published at once;
//  3. the requests of a pass are published (their ring entries written and
//     the ring's tail raised, release) once its copies have completed; the
//     claiming block reads the inputs past the caches (the copy engine
//     wrote them after the worker started);
//  4. makes sure the workers run (they stop by themselves after an idle
//     period): the 1024-thread worker is launched first and waited for
//     until all its blocks have started, so that the 256-thread worker,
//     launched next, takes only the CUs it leaves.
// All device and pinned memory is allocated by pm_server_create.
#include <hip/hip_runtime.h>
#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/polymodp.h"
#include "internal.hpp"

namespace pm {
pm_status server_field(uint32_t p, Field* out);  // capi.cpp
pm_status server_fail(pm_status st, const char* msg);
int server_num_cus();
}  // namespace pm

namespace {

// Sequence numbers index a ring modulo ORDER_CAP. A block reads its ring
// entry right after claiming it; the host can only overwrite that entry
// after publishing ORDER_CAP more requests on the ring, which needs
// ORDER_CAP - max_inflight of them to finish in between, so it is intact.
constexpr uint32_t ORDER_CAP = 1u << 16;
constexpr double IDLE_SECONDS = 0.5;
constexpr int NKIND = 2;  // worker shapes: 0 = 256 threads, 1 = 1024 threads
constexpr int SIGNALS = 64;

struct Pending {
    uint64_t ticket;
    uint64_t tag;
    int32_t op;
    std::vector<uint32_t> ab;  // a then b
    int64_t na, nb;
    uint32_t *g_user, *r_user;
    int64_t g_cap, r_cap;
    pm::Field F;
    double t_submit;
};

struct Slot {
    bool busy = false;
    int kind = 1;
    int32_t op = pm::JOB_GCD;
    uint64_t ticket = 0, tag = 0;
    int64_t in_off = 0, in_len = 0, out_off = 0, out_len = 0, r_off = 0;
    bool published = false;
    uint32_t *g_user = nullptr, *r_user = nullptr;
    int64_t g_cap = 0, r_cap = 0;
    double t_submit = 0, t_start = 0;
};

// First-fit allocator over [0, cap) words with coalescing (64-word grain).
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

// A host copy of one request's inputs into the pinned mirror.
struct CopyTask {
    uint32_t* dst;
    const uint32_t* a;
    int64_t na;
    const uint32_t* b;
    int64_t nb;
};

// Host threads that share the copies of an admission pass: the inputs of a
// batch of requests are tens of megabytes, and one thread's memcpy would
// bound the rate at which a saturated server can start them.
class CopyPool {
public:
    explicit CopyPool(int n) {
        for (int i = 0; i < n; i++) th_.emplace_back([this] { loop(); });
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    // Runs every task (the calling thread takes part) and returns when all
    // are done and no pool thread still holds the task list.
    void run(const std::vector<CopyTask>& tasks) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            tasks_ = &tasks;
            next_.store(0);
            left_ = tasks.size();
            gen_++;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [this] { return left_ == 0 && active_ == 0; });
        tasks_ = nullptr;
    }

private:
    static void copy(const CopyTask& t) {
        if (t.na) std::memcpy(t.dst, t.a, (size_t)t.na * 4);
        if (t.nb) std::memcpy(t.dst + t.na, t.b, (size_t)t.nb * 4);
    }
    void work() {
        const std::vector<CopyTask>* t;
        {
            std::lock_guard<std::mutex> lk(mu_);
            t = tasks_;
            if (!t) return;
            active_++;
        }
        size_t mine = 0, i;
        while ((i = next_.fetch_add(1)) < t->size()) {
            copy((*t)[i]);
            mine++;
        }
        std::lock_guard<std::mutex> lk(mu_);
        left_ -= mine;
        active_--;
        if (left_ == 0 && active_ == 0) done_.notify_all();
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
            }
            work();
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_;
    const std::vector<CopyTask>* tasks_ = nullptr;
    std::atomic<size_t> next_{0};
    size_t left_ = 0;
    int active_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

// One worker shape: its kernel's stream, ring and claim counter.
struct Worker {
    int blocks = 0;
    int64_t cap = 0;
    hipStream_t stream = nullptr;
    bool launched = false;
    uint32_t* d_head = nullptr;   // device: next sequence number to claim
    uint32_t* h_order = nullptr;  // pinned: ORDER_CAP slot ids
    uint32_t tail = 0;            // host copy of the published tail
    int64_t inflight = 0;
};

// The requests of one admission pass, published when their copy is done
// (the signal reaches 0; a null signal: nothing to wait for).
struct Pass {
    hsa_signal_t done;
    std::vector<int> slots;
};

// The copy engine: the SDMA engine of the server's GPU for host-to-device
// copies, through ROCr (the CUs stay with the workers).
struct Copier {
    bool ok = false;
    bool inited = false;
    hsa_agent_t gpu{}, cpu{};
    hsa_amd_sdma_engine_id_t engines[16];  // the available engines, taken in turn
    int n_engines = 0;
};

struct AgentSearch {
    uint32_t bdf, domain;
    bool have_gpu = false, have_cpu = false;
    hsa_agent_t gpu{}, cpu{};
};

hsa_status_t find_agents(hsa_agent_t agent, void* data) {
    AgentSearch* A = (AgentSearch*)data;
    hsa_device_type_t type;
    if (hsa_agent_get_info(agent, HSA_AGENT_INFO_DEVICE, &type) != HSA_STATUS_SUCCESS) return HSA_STATUS_SUCCESS;
    if (type == HSA_DEVICE_TYPE_CPU && !A->have_cpu) {
        A->cpu = agent;
        A->have_cpu = true;
    } else if (type == HSA_DEVICE_TYPE_GPU && !A->have_gpu) {
        uint32_t bdf = 0, dom = 0;
        if (hsa_agent_get_info(agent, (hsa_agent_info_t)HSA_AMD_AGENT_INFO_BDFID, &bdf) == HSA_STATUS_SUCCESS &&
            hsa_agent_get_info(agent, (hsa_agent_info_t)HSA_AMD_AGENT_INFO_DOMAIN, &dom) == HSA_STATUS_SUCCESS &&
            bdf == A->bdf && dom == A->domain) {
            A->gpu = agent;
            A->have_gpu = true;
        }
    }
    return HSA_STATUS_SUCCESS;
}

// The GPU agent of HIP device `dev` (matched by PCI domain and bus, device,
// function) and a host agent, and an SDMA engine that copies host to it.
bool copier_init(Copier* C, int dev) {
    int bus = 0, slot = 0, dom = 0;
    if (hipDeviceGetAttribute(&bus, hipDeviceAttributePciBusId, dev) != hipSuccess ||
        hipDeviceGetAttribute(&slot, hipDeviceAttributePciDeviceId, dev) != hipSuccess ||
        hipDeviceGetAttribute(&dom, hipDeviceAttributePciDomainID, dev) != hipSuccess)
        return false;
    if (hsa_init() != HSA_STATUS_SUCCESS) return false;
    C->inited = true;
    AgentSearch A;
    A.bdf = ((uint32_t)bus << 8) | ((uint32_t)slot << 3);
    A.domain = (uint32_t)dom;
    if (hsa_iterate_agents(find_agents, &A) != HSA_STATUS_SUCCESS || !A.have_gpu || !A.have_cpu) return false;
    uint32_t mask = 0;
    if (hsa_amd_memory_copy_engine_status(A.gpu, A.cpu, &mask) != HSA_STATUS_SUCCESS || mask == 0) return false;
    C->gpu = A.gpu;
    C->cpu = A.cpu;
    // up to four engines, taken in turn by the admission passes
    for (int i = 0; i < 16 && C->n_engines < 4; i++)
        if (mask & (1u << i)) C->engines[C->n_engines++] = (hsa_amd_sdma_engine_id_t)(1u << i);
    C->ok = C->n_engines > 0;
    return true;
}

// Pinned control words: the published tail of each ring, the stop flag and
// each worker's count of started blocks.
enum { CTL_TAIL0 = 0, CTL_TAIL1 = 1, CTL_STOP = 2, CTL_STARTED0 = 3, CTL_STARTED1 = 4, CTL_WORDS = 8 };

}  // namespace

struct pm_server {
    pm_server_opts opt{};
    int device = 0;
    Worker w[NKIND];
    Copier copier;
    bool device_inputs = false;          // inputs copied to d_in (else read from h_mirror)
    uint32_t* d_in = nullptr;            // device input arena (arena_words)
    uint32_t* h_mirror = nullptr;        // pinned, the inputs as staged for the copy
    uint32_t* h_out = nullptr;           // pinned output arena (arena_words)
    Arena* in_arena = nullptr;
    Arena* out_arena = nullptr;
    pm::GcdJob* h_jobs = nullptr;        // pinned, one per slot
    pm::GcdResult* h_results = nullptr;  // pinned, one per slot
    uint32_t* h_ctl = nullptr;           // pinned control words
    std::vector<Slot> slots;
    std::vector<int> free_slots;
    std::deque<Pending> queue;
    std::deque<Pass> passes;             // copies in flight, oldest first
    std::vector<hsa_signal_t> free_signals;
    std::vector<int> staged;             // slots placed in the current pass
    std::vector<CopyTask> copies;        // their host copies, not yet made
    std::vector<std::vector<uint32_t>> holding;  // queued inputs those copies read
    int64_t copy_words = 0;
    CopyPool* pool = nullptr;            // created by the first large pass
    int next_engine = 0;                 // SDMA engines taken in turn
    std::vector<std::pair<int64_t, int64_t>> runs;  // its input ranges (offset, words)
    uint64_t next_ticket = 1;
    int64_t inflight = 0;                // admitted (staged, copied or on the GPU)
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
    if (S->h_ctl) __atomic_store_n(&S->h_ctl[CTL_STOP], 1u, __ATOMIC_RELEASE);  // stop the workers
    for (Worker& W : S->w) {
        if (W.stream) (void)hipStreamSynchronize(W.stream);
        if (W.stream) (void)hipStreamDestroy(W.stream);
        if (W.d_head) (void)hipFree(W.d_head);
        if (W.h_order) (void)hipHostFree(W.h_order);
    }
    for (Pass& P : S->passes) {
        if (!P.done.handle) continue;
        while (hsa_signal_wait_scacquire(P.done, HSA_SIGNAL_CONDITION_LT, 1, UINT64_MAX, HSA_WAIT_STATE_BLOCKED) > 0)
            ;
        (void)hsa_signal_destroy(P.done);
    }
    for (hsa_signal_t g : S->free_signals) (void)hsa_signal_destroy(g);
    if (S->copier.inited) (void)hsa_shut_down();
    if (S->d_in) (void)hipFree(S->d_in);
    for (void* p : {(void*)S->h_mirror, (void*)S->h_out, (void*)S->h_jobs, (void*)S->h_results, (void*)S->h_ctl})
        if (p) (void)hipHostFree(p);
    delete S->pool;
    delete S->in_arena;
    delete S->out_arena;
    (void)hipSetDevice(cur);
    delete S;
}

int kind_of(const pm_server* S, int64_t na, int64_t nb) {
    const int64_t n = na > nb ? na : nb;
    return (S->w[0].blocks > 0 && n <= S->w[0].cap) ? 0 : 1;
}

// Output words a request needs in the pinned output arena.
int64_t out_words(int32_t op, int64_t na, int64_t nb) { return op == pm::JOB_DIVREM ? na + nb : (na > nb ? na : nb); }

pm_status launch_worker(pm_server* S, int k) {
    Worker& W = S->w[k];
    uint32_t* started = &S->h_ctl[k == 0 ? CTL_STARTED0 : CTL_STARTED1];
    __atomic_store_n(started, 0u, __ATOMIC_RELAXED);
    const uint32_t* tail = &S->h_ctl[k == 0 ? CTL_TAIL0 : CTL_TAIL1];
    if (pm::gcd_worker_launch(k, S->h_jobs, W.h_order, ORDER_CAP, tail, &S->h_ctl[CTL_STOP], W.d_head, started,
                              S->opt.s, W.blocks, IDLE_SECONDS, W.stream) != hipSuccess)
        return pm::server_fail(PM_EDEVICE, "worker launch");
    W.launched = true;
    if (k == 1) {
        // every block of the 1024-thread worker holds its CU before the other
        // worker's blocks are placed (bounded wait: another process's work
        // may hold the GPU)
        const auto t = std::chrono::steady_clock::now();
        while (__atomic_load_n(started, __ATOMIC_ACQUIRE) < (uint32_t)W.blocks &&
               std::chrono::steady_clock::now() - t < std::chrono::seconds(2))
            ;
    }
    return PM_OK;
}

bool running(const Worker& W) { return W.launched && hipStreamQuery(W.stream) == hipErrorNotReady; }

// Makes sure the workers that have work run: the 1024-thread one first
// whenever the 256-thread one is (re)launched, so that the latter never
// spreads over CUs the former needs.
pm_status ensure_workers(pm_server* S) {
    const bool need0 = S->w[0].blocks > 0 && S->w[0].inflight > 0;
    const bool need1 = S->w[1].inflight > 0;
    const bool run0 = running(S->w[0]);
    if ((need1 || (need0 && !run0)) && !running(S->w[1])) {
        pm_status st = launch_worker(S, 1);
        if (st) return st;
    }
    if (need0 && !run0) return launch_worker(S, 0);
    return PM_OK;
}

// Writes one word of every page of a new pinned buffer, on several host
// threads. The runtime maps such memory into the process lazily: the first
// write to each page takes a page fault, and left to the admission copies
// those faults ran them at about 3.6 GB/s (28 GB/s once mapped).
void prefault(void* p, size_t bytes) {
    constexpr size_t PAGE = 4096;
    volatile char* base = (volatile char*)p;
    const size_t pages = (bytes + PAGE - 1) / PAGE;
    const unsigned hc = std::thread::hardware_concurrency();
    const size_t nt = std::min<size_t>(pages / 1024 + 1, std::min(8u, hc > 1 ? hc : 1u));
    auto touch = [=](size_t t, size_t step) {
        for (size_t i = t; i < pages; i += step) base[i * PAGE] = 0;
    };
    std::vector<std::thread> th;
    try {
        for (size_t t = 1; t < nt; t++) th.emplace_back(touch, t, nt);
    } catch (...) {
        // no more threads: the calling thread takes the pages of those
        // that did not start (no exception crosses the C interface)
        for (size_t t = th.size() + 1; t < nt; t++) touch(t, nt);
    }
    touch(0, nt);
    for (auto& x : th) x.join();
}

// Puts one request into slot si: its inputs into the pinned mirror at its
// arena offset, its job record, and the slot into the current pass.
void place(pm_server* S, int si, int64_t in_off, int64_t out_off, uint64_t ticket, uint64_t tag, int32_t op,
           const uint32_t* a, int64_t na, const uint32_t* b, int64_t nb, uint32_t* g_user, int64_t g_cap,
           uint32_t* r_user, int64_t r_cap, const pm::Field& F, double t_submit) {
    Slot& sl = S->slots[si];
    sl.busy = true;
    sl.kind = kind_of(S, na, nb);
    sl.op = op;
    sl.ticket = ticket;
    sl.tag = tag;
    sl.in_off = in_off;
    sl.in_len = na + nb;
    sl.out_off = out_off;
    sl.out_len = out_words(op, na, nb);
    sl.r_off = out_off + na;  // a division's r follows its q
    sl.published = false;
    sl.g_user = g_user;
    sl.g_cap = g_cap;
    sl.r_user = r_user;
    sl.r_cap = r_cap;
    sl.t_submit = t_submit;
    sl.t_start = 0;
    std::memset(&S->h_results[si], 0, sizeof(pm::GcdResult));
    // the caller's arrays are copied when the pass closes (submit copies
    // every input before it returns)
    S->copies.push_back(CopyTask{S->h_mirror + in_off, a, na, b, nb});
    S->copy_words += na + nb;
    const uint32_t* da = (S->device_inputs ? S->d_in : S->h_mirror) + in_off;
    uint32_t* out = S->h_out + out_off;
    // outputs: the gcd, or q then r, each within the request's own words
    const int64_t gw = op == pm::JOB_DIVREM ? na : sl.out_len;
    S->h_jobs[si] = pm::GcdJob{da, da + na, na, nb, out, std::min(g_cap, gw), &S->h_results[si], F, 1,
                               op, op == pm::JOB_DIVREM ? out + na : nullptr,
                               op == pm::JOB_DIVREM ? std::min(r_cap, nb) : 0};
    if (!S->runs.empty() && S->runs.back().first + S->runs.back().second == in_off)
        S->runs.back().second += Arena::grain(na + nb);
    else
        S->runs.push_back({in_off, Arena::grain(na + nb)});
    S->staged.push_back(si);
    S->w[sl.kind].inflight++;
    S->inflight++;
}

// Requests whose inputs could not be copied: finished at once with
// PM_EDEVICE (harvested by the next poll), never published.
void fail_slots(pm_server* S, const std::vector<int>& slots) {
    const double t = S->now_ms();
    for (int si : slots) {
        Slot& sl = S->slots[si];
        sl.t_start = t;
        sl.published = true;
        S->h_results[si].status = PM_EDEVICE;
        __atomic_store_n(&S->h_results[si].done, 1, __ATOMIC_RELEASE);
    }
}

// Publishes the passes whose copies have completed, oldest first.
void publish_ready(pm_server* S) {
    bool any[NKIND] = {false, false};
    const double t = S->now_ms();
    while (!S->passes.empty()) {
        const hsa_signal_t g = S->passes.front().done;
        hsa_signal_value_t v = 0;
        if (g.handle) {
            v = hsa_signal_load_scacquire(g);
            if (v > 0) break;  // copies still running
        }
        Pass P = std::move(S->passes.front());
        S->passes.pop_front();
        if (v < 0) {  // the copy engine reported an error
            fail_slots(S, P.slots);
            continue;     // its signal is not reused
        }
        for (int si : P.slots) {
            Slot& sl = S->slots[si];
            Worker& W = S->w[sl.kind];
            sl.t_start = t;
            sl.published = true;
            W.h_order[W.tail & (ORDER_CAP - 1)] = (uint32_t)si;
            W.tail++;
            any[sl.kind] = true;
        }
        if (g.handle) S->free_signals.push_back(g);
    }
    for (int k = 0; k < NKIND; k++)
        if (any[k]) __atomic_store_n(&S->h_ctl[k == 0 ? CTL_TAIL0 : CTL_TAIL1], S->w[k].tail, __ATOMIC_RELEASE);
}

// Ends the current admission pass: its input runs are copied to the device
// on the SDMA engine, one completion signal for the pass (with the inputs
// read from the pinned mirror there is nothing to copy).
pm_status close_pass(pm_server* S) {
    if (S->staged.empty()) return PM_OK;
    // the host copies of the pass: on the pool when they are large
    if (S->copy_words > (INT64_C(1) << 18) && S->copies.size() > 1) {
        if (!S->pool) {
            const unsigned hc = std::thread::hardware_concurrency();
            S->pool = new CopyPool((int)std::min(7u, hc > 2 ? hc / 2 : 1u));
        }
        S->pool->run(S->copies);
    } else {
        for (const CopyTask& t : S->copies) {
            if (t.na) std::memcpy(t.dst, t.a, (size_t)t.na * 4);
            if (t.nb) std::memcpy(t.dst + t.na, t.b, (size_t)t.nb * 4);
        }
    }
    S->copies.clear();
    S->holding.clear();
    S->copy_words = 0;
    hsa_signal_t sig{0};
    if (S->device_inputs) {
        if (S->free_signals.empty()) {
            // every signal in use: the oldest pass must finish first
            hsa_signal_t old = S->passes.front().done;
            while (hsa_signal_wait_scacquire(old, HSA_SIGNAL_CONDITION_LT, 1, UINT64_MAX, HSA_WAIT_STATE_ACTIVE) > 0)
                ;
            publish_ready(S);
        }
        sig = S->free_signals.back();
        S->free_signals.pop_back();
        hsa_signal_store_relaxed(sig, (hsa_signal_value_t)S->runs.size());
        for (const auto& run : S->runs) {
            const hsa_amd_sdma_engine_id_t eng = S->copier.engines[S->next_engine++ % S->copier.n_engines];
            if (hsa_amd_memory_async_copy_on_engine(S->d_in + run.first, S->copier.gpu, S->h_mirror + run.first,
                                                    S->copier.cpu, (size_t)run.second * 4, 0, nullptr, sig, eng,
                                                    false) != HSA_STATUS_SUCCESS) {
                // copies already issued may still count the signal down: it
                // is not reused, and the pass's requests fail
                fail_slots(S, S->staged);
                S->staged.clear();
                S->runs.clear();
                return pm::server_fail(PM_EDEVICE, "input copy");
            }
        }
    }
    S->runs.clear();
    S->passes.push_back(Pass{sig, std::move(S->staged)});
    S->staged.clear();
    return PM_OK;
}

// Admits queued requests in FIFO order while a slot and arena room are
// free, starts their copy, publishes what has arrived, and makes sure the
// workers run.
pm_status admit(pm_server* S) {
    while (!S->queue.empty() && !S->free_slots.empty()) {
        Pending& P = S->queue.front();
        int64_t in_off = 0, out_off = 0;
        if (!S->in_arena->alloc(P.na + P.nb, &in_off)) break;  // FIFO: wait for room, no overtaking
        if (!S->out_arena->alloc(out_words(P.op, P.na, P.nb), &out_off)) {
            S->in_arena->release(in_off, P.na + P.nb);
            break;
        }
        const int si = S->free_slots.back();
        S->free_slots.pop_back();
        place(S, si, in_off, out_off, P.ticket, P.tag, P.op, P.ab.data(), P.na, P.ab.data() + P.na, P.nb, P.g_user,
              P.g_cap, P.r_user, P.r_cap, P.F, P.t_submit);
        S->holding.push_back(std::move(P.ab));  // copied from when the pass closes
        S->queue.pop_front();
    }
    pm_status st = close_pass(S);
    if (st) return st;
    publish_ready(S);
    return ensure_workers(S);
}

// Host checks of one request; *op gets the job kind.
pm_status check_request(const pm_server* S, const pm_gcd_request* r, pm::Field* F, int32_t* op) {
    if (r->op != 0 && r->op != PM_OP_GCD && r->op != PM_OP_DIVREM)
        return pm::server_fail(PM_EINVAL, "op must be PM_OP_GCD or PM_OP_DIVREM");
    *op = r->op == PM_OP_DIVREM ? pm::JOB_DIVREM : pm::JOB_GCD;
    if (r->na < 0 || r->nb < 0 || (r->na > 0 && !r->a) || (r->nb > 0 && !r->b) || r->g_cap < 0 ||
        (r->g_cap > 0 && !r->g))
        return pm::server_fail(PM_EINVAL, "bad request buffers");
    if (*op == pm::JOB_DIVREM && (r->r_cap < 0 || (r->r_cap > 0 && !r->r)))
        return pm::server_fail(PM_EINVAL, "bad remainder buffer");
    const int64_t n = r->na > r->nb ? r->na : r->nb;
    if (n > S->w[1].cap) return pm::server_fail(PM_EINVAL, "request exceeds PM_GCD_BATCH_MAX terms");
    if (Arena::grain(r->na + r->nb) > S->opt.arena_words ||
        Arena::grain(out_words(*op, r->na, r->nb)) > S->opt.arena_words)
        return pm::server_fail(PM_ENOMEM, "request larger than the whole arena");
    if (*op == pm::JOB_DIVREM && r->nb == 0) return pm::server_fail(PM_EDIVZERO, "division by the zero polynomial");
    return pm::server_field(r->p, F);
}

pm_status enqueue(pm_server* S, const pm_gcd_request* r, uint64_t* ticket) {
    pm::Field F;
    int32_t op = 0;
    pm_status st = check_request(S, r, &F, &op);
    if (st) return st;
    int64_t in_off = 0, out_off = 0;
    if (S->queue.empty() && !S->free_slots.empty() && S->in_arena->alloc(r->na + r->nb, &in_off)) {
        if (S->out_arena->alloc(out_words(op, r->na, r->nb), &out_off)) {
            // nothing waits ahead of it: straight from the caller's arrays
            // into the pass being built
            const int si = S->free_slots.back();
            S->free_slots.pop_back();
            const uint64_t t = S->next_ticket++;
            place(S, si, in_off, out_off, t, r->tag, op, r->a, r->na, r->b, r->nb, r->g, r->g_cap, r->r, r->r_cap, F,
                  S->now_ms());
            if (ticket) *ticket = t;
            return PM_OK;
        }
        S->in_arena->release(in_off, r->na + r->nb);
    }
    Pending P;
    P.ticket = S->next_ticket++;
    P.tag = r->tag;
    P.op = op;
    P.na = r->na;
    P.nb = r->nb;
    P.ab.resize((size_t)(r->na + r->nb));
    if (r->na) std::memcpy(P.ab.data(), r->a, (size_t)r->na * 4);
    if (r->nb) std::memcpy(P.ab.data() + r->na, r->b, (size_t)r->nb * 4);
    P.g_user = r->g;
    P.g_cap = r->g_cap;
    P.r_user = r->r;
    P.r_cap = r->r_cap;
    P.F = F;
    P.t_submit = S->now_ms();
    if (ticket) *ticket = P.ticket;
    S->queue.push_back(std::move(P));
    return PM_OK;
}

}  // namespace

extern "C" {

pm_status pm_server_create(const pm_server_opts* opts, pm_server** out) {
    PM_API_BEGIN
    if (!out) return pm::server_fail(PM_EINVAL, "null output");
    *out = nullptr;
    pm_server_opts o{};
    if (opts) o = *opts;
    if (o.s < 0 || o.s > 256) return pm::server_fail(PM_EINVAL, "s must be in [0, 256]");
    if (o.max_inflight < 0 || o.large_blocks < 0 || o.small_blocks < -1 || o.arena_words < 0)
        return pm::server_fail(PM_EINVAL, "negative option");
    if (o.staging < 0 || o.staging > 2) return pm::server_fail(PM_EINVAL, "staging must be 0, 1 or 2");
    pm_server* S = new pm_server();
    if (o.max_inflight == 0) o.max_inflight = 4096;
    if (o.max_inflight > (int32_t)(ORDER_CAP / 4)) o.max_inflight = (int32_t)(ORDER_CAP / 4);
    if (o.s == 0) o.s = 128;
    (void)hipGetDevice(&S->device);
    // the input arena is budgeted from the device's free memory
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        delete S;
        return pm::server_fail(PM_EDEVICE, "hipMemGetInfo");
    }
    const int64_t free_words = (int64_t)(free_b / 4);
    if (o.arena_words == 0) o.arena_words = std::min<int64_t>(INT64_C(32) << 20, free_words / 8);
    if (o.arena_words > free_words / 2) {
        delete S;
        return pm::server_fail(PM_ENOMEM, "arena_words above half the device's free memory");
    }
    const int cus = pm::server_num_cus();
    // every CU on the 1024-thread worker by default: on the served trace a
    // static split that gives CUs to the 256-thread worker measured slower
    // (the small requests' share of CUs cannot follow their share of work)
    if (o.large_blocks == 0) o.large_blocks = cus;
    if (o.large_blocks > cus) o.large_blocks = cus;
    if (o.small_blocks == 0) o.small_blocks = (cus - o.large_blocks) * pm::gcd_worker_blocks_per_cu(0);
    if (o.small_blocks < 0) o.small_blocks = 0;
    S->opt = o;
    S->t0 = std::chrono::steady_clock::now();
    S->w[0].blocks = o.small_blocks;
    S->w[0].cap = pm::gcd_batch_cap(0);
    S->w[1].blocks = o.large_blocks;
    S->w[1].cap = pm::gcd_batch_cap(1);
    const size_t M = (size_t)o.max_inflight;
    hipError_t e = hipSuccess;
    for (Worker& W : S->w) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&W.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMalloc((void**)&W.d_head, sizeof(uint32_t));
        if (e == hipSuccess) e = hipMemset(W.d_head, 0, sizeof(uint32_t));
        if (e == hipSuccess) e = hipHostMalloc((void**)&W.h_order, ORDER_CAP * sizeof(uint32_t), hipHostMallocDefault);
        if (e == hipSuccess) std::memset(W.h_order, 0, ORDER_CAP * sizeof(uint32_t));
    }
    // inputs in device memory when an SDMA engine can copy them there
    S->device_inputs = o.staging != 2 && copier_init(&S->copier, S->device);
    if (o.staging == 1 && !S->device_inputs) {
        destroy(S);
        return pm::server_fail(PM_EDEVICE, "no SDMA engine for the device input arena");
    }
    if (e == hipSuccess && S->device_inputs) e = hipMalloc((void**)&S->d_in, (size_t)o.arena_words * 4);
    if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_mirror, (size_t)o.arena_words * 4, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_out, (size_t)o.arena_words * 4, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_jobs, M * sizeof(pm::GcdJob), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_results, M * sizeof(pm::GcdResult), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&S->h_ctl, CTL_WORDS * sizeof(uint32_t), hipHostMallocDefault);
    for (int i = 0; i < SIGNALS && e == hipSuccess && S->device_inputs; i++) {
        hsa_signal_t g;
        if (hsa_signal_create(0, 0, nullptr, &g) != HSA_STATUS_SUCCESS) e = hipErrorOutOfMemory;
        else S->free_signals.push_back(g);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        destroy(S);
        return pm::server_fail(PM_ENOMEM, "cannot allocate the server's buffers");
    }
    if (S->device_inputs) {
        // one small copy on each engine now: the runtime sets an engine's
        // queue up on its first copy, which would otherwise fall on the
        // first requests (measured: a saturated first batch at a fifth of
        // the rate of later ones)
        hsa_signal_t g = S->free_signals.back();
        for (int i = 0; i < S->copier.n_engines; i++) {
            hsa_signal_store_relaxed(g, 1);
            if (hsa_amd_memory_async_copy_on_engine(S->d_in, S->copier.gpu, S->h_mirror, S->copier.cpu, 256, 0,
                                                    nullptr, g, S->copier.engines[i], false) != HSA_STATUS_SUCCESS) {
                destroy(S);
                return pm::server_fail(PM_EDEVICE, "SDMA copy");
            }
            if (hsa_signal_wait_scacquire(g, HSA_SIGNAL_CONDITION_LT, 1, UINT64_MAX, HSA_WAIT_STATE_BLOCKED) != 0) {
                destroy(S);
                return pm::server_fail(PM_EDEVICE, "SDMA copy");
            }
        }
    }
    std::memset(S->h_results, 0, M * sizeof(pm::GcdResult));
    std::memset(S->h_ctl, 0, CTL_WORDS * sizeof(uint32_t));
    prefault(S->h_mirror, (size_t)o.arena_words * 4);
    prefault(S->h_out, (size_t)o.arena_words * 4);
    S->in_arena = new Arena(o.arena_words);
    S->out_arena = new Arena(o.arena_words);
    S->slots.resize(M);
    for (int i = (int)M - 1; i >= 0; i--) S->free_slots.push_back(i);
    *out = S;
    return PM_OK;
    PM_API_END
}

void pm_server_destroy(pm_server* S) { PM_API_BEGIN destroy(S); PM_API_END_VOID }

pm_status pm_server_submit(pm_server* S, const pm_gcd_request* r, uint64_t* ticket) {
    PM_API_BEGIN
    if (!S || !r) return pm::server_fail(PM_EINVAL, "null argument");
    pm_status st = enqueue(S, r, ticket);
    if (st) return st;
    return admit(S);  // on the GPU as soon as its copy is done, when a slot is free
    PM_API_END
}

pm_status pm_server_submit_batch(pm_server* S, const pm_gcd_request* reqs, int32_t count, uint64_t* tickets) {
    PM_API_BEGIN
    if (!S || count < 0 || (count > 0 && !reqs)) return pm::server_fail(PM_EINVAL, "null argument");
    // every request is checked before any is queued: a bad one queues none
    for (int32_t i = 0; i < count; i++) {
        pm::Field F;
        int32_t op = 0;
        pm_status st = check_request(S, &reqs[i], &F, &op);
        if (st) return st;
    }
    // The requests of one call arrive together, so they may start in any
    // order: longest first (work ~ na * nb), which keeps the largest, each
    // bound by its own step chain on one CU, from starting last and setting
    // the span.
    std::vector<int32_t> order((size_t)count);
    for (int32_t i = 0; i < count; i++) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [reqs](int32_t x, int32_t y) {
        return (double)reqs[x].na * (double)reqs[x].nb > (double)reqs[y].na * (double)reqs[y].nb;
    });
    for (int32_t k = 0; k < count; k++) {
        const int32_t i = order[(size_t)k];
        pm_status st = enqueue(S, &reqs[i], tickets ? &tickets[i] : nullptr);
        if (st) {
            (void)close_pass(S);  // the copies of those already placed are made before returning
            return st;
        }
        if ((k & 15) == 15) {  // the first requests start while the rest are copied
            st = admit(S);
            if (st) return st;
        }
    }
    return admit(S);
    PM_API_END
}

int64_t pm_server_pending(pm_server* S) { return S ? (int64_t)S->queue.size() + S->inflight : 0; }

pm_status pm_server_poll(pm_server* S, pm_completion* out, int32_t max, int32_t* n) {
    PM_API_BEGIN
    if (!S || !n || (max > 0 && !out)) return pm::server_fail(PM_EINVAL, "null argument");
    *n = 0;
    publish_ready(S);
    // 1. harvest
    for (int si = 0; si < S->opt.max_inflight && *n < max; si++) {
        Slot& sl = S->slots[si];
        if (!sl.busy || !sl.published) continue;
        pm::GcdResult* R = &S->h_results[si];
        if (__atomic_load_n(&R->done, __ATOMIC_ACQUIRE) == 0) continue;
        pm_completion& c = out[(*n)++];
        c.ticket = sl.ticket;
        c.tag = sl.tag;
        c.status = R->status;
        c.op = sl.op == pm::JOB_DIVREM ? PM_OP_DIVREM : PM_OP_GCD;
        c.ng = R->status == 0 ? R->ng : 0;
        c.nr = R->status == 0 && sl.op == pm::JOB_DIVREM ? R->nr : 0;
        c.steps = R->steps;
        c.updates = R->updates;
        c.t_submit_ms = sl.t_submit;
        c.t_start_ms = sl.t_start;
        c.t_done_ms = S->now_ms();
        const uint32_t* res = S->h_out + sl.out_off;
        if (c.status == 0) {
            // the device checked the capacities the job record gave it
            if (c.ng > 0) std::memcpy(sl.g_user, res, (size_t)c.ng * 4);
            if (c.nr > 0) std::memcpy(sl.r_user, S->h_out + sl.r_off, (size_t)c.nr * 4);
        }
        S->in_arena->release(sl.in_off, sl.in_len);
        S->out_arena->release(sl.out_off, sl.out_len);
        S->w[sl.kind].inflight--;
        S->inflight--;
        sl.busy = false;
        S->free_slots.push_back(si);
    }
    return admit(S);
    PM_API_END
}

}  // extern "C"
