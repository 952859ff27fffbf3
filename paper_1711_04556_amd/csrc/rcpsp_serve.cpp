// Serving runtime behind include/rcpsp.h: a device arena for search state,
// request queues per launch class with admission by footprint, and a host
// thread that runs the device in time slices (k_serve).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rcpsp.h"
#include "rcpsp_internal.h"
#include "rcpsp_launch.h"
#include "rcpsp_runtime.h"

using namespace rcpsp;

extern "C" int64_t rcpsp_server_now_ns(void) {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

namespace {

constexpr size_t kArenaAlign = 256;
constexpr long long kServeWaitTicks = 20ll * 100 * 1000 * 1000;  // 20 s at 100 MHz
constexpr long long kServeTaskCap = 1ll << 20;                    // tasks per class and slice
constexpr size_t kServeMaxClasses = 32;
constexpr long long kServeCarryCopy = 1ll << 16;                   // task slots read back with every slice

// First-fit allocator over one device allocation.
class Arena : public DeviceAllocator {
public:
    hipError_t init(size_t bytes) {
        size_ = bytes;
        hipError_t e = hipMalloc(&base_, bytes);
        if (e == hipSuccess) free_[0] = bytes;
        return e;
    }
    ~Arena() override {
        if (base_) (void)hipFree(base_);
    }
    hipError_t alloc(void **ptr, size_t bytes) override {
        std::lock_guard<std::mutex> g(mu_);
        const size_t need = (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[off + need] = len - need;
            live_[off] = need;
            used_ += need;
            *ptr = static_cast<char *>(base_) + off;
            return hipSuccess;
        }
        return hipErrorOutOfMemory;
    }
    void release(void *ptr) override {
        std::lock_guard<std::mutex> g(mu_);
        const size_t off = static_cast<size_t>(static_cast<char *>(ptr) - static_cast<char *>(base_));
        auto lv = live_.find(off);
        if (lv == live_.end()) return;
        size_t start = off, len = lv->second;
        used_ -= len;
        live_.erase(lv);
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && nx->first == start + len) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
    }
    size_t used() {
        std::lock_guard<std::mutex> g(mu_);
        return used_;
    }
    size_t size() const { return size_; }

private:
    std::mutex mu_;
    void *base_ = nullptr;
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_, live_;
};

// Sums a plan's buffer sizes without allocating (footprint at submission).
class MeasureAllocator : public DeviceAllocator {
public:
    hipError_t alloc(void **ptr, size_t bytes) override {
        total += (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
        *ptr = reinterpret_cast<void *>(static_cast<uintptr_t>(kArenaAlign * ++count));
        return hipSuccess;
    }
    void release(void *) override {}
    size_t total = 0, count = 0;
};

struct Req {
    int64_t ticket = 0;
    const rcpsp_instance *inst = nullptr;
    rcpsp_search_params p{};
    int64_t budget_us = 0;
    size_t bytes = 0;
    int state = RCPSP_REQ_QUEUED, error = 0, slot = -1, cls = -1;
    rcpsp_search *plan = nullptr;
    int64_t submit_ns = 0, admit_ns = 0, done_ns = 0, seen_ns = 0;
    long long key = 0;    // launch class (decoder, profile width, threads, lanes) from the footprint probe
    int best = 0, iters = 0, next_iter = -1;
    int64_t evals = 0;
    bool cancel = false, cancel_sent = false, fresh = false;
    bool seed = false;    // the host must queue iteration next_iter (the device queue was full)
};

struct Req;

struct SClass {
    int dec = 0, nw = 0, T = 0, G = 1;
    unsigned long long *d_tasks = nullptr;
    ServeQueue *d_q = nullptr;
    unsigned long long *h_tasks = nullptr;   // pinned staging
    size_t h_cap = 0;
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;                 // end of the running slice
    bool running = false;
    int64_t t_launch = 0;
    std::vector<Req *> inflight;             // requests of the running slice
    std::vector<unsigned long long> carry;   // tasks queued but not run in the last slice
    ServeReq *h_back = nullptr;              // pinned: control blocks read back after the slice
    ServeQueue *h_q = nullptr;               // pinned: queue header read back after the slice
    int *h_cancel = nullptr;                 // pinned: cancel flags to upload (per slot)
    size_t queued = 0;                       // tasks the running slice started with
    unsigned long long *h_back_tasks = nullptr;  // pinned: the task queue read back after the slice
    size_t h_back_cap = 0;
};

}  // namespace

struct rcpsp_server {
    rcpsp_server_params prm{};
    std::mutex mu;
    std::condition_variable cv_work, cv_idle;
    std::thread th;
    bool stop = false, failed = false;
    rcpsp_status fail_st = RCPSP_OK;
    std::string fail_msg;
    std::map<long long, std::deque<Req *>> queues;   // per launch class, arrival order
    std::map<long long, int> resident_of;            // resident requests per launch class
    size_t queued = 0;
    std::deque<int64_t> finished;   // tickets not yet taken by the caller
    std::unordered_map<int64_t, Req *> reqs;
    int64_t next_ticket = 1;
    std::vector<Req *> slot_req;
    std::vector<int> free_slots;
    int running = 0;
    Arena arena;
    SearchArgs *d_items = nullptr, *h_items = nullptr;
    ServeReq *d_req = nullptr, *h_req = nullptr;
    std::vector<SClass> classes;   // reserved up front: references stay valid
    uint32_t *d_decay = nullptr;
    int decay_len = 0;
    int device = 0, cus = 256;
    hipStream_t st = nullptr;
    long long *d_clock = nullptr;
    long long dev0 = 0, dev_first = 0;   // device wall clock at host0 / host_first
    int64_t host0 = 0, host_first = 0;
    int64_t next_sync_ns = 0;
    double ticks_per_ns = 0.1;
    rcpsp_server_stats stats{};
};

namespace {

long long dev_ticks_at(const rcpsp_server *s, int64_t host_ns) {
    return s->dev0 + (long long)((double)(host_ns - s->host0) * s->ticks_per_ns);
}

int64_t host_ns_at(const rcpsp_server *s, long long ticks) {
    return s->host0 + (int64_t)((double)(ticks - s->dev0) / s->ticks_per_ns);
}

// One reading of the device wall clock against the host clock (the host time
// is the middle of the launch-to-completion interval).
rcpsp_status clock_pair(rcpsp_server *s, int64_t *host_ns, long long *ticks) {
    const int64_t a = rcpsp_server_now_ns();
    HIP_TRY(launch_clock(s->d_clock, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    const int64_t b = rcpsp_server_now_ns();
    HIP_TRY(hipMemcpy(ticks, s->d_clock, sizeof(long long), hipMemcpyDeviceToHost));
    *host_ns = (a + b) / 2;
    return RCPSP_OK;
}

// Refresh the host <-> device clock mapping: the rate from the first reading
// to the newest (measured, not taken from the driver's attribute), the
// offset from the newest.
rcpsp_status sync_clocks(rcpsp_server *s) {
    int64_t h;
    long long d;
    rcpsp_status st = clock_pair(s, &h, &d);
    if (st != RCPSP_OK) return st;
    if (h - s->host_first > 5 * 1000 * 1000 && d > s->dev_first)
        s->ticks_per_ns = (double)(d - s->dev_first) / (double)(h - s->host_first);
    s->host0 = h;
    s->dev0 = d;
    s->next_sync_ns = h + 50 * 1000 * 1000;
    return RCPSP_OK;
}

void set_failed(rcpsp_server *s, rcpsp_status st, const char *msg) {
    std::lock_guard<std::mutex> g(s->mu);
    s->failed = true;
    s->fail_st = st;
    s->fail_msg = msg;
    s->cv_idle.notify_all();
}

rcpsp_status class_of(rcpsp_server *s, const rcpsp_search *plan, int *out) {
    const int nw = plan->dec == kEvalTime ? plan->nw : 1;
    for (size_t k = 0; k < s->classes.size(); ++k)
        if (s->classes[k].dec == plan->dec && s->classes[k].nw == nw && s->classes[k].T == plan->T &&
            s->classes[k].G == plan->G) {
            *out = (int)k;
            return RCPSP_OK;
        }
    if (s->classes.size() >= kServeMaxClasses) return fail(RCPSP_E_TOO_LARGE, "more than %d launch classes", (int)kServeMaxClasses);
    s->classes.emplace_back();
    SClass &c = s->classes.back();
    c.dec = plan->dec;
    c.nw = nw;
    c.T = plan->T;
    c.G = plan->G;
    const size_t slots = s->slot_req.size();
    HIP_TRY(hipMalloc(&c.d_tasks, sizeof(unsigned long long) * kServeTaskCap));
    HIP_TRY(hipMalloc(&c.d_q, sizeof(ServeQueue)));
    HIP_TRY(hipStreamCreateWithFlags(&c.st, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&c.ev, hipEventDisableTiming));
    HIP_TRY(hipHostMalloc(&c.h_back, sizeof(ServeReq) * slots, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(&c.h_q, sizeof(ServeQueue), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(&c.h_cancel, sizeof(int) * slots, hipHostMallocDefault));
    *out = (int)s->classes.size() - 1;
    return RCPSP_OK;
}

// Admit queued requests while slots and arena room are free.  Each launch
// class has its own queue (arrival order) and at most an equal share of the
// slots among the classes with work, so long requests of one class do not
// block the others; classes are visited round-robin.
void admit(rcpsp_server *s, std::vector<Req *> &fresh) {
    std::unique_lock<std::mutex> g(s->mu);
    int classes_with_work = 0;
    for (auto &kv : s->queues)
        if (!kv.second.empty() || s->resident_of[kv.first] > 0) ++classes_with_work;
    const int cap = std::max(1, s->prm.max_active / std::max(classes_with_work, 1));
    std::map<long long, bool> blocked;
    for (bool progress = true; progress && !s->free_slots.empty();) {
        progress = false;
        for (auto &kv : s->queues) {
            std::deque<Req *> &qu = kv.second;
            if (qu.empty() || blocked[kv.first] || s->free_slots.empty()) continue;
            if (s->resident_of[kv.first] >= cap) continue;
            Req *r = qu.front();
            if (r->cancel) {
                qu.pop_front();
                --s->queued;
                r->state = RCPSP_REQ_FAILED;
                r->error = RCPSP_E_ARG;
                s->finished.push_back(r->ticket);
                progress = true;
                continue;
            }
            rcpsp_search *plan = new (std::nothrow) rcpsp_search();
            if (!plan) return;
            plan->inst = r->inst;
            plan->p = r->p;
            plan->reserve = kBatchStaticLds;
            plan->allocator = &s->arena;
            plan->shared_decay = s->d_decay;
            plan->shared_decay_len = s->decay_len;
            rcpsp_status st = alloc_plan(plan);
            if (st == RCPSP_E_NOMEM) {
                rcpsp_search_destroy(plan);
                blocked[kv.first] = true;  // the arena frees up as requests are released
                continue;
            }
            qu.pop_front();
            --s->queued;
            progress = true;
            int cls = -1;
            if (st == RCPSP_OK) st = class_of(s, plan, &cls);
            if (st != RCPSP_OK) {
                rcpsp_search_destroy(plan);
                r->state = RCPSP_REQ_FAILED;
                r->error = st;
                s->finished.push_back(r->ticket);
                continue;
            }
            const int slot = s->free_slots.back();
            s->free_slots.pop_back();
            s->slot_req[slot] = r;
            ++s->resident_of[kv.first];
            r->plan = plan;
            r->slot = slot;
            r->cls = cls;
            r->admit_ns = rcpsp_server_now_ns();
            r->state = RCPSP_REQ_RUNNING;
            r->fresh = true;
            r->next_iter = -1;
            s->h_items[slot] = plan->a;
            ServeReq q{};
            q.next_iter = -1;
            q.max_iters = plan->p.iterations;
            q.deadline = r->budget_us > 0 ? dev_ticks_at(s, r->admit_ns + r->budget_us * 1000) : LLONG_MAX;
            s->h_req[slot] = q;
            ++s->running;
            ++s->stats.admitted;
            fresh.push_back(r);
        }
    }
}

// Classes run independently: each has its own stream, task queue and slice
// loop, so a class of long iterations never holds back the slices (and so
// the admissions and completions) of the others.

// Start a slice of class c: new requests' arguments and control blocks, the
// set-up or next-iteration tasks of its running requests, the launch.
rcpsp_status launch_class(rcpsp_server *s, int c) {
    SClass &C = s->classes[c];
    std::vector<Req *> act;
    std::vector<char> busy(s->classes.size(), 0);
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (Req *r : s->slot_req) {
            if (!r || r->state != RCPSP_REQ_RUNNING) continue;
            busy[r->cls] = 1;
            if (r->cls == c) act.push_back(r);
        }
        if (act.empty()) return RCPSP_OK;
        for (Req *r : act)
            if (r->cancel && !r->cancel_sent && !r->fresh) {
                r->cancel_sent = true;
                C.h_cancel[r->slot] = 1;
                HIP_TRY(hipMemcpyAsync(&s->d_req[r->slot].cancel, C.h_cancel + r->slot, sizeof(int),
                                       hipMemcpyHostToDevice, C.st));
            }
    }
    // queued tasks of the last slice first, then seeds and new requests' set-up
    std::vector<unsigned long long> tasks;
    tasks.swap(C.carry);
    size_t lds = 0;
    for (Req *r : act) {
        if (r->fresh) {
            HIP_TRY(hipMemcpyAsync(s->d_items + r->slot, s->h_items + r->slot, sizeof(SearchArgs),
                                   hipMemcpyHostToDevice, C.st));
            HIP_TRY(hipMemcpyAsync(s->d_req + r->slot, s->h_req + r->slot, sizeof(ServeReq), hipMemcpyHostToDevice,
                                   C.st));
            tasks.push_back(serve_task(r->slot, 0, 0, 0));
            r->fresh = false;
        } else if (r->seed) {
            for (int b = 0; b < r->p.searches; ++b) tasks.push_back(serve_task(r->slot, 1, b, r->next_iter));
            r->seed = false;
        }
        lds = std::max(lds, r->plan->lds);
    }
    const size_t n0 = tasks.size();
    if (n0 == 0) return fail(RCPSP_E_DEVICE, "serving class %d has running requests but no queued task", c);
    if (n0 > (size_t)kServeTaskCap) return fail(RCPSP_E_TOO_LARGE, "slice needs %zu tasks", n0);
    if (C.h_cap < n0) {
        if (C.h_tasks) (void)hipHostFree(C.h_tasks);
        C.h_tasks = nullptr;
        C.h_cap = std::max<size_t>(n0, 4096);
        HIP_TRY(hipHostMalloc(&C.h_tasks, sizeof(unsigned long long) * C.h_cap, hipHostMallocDefault));
    }
    for (size_t i = 0; i < n0; ++i) C.h_tasks[i] = tasks[i] + 1ull;
    HIP_TRY(hipMemcpyAsync(C.d_tasks, C.h_tasks, sizeof(unsigned long long) * n0, hipMemcpyHostToDevice, C.st));
    HIP_TRY(launch_serve_begin(C.d_q, C.d_tasks, kServeTaskCap, (long long)n0, C.st));
    int per_cu = 0;
    HIP_TRY(serve_occupancy(C.T, C.nw, C.dec, C.G, lds, &per_cu));
    if (per_cu < 1) return fail(RCPSP_E_TOO_LARGE, "serving workgroup of %zu B LDS does not fit a CU", lds);
    // the classes with running requests share the CUs equally, so that a
    // class of long tasks cannot hold every CU
    int nbusy = 0;
    for (char b : busy) nbusy += b;
    const int full = per_cu * s->cus;
    const int share = (full + std::max(nbusy, 1) - 1) / std::max(nbusy, 1);
    const int grid = std::max(std::min(full, 8), std::min(share, full));
    ServeArgs A{};
    A.items = s->d_items;
    A.req = s->d_req;
    A.tasks = C.d_tasks;
    A.q = C.d_q;
    A.cap = kServeTaskCap;
    A.slice_end = dev_ticks_at(s, rcpsp_server_now_ns() + (int64_t)s->prm.slice_us * 1000);
    A.wait_ticks = kServeWaitTicks;
    C.t_launch = rcpsp_server_now_ns();
    HIP_TRY(launch_serve(A, grid, C.T, C.nw, C.dec, C.G, lds, C.st));
    HIP_TRY(hipMemcpyAsync(C.h_back, s->d_req, sizeof(ServeReq) * s->slot_req.size(), hipMemcpyDeviceToHost, C.st));
    HIP_TRY(hipMemcpyAsync(C.h_q, C.d_q, sizeof(ServeQueue), hipMemcpyDeviceToHost, C.st));
    // the queue as the slice leaves it (its first kServeCarryCopy slots; the
    // rest, if any, is read synchronously afterwards)
    if (C.h_back_cap < (size_t)kServeCarryCopy) {
        if (C.h_back_tasks) (void)hipHostFree(C.h_back_tasks);
        C.h_back_tasks = nullptr;
        C.h_back_cap = (size_t)kServeCarryCopy;
        HIP_TRY(hipHostMalloc(&C.h_back_tasks, sizeof(unsigned long long) * C.h_back_cap, hipHostMallocDefault));
    }
    HIP_TRY(hipMemcpyAsync(C.h_back_tasks, C.d_tasks, sizeof(unsigned long long) * kServeCarryCopy,
                           hipMemcpyDeviceToHost, C.st));
    HIP_TRY(hipEventRecord(C.ev, C.st));
    C.queued = n0;
    C.inflight = act;
    C.running = true;
    return RCPSP_OK;
}

// End of a slice of class c (its event has completed): results and next
// iterations of the requests it ran.
rcpsp_status finish_class(rcpsp_server *s, int c) {
    SClass &C = s->classes[c];
    C.running = false;
    const int64_t t1 = rcpsp_server_now_ns();
    if (C.h_q->abort) return fail(RCPSP_E_DEVICE, "serving class %d: a wait inside the kernel exceeded its limit", c);
    // tasks queued in the slice that did not run
    const size_t nt = (size_t)std::min<unsigned long long>(C.h_q->tail, (unsigned long long)kServeTaskCap);
    if (nt > (size_t)kServeCarryCopy) {
        if (C.h_back_cap < nt) {
            if (C.h_back_tasks) (void)hipHostFree(C.h_back_tasks);
            C.h_back_tasks = nullptr;
            C.h_back_cap = nt;
            HIP_TRY(hipHostMalloc(&C.h_back_tasks, sizeof(unsigned long long) * C.h_back_cap, hipHostMallocDefault));
        }
        HIP_TRY(hipMemcpyAsync(C.h_back_tasks, C.d_tasks, sizeof(unsigned long long) * nt, hipMemcpyDeviceToHost,
                               C.st));
        HIP_TRY(hipStreamSynchronize(C.st));
    }
    C.carry.clear();
    for (size_t i = 0; i < nt; ++i) {
        const unsigned long long v = C.h_back_tasks[i];
        if (v != 0ull && v != kServeTaskDone) C.carry.push_back(v - 1ull);
    }
    std::lock_guard<std::mutex> g(s->mu);
    ++s->stats.slices;
    s->stats.busy_ms += (double)(t1 - C.t_launch) * 1e-6;
    for (Req *r : C.inflight) {
        const ServeReq &q = C.h_back[r->slot];
        if (q.finished) {
            r->state = RCPSP_REQ_DONE;
            r->best = q.best;
            r->iters = q.replay_iters;
            r->evals = q.evals;
            r->done_ns = host_ns_at(s, q.done_ticks);
            r->seen_ns = t1;
            --s->running;
            ++s->stats.completed;
            s->stats.evaluations += q.evals;
            s->finished.push_back(r->ticket);
        } else if (q.next_iter >= 0) {
            r->next_iter = q.next_iter;
            r->seed = true;
        }
    }
    C.inflight.clear();
    s->cv_idle.notify_all();
    return RCPSP_OK;
}

void loop(rcpsp_server *s) {
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) {
        set_failed(s, RCPSP_E_DEVICE, "hipSetDevice failed in the server thread");
        return;
    }
    rcpsp_status st = RCPSP_OK;
    for (;;) {
        {
            std::unique_lock<std::mutex> g(s->mu);
            bool any_slice = false;
            for (const SClass &C : s->classes) any_slice = any_slice || C.running;
            if (!any_slice)
                s->cv_work.wait_for(g, std::chrono::milliseconds(1),
                                    [&] { return s->stop || s->queued > 0 || s->running > 0; });
            if (s->stop) break;
        }
        // slices that ended
        for (int c = 0; st == RCPSP_OK && c < (int)s->classes.size(); ++c) {
            if (!s->classes[c].running) continue;
            const hipError_t q = hipEventQuery(s->classes[c].ev);
            if (q == hipSuccess) st = finish_class(s, c);
            else if (q != hipErrorNotReady) st = fail(RCPSP_E_DEVICE, "serving slice: %s", hipGetErrorString(q));
        }
        if (st != RCPSP_OK) break;
        // the clock reading waits on the server's own stream, which may share
        // a hardware queue with a running slice: only refresh while idle
        bool idle_now = true;
        for (const SClass &C : s->classes) idle_now = idle_now && !C.running;
        if (idle_now && rcpsp_server_now_ns() >= s->next_sync_ns && (st = sync_clocks(s)) != RCPSP_OK) break;
        std::vector<Req *> fresh;
        admit(s, fresh);
        // idle classes with running requests start their next slice
        bool any_slice = false;
        for (int c = 0; st == RCPSP_OK && c < (int)s->classes.size(); ++c) {
            if (!s->classes[c].running) st = launch_class(s, c);
            any_slice = any_slice || s->classes[c].running;
        }
        if (st != RCPSP_OK) break;
        if (any_slice) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    if (st != RCPSP_OK) set_failed(s, st, rcpsp_last_error());
    for (SClass &C : s->classes)
        if (C.running) (void)hipStreamSynchronize(C.st);
}

}  // namespace

extern "C" rcpsp_status rcpsp_server_create(const rcpsp_server_params *params, rcpsp_server **out) {
    if (!out) return fail(RCPSP_E_ARG, "null pointer");
    *out = nullptr;
    rcpsp_server *s = new (std::nothrow) rcpsp_server();
    if (!s) return fail(RCPSP_E_NOMEM, "out of host memory");
    if (params) s->prm = *params;
    if (s->prm.max_active <= 0) s->prm.max_active = 256;
    if (s->prm.slice_us <= 0) s->prm.slice_us = 2000;
    if (s->prm.arena_bytes <= 0) s->prm.arena_bytes = 2ll << 30;
    if (s->prm.max_active > (1 << 20)) {
        delete s;
        return fail(RCPSP_E_ARG, "max_active above 2^20");
    }
    auto bail = [&](rcpsp_status st) {
        rcpsp_server_destroy(s);
        return st;
    };
#define SRV_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return bail(fail(e_ == hipErrorOutOfMemory ? RCPSP_E_NOMEM : RCPSP_E_DEVICE, "%s: %s", #expr, \
                             hipGetErrorString(e_)));                                           \
    } while (0)
    SRV_TRY(hipGetDevice(&s->device));
    SRV_TRY(hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device));
    SRV_TRY(s->arena.init((size_t)s->prm.arena_bytes));
    const size_t slots = (size_t)s->prm.max_active;
    SRV_TRY(hipMalloc(&s->d_items, sizeof(SearchArgs) * slots));
    SRV_TRY(hipMalloc(&s->d_req, sizeof(ServeReq) * slots));
    SRV_TRY(hipHostMalloc(&s->h_items, sizeof(SearchArgs) * slots, hipHostMallocDefault));
    SRV_TRY(hipHostMalloc(&s->h_req, sizeof(ServeReq) * slots, hipHostMallocDefault));
    std::memset(s->h_req, 0, sizeof(ServeReq) * slots);
    SRV_TRY(hipMemcpy(s->d_req, s->h_req, sizeof(ServeReq) * slots, hipMemcpyHostToDevice));
    SRV_TRY(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
    {
        std::vector<uint32_t> E = decay_table();
        SRV_TRY(hipMalloc(&s->d_decay, sizeof(uint32_t) * E.size()));
        SRV_TRY(hipMemcpy(s->d_decay, E.data(), sizeof(uint32_t) * E.size(), hipMemcpyHostToDevice));
        s->decay_len = (int)E.size();
    }
    // host <-> device wall-clock mapping: two readings 20 ms apart give the
    // first rate; the server thread refines it every 50 ms
    SRV_TRY(hipMalloc(&s->d_clock, sizeof(long long)));
    {
        rcpsp_status st = clock_pair(s, &s->host_first, &s->dev_first);
        if (st != RCPSP_OK) return bail(st);
        std::this_thread::sleep_for(std::chrono::milliseconds(20));
        st = sync_clocks(s);
        if (st != RCPSP_OK) return bail(st);
        if (!(s->ticks_per_ns > 0.0)) return bail(fail(RCPSP_E_DEVICE, "device wall clock does not advance"));
    }
#undef SRV_TRY
    s->slot_req.assign(slots, nullptr);
    s->classes.reserve(kServeMaxClasses);
    for (int i = (int)slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->stats.arena_bytes = (int64_t)s->arena.size();
    s->th = std::thread(loop, s);
    *out = s;
    return RCPSP_OK;
}

extern "C" void rcpsp_server_destroy(rcpsp_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->th.joinable()) s->th.join();
    for (auto &kv : s->reqs) {
        if (kv.second->plan) rcpsp_search_destroy(kv.second->plan);
        delete kv.second;
    }
    for (SClass &c : s->classes) {
        if (c.st) (void)hipStreamSynchronize(c.st);
        if (c.st) (void)hipStreamDestroy(c.st);
        if (c.d_tasks) (void)hipFree(c.d_tasks);
        if (c.d_q) (void)hipFree(c.d_q);
        if (c.h_tasks) (void)hipHostFree(c.h_tasks);
        if (c.ev) (void)hipEventDestroy(c.ev);
        if (c.h_back) (void)hipHostFree(c.h_back);
        if (c.h_q) (void)hipHostFree(c.h_q);
        if (c.h_cancel) (void)hipHostFree(c.h_cancel);
        if (c.h_back_tasks) (void)hipHostFree(c.h_back_tasks);
    }
    if (s->st) (void)hipStreamDestroy(s->st);
    if (s->d_items) (void)hipFree(s->d_items);
    if (s->d_req) (void)hipFree(s->d_req);
    if (s->h_items) (void)hipHostFree(s->h_items);
    if (s->h_req) (void)hipHostFree(s->h_req);
    if (s->d_decay) (void)hipFree(s->d_decay);
    if (s->d_clock) (void)hipFree(s->d_clock);
    delete s;
}

extern "C" rcpsp_status rcpsp_server_submit(rcpsp_server *s, const rcpsp_instance *inst,
                                            const rcpsp_search_params *params, int64_t budget_us, int64_t *ticket) {
    if (!s || !inst || !params || !ticket) return fail(RCPSP_E_ARG, "null pointer");
    rcpsp_status st = validate_params(*params);
    if (st != RCPSP_OK) return st;
    if (params->iterations < 1 || params->iterations >= kServeNoIteration)
        return fail(RCPSP_E_ARG, "a served request needs an iteration allowance in 1..%d", kServeNoIteration - 1);
    if (params->fbi) return fail(RCPSP_E_ARG, "forward-backward improvement is for search plans only");
    if (params->exchange_every > 1) return fail(RCPSP_E_ARG, "served requests exchange after every iteration");
    if (budget_us < 0) return fail(RCPSP_E_ARG, "negative budget");
    // the request's budget (the parameters' one when none is given here) is
    // checked by the serving kernel, not by the plan's own rounds
    if (budget_us == 0) budget_us = params->time_budget_us;
    rcpsp_search_params q = *params;
    q.time_budget_us = 0;
    params = &q;
    // footprint: the plan's state in the arena and its workgroup's LDS
    MeasureAllocator m;
    rcpsp_search probe;
    probe.inst = inst;
    probe.p = *params;
    probe.reserve = kBatchStaticLds;
    probe.allocator = &m;
    probe.shared_decay = reinterpret_cast<const uint32_t *>(&m);  // not dereferenced
    probe.shared_decay_len = 1;
    st = alloc_plan(&probe);
    probe.allocs.clear();
    if (st != RCPSP_OK) return st;
    if (params->elite > 0 && 6 * params->searches + 5 * params->elite > probe.Ly.cands * probe.Ly.per_lane)
        return fail(RCPSP_E_TOO_LARGE, "exchange bookkeeping does not fit the workgroup's LDS");
    if (m.total > s->arena.size())
        return fail(RCPSP_E_TOO_LARGE, "request state of %zu B exceeds the arena (%zu B)", m.total, s->arena.size());
    const long long key = (long long)probe.dec | ((long long)(probe.dec == kEvalTime ? probe.nw : 1) << 4) |
                          ((long long)probe.T << 8) | ((long long)probe.G << 20);
    Req *r = new (std::nothrow) Req();
    if (!r) return fail(RCPSP_E_NOMEM, "out of host memory");
    r->inst = inst;
    r->p = *params;
    r->budget_us = budget_us;
    r->bytes = m.total;
    r->key = key;
    r->submit_ns = rcpsp_server_now_ns();
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->failed) {
            delete r;
            return fail(s->fail_st, "server failed: %s", s->fail_msg.c_str());
        }
        r->ticket = s->next_ticket++;
        s->reqs[r->ticket] = r;
        s->queues[r->key].push_back(r);
        ++s->queued;
        ++s->stats.submitted;
        *ticket = r->ticket;
    }
    s->cv_work.notify_all();
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_server_poll(rcpsp_server *s, int64_t ticket, rcpsp_request_status *out) {
    if (!s || !out) return fail(RCPSP_E_ARG, "null pointer");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(RCPSP_E_ARG, "unknown ticket %lld", (long long)ticket);
    const Req *r = it->second;
    *out = rcpsp_request_status{};
    out->state = r->state;
    out->best_makespan = r->best;
    out->iterations = r->iters;
    out->error = r->error;
    out->evaluations = r->evals;
    out->submit_ns = r->submit_ns;
    out->admit_ns = r->admit_ns;
    out->done_ns = r->done_ns;
    out->seen_ns = r->seen_ns;
    if (s->failed && r->state != RCPSP_REQ_DONE)
        return fail(s->fail_st, "server failed: %s", s->fail_msg.c_str());
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_server_results(rcpsp_server *s, int64_t ticket, rcpsp_search_result *res) {
    if (!s || !res) return fail(RCPSP_E_ARG, "null pointer");
    rcpsp_search *plan = nullptr;
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return fail(RCPSP_E_ARG, "unknown ticket %lld", (long long)ticket);
        if (it->second->state != RCPSP_REQ_DONE) return fail(RCPSP_E_ARG, "request %lld has not finished", (long long)ticket);
        plan = it->second->plan;
    }
    // the request's state is no longer written by any kernel
    return rcpsp_search_results(plan, res, nullptr);
}

extern "C" rcpsp_status rcpsp_server_cancel(rcpsp_server *s, int64_t ticket) {
    if (!s) return fail(RCPSP_E_ARG, "null pointer");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(RCPSP_E_ARG, "unknown ticket %lld", (long long)ticket);
    it->second->cancel = true;
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_server_release(rcpsp_server *s, int64_t ticket) {
    if (!s) return fail(RCPSP_E_ARG, "null pointer");
    Req *r = nullptr;
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return fail(RCPSP_E_ARG, "unknown ticket %lld", (long long)ticket);
        r = it->second;
        if (r->state != RCPSP_REQ_DONE && r->state != RCPSP_REQ_FAILED)
            return fail(RCPSP_E_ARG, "request %lld is still queued or running", (long long)ticket);
        s->reqs.erase(it);
        for (auto f = s->finished.begin(); f != s->finished.end(); ++f)
            if (*f == ticket) {
                s->finished.erase(f);
                break;
            }
        if (r->slot >= 0) {
            s->slot_req[r->slot] = nullptr;
            s->free_slots.push_back(r->slot);
            --s->resident_of[r->key];
        }
    }
    if (r->plan) rcpsp_search_destroy(r->plan);
    delete r;
    s->cv_work.notify_all();
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_server_drain(rcpsp_server *s, int64_t timeout_ms) {
    if (!s) return fail(RCPSP_E_ARG, "null pointer");
    std::unique_lock<std::mutex> g(s->mu);
    auto idle = [&] { return s->failed || (s->queued == 0 && s->running == 0); };
    if (timeout_ms > 0) {
        if (!s->cv_idle.wait_for(g, std::chrono::milliseconds(timeout_ms), idle))
            return fail(RCPSP_E_ARG, "drain timed out");
    } else {
        s->cv_idle.wait(g, idle);
    }
    if (s->failed) return fail(s->fail_st, "server failed: %s", s->fail_msg.c_str());
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_server_take_finished(rcpsp_server *s, int64_t *tickets, int32_t cap, int32_t *n) {
    if (!s || !n || (cap > 0 && !tickets)) return fail(RCPSP_E_ARG, "null pointer");
    std::lock_guard<std::mutex> g(s->mu);
    int32_t k = 0;
    while (k < cap && !s->finished.empty()) {
        tickets[k++] = s->finished.front();
        s->finished.pop_front();
    }
    *n = k;
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_server_get_stats(rcpsp_server *s, rcpsp_server_stats *out) {
    if (!s || !out) return fail(RCPSP_E_ARG, "null pointer");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    out->resident = (int32_t)(s->slot_req.size() - s->free_slots.size());
    out->queued = (int32_t)s->queued;
    out->arena_used = (int64_t)s->arena.used();
    out->arena_bytes = (int64_t)s->arena.size();
    out->device_clock_mhz = s->ticks_per_ns * 1000.0;
    return RCPSP_OK;
}
