// Serving runtime behind include/rcpsp.h: a device arena for search state,
// a request queue with admission by footprint, and a host thread that runs
// the device in time slices (k_serve).
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
    int best = 0, iters = 0, next_iter = -1;
    int64_t evals = 0;
    bool cancel = false, cancel_sent = false, fresh = false;
};

struct SClass {
    int dec = 0, nw = 0, T = 0, G = 1;
    unsigned long long *d_tasks = nullptr;
    ServeQueue *d_q = nullptr;
    unsigned long long *h_tasks = nullptr;   // pinned staging
    size_t h_cap = 0;
    hipStream_t st = nullptr;
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
    std::deque<Req *> queue;
    std::deque<int64_t> finished;   // tickets not yet taken by the caller
    std::unordered_map<int64_t, Req *> reqs;
    int64_t next_ticket = 1;
    std::vector<Req *> slot_req;
    std::vector<int> free_slots;
    int running = 0;
    Arena arena;
    SearchArgs *d_items = nullptr, *h_items = nullptr;
    ServeReq *d_req = nullptr, *h_req = nullptr;
    int *h_one = nullptr;
    std::vector<SClass> classes;
    uint32_t *d_decay = nullptr;
    int decay_len = 0;
    int device = 0, cus = 256;
    hipStream_t st = nullptr;
    long long *d_clock = nullptr;
    long long dev0 = 0;
    int64_t host0 = 0;
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
    SClass c;
    c.dec = plan->dec;
    c.nw = nw;
    c.T = plan->T;
    c.G = plan->G;
    HIP_TRY(hipMalloc(&c.d_tasks, sizeof(unsigned long long) * kServeTaskCap));
    HIP_TRY(hipMalloc(&c.d_q, sizeof(ServeQueue)));
    HIP_TRY(hipStreamCreateWithFlags(&c.st, hipStreamNonBlocking));
    s->classes.push_back(c);
    *out = (int)s->classes.size() - 1;
    return RCPSP_OK;
}

// Admit queued requests in order while a slot and arena room are free.
void admit(rcpsp_server *s, std::vector<Req *> &fresh) {
    std::unique_lock<std::mutex> g(s->mu);
    while (!s->queue.empty() && !s->free_slots.empty()) {
        Req *r = s->queue.front();
        if (r->cancel) {
            s->queue.pop_front();
            r->state = RCPSP_REQ_FAILED;
            r->error = RCPSP_E_ARG;
            s->finished.push_back(r->ticket);
            continue;
        }
        rcpsp_search *plan = new (std::nothrow) rcpsp_search();
        if (!plan) break;
        plan->inst = r->inst;
        plan->p = r->p;
        plan->p.count_work = r->p.count_work;
        plan->reserve = kBatchStaticLds;
        plan->allocator = &s->arena;
        plan->shared_decay = s->d_decay;
        plan->shared_decay_len = s->decay_len;
        rcpsp_status st = alloc_plan(plan);
        if (st == RCPSP_E_NOMEM) {
            rcpsp_search_destroy(plan);
            break;  // the arena frees up as requests are released
        }
        s->queue.pop_front();
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

// One slice: set-up and iteration tasks per class, launches, read-back.
rcpsp_status run_slice(rcpsp_server *s, const std::vector<Req *> &fresh) {
    // new requests' arguments and control blocks
    for (Req *r : fresh) {
        HIP_TRY(hipMemcpyAsync(s->d_items + r->slot, s->h_items + r->slot, sizeof(SearchArgs),
                               hipMemcpyHostToDevice, s->st));
        HIP_TRY(hipMemcpyAsync(s->d_req + r->slot, s->h_req + r->slot, sizeof(ServeReq), hipMemcpyHostToDevice,
                               s->st));
    }
    std::vector<Req *> active;
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (Req *r : s->slot_req)
            if (r && r->state == RCPSP_REQ_RUNNING) {
                active.push_back(r);
                if (r->cancel && !r->cancel_sent) {
                    r->cancel_sent = true;
                    *s->h_one = 1;
                    HIP_TRY(hipMemcpyAsync(&s->d_req[r->slot].cancel, s->h_one, sizeof(int), hipMemcpyHostToDevice,
                                           s->st));
                }
            }
    }
    HIP_TRY(hipStreamSynchronize(s->st));
    const int nc = (int)s->classes.size();
    std::vector<std::vector<unsigned long long>> tasks(nc);
    std::vector<size_t> lds(nc, 0);
    for (Req *r : active) {
        std::vector<unsigned long long> &t = tasks[r->cls];
        if (r->fresh) t.push_back(serve_task(r->slot, 0, 0, 0));
        else
            for (int b = 0; b < r->p.searches; ++b) t.push_back(serve_task(r->slot, 1, b, r->next_iter));
        lds[r->cls] = std::max(lds[r->cls], r->plan->lds);
        r->fresh = false;
    }
    const long long slice_end = dev_ticks_at(s, rcpsp_server_now_ns() + (int64_t)s->prm.slice_us * 1000);
    const int64_t t0 = rcpsp_server_now_ns();
    int launched = 0;
    for (int c = 0; c < nc; ++c) {
        SClass &C = s->classes[c];
        const size_t n0 = tasks[c].size();
        if (n0 == 0) continue;
        if (n0 > (size_t)kServeTaskCap) return fail(RCPSP_E_TOO_LARGE, "slice needs %zu tasks", n0);
        if (C.h_cap < n0) {
            if (C.h_tasks) (void)hipHostFree(C.h_tasks);
            C.h_tasks = nullptr;
            C.h_cap = std::max<size_t>(n0, 4096);
            HIP_TRY(hipHostMalloc(&C.h_tasks, sizeof(unsigned long long) * C.h_cap, hipHostMallocDefault));
        }
        for (size_t i = 0; i < n0; ++i) C.h_tasks[i] = tasks[c][i] + 1ull;
        HIP_TRY(hipMemcpyAsync(C.d_tasks, C.h_tasks, sizeof(unsigned long long) * n0, hipMemcpyHostToDevice, C.st));
        HIP_TRY(launch_serve_begin(C.d_q, C.d_tasks, kServeTaskCap, (long long)n0, C.st));
        int per_cu = 0;
        HIP_TRY(serve_occupancy(C.T, C.nw, C.dec, C.G, lds[c], &per_cu));
        if (per_cu < 1) return fail(RCPSP_E_TOO_LARGE, "serving workgroup of %zu B LDS does not fit a CU", lds[c]);
        ServeArgs A{};
        A.items = s->d_items;
        A.req = s->d_req;
        A.tasks = C.d_tasks;
        A.q = C.d_q;
        A.cap = kServeTaskCap;
        A.slice_end = slice_end;
        A.wait_ticks = kServeWaitTicks;
        HIP_TRY(launch_serve(A, per_cu * s->cus, C.T, C.nw, C.dec, C.G, lds[c], C.st));
        ++launched;
    }
    for (int c = 0; c < nc; ++c) HIP_TRY(hipStreamSynchronize(s->classes[c].st));
    const int64_t t1 = rcpsp_server_now_ns();
    // read back the control blocks and the queues' abort flags
    HIP_TRY(hipMemcpy(s->h_req, s->d_req, sizeof(ServeReq) * s->slot_req.size(), hipMemcpyDeviceToHost));
    for (int c = 0; c < nc; ++c) {
        ServeQueue q{};
        HIP_TRY(hipMemcpy(&q, s->classes[c].d_q, sizeof(ServeQueue), hipMemcpyDeviceToHost));
        if (q.abort) return fail(RCPSP_E_DEVICE, "serving class %d: a wait inside the kernel exceeded its limit", c);
    }
    std::lock_guard<std::mutex> g(s->mu);
    if (launched) {
        ++s->stats.slices;
        s->stats.busy_ms += (double)(t1 - t0) * 1e-6;
    }
    for (Req *r : active) {
        const ServeReq &q = s->h_req[r->slot];
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
        } else {
            return fail(RCPSP_E_DEVICE, "request %lld left a slice without a next iteration", (long long)r->ticket);
        }
    }
    s->cv_idle.notify_all();
    return RCPSP_OK;
}

void loop(rcpsp_server *s) {
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) {
        set_failed(s, RCPSP_E_DEVICE, "hipSetDevice failed in the server thread");
        return;
    }
    for (;;) {
        {
            std::unique_lock<std::mutex> g(s->mu);
            s->cv_work.wait(g, [&] { return s->stop || !s->queue.empty() || s->running > 0; });
            if (s->stop) return;
        }
        std::vector<Req *> fresh;
        admit(s, fresh);
        bool any;
        {
            std::lock_guard<std::mutex> g(s->mu);
            any = s->running > 0;
        }
        if (!any) {
            // queue blocked by arena room or slots held by unreleased requests
            std::unique_lock<std::mutex> g(s->mu);
            s->cv_idle.notify_all();
            s->cv_work.wait_for(g, std::chrono::milliseconds(1));
            continue;
        }
        rcpsp_status st = run_slice(s, fresh);
        if (st != RCPSP_OK) {
            set_failed(s, st, rcpsp_last_error());
            return;
        }
    }
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
    int khz = 0;
    SRV_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device));
    if (khz <= 0) return bail(fail(RCPSP_E_DEVICE, "device wall clock rate unknown"));
    s->ticks_per_ns = (double)khz * 1e-6;
    SRV_TRY(s->arena.init((size_t)s->prm.arena_bytes));
    const size_t slots = (size_t)s->prm.max_active;
    SRV_TRY(hipMalloc(&s->d_items, sizeof(SearchArgs) * slots));
    SRV_TRY(hipMalloc(&s->d_req, sizeof(ServeReq) * slots));
    SRV_TRY(hipHostMalloc(&s->h_items, sizeof(SearchArgs) * slots, hipHostMallocDefault));
    SRV_TRY(hipHostMalloc(&s->h_req, sizeof(ServeReq) * slots, hipHostMallocDefault));
    SRV_TRY(hipHostMalloc(&s->h_one, sizeof(int), hipHostMallocDefault));
    std::memset(s->h_req, 0, sizeof(ServeReq) * slots);
    SRV_TRY(hipMemcpy(s->d_req, s->h_req, sizeof(ServeReq) * slots, hipMemcpyHostToDevice));
    SRV_TRY(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
    {
        std::vector<uint32_t> E = decay_table();
        SRV_TRY(hipMalloc(&s->d_decay, sizeof(uint32_t) * E.size()));
        SRV_TRY(hipMemcpy(s->d_decay, E.data(), sizeof(uint32_t) * E.size(), hipMemcpyHostToDevice));
        s->decay_len = (int)E.size();
    }
    // host <-> device wall-clock mapping
    SRV_TRY(hipMalloc(&s->d_clock, sizeof(long long)));
    {
        const int64_t a = rcpsp_server_now_ns();
        SRV_TRY(launch_clock(s->d_clock, s->st));
        SRV_TRY(hipStreamSynchronize(s->st));
        const int64_t b = rcpsp_server_now_ns();
        SRV_TRY(hipMemcpy(&s->dev0, s->d_clock, sizeof(long long), hipMemcpyDeviceToHost));
        s->host0 = (a + b) / 2;
    }
#undef SRV_TRY
    s->slot_req.assign(slots, nullptr);
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
    }
    if (s->st) (void)hipStreamDestroy(s->st);
    if (s->d_items) (void)hipFree(s->d_items);
    if (s->d_req) (void)hipFree(s->d_req);
    if (s->h_items) (void)hipHostFree(s->h_items);
    if (s->h_req) (void)hipHostFree(s->h_req);
    if (s->h_one) (void)hipHostFree(s->h_one);
    if (s->d_decay) (void)hipFree(s->d_decay);
    if (s->d_clock) (void)hipFree(s->d_clock);
    delete s;
}

extern "C" rcpsp_status rcpsp_server_submit(rcpsp_server *s, const rcpsp_instance *inst,
                                            const rcpsp_search_params *params, int64_t budget_us, int64_t *ticket) {
    if (!s || !inst || !params || !ticket) return fail(RCPSP_E_ARG, "null pointer");
    rcpsp_status st = validate_params(*params);
    if (st != RCPSP_OK) return st;
    if (params->iterations < 1) return fail(RCPSP_E_ARG, "a served request needs an iteration allowance >= 1");
    if (budget_us < 0) return fail(RCPSP_E_ARG, "negative budget");
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
    Req *r = new (std::nothrow) Req();
    if (!r) return fail(RCPSP_E_NOMEM, "out of host memory");
    r->inst = inst;
    r->p = *params;
    r->budget_us = budget_us;
    r->bytes = m.total;
    r->submit_ns = rcpsp_server_now_ns();
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->failed) {
            delete r;
            return fail(s->fail_st, "server failed: %s", s->fail_msg.c_str());
        }
        r->ticket = s->next_ticket++;
        s->reqs[r->ticket] = r;
        s->queue.push_back(r);
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
    auto idle = [&] { return s->failed || (s->queue.empty() && s->running == 0); };
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
    out->queued = (int32_t)s->queue.size();
    out->arena_used = (int64_t)s->arena.used();
    out->arena_bytes = (int64_t)s->arena.size();
    return RCPSP_OK;
}
