// Host runtime objects shared by the library's translation units
// (library-internal): instances, search plans, error reporting.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "rcpsp.h"
#include "rcpsp_internal.h"

namespace rcpsp {

// Sets the calling thread's last-error message; returns st.
rcpsp_status fail(rcpsp_status st, const char *fmt, ...);

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::rcpsp::fail(e_ == hipErrorOutOfMemory ? RCPSP_E_NOMEM : RCPSP_E_DEVICE, "%s: %s (%s:%d)", \
                                 #expr, hipGetErrorString(e_), __FILE__, __LINE__);           \
    } while (0)

// Source of a plan's device buffers other than hipMalloc (a server's arena).
struct DeviceAllocator {
    virtual hipError_t alloc(void **ptr, size_t bytes) = 0;
    virtual void release(void *ptr) = 0;
    virtual ~DeviceAllocator() = default;
};

int potential_moves(int n, int delta);
std::vector<uint32_t> decay_table();

}  // namespace rcpsp

struct rcpsp_instance {
    int n = 0, m = 0, n_arcs = 0, H = 0, cp = 0, eval = 0, dmax = 0;
    std::vector<int> d, R, r, succ_off, succ, pred_off, pred;
    rcpsp::InstDesc desc{};
    uint32_t *d_blob = nullptr;
    int device = 0;
    rcpsp_info info{};
};

struct rcpsp_search {
    const rcpsp_instance *inst = nullptr;
    rcpsp_search_params p{};
    int T = 64, L = 0, nw = 1, dec = 1, tcw = 1, P = 0;
    int G = 1;            // layout: 1 one candidate per lane, 2 the same with 8-bit finish
                          // times, 16 one candidate per 16 lanes (time-indexed)
    int reserve = 256;    // static LDS of the kernel the plan runs in
    rcpsp::Layout Ly{};
    size_t lds = 0;
    rcpsp::SearchArgs a{};
    std::vector<void *> allocs;
    rcpsp::DeviceAllocator *allocator = nullptr;   // null: hipMalloc / hipFree
    const uint32_t *shared_decay = nullptr;        // eq. 8 table owned elsewhere
    int shared_decay_len = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int iteration_launches = 0, round_launches = 0;
};

namespace rcpsp {

// Layout and device state of a plan (no launches, no graph).
rcpsp_status alloc_plan(rcpsp_search *s);
// Neighbourhood evaluation of device arrays (allocates nothing): launch shape
// chosen for the instance, one workgroup, asynchronous on st.
rcpsp_status eval_device(const rcpsp_instance *I, const int32_t *order, int32_t delta, const uint8_t *tabu,
                         int32_t asp, int32_t *makespan, rcpsp_move *best, hipStream_t st);
// order is a precedence-feasible permutation with w_0 = 0 and w_{N-1} = N-1.
bool feasible_order(const rcpsp_instance *I, const int32_t *order);
rcpsp_status validate_params(const rcpsp_search_params &p);

}  // namespace rcpsp
