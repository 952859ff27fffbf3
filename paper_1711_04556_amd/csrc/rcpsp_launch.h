// Host-side launch entry points of the HIP kernels (library-internal).
#pragma once

#include <hip/hip_runtime.h>

#include "rcpsp_internal.h"

namespace rcpsp {

struct EvalArgs {
    InstDesc D;
    Layout Ly;
    int delta, L, aspiration, P;
    const int32_t *order;   // device [N]
    const uint8_t *tabu;    // device [N*N] or null
    int32_t *makespan;      // device [P] or null
    int32_t *best;          // device [4]
};

hipError_t launch_eval(const EvalArgs &A, int T, int nw, int dec, int G, size_t lds, hipStream_t st);
hipError_t launch_reset(const SearchArgs &A, hipStream_t st);
hipError_t launch_decode_records(const SearchArgs &A, int T, int nw, int dec, size_t lds, hipStream_t st);
hipError_t launch_fbi(const SearchArgs &A, int T, int nw, int dec, size_t lds, hipStream_t st);
hipError_t search_occupancy(int T, int nw, int dec, int G, size_t lds, int *per_cu);
hipError_t launch_search(const SearchArgs &A, int T, int nw, int dec, int G, size_t lds, hipStream_t st);
hipError_t launch_round(const SearchArgs &A, int parity, int init, hipStream_t st);
size_t round_lds_bytes(int B, int NF);
hipError_t prepare_search(int T, int nw, int dec, int G, size_t lds, int B, int NF);
// parts of the two above that live in the iteration-kernel translation units
hipError_t prepare_search_kernels(int T, int nw, int dec, int G, size_t lds);
hipError_t prepare_count_kernels(int T, int nw, int dec, int G, size_t lds);
hipError_t launch_search_plain(const SearchArgs &A, int T, int nw, int dec, int G, size_t lds, hipStream_t st);
hipError_t launch_search_count(const SearchArgs &A, int T, int nw, int dec, int G, size_t lds, hipStream_t st);

struct BatchQueue;

// Static LDS of the batch kernel (its plan arguments and step scratch) is below this.
constexpr int kBatchStaticLds = 1024;

// One class of a batch: the tasks of its members (see k_batch).
struct BatchClassArgs {
    const SearchArgs *items;   // every plan of the batch
    const int *order;          // [count] plan index of member j; members sorted by steps, descending
    const int *cumB;           // [count + 1] searches of members before j
    const long long *off;      // [max_steps + 1] first task of each iteration (set-up tasks come first)
    const int *act;            // [max_steps] members taking part in iteration it (a prefix of order)
    int *epoch;                // [count] 1 + exchange rounds completed (0: not set up)
    int *done;                 // [count] search tasks completed
    BatchQueue *q;             // next task, abort flag
    int count, max_steps;
    long long total;           // tasks
    long long wait_ticks;      // limit of one wait, in wall-clock ticks (100 MHz)
};

size_t batch_queue_bytes();
hipError_t prepare_batch(int T, int nw, int dec, int G, size_t lds);
hipError_t batch_occupancy(int T, int nw, int dec, int G, size_t lds, int *per_cu);
hipError_t launch_batch(const BatchClassArgs &C, int grid, int T, int nw, int dec, int G, size_t lds,
                        hipStream_t st);
hipError_t launch_fill_zero(int *p, long long n, hipStream_t st);

// Serving: per-request control block in device memory (64 bytes).
struct ServeReq {
    int next_iter;       // iteration the host must queue (task queue was full); -1 set-up or none, -2 queued on the device
    int done;            // searches done in the current iteration
    int finished;        // 1 once the request's search has ended
    int replay_iters;    // search steps run per search (iterations of an equal plain run)
    int best;            // global best at the end
    int max_iters;       // iteration allowance (eq. 8's I_block)
    int cancel;          // set by the host: end at the next iteration boundary
    int pad0;
    long long deadline;  // wall-clock ticks: no iteration starts after it
    long long done_ticks;
    long long evals;
    long long pad1;
};

struct ServeQueue {
    unsigned long long head, tail;
    long long pending;   // tasks published and not finished
    int abort;
    int pad[9];
};

// One class of a serving slice (see k_serve).
struct ServeArgs {
    const SearchArgs *items;    // [slots] plan arguments per request slot
    ServeReq *req;              // [slots]
    unsigned long long *tasks;  // [cap] 0 = empty, else task + 1
    ServeQueue *q;
    long long cap;
    long long slice_end;        // wall-clock ticks: no task is taken after it
    long long wait_ticks;       // limit of one wait
};

// Marks a task slot whose task has run.
constexpr unsigned long long kServeTaskDone = ~0ull;

// Iteration field of the search tasks of a request that ends before its
// first iteration (its budget ran out during set-up): each task completes
// its search's set-up (initial decode, first read) and runs no iteration.
constexpr int kServeNoIteration = (1 << 27) - 1;

// task: slot (20 bits) | kind (1: search step, 0: set-up) | search (16 bits) | iteration (27 bits)
__host__ __device__ inline unsigned long long serve_task(int slot, int kind, int b, int it) {
    return ((unsigned long long)slot << 44) | ((unsigned long long)kind << 43) | ((unsigned long long)b << 27) |
           (unsigned long long)it;
}

hipError_t serve_occupancy(int T, int nw, int dec, int G, size_t lds, int *per_cu);
hipError_t launch_serve(const ServeArgs &C, int grid, int T, int nw, int dec, int G, size_t lds, hipStream_t st);
hipError_t launch_serve_begin(ServeQueue *q, unsigned long long *tasks, long long cap, long long n0,
                              hipStream_t st);
hipError_t launch_clock(long long *out, hipStream_t st);

}  // namespace rcpsp
