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

hipError_t launch_eval(const EvalArgs &A, int T, int nw, int dec, size_t lds, hipStream_t st);
hipError_t launch_reset(const SearchArgs &A, hipStream_t st);
hipError_t launch_decode_records(const SearchArgs &A, int T, int nw, int dec, size_t lds, hipStream_t st);
hipError_t launch_search(const SearchArgs &A, int T, int nw, int dec, size_t lds, hipStream_t st);
hipError_t launch_round(const SearchArgs &A, int parity, int init, hipStream_t st);
size_t round_lds_bytes(int B, int NF);
hipError_t prepare_search(int T, int nw, int dec, size_t lds, int B, int NF);

struct BatchQueue;
size_t batch_queue_bytes();
hipError_t prepare_batch(int T, int nw, int dec, size_t lds);
hipError_t launch_batch(const SearchArgs *items, const int *order, int count, BatchQueue *q, int grid, int T, int nw,
                        int dec, size_t lds, hipStream_t st);
hipError_t launch_batch_queue_reset(BatchQueue *q, int n, hipStream_t st);

}  // namespace rcpsp
