// rcpsp_evaluate_neighbourhood_noalloc: the host-array neighbourhood
// evaluation staged through a fixed device array instead of allocations.
//
// `scratch` is a file-scope device array.  Its name in host code is only a
// host-side stand-in for the symbol; the device address of each GPU's copy
// comes from hipGetSymbolAddress (called once per device, with that device
// current) and is the only address host code hands to copies and kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rcpsp.h"
#include "rcpsp_internal.h"
#include "rcpsp_launch.h"
#include "rcpsp_runtime.h"

namespace rcpsp {
namespace {

constexpr size_t kScratchBytes = RCPSP_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device).
rcpsp_status scratch_address(void **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(RCPSP_E_DEVICE, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RCPSP_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RCPSP_OK;
}

size_t round256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
}  // namespace rcpsp

using namespace rcpsp;

extern "C" rcpsp_status rcpsp_evaluate_neighbourhood_noalloc(const rcpsp_instance *inst, const int32_t *order,
                                                             int32_t swap_range, const uint8_t *tabu,
                                                             int32_t aspiration, int32_t *makespan, int32_t cap,
                                                             int32_t *n_potential, rcpsp_move *best,
                                                             void *hip_stream) {
    if (!inst || !order) return fail(RCPSP_E_ARG, "null pointer");
    if (swap_range < 1 || swap_range > kMaxDelta)
        return fail(RCPSP_E_ARG, "swap_range %d outside 1..%d", swap_range, kMaxDelta);
    const int n = inst->n;
    const int P = potential_moves(n, swap_range);
    if (n_potential) *n_potential = P;
    if (makespan && cap < P) return fail(RCPSP_E_BUFFER, "makespan buffer holds %d entries, %d needed", cap, P);
    if (!feasible_order(inst, order)) return fail(RCPSP_E_ORDER, "order is not a precedence-feasible permutation");
    // parts of the scratch array: order, makespans, best move, tabu matrix
    const size_t o_order = 0;
    const size_t o_mk = o_order + round256(sizeof(int32_t) * (size_t)n);
    const size_t o_best = o_mk + round256(sizeof(int32_t) * (size_t)(P > 0 ? P : 1));
    const size_t o_tabu = o_best + round256(sizeof(rcpsp_move));
    const size_t need = o_tabu + (tabu ? round256((size_t)n * n) : 0);
    if (need > kScratchBytes)
        return fail(RCPSP_E_TOO_LARGE, "needs %zu bytes of scratch, the fixed array holds %zu", need, kScratchBytes);
    void *base = nullptr;
    rcpsp_status st = scratch_address(&base);
    if (st != RCPSP_OK) return st;
    unsigned char *b = static_cast<unsigned char *>(base);
    int32_t *d_order = reinterpret_cast<int32_t *>(b + o_order);
    int32_t *d_mk = reinterpret_cast<int32_t *>(b + o_mk);
    rcpsp_move *d_best = reinterpret_cast<rcpsp_move *>(b + o_best);
    uint8_t *d_tabu = tabu ? b + o_tabu : nullptr;
    hipStream_t hs = (hipStream_t)hip_stream;
    HIP_TRY(hipMemcpyAsync(d_order, order, sizeof(int32_t) * n, hipMemcpyHostToDevice, hs));
    if (tabu) HIP_TRY(hipMemcpyAsync(d_tabu, tabu, (size_t)n * n, hipMemcpyHostToDevice, hs));
    // the kernel writes every makespan (-1 for infeasible moves) and the best move
    st = eval_device(inst, d_order, swap_range, d_tabu, aspiration, d_mk, d_best, hs);
    if (st != RCPSP_OK) return st;
    rcpsp_move hb{};
    HIP_TRY(hipMemcpyAsync(&hb, d_best, sizeof(rcpsp_move), hipMemcpyDeviceToHost, hs));
    if (makespan && P > 0) HIP_TRY(hipMemcpyAsync(makespan, d_mk, sizeof(int32_t) * P, hipMemcpyDeviceToHost, hs));
    HIP_TRY(hipStreamSynchronize(hs));
    if (best) *best = hb;
    return RCPSP_OK;
}
