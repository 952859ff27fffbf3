// Kernel translation unit: the persistent batch kernel k_batch.
#include "rcpsp_device.h"

namespace rcpsp {

hipError_t prepare_batch(int T, int nw, int dec, int G, size_t lds) {
    RCPSP_DISPATCH(nw, T, dec, G, {
        hipError_t e = set_lds(k_batch<NW_, T_, DEC_, G_>, lds);
        if (e != hipSuccess) return e;
    });
    return hipSuccess;
}

hipError_t batch_occupancy(int T, int nw, int dec, int G, size_t lds, int *per_cu) {
    *per_cu = 0;
    RCPSP_DISPATCH(nw, T, dec, G, {
        hipError_t e = set_lds(k_batch<NW_, T_, DEC_, G_>, lds);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch<NW_, T_, DEC_, G_>, T_, lds);
        if (e != hipSuccess) return e;
    });
    return hipSuccess;
}

hipError_t launch_batch(const BatchClassArgs &C, int grid, int T, int nw, int dec, int G, size_t lds,
                        hipStream_t st) {
    RCPSP_DISPATCH(nw, T, dec, G, {
        hipLaunchKernelGGL((k_batch<NW_, T_, DEC_, G_>), dim3(grid), dim3(T_), lds, st, C);
    });
    return hipGetLastError();
}

}  // namespace rcpsp
