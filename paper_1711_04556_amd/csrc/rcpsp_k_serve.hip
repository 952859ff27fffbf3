// Kernel translation unit: the serving kernel k_serve.
#include "rcpsp_device.h"

namespace rcpsp {

hipError_t serve_occupancy(int T, int nw, int dec, int G, size_t lds, int *per_cu) {
    *per_cu = 0;
    RCPSP_DISPATCH(nw, T, dec, G, {
        hipError_t e = set_lds(k_serve<NW_, T_, DEC_, G_>, lds);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_serve<NW_, T_, DEC_, G_>, T_, lds);
        if (e != hipSuccess) return e;
    });
    return hipSuccess;
}

hipError_t launch_serve(const ServeArgs &C, int grid, int T, int nw, int dec, int G, size_t lds, hipStream_t st) {
    RCPSP_DISPATCH(nw, T, dec, G, {
        hipLaunchKernelGGL((k_serve<NW_, T_, DEC_, G_>), dim3(grid), dim3(T_), lds, st, C);
    });
    return hipGetLastError();
}

}  // namespace rcpsp
