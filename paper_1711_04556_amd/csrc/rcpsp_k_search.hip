// Kernel translation unit: the iteration kernel k_search (plain runs).
#include "rcpsp_device.h"

namespace rcpsp {

hipError_t prepare_search_kernels(int T, int nw, int dec, int G, size_t lds) {
    RCPSP_DISPATCH(nw, T, dec, G, {
        hipError_t e = set_lds(k_search<NW_, T_, DEC_, G_, false>, lds);
        if (e != hipSuccess) return e;
    });
    return hipSuccess;
}

hipError_t launch_search_plain(const SearchArgs &A, int T, int nw, int dec, int G, size_t lds, hipStream_t st) {
    RCPSP_DISPATCH(nw, T, dec, G, {
        const int grid = A.grid > 0 ? A.grid : A.B;
        hipLaunchKernelGGL((k_search<NW_, T_, DEC_, G_, false>), dim3(grid), dim3(T_), lds, st, A);
    });
    return hipGetLastError();
}

hipError_t search_occupancy(int T, int nw, int dec, int G, size_t lds, int *per_cu) {
    *per_cu = 0;
    RCPSP_DISPATCH(nw, T, dec, G, {
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_search<NW_, T_, DEC_, G_, false>, T_, lds);
        if (e != hipSuccess) return e;
    });
    return hipSuccess;
}

}  // namespace rcpsp
