// Kernel translation unit: the work-counting iteration kernel and the
// single-neighbourhood kernel k_eval.
#include "rcpsp_device.h"

namespace rcpsp {

hipError_t prepare_count_kernels(int T, int nw, int dec, int G, size_t lds) {
    RCPSP_DISPATCH(nw, T, dec, G, {
        hipError_t e = set_lds(k_search<NW_, T_, DEC_, G_, true>, lds);
        if (e != hipSuccess) return e;
    });
    return hipSuccess;
}

hipError_t launch_search_count(const SearchArgs &A, int T, int nw, int dec, int G, size_t lds, hipStream_t st) {
    RCPSP_DISPATCH(nw, T, dec, G, {
        const int grid = A.grid > 0 ? A.grid : A.B;
        hipLaunchKernelGGL((k_search<NW_, T_, DEC_, G_, true>), dim3(grid), dim3(T_), lds, st, A);
    });
    return hipGetLastError();
}

hipError_t launch_eval(const EvalArgs &A, int T, int nw, int dec, int G, size_t lds, hipStream_t st) {
    RCPSP_DISPATCH(nw, T, dec, G, {
        hipError_t e = set_lds(k_eval<NW_, T_, DEC_, G_>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_eval<NW_, T_, DEC_, G_>), dim3(1), dim3(T_), lds, st, A);
    });
    return hipGetLastError();
}

}  // namespace rcpsp
