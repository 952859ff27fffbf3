// Kernel translation unit: the plain kernels (reset, exchange round, fills,
// device clock), the set-up kernels (forward-backward improvement, record
// decodes) and their launchers; the iteration, batch and serving kernels
// live in translation units of their own (rcpsp_k_*.hip) so that they
// compile side by side.
#define RCPSP_PLAIN_KERNELS
#include "rcpsp_device.h"

namespace rcpsp {

hipError_t launch_reset(const SearchArgs &A, hipStream_t st) {
    const int g = A.B > A.NF ? A.B : A.NF;
    hipLaunchKernelGGL(k_reset, dim3(g), dim3(64), 0, st, A);
    return hipGetLastError();
}

size_t round_lds_bytes(int B, int NF) { return sizeof(int) * (6 * (size_t)B + 5 * (size_t)NF); }

// Raise the dynamic LDS limit of the search kernels (outside graph capture).
hipError_t prepare_search(int T, int nw, int dec, int G, size_t lds, int B, int NF) {
    RCPSP_DISPATCH(nw, T, dec, G, {
        hipError_t e = set_lds(k_decode_records<NW_, T_, DEC_>, lds);
        if (e != hipSuccess) return e;
        e = set_lds(k_fbi<NW_, T_, DEC_>, lds);
        if (e != hipSuccess) return e;
    });
    hipError_t e = prepare_search_kernels(T, nw, dec, G, lds);
    if (e != hipSuccess) return e;
    if ((e = prepare_count_kernels(T, nw, dec, G, lds)) != hipSuccess) return e;
    if (NF > 0) return set_lds(k_round, round_lds_bytes(B, NF));
    return hipSuccess;
}

hipError_t launch_search(const SearchArgs &A, int T, int nw, int dec, int G, size_t lds, hipStream_t st) {
    return A.count_work ? launch_search_count(A, T, nw, dec, G, lds, st) : launch_search_plain(A, T, nw, dec, G, lds, st);
}

hipError_t launch_fbi(const SearchArgs &A, int T, int nw, int dec, size_t lds, hipStream_t st) {
    const int units = A.NF > 0 ? A.NF : A.B;
    if (units < 2) return hipSuccess;
    // the set-up kernels run at the plan's threads (512 exist for two layouts only)
    RCPSP_DISPATCH(nw, T, dec, setup_layout(T, dec), {
        hipLaunchKernelGGL((k_fbi<NW_, T_, DEC_>), dim3(units / 2), dim3(T_), lds, st, A);
    });
    return hipGetLastError();
}

hipError_t launch_decode_records(const SearchArgs &A, int T, int nw, int dec, size_t lds, hipStream_t st) {
    RCPSP_DISPATCH(nw, T, dec, setup_layout(T, dec), {
        hipLaunchKernelGGL((k_decode_records<NW_, T_, DEC_>), dim3(A.NF), dim3(T_), lds, st, A);
    });
    return hipGetLastError();
}

hipError_t launch_fill_zero(int *p, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

size_t batch_queue_bytes() { return sizeof(BatchQueue); }

hipError_t launch_serve_begin(ServeQueue *q, unsigned long long *tasks, long long cap, long long n0,
                              hipStream_t st) {
    const long long n = cap > 1 ? cap : 1;
    hipLaunchKernelGGL(k_serve_begin, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, q, tasks, cap, n0);
    return hipGetLastError();
}

hipError_t launch_clock(long long *out, hipStream_t st) {
    hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, st, out);
    return hipGetLastError();
}

hipError_t launch_round(const SearchArgs &A, int parity, int init, hipStream_t st) {
    const size_t lds = round_lds_bytes(A.B, A.NF);
    hipLaunchKernelGGL(k_round, dim3(1), dim3(256), lds, st, A, parity, init);
    return hipGetLastError();
}

}  // namespace rcpsp
