// Kernel wrappers and variant dispatch of the fused fit for one product
// precision (included once per precision by fit_f32.hip, fit_bf16.hip,
// fit_f16.hip so the variants compile in parallel).
#pragma once

#include "fit_body.h"

namespace isnmf {
namespace {

template <int NW, int CPW, int KMAX, int PREC, bool WG>
__global__ __launch_bounds__(NW * 64) void fit_single_kernel(FitDesc a) {
    fit_body<NW, CPW, KMAX, PREC, WG>(a, blockIdx.x);
}

// Batched form: item = (stream, tile); the tile's frames start at
// cursor[stream] in that stream's V; beff[stream] frames are fitted this step.
template <int NW, int CPW, int KMAX, int PREC, bool WG>
__global__ __launch_bounds__(NW * 64) void fit_multi_kernel(const FitDesc *__restrict__ descs,
                                                            const int2 *__restrict__ items,
                                                            const long long *__restrict__ cursor,
                                                            const int *__restrict__ beff) {
    const int2 it = items[blockIdx.x];
    const int b = beff[it.x];
    if (it.y * NF >= b) return;   // tile past this step's minibatch (uniform per block)
    FitDesc a = descs[it.x];
    const long long c = cursor[it.x];
    a.b = b;
    a.V += c * a.ldv;
    if (a.Hb) a.Hb += c * a.ldh;
    fit_body<NW, CPW, KMAX, PREC, WG>(a, it.y);
}

template <int NW, int CPW, int KMAX, int PREC, bool WG>
struct Launch {
    static hipError_t single(const FitDesc &a, int grid, hipStream_t s) {
        fit_single_kernel<NW, CPW, KMAX, PREC, WG><<<grid, NW * 64, 0, s>>>(a);
        return hipGetLastError();
    }
    static hipError_t multi(const FitDesc *d, const int2 *it, int n, const long long *cur,
                            const int *beff, hipStream_t s) {
        fit_multi_kernel<NW, CPW, KMAX, PREC, WG><<<n, NW * 64, 0, s>>>(d, it, cur, beff);
        return hipGetLastError();
    }
};

// Calls F<NW, CPW, KMAX, PREC, WG> for the class, or returns hipErrorNotSupported.
template <int PREC, template <int, int, int, int, bool> class L, typename... Args>
hipError_t dispatch(const FitClass &c, Args... args) {
#define ISNMF_K(NW, CPW, WG)                                                            \
    switch (c.kmax) {                                                                   \
        case 8: return L<NW, CPW, 8, PREC, WG>::run(args...);                           \
        case 16: return L<NW, CPW, 16, PREC, WG>::run(args...);                         \
        case 24: return L<NW, CPW, 24, PREC, WG>::run(args...);                         \
        case 32: return L<NW, CPW, 32, PREC, WG>::run(args...);                         \
        case 40: return L<NW, CPW, 40, PREC, WG>::run(args...);                         \
        case 52: return L<NW, CPW, 52, PREC, WG>::run(args...);                         \
        case 64: return L<NW, CPW, 64, PREC, WG>::run(args...);                         \
        default: break;                                                                 \
    }
#define ISNMF_K16(NW, CPW, WG)                                                          \
    switch (c.kmax) {                                                                   \
        case 80: return L<NW, CPW, 80, PREC, WG>::run(args...);                         \
        case 96: return L<NW, CPW, 96, PREC, WG>::run(args...);                         \
        case 112: return L<NW, CPW, 112, PREC, WG>::run(args...);                       \
        case 128: return L<NW, CPW, 128, PREC, WG>::run(args...);                       \
        default: break;                                                                 \
    }
    if (!c.wg && c.cpw == 1) {
        switch (c.nw) {
            case 1: { ISNMF_K(1, 1, false) if constexpr (PREC != 0) { ISNMF_K16(1, 1, false) } break; }
            case 2: { ISNMF_K(2, 1, false) if constexpr (PREC != 0) { ISNMF_K16(2, 1, false) } break; }
            case 4: { ISNMF_K(4, 1, false) if constexpr (PREC != 0) { ISNMF_K16(4, 1, false) } break; }
            case 8: { ISNMF_K(8, 1, false) if constexpr (PREC != 0) { ISNMF_K16(8, 1, false) } break; }
            default: break;
        }
    }
    if constexpr (PREC != 0) {
        if (!c.wg && c.cpw == 2 && c.nw == 8) { ISNMF_K(8, 2, false) }
        if (!c.wg && c.cpw == 2 && c.nw == 4) { ISNMF_K(4, 2, false) }
        if (c.wg && c.cpw == 1 && c.nw == 16) { ISNMF_K(16, 1, true) ISNMF_K16(16, 1, true) }
    }
#undef ISNMF_K
#undef ISNMF_K16
    return hipErrorNotSupported;
}

template <int NW, int CPW, int KMAX, int PREC, bool WG>
struct SingleL {
    static hipError_t run(const FitDesc &a, int grid, hipStream_t s) {
        return Launch<NW, CPW, KMAX, PREC, WG>::single(a, grid, s);
    }
};
template <int NW, int CPW, int KMAX, int PREC, bool WG>
struct MultiL {
    static hipError_t run(const FitDesc *d, const int2 *it, int n, const long long *cur,
                          const int *beff, hipStream_t s) {
        return Launch<NW, CPW, KMAX, PREC, WG>::multi(d, it, n, cur, beff, s);
    }
};

}  // namespace

#define ISNMF_INSTANTIATE_FIT(PREC)                                                         \
    template <>                                                                             \
    hipError_t launch_fit_single_p<PREC>(const FitDesc &a, const FitClass &c, int grid,    \
                                         hipStream_t s) {                                   \
        return dispatch<PREC, SingleL>(c, a, grid, s);                                      \
    }                                                                                       \
    template <>                                                                             \
    hipError_t launch_fit_multi_p<PREC>(const FitClass &c, const FitDesc *d, const int2 *it, \
                                        int n, const long long *cur, const int *beff,       \
                                        hipStream_t s) {                                    \
        return dispatch<PREC, MultiL>(c, d, it, n, cur, beff, s);                           \
    }

}  // namespace isnmf
