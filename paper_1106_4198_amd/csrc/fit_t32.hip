// Host side of the FP32 16-frame tile variant (kernel in fit_t32.h): its class
// for a shape and the launches.
#include "fit_t32.h"

namespace isnmf {
namespace {

template <int MT>
hipError_t run(const FitDesc *a, int b, const FitDesc *d, const int2 *items, int n,
               const long long *cur, const int *beff, const FitDesc *tab, const ServeWork *work,
               int tiles, int T, hipStream_t s) {
    const size_t lds = t32::lds_bytes(T, MT);
    if (T < 1 || T > t32::t_max(MT)) return hipErrorInvalidValue;
    // the largest dynamic LDS any launch of the kernel asks for, set once
    static const hipError_t a1 = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&t32::fit_t32_kernel<MT>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)t32::LDS_MAX);
    static const hipError_t a2 = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&t32::fit_t32_multi_kernel<MT>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)t32::LDS_MAX);
    static const hipError_t a3 = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&t32::fit_t32_work_kernel<MT>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)t32::LDS_MAX);
    if (work) {
        if (a3 != hipSuccess) return a3;
        t32::fit_t32_work_kernel<MT><<<dim3(n, tiles), t32::NWT * 64, lds, s>>>(tab, work);
    } else if (d) {
        if (a2 != hipSuccess) return a2;
        t32::fit_t32_multi_kernel<MT><<<n, t32::NWT * 64, lds, s>>>(d, items, cur, beff);
    } else {
        if (a1 != hipSuccess) return a1;
        t32::fit_t32_kernel<MT><<<(b + t32::FPW - 1) / t32::FPW, t32::NWT * 64, lds, s>>>(*a);
    }
    return hipGetLastError();
}

// T comes from the class (rf): every stream of a launch has that many row tiles.
hipError_t launch(const FitClass &c, const FitDesc *a, int b, const FitDesc *d, const int2 *items,
                  int n, const long long *cur, const int *beff, const FitDesc *tab,
                  const ServeWork *work, int tiles, hipStream_t s) {
    if (!c.ok || c.cpw != -3 || c.nw != t32::NWT) return hipErrorNotSupported;
    switch (c.kmax) {
        case 16: return run<1>(a, b, d, items, n, cur, beff, tab, work, tiles, c.rf, s);
        case 32: return run<2>(a, b, d, items, n, cur, beff, tab, work, tiles, c.rf, s);
        case 48: return run<3>(a, b, d, items, n, cur, beff, tab, work, tiles, c.rf, s);
        case 64: return run<4>(a, b, d, items, n, cur, beff, tab, work, tiles, c.rf, s);
        default: return hipErrorNotSupported;
    }
}

}  // namespace

// FP32 16-frame tile variant: 8 waves of 16 frames on 16x16x4 FP32 MFMA, W in
// LDS; K <= 64 and F <= 16 t_max(ceil(K / 16)) (592 at K <= 64, 784 at K <= 48,
// 1136 at K <= 32, 2048 at K <= 16).  rf = ceil(F / 16) row tiles.
FitClass t32_class(int F, int K) {
    FitClass c = {};
    if (F < 1 || K < 1 || K > 16 * t32::MT_MAX) return c;
    const int MT = (K + 15) / 16;
    const int T = (F + 15) / 16;
    if (T > t32::t_max(MT)) return c;
    c.ok = 1;
    c.nw = t32::NWT;
    c.cpw = -3;
    c.kmax = 16 * MT;
    c.wg = 0;
    c.rf = T;
    return c;
}

hipError_t launch_fit_t32(const FitDesc &a, const FitClass &c, int b, hipStream_t s) {
    const FitClass e = t32_class(a.F, a.K);
    if (!e.ok || e.rf != c.rf || e.kmax != c.kmax || !a.W) return hipErrorInvalidValue;
    return launch(c, &a, b, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, 0, s);
}

hipError_t launch_fit_t32_multi(const FitClass &c, const FitDesc *d, const int2 *items, int n,
                                const long long *cur, const int *beff, hipStream_t s) {
    return launch(c, nullptr, 0, d, items, n, cur, beff, nullptr, nullptr, 0, s);
}

hipError_t launch_fit_t32_work(const FitClass &c, const FitDesc *tab, const ServeWork *work, int n,
                               int tiles, hipStream_t s) {
    return launch(c, nullptr, 0, nullptr, nullptr, n, nullptr, nullptr, tab, work, tiles, s);
}

}  // namespace isnmf
