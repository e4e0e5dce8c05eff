// Host side of the streamed 16-frame tile variant (kernel in fit_stile.h): its
// class for a shape and the launches.
#include "fit_stile.h"

namespace isnmf {
namespace {

template <int KS>
hipError_t run(const FitDesc *a, int b, const FitDesc *d, const int2 *items, int n,
               const long long *cur, const int *beff, const FitDesc *tab, const ServeWork *work,
               int tiles, hipStream_t s) {
    constexpr size_t lds = stile::lds_bytes(KS);
    if (work) {
        stile::fit_stile_work_kernel<KS><<<dim3(n, tiles), stile::NWT * 64, lds, s>>>(tab, work);
    } else if (d) {
        stile::fit_stile_multi_kernel<KS><<<n, stile::NWT * 64, lds, s>>>(d, items, cur, beff);
    } else {
        stile::fit_stile_kernel<KS><<<(b + stile::FPW - 1) / stile::FPW, stile::NWT * 64, lds, s>>>(*a);
    }
    return hipGetLastError();
}

hipError_t launch(const FitClass &c, const FitDesc *a, int b, const FitDesc *d, const int2 *items,
                  int n, const long long *cur, const int *beff, const FitDesc *tab,
                  const ServeWork *work, int tiles, hipStream_t s) {
    if (!c.ok || c.cpw != -2 || c.nw != stile::NWT) return hipErrorNotSupported;
    switch (c.kmax) {
        case 32: return run<1>(a, b, d, items, n, cur, beff, tab, work, tiles, s);
        case 64: return run<2>(a, b, d, items, n, cur, beff, tab, work, tiles, s);
        case 96: return run<3>(a, b, d, items, n, cur, beff, tab, work, tiles, s);
        case 128: return run<4>(a, b, d, items, n, cur, beff, tab, work, tiles, s);
        default: return hipErrorNotSupported;
    }
}

}  // namespace

// Streamed 16-frame tile variant (BF16 products): 8 waves of 16 frames, the W
// operands streamed through LDS one 32-row step at a time; F <= 2048, K <= 128.
// The class does not depend on F (rf = 0), so streams of any F share a launch.
FitClass stile_class(int F, int K) {
    FitClass c = {};
    const int S = (F + 31) / 32;
    if (F < 1 || K < 1 || K > 32 * stile::KS_MAX || S > stile::S_MAX) return c;
    c.ok = 1;
    c.nw = stile::NWT;
    c.cpw = -2;
    c.kmax = 32 * ((K + 31) / 32);
    c.wg = 0;
    c.rf = 0;
    return c;
}

hipError_t launch_fit_stile(const FitDesc &a, const FitClass &c, int b, hipStream_t s) {
    const FitClass e = stile_class(a.F, a.K);
    if (!e.ok || e.kmax != c.kmax || !a.W16r || !a.W16c) return hipErrorInvalidValue;
    return launch(c, &a, b, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, 0, s);
}

hipError_t launch_fit_stile_multi(const FitClass &c, const FitDesc *d, const int2 *items, int n,
                                  const long long *cur, const int *beff, hipStream_t s) {
    return launch(c, nullptr, 0, d, items, n, cur, beff, nullptr, nullptr, 0, s);
}

hipError_t launch_fit_stile_work(const FitClass &c, const FitDesc *tab, const ServeWork *work, int n,
                                 int tiles, hipStream_t s) {
    return launch(c, nullptr, 0, nullptr, nullptr, n, nullptr, nullptr, tab, work, tiles, s);
}

}  // namespace isnmf
