// Host side of the FP32 16-frame tile variant (kernel in fit_t32.h): its class
// for a shape and the launches.
#include "fit_t32.h"

namespace isnmf {
namespace t32 {
ISNMF_T32_EXTERN(1)
ISNMF_T32_EXTERN(2)
ISNMF_T32_EXTERN(3)
ISNMF_T32_EXTERN(4)
}  // namespace t32

namespace {

// Split of K components: MT m-tiles on the matrix pipe and KR <= 4 on the
// VALU (K = 16 MT + KR when K mod 16 <= 4, else MT = ceil(K / 16), KR = 0).
void split_k(int K, int &MT, int &KR) {
    const int q = K / 16, r = K % 16;
    if (q >= 1 && r <= 4) {
        MT = q;
        KR = r;
    } else {
        MT = q + 1;
        KR = 0;
    }
}

// The class's kmax is K itself, so streams that share a launch share the split.
hipError_t launch(const FitClass &c, const FitDesc *a, int b, const FitDesc *d, const int2 *items,
                  int n, const long long *cur, const int *beff, const FitDesc *tab,
                  const ServeWork *work, int tiles, bool fold, hipStream_t s) {
    if (!c.ok || c.cpw != -3 || c.nw != t32::NWT || c.kmax < 1 || c.kmax > 16 * t32::MT_MAX)
        return hipErrorNotSupported;
    int MT, KR;
    split_k(c.kmax, MT, KR);
    switch (MT) {
#define ISNMF_T32_MT(M)                                                                          \
    case M:                                                                                      \
        return t32::launch_mt<M>(KR, a, b, d, items, n, cur, beff, tab, work, tiles, c.rf, fold, s);
        ISNMF_T32_MT(1) ISNMF_T32_MT(2) ISNMF_T32_MT(3) ISNMF_T32_MT(4)
#undef ISNMF_T32_MT
        default: return hipErrorNotSupported;
    }
}

}  // namespace

// FP32 16-frame tile variant: 8 waves of 16 frames on 16x16x4 FP32 MFMA (and
// up to 4 remainder components on the VALU), W in LDS; K <= 64 and F <= 16
// t_max(MT): 592 at K > 52, 784 at K <= 52, 1136 at K <= 36, 2048 at K <= 20.
// rf = ceil(F / 16) row tiles, kmax = K.
FitClass t32_class(int F, int K) {
    FitClass c = {};
    if (F < 1 || K < 1 || K > 16 * t32::MT_MAX) return c;
    int MT, KR;
    split_k(K, MT, KR);
    const int T = (F + 15) / 16;
    if (T > t32::t_max(MT)) return c;
    c.ok = 1;
    c.nw = t32::NWT;
    c.cpw = -3;
    c.kmax = K;
    c.wg = 0;
    c.rf = T;
    return c;
}

hipError_t launch_fit_t32(const FitDesc &a, const FitClass &c, int b, hipStream_t s) {
    const FitClass e = t32_class(a.F, a.K);
    if (!e.ok || e.rf != c.rf || e.kmax != c.kmax || !a.W) return hipErrorInvalidValue;
    return launch(c, &a, b, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, 0, false, s);
}

hipError_t launch_fit_t32_multi(const FitClass &c, const FitDesc *d, const int2 *items, int n,
                                const long long *cur, const int *beff, bool fold, hipStream_t s) {
    if (fold && !t32_fold_fits(c)) return hipErrorNotSupported;
    return launch(c, nullptr, 0, d, items, n, cur, beff, nullptr, nullptr, 0, fold, s);
}

hipError_t launch_fit_t32_work(const FitClass &c, const FitDesc *tab, const ServeWork *work, int n,
                               int tiles, hipStream_t s) {
    return launch(c, nullptr, 0, nullptr, nullptr, n, nullptr, nullptr, tab, work, tiles, false, s);
}

bool t32_fold_fits(const FitClass &c) {
    if (!c.ok || c.cpw != -3 || c.kmax < 1 || c.kmax > 16 * t32::MT_MAX) return false;
    int MT, KR;
    split_k(c.kmax, MT, KR);
    return t32::lds_fold_bytes(c.rf, MT) <= t32::LDS_MAX;
}

}  // namespace isnmf
