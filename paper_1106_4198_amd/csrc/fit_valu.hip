// Host side of the VALU fit variant (kernel in fit_valu.h): its class for a
// shape and the launches.
#include "fit_valu.h"

namespace isnmf {
namespace valu {
ISNMF_VALU_EXTERN(1)
ISNMF_VALU_EXTERN(2)
ISNMF_VALU_EXTERN(3)
ISNMF_VALU_EXTERN(4)
ISNMF_VALU_EXTERN(5)
ISNMF_VALU_EXTERN(6)
ISNMF_VALU_EXTERN(7)
ISNMF_VALU_EXTERN(8)
}  // namespace valu

namespace {
constexpr int VALU_RF_MAX = 17;   // F <= 1088
constexpr int VALU_CK_MAX = 8;    // K <= 64

hipError_t launch(const FitClass &c, const FitDesc *a, int b, const FitDesc *d, const int2 *items,
                  int n, const long long *cur, const int *beff, hipStream_t s) {
    if (!c.ok || c.cpw != 0 || c.kmax % 8 != 0) return hipErrorNotSupported;
    switch (c.kmax / 8) {
        case 1: return valu::launch_any<1>(a, c.rf, b, d, items, n, cur, beff, s);
        case 2: return valu::launch_any<2>(a, c.rf, b, d, items, n, cur, beff, s);
        case 3: return valu::launch_any<3>(a, c.rf, b, d, items, n, cur, beff, s);
        case 4: return valu::launch_any<4>(a, c.rf, b, d, items, n, cur, beff, s);
        case 5: return valu::launch_any<5>(a, c.rf, b, d, items, n, cur, beff, s);
        case 6: return valu::launch_any<6>(a, c.rf, b, d, items, n, cur, beff, s);
        case 7: return valu::launch_any<7>(a, c.rf, b, d, items, n, cur, beff, s);
        case 8: return valu::launch_any<8>(a, c.rf, b, d, items, n, cur, beff, s);
        default: return hipErrorNotSupported;
    }
}
}  // namespace

FitClass valu_class(int F, int K) {
    FitClass c = {};
    const int rf = (F + 63) / 64, ck = (K + 7) / 8;
    if (F < 1 || K < 1 || rf > VALU_RF_MAX || ck > VALU_CK_MAX) return c;
    c.ok = 1;
    c.nw = valu::VT / 64;
    c.cpw = 0;
    c.kmax = 8 * ck;
    c.wg = 0;
    c.rf = rf;
    return c;
}

hipError_t launch_fit_valu(const FitDesc &a, const FitClass &c, int b, hipStream_t s) {
    if (c.rf != (a.F + 63) / 64 || c.kmax < a.K || !a.Wv) return hipErrorInvalidValue;
    return launch(c, &a, b, nullptr, nullptr, 0, nullptr, nullptr, s);
}

hipError_t launch_fit_valu_multi(const FitClass &c, const FitDesc *d, const int2 *items, int n,
                                 const long long *cur, const int *beff, hipStream_t s) {
    return launch(c, nullptr, 0, d, items, n, cur, beff, s);
}

}  // namespace isnmf
