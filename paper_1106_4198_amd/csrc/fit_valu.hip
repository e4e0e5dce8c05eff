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
constexpr int VALU_RF_MAX = 17;     // F <= 1088 (8 waves)
constexpr int VALU16_RF_MAX = 9;    // 1088 < F <= 1152 (16 waves)
constexpr int VALU_CK_MAX = 8;      // K <= 64

// rows per row set of the class's workgroup
int rows_per_set(const FitClass &c) { return 8 * c.nw; }

// cpw 0: FP32 products (8 or 16 waves); cpw -4: bf16 products on
// v_dot2c_f32_bf16 (8 waves).
hipError_t launch(const FitClass &c, const FitDesc *a, int b, const FitDesc *d, const int2 *items,
                  int n, const long long *cur, const int *beff, const FitDesc *tab,
                  const ServeWork *work, int max_b, hipStream_t s) {
    if (!c.ok || (c.cpw != 0 && c.cpw != -4) || c.kmax % 8 != 0) return hipErrorNotSupported;
    if (c.nw != 8 && !(c.nw == 16 && c.cpw == 0)) return hipErrorNotSupported;
    const bool bf = c.cpw == -4, w16 = c.nw == 16;
    switch (c.kmax / 8) {
#define ISNMF_VALU_CK(CKV)                                                                          \
    case CKV:                                                                                       \
        return bf    ? valu::launch_any<CKV, true, 8>(a, c.rf, b, d, items, n, cur, beff, tab, work, \
                                                      max_b, s)                                     \
               : w16 ? valu::launch_any<CKV, false, 16>(a, c.rf, b, d, items, n, cur, beff, tab,    \
                                                        work, max_b, s)                             \
                     : valu::launch_any<CKV, false, 8>(a, c.rf, b, d, items, n, cur, beff, tab,     \
                                                       work, max_b, s);
        ISNMF_VALU_CK(1) ISNMF_VALU_CK(2) ISNMF_VALU_CK(3) ISNMF_VALU_CK(4)
        ISNMF_VALU_CK(5) ISNMF_VALU_CK(6) ISNMF_VALU_CK(7) ISNMF_VALU_CK(8)
#undef ISNMF_VALU_CK
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

FitClass valu16_class(int F, int K) {
    FitClass c = {};
    const int rf = (F + 127) / 128, ck = (K + 7) / 8;
    if (F <= 64 * VALU_RF_MAX || K < 1 || rf > VALU16_RF_MAX || ck > VALU_CK_MAX) return c;
    c.ok = 1;
    c.nw = 16;
    c.cpw = 0;
    c.kmax = 8 * ck;
    c.wg = 0;
    c.rf = rf;
    return c;
}

FitClass vbf_class(int F, int K) {
    FitClass c = valu_class(F, K);
    if (c.ok) c.cpw = -4;
    return c;
}

hipError_t launch_fit_valu(const FitDesc &a, const FitClass &c, int b, hipStream_t s) {
    const int pr = rows_per_set(c);
    if (c.rf != (a.F + pr - 1) / pr || c.kmax < a.K || (c.nw == 8 && !a.Wv))
        return hipErrorInvalidValue;
    return launch(c, &a, b, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, 0, s);
}

hipError_t launch_fit_valu_multi(const FitClass &c, const FitDesc *d, const int2 *items, int n,
                                 const long long *cur, const int *beff, hipStream_t s) {
    return launch(c, nullptr, 0, d, items, n, cur, beff, nullptr, nullptr, 0, s);
}

hipError_t launch_fit_valu_work(const FitClass &c, const FitDesc *tab, const ServeWork *work, int n,
                                int max_b, hipStream_t s) {
    if (n < 1 || max_b < 1) return hipSuccess;
    return launch(c, nullptr, 0, nullptr, nullptr, n, nullptr, nullptr, tab, work, max_b, s);
}

}  // namespace isnmf
