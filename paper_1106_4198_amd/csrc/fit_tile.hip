// Host side of the 16-frame tile variant (kernel in fit_tile.h): its class
// for a shape and the launches.
#include "fit_tile.h"

namespace isnmf {
namespace tile {
ISNMF_TILE_EXTERN(1)
ISNMF_TILE_EXTERN(2)
}  // namespace tile

namespace {
hipError_t launch(const FitClass &c, const FitDesc *a, int b, const FitDesc *d, const int2 *items,
                  int n, const long long *cur, const int *beff, bool fold, hipStream_t s) {
    if (!c.ok || c.cpw != -1 || c.nw != tile::NWT) return hipErrorNotSupported;
    if (c.kmax == 32) return tile::launch_ks<1>(c.rf, a, b, d, items, n, cur, beff, fold, s);
    if (c.kmax == 64) return tile::launch_ks<2>(c.rf, a, b, d, items, n, cur, beff, fold, s);
    return hipErrorNotSupported;
}
}  // namespace

// 16-frame tile variant (BF16 products): 8 waves of 16 frames, F <= 640, K <= 64.
FitClass tile_class(int F, int K) {
    FitClass c = {};
    const int S = (F + 31) / 32;
    if (F < 1 || K < 1 || K > 64 || S > tile::S_MAX) return c;
    c.ok = 1;
    c.nw = tile::NWT;
    c.cpw = -1;
    c.kmax = 32 * ((K + 31) / 32);
    c.wg = 0;
    c.rf = S;
    return c;
}

hipError_t launch_fit_tile(const FitDesc &a, const FitClass &c, int b, hipStream_t s) {
    const FitClass e = tile_class(a.F, a.K);
    if (!e.ok || e.rf != c.rf || e.kmax != c.kmax || !a.W16r || !a.W16c) return hipErrorInvalidValue;
    return launch(c, &a, b, nullptr, nullptr, 0, nullptr, nullptr, false, s);
}

hipError_t launch_fit_tile_multi(const FitClass &c, const FitDesc *d, const int2 *items, int n,
                                 const long long *cur, const int *beff, bool fold, hipStream_t s) {
    if (fold && !tile_fold_fits(c)) return hipErrorNotSupported;
    return launch(c, nullptr, 0, d, items, n, cur, beff, fold, s);
}

bool tile_fold_fits(const FitClass &c) {
    return c.ok && c.cpw == -1 && (c.kmax == 32 || c.kmax == 64) &&
           tile::lds_fold_bytes(c.rf, c.kmax / 32) <= tile::LDS_MAX;
}

hipError_t launch_fit_tile_work(const FitClass &c, const FitDesc *tab, const ServeWork *work, int n,
                                int tiles, hipStream_t s) {
    if (!c.ok || c.cpw != -1 || c.nw != tile::NWT) return hipErrorNotSupported;
    if (c.kmax == 32) return tile::launch_work_ks<1>(c.rf, tab, work, n, tiles, s);
    if (c.kmax == 64) return tile::launch_work_ks<2>(c.rf, tab, work, n, tiles, s);
    return hipErrorNotSupported;
}

}  // namespace isnmf
