// Device bodies of the dictionary update shared by the single-stream and the
// batched kernels (Algorithm 1, rescaling of W, section 2.3).
#pragma once

#include "common.h"
#include "devmath.h"

namespace isnmf {

// 16-bit copies of W for the precision forms: W * 2^wexp, rounded to nearest
// even, row-major (F x KP) and column-major (K x FR).
__device__ inline uint16_t w16_bits(double v, int kind, int wexp) {
    const float f = ldexpf(float(v), wexp);
    if (kind == 1) {
        unsigned u = __float_as_uint(f);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    }
    return __builtin_bit_cast(uint16_t, (_Float16)f);
}

struct W16Out {
    uint16_t *r, *c;   // null when the handle has no such 16-bit copy
    int kind, wexp, KP, FR;
};

__device__ inline void store_w16(const W16Out &o, int f, int k, double w) {
    if (!o.c) return;
    const uint16_t b = w16_bits(w, o.kind, o.wexp);
    if (o.r) o.r[(size_t)f * o.KP + k] = b;
    o.c[(size_t)k * o.FR + f] = b;
}

// The VALU fit's register-order copy of W (null when the handle has none).
struct WvOut {
    float *p;
    int ck;
};

__device__ inline void store_wv(const WvOut &o, int f, int k, double w) {
    if (o.p) o.p[wv_index(f, k, o.ck)] = float(w);
}

struct RescaleArgs {
    int F, K;
    const double *Wn;
    double *W64;
    float *W32;
    W16Out w16;
    WvOut wv;
    double *sc;     // K: pending column scale of A and B, set to s_k (1 without normalize)
    int normalize, warm;
    float *Hb;      // warm-start activations to compensate (or null)
    int ldh;
    double *dwpart; // per-column squared change of W, or null (not computed)
    int *flags;
};

// One wave per column k: s_k = sum_f Wn_fk, W = Wn / s, warm H[k,:] *= s,
// and the column's squared change of W when dwpart is set.  A /= s and B *= s
// are not applied here: sc[k] = s records them for the next reader of A and B
// (the fold applies them as it loads, with the same FP64 operations).  Lane l
// takes rows l, l + 64, ... in order; the lane values are combined by
// wave_sum_f64.
__device__ __forceinline__ void rescale_body(const RescaleArgs &a, int k, int b) {
    const int lane = threadIdx.x & 63;
    const int F = a.F;
    const size_t col = (size_t)k * F;
    const bool dw_on = a.dwpart != nullptr;
    constexpr int RW = 9;   // rows per lane held in registers (F <= 576); the rest loop
    double wn[RW], wo[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {   // every load of the column in one round trip
        const int f = lane + 64 * r;
        const bool ok = f < F;
        wn[r] = ok ? a.Wn[col + f] : 0.0;
        wo[r] = ok && dw_on ? a.W64[col + f] : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < RW; ++r) s += wn[r];
    for (int f = lane + 64 * RW; f < F; f += 64) s += a.Wn[col + f];
    s = wave_sum_f64(s);
    double scale = 1.0;
    if (a.normalize) {
        if (s > 0.0)
            scale = s;
        else if (lane == 0)
            atomicOr(a.flags, FLAG_GUARD_W);
    }
    double dw = 0.0;
    auto update = [&](int f, double wnv, double wo) {
        const double w = wnv / scale;
        const double dlt = w - wo;
        dw += dlt * dlt;
        a.W64[col + f] = w;
        a.W32[col + f] = float(w);
        store_w16(a.w16, f, k, w);
        store_wv(a.wv, f, k, w);
    };
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int f = lane + 64 * r;
        if (f < F) update(f, wn[r], wo[r]);
    }
    for (int f = lane + 64 * RW; f < F; f += 64)
        update(f, a.Wn[col + f], dw_on ? a.W64[col + f] : 0.0);
    if (lane == 0) a.sc[k] = scale;
    if (a.warm && a.Hb && a.normalize)
        for (int n = lane; n < b; n += 64) a.Hb[(size_t)n * a.ldh + k] *= float(scale);
    if (dw_on) {
        dw = wave_sum_f64(dw);
        if (lane == 0) a.dwpart[k] = dw;
    }
}

// The column rescale of a stream whose fold ran in this workgroup (the
// batched form's folding fits: one workgroup holds the stream's whole
// minibatch, statistics and W).  A barrier first makes the workgroup's stores
// of the unscaled W, of A and of B visible to all its waves; then wave w
// rescales columns w, w + NW, ... with rescale_body, so the bits are those of
// the separate rescale launch.  Without a W update the fold stored A and B
// with no pending scale: sc = 1.
template <int NW>
__device__ inline void rescale_in_workgroup(const FitDesc &a, int b, bool update_w) {
    if (!a.rs) return;   // uniform per workgroup
    __syncthreads();
    const RescaleArgs &ra = *a.rs;
    if (!update_w) {
        for (int k = threadIdx.x; k < ra.K; k += NW * 64) ra.sc[k] = 1.0;
        return;
    }
    for (int k = threadIdx.x >> 6; k < ra.K; k += NW) rescale_body(ra, k, b);
}

inline W16Out w16_out(const OnlineDev &d) {
    W16Out o;
    o.r = d.w16_kind && d.w16_rows ? d.W16r : nullptr;
    o.c = d.w16_kind ? d.W16c : nullptr;
    o.kind = d.w16_kind;
    o.wexp = d.wexp;
    o.KP = d.KP;
    o.FR = d.FR;
    return o;
}

inline WvOut wv_out(const OnlineDev &d) { return WvOut{d.wv_live ? d.Wv : nullptr, d.wv_ck}; }

inline RescaleArgs rescale_args(const OnlineDev &d, int normalize, int warm, float *Hb, int ldh) {
    RescaleArgs a;
    a.F = d.F;
    a.K = d.K;
    a.Wn = d.Wn;
    a.W64 = d.W64;
    a.W32 = d.W32;
    a.w16 = w16_out(d);
    a.wv = wv_out(d);
    a.sc = d.sc;
    a.normalize = normalize;
    a.warm = warm;
    a.Hb = Hb;
    a.ldh = ldh;
    a.dwpart = d.dwpart;
    a.flags = d.flags;
    return a;
}

}  // namespace isnmf
