// Device bodies of the dictionary update shared by the single-stream and the
// batched kernels (Algorithm 1, rescaling of W, section 2.3).
#pragma once

#include "common.h"

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
    uint16_t *r, *c;   // null when the handle has no 16-bit copies
    int kind, wexp, KP, FR;
};

__device__ inline void store_w16(const W16Out &o, int f, int k, double w) {
    if (!o.r) return;
    const uint16_t b = w16_bits(w, o.kind, o.wexp);
    o.r[(size_t)f * o.KP + k] = b;
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

// Sum over a 256-thread block in a fixed order: per-wave xor butterfly (the
// same value in every lane), then the four wave sums in index order.
__device__ inline double block_sum256(double v, double *red4) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((red4[0] + red4[1]) + red4[2]) + red4[3];
}

struct RescaleArgs {
    int F, K;
    const double *Wn;
    double *W64;
    float *W32;
    W16Out w16;
    WvOut wv;
    double *A, *B;
    int normalize, warm;
    float *Hb;      // warm-start activations to compensate (or null)
    int ldh;
    double *dwpart;
    int *flags;
};

// Block (256 threads) per column k: s_k = sum_f Wn_fk, W = Wn / s, A /= s,
// B *= s, warm H[k,:] *= s, and the column's squared change of W.
__device__ __forceinline__ void rescale_body(const RescaleArgs &a, int k, int b) {
    __shared__ double red4[4];
    const int tid = threadIdx.x;
    const int F = a.F;
    const size_t col = (size_t)k * F;
    // all loads first (one memory round trip), then the column sum
    constexpr int RMAX = 8;   // rows per thread held in registers (F <= 2048)
    double wn[RMAX], wo[RMAX], av[RMAX], bv[RMAX];
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
        const int f = tid + 256 * r;
        const bool ok = f < F;
        wn[r] = ok ? a.Wn[col + f] : 0.0;
        wo[r] = ok ? a.W64[col + f] : 0.0;
        av[r] = ok ? a.A[col + f] : 0.0;
        bv[r] = ok ? a.B[col + f] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RMAX; ++r) s += wn[r];
    for (int f = tid + 256 * RMAX; f < F; f += 256) s += a.Wn[col + f];
    s = block_sum256(s, red4);
    double scale = 1.0;
    if (a.normalize) {
        if (s > 0.0)
            scale = s;
        else if (tid == 0)
            atomicOr(a.flags, FLAG_GUARD_W);
    }
    double dw = 0.0;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
        const int f = tid + 256 * r;
        if (f < F) {
            const double w = wn[r] / scale;
            const double dlt = w - wo[r];
            dw += dlt * dlt;
            a.W64[col + f] = w;
            a.W32[col + f] = float(w);
            store_w16(a.w16, f, k, w);
            store_wv(a.wv, f, k, w);
            if (a.normalize) {
                a.A[col + f] = av[r] / scale;
                a.B[col + f] = bv[r] * scale;
            }
        }
    }
    for (int f = tid + 256 * RMAX; f < F; f += 256) {
        const double w = a.Wn[col + f] / scale;
        const double dlt = w - a.W64[col + f];
        dw += dlt * dlt;
        a.W64[col + f] = w;
        a.W32[col + f] = float(w);
        store_w16(a.w16, f, k, w);
        store_wv(a.wv, f, k, w);
        if (a.normalize) {
            a.A[col + f] /= scale;
            a.B[col + f] *= scale;
        }
    }
    if (a.warm && a.Hb && a.normalize)
        for (int n = tid; n < b; n += 256) a.Hb[(size_t)n * a.ldh + k] *= float(scale);
    dw = block_sum256(dw, red4);
    if (tid == 0) a.dwpart[k] = dw;
}

inline W16Out w16_out(const OnlineDev &d) {
    W16Out o;
    o.r = d.w16_kind ? d.W16r : nullptr;
    o.c = d.w16_kind ? d.W16c : nullptr;
    o.kind = d.w16_kind;
    o.wexp = d.wexp;
    o.KP = d.KP;
    o.FR = d.FR;
    return o;
}

inline WvOut wv_out(const OnlineDev &d) { return WvOut{d.Wv, d.wv_ck}; }

inline RescaleArgs rescale_args(const OnlineDev &d, int normalize, int warm, float *Hb, int ldh) {
    RescaleArgs a;
    a.F = d.F;
    a.K = d.K;
    a.Wn = d.Wn;
    a.W64 = d.W64;
    a.W32 = d.W32;
    a.w16 = w16_out(d);
    a.wv = wv_out(d);
    a.A = d.A;
    a.B = d.B;
    a.normalize = normalize;
    a.warm = warm;
    a.Hb = Hb;
    a.ldh = ldh;
    a.dwpart = d.dwpart;
    a.flags = d.flags;
    return a;
}

}  // namespace isnmf
