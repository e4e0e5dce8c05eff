// Throughput variant of the fused fit for BF16 products: each wave fits 16
// frames on v_mfma_f32_16x16x32_bf16, 8 waves (128 frames) per workgroup.
//
// It computes what fit_body.h computes (the inner problem of Algorithm 1: I
// multiplicative updates of Section 2.1, then the final model, the ratios
// 1/x and (eps+v)/x^2 for the fold, the frame loss and the fitted h), with
// the three products of an update as matrix-matrix products whose N
// dimension is a wave's 16 frames:
//   X   [F x 16] = W [F x K] . H [K x 16]        (M = rows, K = components)
//   NUM [K x 16] = W^T [K x F] . R2 [F x 16]     (M = components, K = rows)
//   DEN [K x 16] = W^T [K x F] . R1 [F x 16]
// A wave owns all rows and components of its frames, so an update needs no
// exchange with other waves: the X accumulators become the B operand of
// NUM/DEN in registers, and the NUM/DEN accumulators become the B operand of
// the next X.  That works because an MFMA sums over its K index in whatever
// order the (lane, slot) pairs give: the rows of a 32-row contraction step
// are taken in the order the X accumulators of tiles 2s and 2s+1 hold them
// (lane (g, n), slot j < 4 -> row 32s + 4g + j, slot j >= 4 -> row 32s + 16 +
// 4g + j - 4), the components of a 32-component step in the order the
// NUM/DEN accumulators of m-tiles 2c and 2c+1 hold them (the same pattern),
// and both W operands are stored in LDS in those orders.
//
// W enters as the 16-bit copies W * 2^s and h as h * 2^-s, so X is unscaled
// and NUM, DEN share the factor 2^s, which cancels in num/den.  Accumulation
// is FP32, the ratios and h are FP32, the frame loss terms FP32 summed in
// FP64 per frame.
#pragma once

#include "common.h"
#include "devmath.h"
#include "fold_body.h"
#include "state_body.h"

namespace isnmf {
namespace tile {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef const float __attribute__((address_space(1))) gfloat;

constexpr int WF = 16;       // frames per wave
constexpr int NWT = 8;       // waves per workgroup
constexpr int FPW = WF * NWT;  // frames per workgroup
constexpr int PIPE_S_MAX = 17;  // contraction steps up to which the update loop is pipelined

__device__ inline f4 mfma(bf16x8 a, bf16x8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 4 consecutive 16-bit values (8 bytes, 8-byte aligned) or zeros
__device__ inline uint2 ld4(const uint16_t *p, bool ok) {
    return ok ? *reinterpret_cast<const uint2 *>(p) : uint2{0u, 0u};
}

// Components k0 .. k0 + 3 of row `row` from the column-major copy (K x FR),
// zero past K: what the row-major copy holds there, whose padding is zero.
__device__ inline uint2 ld4_cols(const uint16_t *W16c, int FR, int K, int row, int k0, bool rok) {
    uint32_t h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        h[j] = (rok && k0 + j < K) ? (uint32_t)W16c[(size_t)(k0 + j) * FR + row] : 0u;
    return uint2{h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));

// two FP32 -> two bf16 (round to nearest even), a in the low half
__device__ inline uint32_t pack2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){a, b}, bf16x2));
}

// LDS bytes of the two W operand arrays for (S contraction steps of 32
// rows, KS steps of 32 components): X operands [2S][KS][64] and W^T operands
// [S][2 KS][64], 16 bytes each.
__host__ __device__ constexpr size_t lds_bytes(int S, int KS) {
    return (size_t)(2 * S * KS + S * 2 * KS) * 64 * 16;
}

// The folding final pass (FOLD) keeps the X operands and, past them, over the
// W^T operands: the ratios of two row tiles for all 128 frames in two buffers
// ([buffer][tile][r2, r1][frame][16 rows] floats; buffer 1 first carries h of
// every frame), a per-wave slab pair for the epilogue, the 128 frame losses.
constexpr size_t FOLD_STAGE = (size_t)2 * 2 * 2 * FPW * 16 * 4;
constexpr size_t FOLD_EXTRA = FOLD_STAGE + (size_t)NWT * 2 * RSLAB * 4 + (size_t)FPW * 8;
constexpr size_t LDS_MAX = 160 * 1024;
__host__ __device__ constexpr size_t lds_fold_bytes(int S, int KS) {
    return lds_bytes(S, KS) > (size_t)2 * S * KS * 64 * 16 + FOLD_EXTRA
               ? lds_bytes(S, KS)
               : (size_t)2 * S * KS * 64 * 16 + FOLD_EXTRA;
}

// S = ceil(F / 32) contraction steps, KS = ceil(K / 32) component steps.
// FOLD: the workgroup holds the stream's whole minibatch (b <= 128, n_first =
// 0) and folds it (a.fold) instead of writing R1 and R2.
template <int S, int KS, bool FOLD>
__device__ inline void body(const FitDesc &a, int n_first) {
    constexpr int T = 2 * S;        // 16-row tiles (the last may be past F)
    constexpr int MT = 2 * KS;      // 16-component m-tiles
    extern __shared__ uint4 wl[];
    uint4 *wxl = wl;                        // [T][KS][64]: X A operands
    uint4 *wnl = wl + T * KS * 64;          // [S][MT][64]: W^T A operands
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int n = lane & 15;
    const int F = a.F, K = a.K;
    const int fr = n_first + WF * w + n;     // this lane's frame (B/C column)
    const bool fok = fr < a.b;
    const float eps = a.eps;

    // ---- W operands into LDS (bf16 bits of W * 2^s; zero past F and K), both
    // from the column-major copy: this variant needs no row-major copy
    for (int e = threadIdx.x; e < T * KS * 64; e += NWT * 64) {
        const int l = e & 63, c = (e >> 6) % KS, t = (e >> 6) / KS;
        const int row = 16 * t + (l & 15), k0 = 32 * c + 4 * (l >> 4);
        const uint2 lo = ld4_cols(a.W16c, a.FR, K, row, k0, row < F);
        const uint2 hi = ld4_cols(a.W16c, a.FR, K, row, k0 + 16, row < F);
        wxl[e] = uint4{lo.x, lo.y, hi.x, hi.y};
    }
    for (int e = threadIdx.x; e < S * MT * 64; e += NWT * 64) {
        const int l = e & 63, mt = (e >> 6) % MT, s = (e >> 6) / MT;
        const int k = 16 * mt + (l & 15), r0 = 32 * s + 4 * (l >> 4);
        const uint16_t *pc = a.W16c + (size_t)k * a.FR;
        // rows r0.. and r0 + 16..: below FR (a multiple of 64), zero past F
        const uint2 lo = ld4(pc + r0, k < K && r0 < a.FR);
        const uint2 hi = ld4(pc + r0 + 16, k < K && r0 + 16 < a.FR);
        wnl[e] = uint4{lo.x, lo.y, hi.x, hi.y};
    }

    // ---- eps + v at the lane's rows (C layout: rows 16t + 4g + j, frame n),
    // rounded to bf16 for the update loop (the ratios it feeds are bf16
    // operands); the final pass reads v again in FP32
    uint32_t vp[T][2];
    int bad = 0;
    auto load_v = [&](int t, int j) {
        const int row = 16 * t + 4 * g + j;
        return (row < F && fok) ? a.V[(size_t)fr * a.ldv + row] : 0.f;
    };
    auto vprime = [&](int t, int j, float v) { return 16 * t + 4 * g + j < F && fok ? eps + v : 0.f; };
#pragma unroll
    for (int t = 0; t < T; ++t) {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = load_v(t, j);
            bad |= !isfinite(v[j]);
        }
        vp[t][0] = pack2(vprime(t, 0, v[0]), vprime(t, 1, v[1]));
        vp[t][1] = pack2(vprime(t, 2, v[2]), vprime(t, 3, v[3]));
    }
    if (bad) atomicOr(a.flags, FLAG_NONFINITE_V);
    // unpacked where used; the packed words are redefined by an empty asm at
    // the start of every update (in place, no copies), which keeps the
    // compiler from hoisting the FP32 values out of the update loop (that
    // would undo the packing)
    auto vq = [&](int t, int j) {
        const uint32_t u = vp[t][j >> 1];
        return __uint_as_float((j & 1) ? (u & 0xffff0000u) : (u << 16));
    };
    // X accumulator start: eps, or 1 on rows past F (W = 0 there, x only needs to be > 0)
    const f4 ce = {eps, eps, eps, eps};
    auto cinit = [&](int t) {
        f4 c = ce;
        // F > 32 (S - 1): only the last two tiles can reach past F
        if (t >= T - 2 && 16 * t + 15 >= F) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (16 * t + 4 * g + j >= F) c[j] = 1.f;
        }
        return c;
    };

    // ---- h (FP32): lane (g, n) holds components 16 mt + 4g + j of frame n
    float hq[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 16 * mt + 4 * g + j;
            hq[mt][j] = k < K ? ((a.warm && fok) ? a.Hb[(size_t)fr * a.ldh + k] : 1.f) : 0.f;
        }
    // the X B operand: slot j of step c is m-tile 2c (j < 4) or 2c + 1 (j >= 4)
    bf16x8 hb[KS];
    auto pack_h = [&]() {
#pragma unroll
        for (int c = 0; c < KS; ++c) {
            const float sc = a.hscale;
            const uint4 u = {pack2(hq[2 * c][0] * sc, hq[2 * c][1] * sc),
                             pack2(hq[2 * c][2] * sc, hq[2 * c][3] * sc),
                             pack2(hq[2 * c + 1][0] * sc, hq[2 * c + 1][1] * sc),
                             pack2(hq[2 * c + 1][2] * sc, hq[2 * c + 1][3] * sc)};
            hb[c] = __builtin_bit_cast(bf16x8, u);
        }
    };
    pack_h();
    __syncthreads();   // W operands in LDS

    auto model = [&](int t) {
        f4 x = cinit(t);
#pragma unroll
        for (int c = 0; c < KS; ++c)
            x = mfma(__builtin_bit_cast(bf16x8, wxl[(t * KS + c) * 64 + lane]), hb[c], x);
        return x;
    };

    // X operands of row tiles 2s and 2s + 1 (contraction step s), and the
    // model products of those tiles from them
    auto load_wx = [&](int s, bf16x8 (&o)[2][KS]) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int c = 0; c < KS; ++c)
                o[u][c] = __builtin_bit_cast(bf16x8, wxl[((2 * s + u) * KS + c) * 64 + lane]);
    };
    auto model_ops = [&](int t, const bf16x8 (&ops)[KS]) {
        f4 x = cinit(t);
#pragma unroll
        for (int c = 0; c < KS; ++c) x = mfma(ops[c], hb[c], x);
        return x;
    };

    int guard = 0;
    for (int it = 0; it < a.iters; ++it) {
#pragma unroll
        for (int t = 0; t < T; ++t) asm volatile("" : "+v"(vp[t][0]), "+v"(vp[t][1]));
        f4 na[MT], da[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            na[mt] = f4{0.f, 0.f, 0.f, 0.f};
            da[mt] = f4{0.f, 0.f, 0.f, 0.f};
        }
        // ratios r1 = 1/x, r2 = (eps + v)/x^2 of step s's rows from its model
        // products, as the two bf16 B operands of NUM and DEN
        auto ratios = [&](int s, const f4 &x0, const f4 &x1, bf16x8 &b1, bf16x8 &b2) {
            float r1[8], r2[8];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                r1[j] = __builtin_amdgcn_rcpf(x0[j]);
                r2[j] = vq(2 * s, j) * r1[j] * r1[j];
                r1[4 + j] = __builtin_amdgcn_rcpf(x1[j]);
                r2[4 + j] = vq(2 * s + 1, j) * r1[4 + j] * r1[4 + j];
            }
            b1 = __builtin_bit_cast(
                bf16x8, uint4{pack2(r1[0], r1[1]), pack2(r1[2], r1[3]), pack2(r1[4], r1[5]),
                              pack2(r1[6], r1[7])});
            b2 = __builtin_bit_cast(
                bf16x8, uint4{pack2(r2[0], r2[1]), pack2(r2[2], r2[3]), pack2(r2[4], r2[5]),
                              pack2(r2[6], r2[7])});
        };
        if constexpr (S <= PIPE_S_MAX) {
            // Software pipeline over the contraction steps: step s + 1's model
            // products are issued to the matrix pipe before step s's ratios are
            // formed on the VALU, from X operands read from LDS one step ahead
            // (register sets wx[s & 1]).  The products and sums are those of
            // the plain order below, so the results are the same bits.
            bf16x8 wx[2][2][KS];
            load_wx(0, wx[0]);
            f4 x0 = model_ops(0, wx[0][0]), x1 = model_ops(1, wx[0][1]);
            if (S > 1) load_wx(1, wx[1]);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                // the W operands are re-read from LDS at every step (kept from
                // being hoisted into registers: all of them would not fit), and
                // the steps are not interleaved by the scheduler (live ranges)
                asm volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                f4 y0 = ce, y1 = ce;
                if (s + 1 < S) {
                    y0 = model_ops(2 * s + 2, wx[(s + 1) & 1][0]);
                    y1 = model_ops(2 * s + 3, wx[(s + 1) & 1][1]);
                }
                // this step's W^T operands, then the X operands of step s + 2:
                // in that order the wait for the first leaves the second in flight
                bf16x8 wt[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    wt[mt] = __builtin_bit_cast(bf16x8, wnl[(s * MT + mt) * 64 + lane]);
                __builtin_amdgcn_sched_barrier(0);
                if (s + 2 < S) load_wx(s + 2, wx[s & 1]);
                __builtin_amdgcn_sched_barrier(0);
                bf16x8 b1, b2;
                ratios(s, x0, x1, b1, b2);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    na[mt] = mfma(wt[mt], b2, na[mt]);
                    da[mt] = mfma(wt[mt], b1, da[mt]);
                }
                x0 = y0;
                x1 = y1;
            }
        } else {
            // plain order (larger S: the pipeline's registers would spill)
#pragma unroll
            for (int s = 0; s < S; ++s) {
                asm volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                const f4 x0 = model(2 * s), x1 = model(2 * s + 1);
                bf16x8 b1, b2;
                ratios(s, x0, x1, b1, b2);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const bf16x8 wt = __builtin_bit_cast(bf16x8, wnl[(s * MT + mt) * 64 + lane]);
                    na[mt] = mfma(wt, b2, na[mt]);
                    da[mt] = mfma(wt, b1, da[mt]);
                }
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (16 * mt + 4 * g + j < K) {
                    const float N = na[mt][j], D = da[mt][j];
                    if (D > 0.f && N >= 0.f)
                        hq[mt][j] *= __builtin_amdgcn_sqrtf(N * __builtin_amdgcn_rcpf(D));
                    else if (fok)
                        guard = 1;
                }
            }
        pack_h();
    }
    if (guard) atomicOr(a.flags, FLAG_GUARD_H);

    // ---- final model: R1, R2 for the fold (FP32), or the fold itself, and the
    // frame loss.
    // the fitted h: internal copy and the caller's H
    auto store_h = [&]() {
        if (fok) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = 16 * mt + 4 * g + j;
                    if (k < K) {
                        a.Hi[(size_t)fr * a.KP + k] = hq[mt][j];
                        if (a.Hb) a.Hb[(size_t)fr * a.ldh + k] = hq[mt][j];
                    }
                }
        }
    };
    double ls = 0.0;
    if constexpr (FOLD) {
        // The fold of the minibatch (Algorithm 1's statistics update and W =
        // sqrt(A/B)) in this workgroup.  Round r takes row tiles 2r and 2r + 1:
        // every wave forms its frames' ratios there and stages them in LDS,
        // then wave w folds row tile 2r + (w & 1) over component tile w >> 1
        // for all frames, with the separate fold's MFMA chains (frames with
        // (n / 4) mod 4 = v in increasing n), chain sums and epilogue
        // (fold_rows_body), so the bits are those of the fit followed by that
        // fold.  The ratio buffers alternate, one barrier per round.
        const FoldArgs &fa0 = *a.fold;
        FoldArgs fa = fa0;
        fa.b = a.b;
        constexpr int CW = 32 * KS;                  // LDS floats per frame of h
        constexpr int RB = 2 * FPW * 16;             // floats per staged row tile (r2, r1)
        float *stg = reinterpret_cast<float *>(wl + 2 * S * KS * 64);
        float *slab = stg + 4 * RB + w * 2 * RSLAB;
        const int KT = (K + 15) / 16;
        const int kt = w >> 1, uw = w & 1;
        const bool kact = kt < KT;   // uniform per wave
        // h of every frame through buffer 1 (zero past the minibatch and past
        // K, as the separate fold stages it); wave w keeps the column of its
        // component tile for all 128 frames.  The barrier first: the W^T
        // operands under the buffers may still be read by the last update.
        __syncthreads();
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            f4 hv;
#pragma unroll
            for (int j = 0; j < 4; ++j) hv[j] = (fok && 16 * mt + 4 * g + j < K) ? hq[mt][j] : 0.f;
            *reinterpret_cast<f4 *>(stg + 2 * RB + (WF * w + n) * CW + 16 * mt + 4 * g) = hv;
        }
        __syncthreads();
        float hh[32];
#pragma unroll
        for (int m = 0; m < 32; ++m) hh[m] = kact ? stg[2 * RB + (4 * m + g) * CW + 16 * kt + n] : 0.f;
        store_h();
        // v (FP32) of a round's two row tiles and the epilogue operands of the
        // wave's fold tile (element (16 tf + n, 16 kt + 4 g + j) in pass j: W,
        // A, B), read one round ahead; the pending column scales of its columns
        float vc[2][4], vn[2][4];
        double eo[3][4], en[3][4];   // [W, A, B][j]
        double scq[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int kc = 16 * kt + 4 * g + j;
            scq[j] = kact && kc < K ? fa.sc[kc] : 1.0;
        }
        // (global-memory loads: flat ones would hold up every LDS wait of the
        // round until they arrive)
        const gdouble *gW = (const gdouble *)fa.W64;
        const gdouble *gA = (const gdouble *)fa.A;
        const gdouble *gB = (const gdouble *)fa.B;
        const gfloat *gV = (const gfloat *)a.V;
        auto load_vg = [&](int t, int j) {
            const int row = 16 * t + 4 * g + j;
            return (row < F && fok) ? gV[(size_t)fr * a.ldv + row] : 0.f;
        };
        auto load_eo = [&](int r, double (&o)[3][4]) {
            const int tf = 2 * r + uw, fe = 16 * tf + n;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int kc = 16 * kt + 4 * g + j;
                const bool ok = kact && fe < F && kc < K;
                const size_t e = ok ? (size_t)fe + (size_t)kc * F : 0;
                o[0][j] = ok ? gW[e] : 0.0;
                o[1][j] = ok ? gA[e] : 0.0;
                o[2][j] = ok ? gB[e] : 0.0;
            }
        };
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j) vc[u][j] = load_vg(u, j);
        load_eo(0, eo);
#pragma unroll 1
        for (int r = 0; r < S; ++r) {
            float *sb0 = stg + (r & 1) * 2 * RB;
            const int tf = 2 * r + uw;                 // this wave's fold row tile
            const bool fact = kact && 16 * tf < F;     // uniform per wave
            const int fe = 16 * tf + n;
            if (r + 1 < S) load_eo(r + 1, en);
            if (r + 1 < S) {
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int j = 0; j < 4; ++j) vn[u][j] = load_vg(2 * r + 2 + u, j);
            }
            // ratios of row tiles 2r and 2r + 1 of this wave's frames (zero for
            // frames past the minibatch) and the frame loss terms
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int t = 2 * r + u;
                asm volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
                const f4 x = model(t);
                const int row0 = 16 * t + 4 * g;
                f4 r1, r2;
                float l = 0.f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float rr = __builtin_amdgcn_rcpf(x[j]);
                    const float ve = vprime(t, j, vc[u][j]);
                    r1[j] = fok ? rr : 0.f;
                    r2[j] = fok ? ve * rr * rr : 0.f;
                    if (row0 + j < F) l += dis_term32(ve, rr);
                }
                ls += double(l);
                float *sr = sb0 + u * RB;
                *reinterpret_cast<f4 *>(sr + (WF * w + n) * 16 + 4 * g) = r2;
                *reinterpret_cast<f4 *>(sr + FPW * 16 + (WF * w + n) * 16 + 4 * g) = r1;
            }
            __syncthreads();
            if (fact) {
                const float *sr2 = sb0 + uw * RB, *sr1 = sr2 + FPW * 16;
                floatx4 ca[4], cb[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    ca[v] = floatx4{0.f, 0.f, 0.f, 0.f};
                    cb[v] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
                // every group of 4 frames: those past the minibatch hold r = h =
                // 0, whose products add exactly zero to the non-negative chains,
                // as the separate fold's skipping them does
#pragma unroll
                for (int m = 0; m < 32; ++m) {
                    if ((m & 7) == 0) __builtin_amdgcn_sched_barrier(0);   // bounds the reads in flight
                    const int nl = 4 * m + g;
                    ca[m & 3] = mfma16(sr2[nl * 16 + n], hh[m], ca[m & 3]);
                    cb[m & 3] = mfma16(sr1[nl * 16 + n], hh[m], cb[m & 3]);
                }
                const floatx4 sa = ((ca[0] + ca[1]) + ca[2]) + ca[3];
                const floatx4 sb = ((cb[0] + cb[1]) + cb[2]) + cb[3];
                reinterpret_cast<floatx4 *>(slab)[red_pos(lane)] = sa;
                reinterpret_cast<floatx4 *>(slab + RSLAB)[red_pos(lane)] = sb;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int cl = 4 * g + j;
                    const float ea = red_elem(slab, n, cl);
                    const float eb = red_elem(slab + RSLAB, n, cl);
                    const int kc = 16 * kt + cl;
                    if (fe < F && kc < K)
                        epilogue<true>(fa, fe, kc, double(ea), double(eb), eo[0][j],
                                       eo[1][j] / scq[j], eo[2][j] * scq[j]);
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int j = 0; j < 4; ++j) vc[u][j] = vn[u][j];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) eo[i][j] = en[i][j];
        }
    } else {
    // v (FP32) is read FPD row tiles ahead of its use, so that the loads are in
    // flight during the tiles before (the update loop's registers are free here)
    constexpr int FPD = 8;
    float vf[T][4];
#pragma unroll
    for (int t = 0; t < FPD && t < T; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) vf[t][j] = load_v(t, j);
#pragma unroll
    for (int t = 0; t < T; ++t) {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        if (t + FPD < T) {
#pragma unroll
            for (int j = 0; j < 4; ++j) vf[t + FPD][j] = load_v(t + FPD, j);
        }
        const f4 x = model(t);
        const int row0 = 16 * t + 4 * g;
        f4 r1, r2;
        float l = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float r = __builtin_amdgcn_rcpf(x[j]);
            const float ve = vprime(t, j, vf[t][j]);
            r1[j] = r;
            r2[j] = ve * r * r;
            if (row0 + j < F) l += dis_term32(ve, r);
        }
        ls += double(l);
        if (fok && row0 < F) {   // FR is a multiple of 64: rows row0..row0+3 are in the buffer
            *reinterpret_cast<f4 *>(a.R1 + (size_t)fr * a.FR + row0) = r1;
            *reinterpret_cast<f4 *>(a.R2 + (size_t)fr * a.FR + row0) = r2;
        }
    }
    }
    // frame n's loss: lanes n, n + 16, n + 32, n + 48, in that order
    const double l1 = __shfl_xor(ls, 16, 64);
    const double l2 = __shfl_xor(ls, 32, 64);
    const double l3 = __shfl_xor(ls, 48, 64);
    const double lframe = ((ls + l1) + l2) + l3;
    if (g == 0 && fok) a.lossf[fr] = lframe;
    if constexpr (FOLD) {
        // the minibatch loss as the separate fold adds it: wave 1, lane l sums
        // frames l, l + 64 in order, then a fixed xor butterfly over the lanes
        double *lsh = reinterpret_cast<double *>(reinterpret_cast<char *>(wl) + 2 * S * KS * 64 * 16 +
                                                 FOLD_STAGE + NWT * 2 * RSLAB * 4);
        if (g == 0) lsh[WF * w + n] = lframe;
        __syncthreads();
        const FoldArgs *fa = a.fold;
        if (fa->d_loss_sum && w == 1) {
            double sl = 0.0;
            for (int m = lane; m < a.b; m += 64) sl += lsh[m];
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) sl += __shfl_xor(sl, m, 64);
            if (lane == 0) *fa->d_loss_sum += sl;
        }
    }
    if (!FOLD) store_h();   // the folding pass stores h before its rounds
}

template <int S, int KS>
__global__ __launch_bounds__(NWT * 64) void fit_tile_kernel(FitDesc a) {
    body<S, KS, false>(a, blockIdx.x * FPW);
}

// Batched form: item = (stream, tile of 128 frames); tiles past the stream's
// minibatch of this step exit.  FOLD: every stream of the launch has one tile
// (b <= 128) and a fold descriptor, and the workgroup also rescales W when the
// descriptor carries the rescale.
template <int S, int KS, bool FOLD>
__global__ __launch_bounds__(NWT * 64) void fit_tile_multi_kernel(const FitDesc *__restrict__ descs,
                                                                  const int2 *__restrict__ items,
                                                                  const long long *__restrict__ cursor,
                                                                  const int *__restrict__ beff) {
    const int2 it = items[blockIdx.x];
    const int b = beff[it.x];
    if (it.y * FPW >= b) return;   // uniform per workgroup
    FitDesc a = descs[it.x];
    const long long c = cursor[it.x];
    a.b = b;
    a.V += c * a.ldv;
    if (a.Hb) a.Hb += c * a.ldh;
    body<S, KS, FOLD>(a, it.y * FPW);
    if constexpr (FOLD) rescale_in_workgroup<NWT>(a, b, a.fold->update_w);
}

// Served form: grid (chunk i, 128-frame tile j) over a step's work list.
template <int S, int KS>
__global__ __launch_bounds__(NWT * 64) void fit_tile_work_kernel(const FitDesc *__restrict__ tab,
                                                                 const ServeWork *__restrict__ work) {
    const ServeWork wk = work[blockIdx.x];
    if ((int)blockIdx.y * FPW >= wk.b) return;   // uniform per workgroup
    FitDesc a = tab[wk.sess];
    a.b = wk.b;
    a.V = wk.V;
    a.ldv = wk.ldv;
    body<S, KS, false>(a, blockIdx.y * FPW);
}

template <int S, int KS>
hipError_t launch_work_one(const FitDesc *tab, const ServeWork *work, int n, int tiles,
                           hipStream_t s) {
    constexpr size_t lds = lds_bytes(S, KS);
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&fit_tile_work_kernel<S, KS>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
    fit_tile_work_kernel<S, KS><<<dim3(n, tiles), NWT * 64, lds, s>>>(tab, work);
    return hipGetLastError();
}

template <int S, int KS>
hipError_t launch_one(const FitDesc *a, int b, const FitDesc *d, const int2 *items, int n,
                      const long long *cur, const int *beff, bool fold, hipStream_t s) {
    constexpr size_t lds = lds_bytes(S, KS);
    if (d && fold) {
        constexpr size_t lf = lds_fold_bytes(S, KS);
        if constexpr (lf <= LDS_MAX) {
            static const hipError_t attr = hipFuncSetAttribute(
                reinterpret_cast<const void *>(&fit_tile_multi_kernel<S, KS, true>),
                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lf);
            if (attr != hipSuccess) return attr;
            fit_tile_multi_kernel<S, KS, true><<<n, NWT * 64, lf, s>>>(d, items, cur, beff);
        } else {
            return hipErrorNotSupported;
        }
    } else if (d) {
        static const hipError_t attr = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&fit_tile_multi_kernel<S, KS, false>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (attr != hipSuccess) return attr;
        fit_tile_multi_kernel<S, KS, false><<<n, NWT * 64, lds, s>>>(d, items, cur, beff);
    } else {
        static const hipError_t attr = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&fit_tile_kernel<S, KS>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (attr != hipSuccess) return attr;
        fit_tile_kernel<S, KS><<<(b + FPW - 1) / FPW, NWT * 64, lds, s>>>(*a);
    }
    return hipGetLastError();
}

}  // namespace tile
}  // namespace isnmf

namespace isnmf {
namespace tile {

constexpr int S_MAX = 20;   // F <= 640

// Launch of the (S, KS) instance for S = 1..S_MAX; explicitly instantiated per
// KS in fit_tile_k*.hip so the instances build in parallel.
template <int KS>
hipError_t launch_ks(int S, const FitDesc *a, int b, const FitDesc *d, const int2 *items, int n,
                     const long long *cur, const int *beff, bool fold, hipStream_t st) {
    switch (S) {
#define ISNMF_TILE_S(SV) \
    case SV: return launch_one<SV, KS>(a, b, d, items, n, cur, beff, fold, st);
        ISNMF_TILE_S(1) ISNMF_TILE_S(2) ISNMF_TILE_S(3) ISNMF_TILE_S(4) ISNMF_TILE_S(5)
        ISNMF_TILE_S(6) ISNMF_TILE_S(7) ISNMF_TILE_S(8) ISNMF_TILE_S(9) ISNMF_TILE_S(10)
        ISNMF_TILE_S(11) ISNMF_TILE_S(12) ISNMF_TILE_S(13) ISNMF_TILE_S(14) ISNMF_TILE_S(15)
        ISNMF_TILE_S(16) ISNMF_TILE_S(17) ISNMF_TILE_S(18) ISNMF_TILE_S(19) ISNMF_TILE_S(20)
#undef ISNMF_TILE_S
        default: return hipErrorNotSupported;
    }
}

template <int KS>
hipError_t launch_work_ks(int S, const FitDesc *tab, const ServeWork *work, int n, int tiles,
                         hipStream_t st) {
    switch (S) {
#define ISNMF_TILE_S(SV) \
    case SV: return launch_work_one<SV, KS>(tab, work, n, tiles, st);
        ISNMF_TILE_S(1) ISNMF_TILE_S(2) ISNMF_TILE_S(3) ISNMF_TILE_S(4) ISNMF_TILE_S(5)
        ISNMF_TILE_S(6) ISNMF_TILE_S(7) ISNMF_TILE_S(8) ISNMF_TILE_S(9) ISNMF_TILE_S(10)
        ISNMF_TILE_S(11) ISNMF_TILE_S(12) ISNMF_TILE_S(13) ISNMF_TILE_S(14) ISNMF_TILE_S(15)
        ISNMF_TILE_S(16) ISNMF_TILE_S(17) ISNMF_TILE_S(18) ISNMF_TILE_S(19) ISNMF_TILE_S(20)
#undef ISNMF_TILE_S
        default: return hipErrorNotSupported;
    }
}

#define ISNMF_TILE_EXTERN(KSV)                                                                   \
    extern template hipError_t launch_ks<KSV>(int, const FitDesc *, int, const FitDesc *,       \
                                              const int2 *, int, const long long *, const int *, \
                                              bool, hipStream_t);                                \
    extern template hipError_t launch_work_ks<KSV>(int, const FitDesc *, const ServeWork *, int, \
                                                   int, hipStream_t);
#define ISNMF_TILE_INSTANTIATE(KSV)                                                       \
    template hipError_t launch_ks<KSV>(int, const FitDesc *, int, const FitDesc *,       \
                                       const int2 *, int, const long long *, const int *, \
                                       bool, hipStream_t);                                \
    template hipError_t launch_work_ks<KSV>(int, const FitDesc *, const ServeWork *, int, \
                                            int, hipStream_t);

}  // namespace tile
}  // namespace isnmf
