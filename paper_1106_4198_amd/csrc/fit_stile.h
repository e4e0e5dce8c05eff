// Streamed variant of the 16-frame tile fit for BF16 products: the same
// per-wave products as fit_tile.h (16 frames per wave on
// v_mfma_f32_16x16x32_bf16, 8 waves per workgroup, no exchange between waves),
// for shapes whose W operands do not fit in LDS (F > 640 or K > 64).
//
// Per update, the 32-row contraction steps s = 0 .. S-1 run in order.  The W
// operands of one step (X operands of row tiles 2s and 2s+1, W^T operands of
// rows 32s .. 32s+31, for every component) pass through a two-slot LDS
// window: the whole workgroup loads step s+1's operands from the 16-bit
// copies (row-major W16r for X, column-major W16c for W^T) into registers
// while it computes step s, writes them to the other slot, and one barrier
// separates the steps.  eps + v of a step's rows is re-read from V (FP32) at
// every step instead of being held in registers; the registers then hold only
// h, the NUM/DEN accumulators and one step's values, so S is a run-time value
// (F up to 32 * S_MAX rows).
//
// The operand orders, the K-index permutation that lets the X accumulators
// feed NUM/DEN and the NUM/DEN accumulators feed the next X, the scaling by
// 2^s, the final pass and the output layouts are those of fit_tile.h.  The
// update loop uses eps + v in FP32 (not rounded to bf16 first); the ratios
// are rounded to bf16 as MFMA operands either way.
#pragma once

#include "common.h"
#include "devmath.h"

namespace isnmf {
namespace stile {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float float2v __attribute__((ext_vector_type(2)));

constexpr int WF = 16;         // frames per wave
constexpr int NWT = 8;         // waves per workgroup
constexpr int FPW = WF * NWT;  // frames per workgroup
constexpr int S_MAX = 64;      // F <= 2048
constexpr int KS_MAX = 4;      // K <= 128

__device__ inline f4 mfma(bf16x8 a, bf16x8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline uint32_t pack2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){a, b}, bf16x2));
}

// 4 consecutive 16-bit values (8 bytes, 8-byte aligned) or zeros
__device__ inline uint2 ld4(const uint16_t *p, bool ok) {
    return ok ? *reinterpret_cast<const uint2 *>(p) : uint2{0u, 0u};
}

// uint4 elements of one LDS window slot: X operands [2][KS][64], then W^T
// operands [2 KS][64]
__host__ __device__ constexpr int slot_elems(int KS) { return 2 * KS * 64 + 2 * KS * 64; }
__host__ __device__ constexpr size_t lds_bytes(int KS) { return (size_t)2 * slot_elems(KS) * 16; }

// Element e of step s's window: the same operand bits fit_tile.h keeps for
// row tiles 2s, 2s+1 (X) and contraction step s (W^T).
template <int KS>
__device__ inline uint4 window_elem(const FitDesc &a, int s, int e) {
    constexpr int NX = 2 * KS * 64;
    if (e < NX) {
        const int l = e & 63, c = (e >> 6) % KS, t = 2 * s + (e >> 6) / KS;
        const int row = 16 * t + (l & 15), k0 = 32 * c + 4 * (l >> 4);
        const uint16_t *pr = a.W16r + (size_t)row * a.KP;
        const uint2 lo = ld4(pr + k0, row < a.F && k0 < a.KP);
        const uint2 hi = ld4(pr + k0 + 16, row < a.F && k0 + 16 < a.KP);
        return uint4{lo.x, lo.y, hi.x, hi.y};
    }
    e -= NX;
    const int l = e & 63, mt = e >> 6;
    const int k = 16 * mt + (l & 15), r0 = 32 * s + 4 * (l >> 4);
    const uint16_t *pc = a.W16c + (size_t)k * a.FR;
    // rows r0.. and r0 + 16..: below FR (a multiple of 64), zero past F
    const uint2 lo = ld4(pc + r0, k < a.K && r0 < a.FR);
    const uint2 hi = ld4(pc + r0 + 16, k < a.K && r0 + 16 < a.FR);
    return uint4{lo.x, lo.y, hi.x, hi.y};
}

// KS = ceil(K / 32) component steps; S = ceil(F / 32) contraction steps.
template <int KS>
__device__ inline void body(const FitDesc &a, int n_first) {
    constexpr int MT = 2 * KS;                    // 16-component m-tiles
    constexpr int SE = slot_elems(KS);
    constexpr int EPT = (SE + NWT * 64 - 1) / (NWT * 64);   // window elements per thread
    extern __shared__ uint4 win[];                // [2][SE]
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int g = lane >> 4;
    const int n = lane & 15;
    const int F = a.F, K = a.K;
    const int S = (F + 31) / 32;
    const int fr = n_first + WF * w + n;          // this lane's frame (B/C column)
    const bool fok = fr < a.b;
    const float eps = a.eps;
    const float *vrow = a.V + (size_t)(fok ? fr : 0) * a.ldv;

    // eps + v at row `row` of this lane's frame (0 past F or past the minibatch)
    auto vprime = [&](int row) { return (row < F && fok) ? eps + vrow[row] : 0.f; };
    // X accumulator start of row tile t: eps, or 1 on rows past F (W = 0 there)
    auto cinit = [&](int t) {
        f4 c = {eps, eps, eps, eps};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (16 * t + 4 * g + j >= F) c[j] = 1.f;
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

    // ---- window: step q's operands go to slot q & 1
    uint4 pre[EPT];
    auto fetch = [&](int s) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + NWT * 64 * i;
            if (e < SE) pre[i] = window_elem<KS>(a, s, e);
        }
    };
    auto store = [&](int slot) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + NWT * 64 * i;
            if (e < SE) win[slot * SE + e] = pre[i];
        }
    };
    fetch(0);
    store(0);
    __syncthreads();

    // one pass over the steps: X of tiles 2s, 2s+1 from the window, then
    // either the NUM/DEN products (update) or the fold's outputs (final)
    const int passes = a.iters + 1;
    int guard = 0, bad = 0;
    double ls = 0.0;
    f4 na[MT], da[MT];
    for (int q = 0; q < passes * S; ++q) {
        const int it = q / S, s = q - it * S;
        const bool final_pass = it == a.iters;
        const bool more = q + 1 < passes * S;
        if (more) fetch(s + 1 < S ? s + 1 : 0);   // next step (of this or the next pass)
        const uint4 *wx = win + (q & 1) * SE;
        const uint4 *wn = wx + 2 * KS * 64;
        if (s == 0) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                na[mt] = f4{0.f, 0.f, 0.f, 0.f};
                da[mt] = f4{0.f, 0.f, 0.f, 0.f};
            }
        }
        f4 x[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            x[u] = cinit(2 * s + u);
#pragma unroll
            for (int c = 0; c < KS; ++c)
                x[u] = mfma(__builtin_bit_cast(bf16x8, wx[(u * KS + c) * 64 + lane]), hb[c], x[u]);
        }
        if (!final_pass) {
            float r1[8], r2[8];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float r = __builtin_amdgcn_rcpf(x[u][j]);
                    r1[4 * u + j] = r;
                    r2[4 * u + j] = vprime(32 * s + 16 * u + 4 * g + j) * r * r;
                }
            const bf16x8 b1 = __builtin_bit_cast(
                bf16x8, uint4{pack2(r1[0], r1[1]), pack2(r1[2], r1[3]), pack2(r1[4], r1[5]),
                              pack2(r1[6], r1[7])});
            const bf16x8 b2 = __builtin_bit_cast(
                bf16x8, uint4{pack2(r2[0], r2[1]), pack2(r2[2], r2[3]), pack2(r2[4], r2[5]),
                              pack2(r2[6], r2[7])});
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const bf16x8 wt = __builtin_bit_cast(bf16x8, wn[mt * 64 + lane]);
                na[mt] = mfma(wt, b2, na[mt]);
                da[mt] = mfma(wt, b1, da[mt]);
            }
            if (s == S - 1) {   // end of an update: h <- h sqrt(num / den)
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
        } else {
            // final model: R1, R2 for the fold (FP32) and the frame loss
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int row0 = 32 * s + 16 * u + 4 * g;
                f4 r1, r2;
                float l = 0.f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float v = (row0 + j < F && fok) ? vrow[row0 + j] : 0.f;
                    bad |= !isfinite(v);
                    const float ve = (row0 + j < F && fok) ? eps + v : 0.f;
                    const float r = __builtin_amdgcn_rcpf(x[u][j]);
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
        if (more) store((q + 1) & 1);   // the other slot: its last readers passed the barrier below
        __syncthreads();
    }
    if (guard) atomicOr(a.flags, FLAG_GUARD_H);
    if (bad) atomicOr(a.flags, FLAG_NONFINITE_V);
    // frame n's loss: lanes n, n + 16, n + 32, n + 48, in that order
    const double l1 = __shfl_xor(ls, 16, 64);
    const double l2 = __shfl_xor(ls, 32, 64);
    const double l3 = __shfl_xor(ls, 48, 64);
    if (g == 0 && fok) a.lossf[fr] = ((ls + l1) + l2) + l3;
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
}

template <int KS>
__global__ __launch_bounds__(NWT * 64) void fit_stile_kernel(FitDesc a) {
    body<KS>(a, blockIdx.x * FPW);
}

// Batched form: item = (stream, tile of 128 frames); tiles past the stream's
// minibatch of this step exit.
template <int KS>
__global__ __launch_bounds__(NWT * 64) void fit_stile_multi_kernel(const FitDesc *__restrict__ descs,
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
    body<KS>(a, it.y * FPW);
}

// Served form: grid (chunk i, 128-frame tile j) over a step's work list.
template <int KS>
__global__ __launch_bounds__(NWT * 64) void fit_stile_work_kernel(const FitDesc *__restrict__ tab,
                                                                  const ServeWork *__restrict__ work) {
    const ServeWork wk = work[blockIdx.x];
    if ((int)blockIdx.y * FPW >= wk.b) return;   // uniform per workgroup
    FitDesc a = tab[wk.sess];
    a.b = wk.b;
    a.V = wk.V;
    a.ldv = wk.ldv;
    body<KS>(a, blockIdx.y * FPW);
}

}  // namespace stile
}  // namespace isnmf
