// Throughput variant of the fused fit for FP32 products: each wave fits 16
// frames on v_mfma_f32_16x16x4_f32, 8 waves (128 frames) per workgroup.
//
// It computes what the other fused fits compute (the inner problem of
// Algorithm 1: I multiplicative updates of section 2.1, then the final model,
// the ratios 1/x and (eps+v)/x^2 for the fold of eq. (4), the frame loss and
// the fitted h), with the three products of an update as matrix-matrix
// products whose N dimension is a wave's 16 frames:
//   X   [F x 16] = W [F x K] . H [K x 16]        (M = rows, contraction over components)
//   NUM [K x 16] = W^T [K x F] . R2 [F x 16]     (M = components, contraction over rows)
//   DEN [K x 16] = W^T [K x F] . R1 [F x 16]
// in FP32 throughout (operands, products and accumulation).
//
// Operand layout (lane l = 16 g + n, g < 4, n < 16; frame n of the wave):
//   an MFMA's A operand is lane l -> A[n][g], its B operand lane l -> B[g][n],
//   its accumulator lane l, slot j -> C[4g + j][n].
//   X of row tile t: instruction (m-tile mt, slot j) contracts components
//     16 mt + 4 g' + j (g' = 0..3): A = W[16t + n][16mt + 4g + j], B = h of
//     component 16mt + 4g + j, which is slot j of the lane's h registers
//     (hq[mt][j] = h[16mt + 4g + j][n], the layout of the NUM/DEN
//     accumulators).
//   NUM/DEN of row tile t: instruction (slot j, m-tile mt) contracts rows
//     16t + 4g' + j: A = W[16t + 4g + j][16mt + n], B = the lane's own ratio
//     of row 16t + 4g + j (slot j of the X accumulator).
// So a wave owns all rows and components of its frames and an update needs
// no exchange with other waves.  An MFMA sums its four contraction terms in
// a fixed order, so the results do not depend on the launch.
//
// W is staged once per workgroup in LDS, row-major with a pitch of 16 MT + 4
// floats (zero past F and K): the X operand of a lane is one 16-byte read
// (four consecutive components of one row) and the W^T operand one 4-byte
// read (one component of a row); the pitch (4 mod 8) puts the 8 lanes of a
// 16-byte read phase and the 32 lanes of a 4-byte read phase on distinct
// banks.  v is read from memory at every update (16 frames x F floats per
// wave, L2- or MALL-resident), so the kernel holds no per-row registers and
// the number of row tiles T = ceil(F / 16) is a run-time value.
#pragma once

#include <type_traits>

#include "common.h"
#include "devmath.h"
#include "fold_body.h"

namespace isnmf {
namespace t32 {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int WF = 16;          // frames per wave
constexpr int NWT = 8;          // waves per workgroup
constexpr int FPW = WF * NWT;   // frames per workgroup
constexpr int MT_MAX = 4;       // K <= 64
constexpr size_t LDS_MAX = 160 * 1024;

__device__ inline f4 mfma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__host__ __device__ constexpr int pitch(int MT) { return 16 * MT + 4; }
__host__ __device__ constexpr size_t lds_bytes(int T, int MT) {
    return (size_t)16 * T * pitch(MT) * sizeof(float);
}
// Row tiles the LDS holds at MT m-tiles: F <= 16 t_max(MT).
__host__ __device__ constexpr int t_max(int MT) { return (int)(LDS_MAX / lds_bytes(1, MT)); }

// The folding final pass (FOLD) keeps W and, past it, the ratios of two row
// tiles for all 128 frames ([tile][r2, r1][frame][16 rows] floats; it first
// carries h of every frame), a per-wave slab pair for the epilogue and the
// 128 frame losses.
constexpr size_t FOLD_STAGE = (size_t)2 * 2 * FPW * 16 * 4;
constexpr size_t FOLD_EXTRA = FOLD_STAGE + (size_t)NWT * 2 * RSLAB * 4 + (size_t)FPW * 8;
__host__ __device__ constexpr size_t lds_fold_bytes(int T, int MT) {
    return lds_bytes(T, MT) + FOLD_EXTRA;
}

// Word 3 of a raw (unswizzled, stride 0) buffer descriptor on gfx9-family
// chips: 32-bit data format, every out-of-range dword reads as 0.
constexpr int BUFFER_DWORD3 = 0x00020000;

// Global-memory view of a pointer: loads through it are global (vector memory)
// instructions, whose completion counter LDS waits do not include.
typedef const float __attribute__((address_space(1))) gfloat;
__device__ inline gfloat *gptr(const float *p) { return (gfloat *)p; }

// MT m-tiles of 16 components run on the matrix pipe; the KR <= 4 components
// after them (16 MT .. 16 MT + KR - 1: K = 50 is 3 m-tiles and 2 remainder
// components) run on the VALU, instead of a fourth m-tile of which 14 of 16
// rows would be zero.  The remainder columns sit in the pitch padding of the
// LDS rows, so the LDS layout is the same.
// FOLD: the workgroup holds the stream's whole minibatch (b <= 128, n_first =
// 0) and folds it (a.fold) instead of writing R1 and R2.
template <int MT, int KR, bool FOLD>
__device__ inline void body(const FitDesc &a, int n_first) {
    constexpr int P = pitch(MT);
    static_assert(KR >= 0 && KR <= 4 && 16 * MT + KR <= P, "remainder fits the pitch padding");
    extern __shared__ float wl[];   // [16 T][P]
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
    const int g = lane >> 4;
    const int n = lane & 15;
    const int F = a.F, K = a.K;
    const int T = (F + 15) >> 4;
    const int fr = n_first + WF * w + n;   // this lane's frame (B / C column)
    const bool fok = fr < a.b;
    const float eps = a.eps;

    // ---- W into LDS (zero past F and K, every column of the pitch): thread r
    // takes row r, with every load issued before the first is used
    {
        gfloat *W = gptr(a.W);
        for (int r = threadIdx.x; r < 16 * T; r += NWT * 64) {
            const bool rok = r < F;
#pragma unroll
            for (int c4 = 0; c4 < P / 4; ++c4) {
                f4 q;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int c = 4 * c4 + j;
                    const bool ok = rok && c < K;
                    const float x = W[ok ? r + (size_t)c * F : 0];
                    q[j] = ok ? x : 0.f;
                }
                *reinterpret_cast<f4 *>(wl + r * P + 4 * c4) = q;
            }
        }
    }

    // v at the lane's rows 16t + 4g + j of its frame, through a buffer
    // descriptor per wave whose range ends at the last float of the
    // minibatch's last frame: a load past it (rows past F of that frame,
    // frames past the minibatch) returns 0 in hardware, so the loads need no
    // clamps.  Rows past F of the other frames read the next frame; only the
    // last row tile (t = T - 1) has such rows, and TAIL (a compile-time flag)
    // marks the code that may meet it and masks them.  A wave's frames never
    // mix (each is one column of every product), so lanes past the
    // minibatch compute on zeros and their results are dropped.
    const int f0w = n_first + WF * w;
    const int nval = max(0, min(WF, a.b - f0w));
    const int nrec = nval ? (int)(((size_t)(nval - 1) * a.ldv + F) * sizeof(float)) : 0;
    const __amdgpu_buffer_rsrc_t vrsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(a.V + (size_t)f0w * a.ldv), (short)0, nrec, BUFFER_DWORD3);
    const int voff = (n * a.ldv + 4 * g) * (int)sizeof(float);
    // one 16-byte load per tile (each dword range-checked on its own)
    auto load_v = [&](int t) {
        return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(vrsrc, voff + 64 * t, 0, 0));
    };
    // eps + v, and 0 on rows past F
    auto vprime = [&](int t, const f4 &v, auto tail) {
        f4 o;
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = eps + v[j];
        if constexpr (decltype(tail)::value) {
            const int r0 = 16 * t + 4 * g;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (r0 + j >= F) o[j] = 0.f;
        }
        return o;
    };
    // X accumulator start: eps, or 1 on rows past F (W = 0 there; x only needs to be > 0)
    auto cinit = [&](int t, auto tail) {
        f4 c = {eps, eps, eps, eps};
        if constexpr (decltype(tail)::value) {
            const int r0 = 16 * t + 4 * g;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (r0 + j >= F) c[j] = 1.f;
        }
        return c;
    };
    constexpr std::true_type TAIL{};
    constexpr std::false_type FULL{};
    // ---- h (FP32): lane (g, n) holds components 16 mt + 4 g + j of frame n;
    // hr[i] is remainder component 16 MT + i of frame n (the same in the four
    // lanes of the frame)
    float hq[MT][4];
    float hr[KR > 0 ? KR : 1];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 16 * mt + 4 * g + j;
            hq[mt][j] = k < K ? ((a.warm && fok) ? a.Hb[(size_t)fr * a.ldh + k] : 1.f) : 0.f;
        }
#pragma unroll
    for (int i = 0; i < KR; ++i) {
        const int k = 16 * MT + i;
        hr[i] = k < K ? ((a.warm && fok) ? a.Hb[(size_t)fr * a.ldh + k] : 1.f) : 0.f;
    }
    __syncthreads();   // W in LDS

    // remainder operands of a row: KR floats (2 or 4 read at once)
    typedef float RV __attribute__((ext_vector_type(KR <= 2 ? 2 : 4)));

    // X operands of row tile t: components 16 mt + 4g .. + 3 of row 16t + n
    auto load_wx = [&](int t, f4 (&o)[MT]) {
        const float *p = wl + (16 * t + n) * P + 4 * g;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) o[mt] = *reinterpret_cast<const f4 *>(p + 16 * mt);
    };
    // W^T operands of row tile t: component 16 mt + n of rows 16t + 4g + j; and
    // the remainder components of those rows (one 16-byte read per row, the
    // same address in the 16 lanes of a row group)
    auto load_wt = [&](int t, float (&o)[4][MT], RV (&r)[4]) {
        const float *p = wl + (16 * t + 4 * g) * P;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) o[j][mt] = p[j * P + 16 * mt + n];
            if constexpr (KR > 0) r[j] = *reinterpret_cast<const RV *>(p + j * P + 16 * MT);
        }
    };
    // matrix-pipe part of the model: one accumulation chain (the matrix pipe
    // accumulates back to back); its result is read a half trip later
    auto model_ops = [&](int t, const f4 (&o)[MT], auto tail) {
        f4 x = cinit(t, tail);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) x = mfma(o[mt][j], hq[mt][j], x);
        return x;
    };
    // the remainder components' part of the model, added to the matrix part
    auto model_rest = [&](f4 x, const RV (&r)[4]) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < KR; ++i) x[j] = fmaf(r[j][i], hr[i], x[j]);
        return x;
    };

    int guard = 0;
    for (int it = 0; it < a.iters; ++it) {
        f4 na[MT], da[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            na[mt] = f4{0.f, 0.f, 0.f, 0.f};
            da[mt] = f4{0.f, 0.f, 0.f, 0.f};
        }
        float nr[KR > 0 ? KR : 1], dr[KR > 0 ? KR : 1];
#pragma unroll
        for (int i = 0; i < KR; ++i) nr[i] = dr[i] = 0.f;
        // Software pipeline over the row tiles: tile t + 1's model products go
        // to the matrix pipe before tile t's ratios are formed; the LDS
        // operands of the next tiles and v two tiles ahead are in flight
        // meanwhile.  The loop takes two tiles per trip, so the register sets
        // alternate by name (no copies that would wait on the loads).  Same
        // products and sums as tile by tile, so the same bits.
        auto ratios = [&](int t, const f4 &xm, const RV (&wr)[4], const f4 &v, float (&r1)[4],
                          float (&r2)[4], auto tail) {
            const f4 x = model_rest(xm, wr);
            const f4 ve = vprime(t, v, tail);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                r1[j] = __builtin_amdgcn_rcpf(x[j]);
                r2[j] = ve[j] * r1[j] * r1[j];
            }
        };
        auto numden = [&](const float (&wt)[4][MT], const RV (&wr)[4], const float (&r1)[4],
                          const float (&r2)[4]) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    na[mt] = mfma(wt[j][mt], r2[j], na[mt]);
                    da[mt] = mfma(wt[j][mt], r1[j], da[mt]);
                }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < KR; ++i) {
                    nr[i] = fmaf(wr[j][i], r2[j], nr[i]);
                    dr[i] = fmaf(wr[j][i], r1[j], dr[i]);
                }
        };
        f4 wx0[MT], wx1[MT];
        float wt0[4][MT], wt1[4][MT];
        RV wr0[4], wr1[4];
        load_wx(0, wx0);
        f4 x0 = model_ops(0, wx0, TAIL), x1 = x0;
        if (T > 1) load_wx(1, wx1);
        load_wt(0, wt0, wr0);
        // v four tiles ahead: tiles past T read zeros or the next frame, unused
        // (issued in tile order: the loop's waits count them in that order)
        f4 vq[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            vq[i] = load_v(i);
            __builtin_amdgcn_sched_barrier(0);
        }
        // One tile: X(tt) in xc, v(tt) in vc, W^T operands in wtc/wrc, X operands
        // of tile tt + 1 in wxc.  First the LDS reads of the operands of tiles
        // tt + 1 (W^T, into wtn/wrn) and tt + 2 (X, into wxn); then the model of
        // tile tt + 1 on the matrix pipe with this tile's ratios on the VALU
        // beside it, NUM/DEN of this tile, and v of tile tt + 4 into vc.
        // tail: a tile it touches may be T - 1.
        auto tile = [&](int tt, f4 &xc, f4 &xn, f4 &vc, f4 (&wxc)[MT], f4 (&wxn)[MT],
                        float (&wtc)[4][MT], float (&wtn)[4][MT], RV (&wrc)[4], RV (&wrn)[4],
                        auto tail) {
            constexpr bool TL = decltype(tail)::value;   // else tiles tt .. tt + 4 all exist
            float r1[4], r2[4];
            __builtin_amdgcn_sched_barrier(0);
            if (!TL || tt + 2 < T) load_wx(tt + 2, wxn);
            load_wt(TL ? min(tt + 1, T - 1) : tt + 1, wtn, wrn);
            __builtin_amdgcn_sched_barrier(0);   // the next operands in flight first
            if (!TL || tt + 1 < T) xn = model_ops(tt + 1, wxc, tail);
            ratios(tt, xc, wrc, vc, r1, r2, tail);
            vc = load_v(tt + 4);
            numden(wtc, wrc, r1, r2);
        };
        // four tiles per trip, so the register sets rotate by name
        auto trip = [&](int t, auto tail) {
            constexpr bool TL = decltype(tail)::value;
            tile(t, x0, x1, vq[0], wx1, wx0, wt0, wt1, wr0, wr1, tail);
            if (TL && t + 1 >= T) return;
            tile(t + 1, x1, x0, vq[1], wx0, wx1, wt1, wt0, wr1, wr0, tail);
            if (TL && t + 2 >= T) return;
            tile(t + 2, x0, x1, vq[2], wx1, wx0, wt0, wt1, wr0, wr1, tail);
            if (TL && t + 3 >= T) return;
            tile(t + 3, x1, x0, vq[3], wx0, wx1, wt1, wt0, wr1, wr0, tail);
        };
        // trips whose tiles t .. t + 4 all lie before the last tile need no masks
        int t = 0;
        for (; t + 4 < T - 1; t += 4) trip(t, FULL);
        for (; t < T; t += 4) trip(t, TAIL);
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
        // remainder components: the four row groups' partial sums of the
        // frame, combined by a fixed xor butterfly (the same bits in the four
        // lanes), then the same update in each
#pragma unroll
        for (int i = 0; i < KR; ++i) {
            float N = nr[i], D = dr[i];
            N += __shfl_xor(N, 16, 64);
            D += __shfl_xor(D, 16, 64);
            N += __shfl_xor(N, 32, 64);
            D += __shfl_xor(D, 32, 64);
            if (16 * MT + i < K) {
                if (D > 0.f && N >= 0.f)
                    hr[i] *= __builtin_amdgcn_sqrtf(N * __builtin_amdgcn_rcpf(D));
                else if (fok)
                    guard = 1;
            }
        }
    }
    if (guard) atomicOr(a.flags, FLAG_GUARD_H);

    // ---- final model: R1, R2 for the fold, or the fold itself, the frame loss
    // (FP64 terms, as the objective), and the check of v
    double ls = 0.0;
    int bad = 0;
    f4 wx[MT];
    float wt_unused[4][MT];
    RV wr[4];
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
            if (g == 0) {
#pragma unroll
                for (int i = 0; i < KR; ++i) {
                    const int k = 16 * MT + i;
                    if (k < K) {
                        a.Hi[(size_t)fr * a.KP + k] = hr[i];
                        if (a.Hb) a.Hb[(size_t)fr * a.ldh + k] = hr[i];
                    }
                }
            }
        }
    };
    if constexpr (FOLD) {
        // The fold of the minibatch (Algorithm 1's statistics update and W =
        // sqrt(A/B)) in this workgroup, as in the BF16 tile variant's folding
        // pass: round r takes row tiles 2r and 2r + 1, whose ratios every wave
        // forms for its frames (the values the separate fold would read) and
        // stores in LDS; then wave w folds row tile 2r + (w & 1) over
        // component tile w >> 1 for all frames with the separate fold's MFMA
        // chains, chain sums and epilogue, so the bits are those of the fit
        // followed by that fold.  One ratio buffer, two barriers per round.
        const FoldArgs &fa0 = *a.fold;
        FoldArgs fa = fa0;
        fa.b = a.b;
        constexpr int RB = 2 * FPW * 16;             // floats per staged row tile (r2, r1)
        float *stg = wl + 16 * T * P;
        float *slab = stg + 2 * RB + w * 2 * RSLAB;
        double *lsh = reinterpret_cast<double *>(stg + 2 * RB + NWT * 2 * RSLAB);
        const int KT = (K + 15) / 16;
        const int CW = 16 * KT;                      // LDS floats per frame of h
        const int kt = w >> 1, uw = w & 1;
        const bool kact = kt < KT;                   // uniform per wave
        // h of every frame through the ratio buffer (zero past the minibatch
        // and past K, as the separate fold stages it); wave w keeps the column
        // of its component tile for all 128 frames
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = 16 * mt + 4 * g + j;
                if (k < CW) stg[(WF * w + n) * CW + k] = (fok && k < K) ? hq[mt][j] : 0.f;
            }
        if (g == 0) {
            for (int k = 16 * MT; k < CW; ++k) {
                const int i = k - 16 * MT;
                float hv = 0.f;
#pragma unroll
                for (int q = 0; q < KR; ++q)
                    if (q == i) hv = hr[q];
                stg[(WF * w + n) * CW + k] = (fok && k < K) ? hv : 0.f;
            }
        }
        __syncthreads();
        float hh[32];
#pragma unroll
        for (int m = 0; m < 32; ++m) hh[m] = kact ? stg[(4 * m + g) * CW + 16 * kt + n] : 0.f;
        store_h();
        __syncthreads();   // the buffer's next use is the first round's ratios
        const gdouble *gW = (const gdouble *)fa.W64;
        const gdouble *gA = (const gdouble *)fa.A;
        const gdouble *gB = (const gdouble *)fa.B;
        double scq[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int kc = 16 * kt + 4 * g + j;
            scq[j] = kact && kc < K ? fa.sc[kc] : 1.0;
        }
        const int R = (T + 1) / 2;
        for (int r = 0; r < R; ++r) {
            const int tf = 2 * r + uw;                 // this wave's fold row tile
            const bool fact = kact && tf < T;          // uniform per wave
            const int fe = 16 * tf + n;
            // epilogue operands, element (16 tf + n, 16 kt + 4 g + j) in pass j
            double eo[3][4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int kc = 16 * kt + 4 * g + j;
                const bool ok = fact && fe < F && kc < K;
                const size_t e = ok ? (size_t)fe + (size_t)kc * F : 0;
                eo[0][j] = ok ? gW[e] : 0.0;
                eo[1][j] = ok ? gA[e] : 0.0;
                eo[2][j] = ok ? gB[e] : 0.0;
            }
            // ratios of row tiles 2r and 2r + 1 of this wave's frames (zero for
            // frames past the minibatch and rows past F) and the loss terms
            for (int u = 0; u < 2; ++u) {
                const int t = 2 * r + u;
                if (t >= T) break;   // uniform
                load_wx(t, wx);
                load_wt(t, wt_unused, wr);
                const f4 xf = model_rest(model_ops(t, wx, TAIL), wr);
                const f4 v0 = load_v(t);
                const int r0 = 16 * t + 4 * g;
                f4 r1, r2;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bool ok = fok && r0 + j < F;
                    const float v = ok ? v0[j] : 0.f;
                    bad |= !isfinite(v);
                    const float ve = eps + v;
                    const float rr = __builtin_amdgcn_rcpf(xf[j]);
                    r1[j] = ok ? rr : 0.f;
                    r2[j] = ok ? ve * rr * rr : 0.f;
                    if (ok) ls += dis_term(a.epsd + double(v), double(xf[j]));
                }
                float *sr = stg + u * RB;
                *reinterpret_cast<f4 *>(sr + (WF * w + n) * 16 + 4 * g) = r2;
                *reinterpret_cast<f4 *>(sr + FPW * 16 + (WF * w + n) * 16 + 4 * g) = r1;
            }
            __syncthreads();
            if (fact) {
                const float *sr2 = stg + uw * RB, *sr1 = sr2 + FPW * 16;
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
            __syncthreads();   // the ratio buffer is read; the next round rewrites it
        }
        if (bad) atomicOr(a.flags, FLAG_NONFINITE_V);
        // frame n's loss: lanes n, n + 16, n + 32, n + 48, in that order; the
        // minibatch loss as the separate fold adds it (wave 1, lane l sums
        // frames l, l + 64 in order, then a fixed xor butterfly)
        const double l1 = __shfl_xor(ls, 16, 64);
        const double l2 = __shfl_xor(ls, 32, 64);
        const double l3 = __shfl_xor(ls, 48, 64);
        const double lframe = ((ls + l1) + l2) + l3;
        if (g == 0 && fok) a.lossf[fr] = lframe;
        if (g == 0) lsh[WF * w + n] = lframe;
        __syncthreads();
        if (fa.d_loss_sum && w == 1) {
            double sl = 0.0;
            for (int m = lane; m < a.b; m += 64) sl += lsh[m];
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) sl += __shfl_xor(sl, m, 64);
            if (lane == 0) *fa.d_loss_sum += sl;
        }
        return;
    }
    load_wx(0, wx);
    f4 x = model_ops(0, wx, TAIL);
    f4 v0 = load_v(0);
    for (int t = 0; t < T; ++t) {
        load_wt(t, wt_unused, wr);
        f4 xn = x;
        if (t + 1 < T) {
            load_wx(t + 1, wx);
            xn = model_ops(t + 1, wx, TAIL);
        }
        const f4 v1 = load_v(min(t + 1, T - 1));
        const f4 xf = model_rest(x, wr);
        const int r0 = 16 * t + 4 * g;
        f4 r1, r2;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool ok = fok && r0 + j < F;
            const float v = ok ? v0[j] : 0.f;
            bad |= !isfinite(v);
            const float ve = eps + v;
            const float r = __builtin_amdgcn_rcpf(xf[j]);
            r1[j] = ok ? r : 0.f;
            r2[j] = ok ? ve * r * r : 0.f;
            if (ok) ls += dis_term(a.epsd + double(v), double(xf[j]));
        }
        // FR is a multiple of 64, so rows r0 .. r0 + 3 lie in the frame's buffer row
        if (fok) {
            *reinterpret_cast<f4 *>(a.R1 + (size_t)fr * a.FR + r0) = r1;
            *reinterpret_cast<f4 *>(a.R2 + (size_t)fr * a.FR + r0) = r2;
        }
        x = xn;
        v0 = v1;
    }
    if (bad) atomicOr(a.flags, FLAG_NONFINITE_V);
    // frame n's loss: lanes n, n + 16, n + 32, n + 48, in that order
    const double l1 = __shfl_xor(ls, 16, 64);
    const double l2 = __shfl_xor(ls, 32, 64);
    const double l3 = __shfl_xor(ls, 48, 64);
    if (g == 0 && fok) a.lossf[fr] = ((ls + l1) + l2) + l3;
    store_h();
}

template <int MT, int KR>
__global__ __launch_bounds__(NWT * 64) void fit_t32_kernel(FitDesc a) {
    body<MT, KR, false>(a, blockIdx.x * FPW);
}

// Batched form: item = (stream, tile of 128 frames); tiles past the stream's
// minibatch of this step exit.  FOLD: every stream of the launch has one tile
// (b <= 128) and a fold descriptor.
template <int MT, int KR, bool FOLD>
__global__ __launch_bounds__(NWT * 64) void fit_t32_multi_kernel(const FitDesc *__restrict__ descs,
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
    body<MT, KR, FOLD>(a, it.y * FPW);
}

// Served form: grid (chunk i, 128-frame tile j) over a step's work list.
template <int MT, int KR>
__global__ __launch_bounds__(NWT * 64) void fit_t32_work_kernel(const FitDesc *__restrict__ tab,
                                                                const ServeWork *__restrict__ work) {
    const ServeWork wk = work[blockIdx.x];
    if ((int)blockIdx.y * FPW >= wk.b) return;   // uniform per workgroup
    FitDesc a = tab[wk.sess];
    a.b = wk.b;
    a.V = wk.V;
    a.ldv = wk.ldv;
    body<MT, KR, false>(a, blockIdx.y * FPW);
}

template <int MT, int KR>
hipError_t run(const FitDesc *a, int b, const FitDesc *d, const int2 *items, int n,
               const long long *cur, const int *beff, const FitDesc *tab, const ServeWork *work,
               int tiles, int T, bool fold, hipStream_t s) {
    if (T < 1 || T > t_max(MT)) return hipErrorInvalidValue;
    const size_t lds = lds_bytes(T, MT);
    if (fold) {
        if (!d || lds_fold_bytes(T, MT) > LDS_MAX) return hipErrorNotSupported;
        static const hipError_t a4 = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&fit_t32_multi_kernel<MT, KR, true>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX);
        if (a4 != hipSuccess) return a4;
        fit_t32_multi_kernel<MT, KR, true><<<n, NWT * 64, lds_fold_bytes(T, MT), s>>>(d, items, cur,
                                                                                     beff);
        return hipGetLastError();
    }
    // the largest dynamic LDS any launch of the kernel asks for, set once
    static const hipError_t a1 = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&fit_t32_kernel<MT, KR>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX);
    static const hipError_t a2 = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&fit_t32_multi_kernel<MT, KR, false>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX);
    static const hipError_t a3 = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&fit_t32_work_kernel<MT, KR>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX);
    if (work) {
        if (a3 != hipSuccess) return a3;
        fit_t32_work_kernel<MT, KR><<<dim3(n, tiles), NWT * 64, lds, s>>>(tab, work);
    } else if (d) {
        if (a2 != hipSuccess) return a2;
        fit_t32_multi_kernel<MT, KR, false><<<n, NWT * 64, lds, s>>>(d, items, cur, beff);
    } else {
        if (a1 != hipSuccess) return a1;
        fit_t32_kernel<MT, KR><<<(b + FPW - 1) / FPW, NWT * 64, lds, s>>>(*a);
    }
    return hipGetLastError();
}

// Launch of the (MT, KR) instance; explicitly instantiated per MT in
// fit_t32_m*.hip so the instances build in parallel.
template <int MT>
hipError_t launch_mt(int KR, const FitDesc *a, int b, const FitDesc *d, const int2 *items, int n,
                     const long long *cur, const int *beff, const FitDesc *tab,
                     const ServeWork *work, int tiles, int T, bool fold, hipStream_t s) {
    if constexpr (MT == MT_MAX) {
        if (KR != 0) return hipErrorNotSupported;
        return run<MT, 0>(a, b, d, items, n, cur, beff, tab, work, tiles, T, fold, s);
    } else {
        switch (KR) {
            case 0: return run<MT, 0>(a, b, d, items, n, cur, beff, tab, work, tiles, T, fold, s);
            case 1: return run<MT, 1>(a, b, d, items, n, cur, beff, tab, work, tiles, T, fold, s);
            case 2: return run<MT, 2>(a, b, d, items, n, cur, beff, tab, work, tiles, T, fold, s);
            case 3: return run<MT, 3>(a, b, d, items, n, cur, beff, tab, work, tiles, T, fold, s);
            case 4: return run<MT, 4>(a, b, d, items, n, cur, beff, tab, work, tiles, T, fold, s);
            default: return hipErrorNotSupported;
        }
    }
}

#define ISNMF_T32_SIG(MTV)                                                                     \
    hipError_t launch_mt<MTV>(int, const FitDesc *, int, const FitDesc *, const int2 *, int,   \
                              const long long *, const int *, const FitDesc *,                 \
                              const ServeWork *, int, int, bool, hipStream_t)
#define ISNMF_T32_EXTERN(MTV) extern template ISNMF_T32_SIG(MTV);
#define ISNMF_T32_INSTANTIATE(MTV) template ISNMF_T32_SIG(MTV);

}  // namespace t32
}  // namespace isnmf
