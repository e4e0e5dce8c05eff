// Streamed variant of the 16-frame tile fit for BF16 products: the same
// per-wave products as fit_tile.h (16 frames per wave on
// v_mfma_f32_16x16x32_bf16, 8 waves per workgroup, no exchange between waves),
// for shapes whose W operands do not fit in LDS (F > 640 or K > 64).
//
// Per update, the 32-row contraction steps s = 0 .. S-1 run in order.  The W
// operands of one step (X operands of row tiles 2s and 2s+1, W^T operands of
// rows 32s .. 32s+31, for every component) pass through a two-slot LDS
// window: the whole workgroup loads the operands of later steps from the
// 16-bit copies (row-major W16r for X, column-major W16c for W^T) into
// registers while it computes step s, writes step s+1's to the other slot, and one barrier
// separates the steps.  v of a step's rows is re-read from V (FP32) at every
// step instead of being held in registers.  Both are loaded two steps ahead,
// so that a load has two steps' work to arrive in; the registers then hold
// only h, the NUM/DEN accumulators and three steps' loads, so S is a
// run-time value (F up to 32 * S_MAX rows).
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

// Buffer descriptors: a load at a byte offset at or past the descriptor's
// size returns zeros and never faults, so the bounds checks below select an
// offset instead of branching around the load.
constexpr int BUFFER_DWORD3 = 0x00020000;
constexpr unsigned OUTSIDE = 0x80000000u;   // beyond every descriptor's size

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void *base, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0,
                                             (int)(bytes < 0x7fffffff ? bytes : 0x7fffffff),
                                             BUFFER_DWORD3);
}

// 4 consecutive 16-bit values (8 bytes, 8-byte aligned) at element `idx`, or zeros
__device__ inline uint2 ld4(__amdgpu_buffer_rsrc_t r, int idx, bool ok) {
    return __builtin_bit_cast(
        uint2, __builtin_amdgcn_raw_buffer_load_b64(r, ok ? 2u * (unsigned)idx : OUTSIDE, 0, 0));
}

// uint4 elements of one LDS window slot: X operands [2][KS][64], then W^T
// operands [2 KS][64]
__host__ __device__ constexpr int slot_elems(int KS) { return 2 * KS * 64 + 2 * KS * 64; }
__host__ __device__ constexpr size_t lds_bytes(int KS) { return (size_t)2 * slot_elems(KS) * 16; }

// Element e of step s's window: the same operand bits fit_tile.h keeps for
// row tiles 2s, 2s+1 (X) and contraction step s (W^T).
// wr: W16r (F x KP), wc: W16c (K x FR).  A wave's 64 lanes hold 64
// consecutive e from a multiple of 64, so whether e names an X operand
// (e < 2 KS 64) is uniform over the wave: the descriptor is chosen by a
// scalar select and both index forms are computed, with no branch.  e at or
// past the slot size names a component past K and reads zeros.
template <int KS>
__device__ inline uint4 window_elem(const FitDesc &a, __amdgpu_buffer_rsrc_t wr,
                                    __amdgpu_buffer_rsrc_t wc, int s, int e) {
    constexpr int NX = 2 * KS * 64;
    const bool isx = __builtin_amdgcn_readfirstlane(e) < NX;
    const int l = e & 63;
    // X operand: row tile 2 s + (e / 64) / KS, component step (e / 64) mod KS
    const int cx = (e >> 6) % KS, t = 2 * s + (e >> 6) / KS;
    const int row = 16 * t + (l & 15), k0 = 32 * cx + 4 * (l >> 4);
    // W^T operand: m-tile (e - NX) / 64; rows r0.., r0 + 16.. lie below
    // 32 ceil(F / 32) <= FR, and W16c is zero past F
    const int mt = (e - NX) >> 6;
    const int k = 16 * mt + (l & 15), r0 = 32 * s + 4 * (l >> 4);
    const __amdgpu_buffer_rsrc_t r = isx ? wr : wc;
    const int i0 = isx ? row * a.KP + k0 : k * a.FR + r0;
    const bool ok0 = isx ? (row < a.F && k0 < a.KP) : k < a.K;
    const bool ok1 = isx ? (row < a.F && k0 + 16 < a.KP) : k < a.K;
    const uint2 lo = ld4(r, i0, ok0);
    const uint2 hi = ld4(r, i0 + 16, ok1);
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
    __builtin_assume(tid < NWT * 64);
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int g = lane >> 4;
    const int n = lane & 15;
    const int F = a.F, K = a.K;
    const int S = (F + 31) / 32;
    const int fr = n_first + WF * w + n;          // this lane's frame (B/C column)
    const bool fok = fr < a.b;
    const float eps = a.eps;
    // the wave's frames n_first + 16 w .. (nval of them) as one descriptor
    const int f0w = n_first + WF * __builtin_amdgcn_readfirstlane(w);
    const int nval = a.b - f0w < 0 ? 0 : (a.b - f0w < WF ? a.b - f0w : WF);
    const __amdgpu_buffer_rsrc_t vr =
        rsrc(a.V + (size_t)f0w * a.ldv, nval ? ((size_t)(nval - 1) * a.ldv + F) * 4 : 0);
    const __amdgpu_buffer_rsrc_t wr = rsrc(a.W16r, (size_t)F * a.KP * 2);
    const __amdgpu_buffer_rsrc_t wc = rsrc(a.W16c, (size_t)K * a.FR * 2);

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

    // ---- staging: step q's W operands and v are loaded two steps ahead into
    // register set q mod 2 (Stage), its W operands are written to LDS slot
    // q mod 2 at the end of step q - 1, and its v is read from the set at the
    // start of step q.  Loads of step q + 2 are thus in flight during steps q
    // and q + 1.  v: rows 32 s + 16 u + 4 g + j (u < 2, j < 4) of this lane's
    // frame, 0 past F or past the minibatch.
    struct Stage {
        uint4 w[EPT];
        float v[8];
    };
    auto fetch_w = [&](Stage &st, int s) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) st.w[i] = window_elem<KS>(a, wr, wc, s, tid + NWT * 64 * i);
    };
    // The four rows of one u come in one 16-byte load: a lane's frame spans
    // one cache line per step, so this touches a quarter of the lines that
    // four 4-byte loads would.  Rows past F read the next frame, the caller's
    // padding or zeros; every use masks them (not here, which would wait for
    // the load).
    auto fetch_v = [&](Stage &st, int s) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int row = 32 * s + 16 * u + 4 * g;
            const f4 q4 = __builtin_bit_cast(
                f4, __builtin_amdgcn_raw_buffer_load_b128(
                        vr, fok ? 4u * (unsigned)(n * a.ldv + row) : OUTSIDE, 0, 0));
#pragma unroll
            for (int j = 0; j < 4; ++j) st.v[4 * u + j] = q4[j];
        }
    };
    auto fetch = [&](Stage &st, int s) {
        fetch_w(st, s);
        fetch_v(st, s);
    };
    auto store = [&](const Stage &st, int slot) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + NWT * 64 * i;
            if (__builtin_amdgcn_readfirstlane(e) < SE) win[slot * SE + e] = st.w[i];
        }
    };
    const int QU = a.iters * S;   // steps of the update passes
    const int QT = QU + S;        // and of the final pass
    Stage sa, sb;
    fetch(sa, 0);
    if (QT > 1) fetch(sb, 1 % S);
    store(sa, 0);
    __syncthreads();

    int guard = 0, bad = 0;
    double ls = 0.0;
    // Step q on set cur (the other set, nxt, holds step q + 1): cur's W
    // operands are in LDS, so its w registers take step q + 2's first; its v
    // registers take step q + 2's once this step has read them, so that a
    // set's registers keep one place from trip to trip.  The last two steps
    // load operands no step uses (those of steps 0 and 1 again) rather than
    // branch around the loads.
    auto begin_step = [&](int q, Stage &cur) { fetch_w(cur, (q + 2) % S); };
    auto after_v = [&](int q, Stage &cur) { fetch_v(cur, (q + 2) % S); };
    auto end_step = [&](int q, const Stage &nxt) {
        if (q + 1 < QT) store(nxt, (q + 1) & 1);   // its last readers passed the barrier of step q - 1
        __syncthreads();
    };
    auto model = [&](int q, int s, f4 (&x)[2]) {
        const uint4 *wx = win + (q & 1) * SE;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            x[u] = cinit(2 * s + u);
#pragma unroll
            for (int c = 0; c < KS; ++c)
                x[u] = mfma(__builtin_bit_cast(bf16x8, wx[(u * KS + c) * 64 + lane]), hb[c], x[u]);
        }
    };

    // update passes
    f4 na[MT], da[MT];
    auto update_step = [&](int q, int s, Stage &cur, const Stage &nxt) {
        begin_step(q, cur);
        if (s == 0) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                na[mt] = f4{0.f, 0.f, 0.f, 0.f};
                da[mt] = f4{0.f, 0.f, 0.f, 0.f};
            }
        }
        f4 x[2];
        model(q, s, x);
        float r1[8], r2[8];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float r = __builtin_amdgcn_rcpf(x[u][j]);
                r1[4 * u + j] = r;
                const bool in = 32 * s + 16 * u + 4 * g + j < F && fok;
                r2[4 * u + j] = (in ? eps + cur.v[4 * u + j] : 0.f) * r * r;
            }
        after_v(q, cur);
        const bf16x8 b1 = __builtin_bit_cast(
            bf16x8, uint4{pack2(r1[0], r1[1]), pack2(r1[2], r1[3]), pack2(r1[4], r1[5]),
                          pack2(r1[6], r1[7])});
        const bf16x8 b2 = __builtin_bit_cast(
            bf16x8, uint4{pack2(r2[0], r2[1]), pack2(r2[2], r2[3]), pack2(r2[4], r2[5]),
                          pack2(r2[6], r2[7])});
        const uint4 *wn = win + (q & 1) * SE + 2 * KS * 64;
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
        end_step(q, nxt);
    };
    // two steps per trip, so that each set keeps its role in the code
    int q = 0, s = 0;
    while (q < QU) {
        update_step(q, s, sa, sb);
        ++q;
        s = s + 1 == S ? 0 : s + 1;
        if (q == QU) break;
        update_step(q, s, sb, sa);
        ++q;
        s = s + 1 == S ? 0 : s + 1;
    }

    // final model: R1, R2 for the fold (FP32) and the frame loss
    auto final_step = [&](int q, int s, Stage &cur, const Stage &nxt) {
        begin_step(q, cur);
        f4 x[2];
        model(q, s, x);
        float vc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) vc[i] = cur.v[i];
        after_v(q, cur);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int row0 = 32 * s + 16 * u + 4 * g;
            f4 r1, r2;
            float l = 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool in = row0 + j < F && fok;
                const float v = in ? vc[4 * u + j] : 0.f;
                bad |= !isfinite(v);
                const float ve = in ? eps + v : 0.f;
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
        end_step(q, nxt);
    };
    for (s = 0; q < QT; ++q, ++s) {
        if (q & 1)
            final_step(q, s, sb, sa);
        else
            final_step(q, s, sa, sb);
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
