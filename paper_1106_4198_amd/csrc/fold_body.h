// Device body of the MFMA fold (see fold.hip), shared by the single-stream
// and the batched kernels.
#pragma once

#include "common.h"

namespace isnmf {

constexpr int SLICE = 512;

struct FoldArgs {
    int F, K, b, FR, KP;
    const float *R1, *R2, *H;
    const double *W64;
    double *A, *B, *Wn;
    const double *sc;      // K: pending column scale of A and B (see OnlineDev)
    double rho;
    int update_w;
    float *part;           // slices x 2 x F x K partials (multi-slice only)
    const double *lossf;   // frame losses of the minibatch (may be null)
    double *d_loss_sum;    // += sum of lossf (may be null)
    int *flags;
};

__device__ inline floatx4 mfma16(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Wave partials of a 16 x 16 tile in LDS for the epilogue.  The MFMA result
// of lane l, register r is element (row 4 (l / 16) + r, column l % 16); a
// slab stores the 64 lanes' floatx4 with one floatx4 gap after every 16
// lanes (RSLAB floats).  The epilogue reads element (row fl, column cl) with
// lane fl + 16 q taking column cl = 4 q + j in its j-th pass, so a pass
// covers 16 consecutive rows of 4 columns (four 128-byte runs of an F-major
// FP64 array) and its LDS reads fall in 64 distinct banks.
constexpr int RSLAB = 68 * 4;

__device__ inline int red_pos(int l) { return l + (l >> 4); }   // floatx4 index in a slab

__device__ inline float red_elem(const float *slab, int fl, int cl) {
    const int sl = 16 * (fl >> 2) + cl;
    return slab[4 * red_pos(sl) + (fl & 3)];
}

typedef double __attribute__((address_space(1))) gdouble;

// A = rho A + sum_n r2 h W^2, B = rho B + sum_n r1 h (Algorithm 1), W = sqrt(A/B);
// w, a0, b0: the element's current W, A, B (a0, b0 with the pending column
// scale applied).  A and B are stored as computed here, with no pending scale.
// GLOBAL: the stores are global-memory instructions, which only the vector
// memory counter tracks (flat stores also hold up every wait for LDS reads).
template <bool GLOBAL = false>
__device__ inline void epilogue(const FoldArgs &a, int f, int k, double sa, double sb, double w,
                                double a0, double b0) {
    const size_t e = (size_t)f + (size_t)k * a.F;
    const double av = a.rho * a0 + sa * (w * w);
    const double bv = a.rho * b0 + sb;
    auto put = [](double *p, size_t i, double v) {
        if constexpr (GLOBAL)
            ((gdouble *)p)[i] = v;
        else
            p[i] = v;
    };
    put(a.A, e, av);
    put(a.B, e, bv);
    if (a.update_w) {
        double wn = w;
        if (bv > 0.0 && av >= 0.0)
            wn = sqrt(av / bv);
        else
            atomicOr(a.flags, FLAG_GUARD_W);
        put(a.Wn, e, wn);
    }
}

// Batched and served fold: one 16-row tile of f and every component k per
// 256-thread block (4 waves), KTM >= ceil(K / 16) tiles of 16 components, so
// each block reads its r1, r2 rows once for all components.  The frames are the
// contraction dimension of v_mfma_f32_16x16x4f32.  Wave w owns the component
// tiles kt = w (mod 4) and keeps four accumulators per tile, one per class of
// groups of 4 frames with (n / 4) mod 4 == v, each fed in increasing n and
// summed in class order at the end: the same chains and the same sums as the
// single-stream fold's four waves, with no reduction across waves.
// The operands of CH frames at a time are first staged in LDS by the whole
// block with 16-byte loads, all issued before the first is waited for;
// frames past the minibatch and components past K are staged as zeros.  The
// four frames of one MFMA operand fall in disjoint LDS bank ranges: with four
// or more component tiles, component c of local frame n is stored at column
// c ^ 16 (n mod 4) of its row; with fewer, rows are padded to HS floats.
// The epilogue operands are loaded after the frames, which keeps the
// registers, and so the resident blocks per CU, within the LDS bound.
// One slice of at most SLICE frames (the batched forms' limit).
template <int KTM>
struct RowsFold {
    static constexpr int CH = KTM <= 2 ? 128 : 64;             // frames per staged chunk
    static constexpr bool SWZ = KTM >= 4;                       // XOR-swizzled H rows
    static constexpr int HS = SWZ ? 16 * KTM : KTM == 1 ? 16 : 48;   // LDS floats per H row
    __device__ static int hcol(int n, int c) { return SWZ ? c ^ (16 * (n & 3)) : c; }
    static constexpr int HQ = 4 * KTM;                          // float4 of H data per row
    static constexpr int STAGE = CH * (32 + HS);                // floats: r2, r1, H
    static constexpr int TRANS = 4 * 2 * RSLAB;                 // floats: per-wave epilogue slabs
    static constexpr int LDS = STAGE > TRANS ? STAGE : TRANS;
    static constexpr int RQ = CH * 4 / 256;                     // float4 of r2 (and r1) per thread
    static constexpr int HL = CH * HQ / 256;                    // float4 of H per thread
    static_assert(RQ * 256 == CH * 4 && HL * 256 == CH * HQ, "chunk must tile the block");
};

template <int KTM>
__device__ __forceinline__ void fold_rows_body(const FoldArgs &a, int ft) {
    using C = RowsFold<KTM>;
    constexpr int KE = (KTM + 3) / 4;           // component tiles per wave
    __shared__ float4 lds4[C::LDS / 4];
    float *lds = reinterpret_cast<float *>(lds4);
    float *sR2 = lds, *sR1 = lds + C::CH * 16, *sH = lds + C::CH * 32;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int w = t >> 6;
    const int KT = (a.K + 15) / 16;
    const int f0 = ft * 16;
    const int n_hi = min(a.b, SLICE);
    const int sub = lane >> 4;             // frame within the group of 4

    // minibatch loss: wave 1 of tile 0, lane l sums frames l, l + 64, ... in
    // order, then a fixed xor butterfly over the lanes
    if (a.d_loss_sum && ft == 0 && w == 1) {
        double s = 0.0;
        for (int n = lane; n < a.b; n += 64) s += a.lossf[n];
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) s += __shfl_xor(s, m, 64);
        if (lane == 0) *a.d_loss_sum += s;
    }

    floatx4 ca[KE][4], cb[KE][4];
#pragma unroll
    for (int u = 0; u < KE; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            ca[u][v] = floatx4{0.f, 0.f, 0.f, 0.f};
            cb[u][v] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    const float4 z4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int c0 = 0; c0 < n_hi; c0 += C::CH) {
        // stage: every load first, then every LDS store
        float4 v2[C::RQ], v1[C::RQ], vh[C::HL];
#pragma unroll
        for (int i = 0; i < C::RQ; ++i) {
            const int e = t + 256 * i;
            const int n = c0 + (e >> 2);
            const size_t g = (size_t)n * a.FR + f0 + 4 * (e & 3);   // f0 + 16 <= FR
            v2[i] = n < n_hi ? *reinterpret_cast<const float4 *>(a.R2 + g) : z4;
            v1[i] = n < n_hi ? *reinterpret_cast<const float4 *>(a.R1 + g) : z4;
        }
#pragma unroll
        for (int i = 0; i < C::HL; ++i) {
            const int e = t + 256 * i;
            const int n = c0 + e / C::HQ;
            const int k = 4 * (e % C::HQ);
            vh[i] = (n < n_hi && k < a.KP)
                        ? *reinterpret_cast<const float4 *>(a.H + (size_t)n * a.KP + k) : z4;
            if (k + 3 >= a.K && k < a.KP) {   // components K .. KP of a row are padding
                if (k + 0 >= a.K) vh[i].x = 0.f;
                if (k + 1 >= a.K) vh[i].y = 0.f;
                if (k + 2 >= a.K) vh[i].z = 0.f;
                if (k + 3 >= a.K) vh[i].w = 0.f;
            }
        }
#pragma unroll
        for (int i = 0; i < C::RQ; ++i) {
            const int e = t + 256 * i;
            *reinterpret_cast<float4 *>(sR2 + 4 * e) = v2[i];
            *reinterpret_cast<float4 *>(sR1 + 4 * e) = v1[i];
        }
#pragma unroll
        for (int i = 0; i < C::HL; ++i) {
            const int e = t + 256 * i;
            const int nr = e / C::HQ;
            *reinterpret_cast<float4 *>(sH + nr * C::HS + C::hcol(nr, 4 * (e % C::HQ))) = vh[i];
        }
        __syncthreads();
        const int nmax = min(C::CH, n_hi - c0);
#pragma unroll 2
        for (int g0 = 0; g0 < nmax; g0 += 16) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (g0 + 4 * v >= nmax) break;
                const int nl = g0 + 4 * v + sub;
                const float r2 = sR2[nl * 16 + (lane & 15)];
                const float r1 = sR1[nl * 16 + (lane & 15)];
#pragma unroll
                for (int u = 0; u < KE; ++u) {
                    const int kt = w + 4 * u;
                    if (kt < KT) {
                        const float hh = sH[nl * C::HS + C::hcol(nl, 16 * kt + (lane & 15))];
                        ca[u][v] = mfma16(r2, hh, ca[u][v]);
                        cb[u][v] = mfma16(r1, hh, cb[u][v]);
                    }
                }
            }
        }
        __syncthreads();
    }
    // epilogue operands of this wave's component tiles: element
    // (f0 + lane % 16, 16 kt + 4 (lane / 16) + j) in pass j
    const int fe = f0 + (lane & 15);
    double wq[KE][4], aq[KE][4], bq[KE][4];
#pragma unroll
    for (int u = 0; u < KE; ++u) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int kc = 16 * (w + 4 * u) + 4 * sub + j;
            const bool ok = w + 4 * u < KT && fe < a.F && kc < a.K;
            const size_t e = ok ? (size_t)fe + (size_t)kc * a.F : 0;
            wq[u][j] = ok ? a.W64[e] : 0.0;
            aq[u][j] = ok ? a.A[e] / a.sc[kc] : 0.0;
            bq[u][j] = ok ? a.B[e] * a.sc[kc] : 0.0;
        }
    }

    // epilogue through a wave-private slab pair (the staging area is free
    // after the last chunk's barrier; a wave's own LDS accesses stay in order)
    float *slab = lds + w * 2 * RSLAB;
#pragma unroll
    for (int u = 0; u < KE; ++u) {
        const int kt = w + 4 * u;
        if (kt >= KT) continue;
        const floatx4 sa = ((ca[u][0] + ca[u][1]) + ca[u][2]) + ca[u][3];
        const floatx4 sb = ((cb[u][0] + cb[u][1]) + cb[u][2]) + cb[u][3];
        reinterpret_cast<floatx4 *>(slab)[red_pos(lane)] = sa;
        reinterpret_cast<floatx4 *>(slab + RSLAB)[red_pos(lane)] = sb;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int cl = 4 * sub + j;
            const float ea = red_elem(slab, lane & 15, cl);
            const float eb = red_elem(slab + RSLAB, lane & 15, cl);
            const int kc = 16 * kt + cl;
            if (fe < a.F && kc < a.K)
                epilogue(a, fe, kc, double(ea), double(eb), wq[u][j], aq[u][j], bq[u][j]);
        }
    }
}

// Single-stream fold: one 16 x 16 tile of (f, k) per 256-thread block (4
// waves), so a single minibatch spreads over ceil(F/16) ceil(K/16) blocks.
// Each element is computed exactly as fold_rows_body computes it (the same
// MFMA chain per wave over the frames with (n / 4) mod 4 == w, the same wave
// order, the same epilogue), so both give the same bits.  The four waves
// share the tile's epilogue: wave w takes its columns 4 q + w.
// nslices > 1: write the FP32 partial tile of slice `slice` instead of the
// epilogue.
__device__ __forceinline__ void fold_tile16_body(const FoldArgs &a, int tile, int slice,
                                                 int nslices) {
    __shared__ float4 red4[4 * 2 * RSLAB / 4];   // wave partials, slabs [4][2]
    float *red = reinterpret_cast<float *>(red4);
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int tiles_f = (a.F + 15) / 16;
    const int f0 = (tile % tiles_f) * 16;
    const int k0 = (tile / tiles_f) * 16;
    const int n_lo = slice * SLICE;
    const int n_hi = min(a.b, n_lo + SLICE);
    const int fa = f0 + (lane & 15);       // A operand row
    const int kb = k0 + (lane & 15);       // B operand column
    const int sub = lane >> 4;             // frame within the group of 4
    const bool fok = fa < a.F, kok = kb < a.K;

    // epilogue: wave w takes element (f0 + lane % 16, k0 + 4 (lane / 16) + w);
    // its operands are loaded before the frame rounds
    const int fe = f0 + (lane & 15);
    const int cl = 4 * sub + w;
    const int kc = k0 + cl;
    const bool eok = fe < a.F && kc < a.K;
    double wq = 0.0, aq = 0.0, bq = 0.0;
    if (eok && nslices == 1) {
        const size_t e = (size_t)fe + (size_t)kc * a.F;
        wq = a.W64[e];
        aq = a.A[e] / a.sc[kc];
        bq = a.B[e] * a.sc[kc];
    }

    // minibatch loss: wave 1 of tile 0, lane l sums frames l, l + 64, ... in
    // order, then a fixed xor butterfly over the lanes
    if (a.d_loss_sum && tile == 0 && slice == 0 && w == 1) {
        double s = 0.0;
        for (int n = lane; n < a.b; n += 64) s += a.lossf[n];
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) s += __shfl_xor(s, m, 64);
        if (lane == 0) *a.d_loss_sum += s;
    }

    floatx4 ca = {0.f, 0.f, 0.f, 0.f}, cb = {0.f, 0.f, 0.f, 0.f};
    // rounds of 8 groups per wave: every load of a round is issued before its MFMAs
    for (int g0 = n_lo + 4 * w; g0 < n_hi; g0 += 4 * 4 * 8) {
        float r2[8], r1[8], hh[8];
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            const int n = g0 + 16 * g + sub;
            const bool ok = n < n_hi;
            r2[g] = (ok && fok) ? a.R2[(size_t)n * a.FR + fa] : 0.f;
            r1[g] = (ok && fok) ? a.R1[(size_t)n * a.FR + fa] : 0.f;
            hh[g] = (ok && kok) ? a.H[(size_t)n * a.KP + kb] : 0.f;
        }
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            ca = mfma16(r2[g], hh[g], ca);
            cb = mfma16(r1[g], hh[g], cb);
        }
    }
    reinterpret_cast<floatx4 *>(red + (w * 2 + 0) * RSLAB)[red_pos(lane)] = ca;
    reinterpret_cast<floatx4 *>(red + (w * 2 + 1) * RSLAB)[red_pos(lane)] = cb;
    __syncthreads();
    auto at = [&](int v, int c) { return red_elem(red + (v * 2 + c) * RSLAB, lane & 15, cl); };
    const float sa = ((at(0, 0) + at(1, 0)) + at(2, 0)) + at(3, 0);
    const float sb = ((at(0, 1) + at(1, 1)) + at(2, 1)) + at(3, 1);
    if (!eok) return;
    if (nslices == 1) {
        epilogue(a, fe, kc, double(sa), double(sb), wq, aq, bq);
    } else {
        const size_t fk = (size_t)a.F * a.K;
        float *pa = a.part + (size_t)slice * 2 * fk;
        pa[fe + (size_t)kc * a.F] = sa;
        pa[fk + fe + (size_t)kc * a.F] = sb;
    }
}


// The fold instance for K components: the smallest of 1, 2, 4, 8 component
// tiles (K <= 128) that covers them.
inline int fold_ktm(int K) {
    const int kt = (K + 15) / 16;
    return kt <= 1 ? 1 : kt <= 2 ? 2 : kt <= 4 ? 4 : kt <= 8 ? 8 : 0;
}

inline FoldArgs fold_args(const OnlineDev &d, int b, double rho, int update_w, float *part,
                          double *d_loss_sum) {
    FoldArgs a;
    a.F = d.F;
    a.K = d.K;
    a.b = b;
    a.FR = d.FR;
    a.KP = d.KP;
    a.R1 = (const float *)d.R1;
    a.R2 = (const float *)d.R2;
    a.H = (const float *)d.Hi;
    a.W64 = d.W64;
    a.A = d.A;
    a.B = d.B;
    a.sc = d.sc;
    a.Wn = d.Wn;
    a.rho = rho;
    a.update_w = update_w;
    a.part = part;
    a.lossf = d.lossf;
    a.d_loss_sum = d_loss_sum;
    a.flags = d.flags;
    return a;
}

// Blocks of the fold: per 16-row tile (fold_rows_body), per 16 x 16 tile
// (fold_tile16_body).
inline int fold_tiles(const OnlineDev &d) { return (d.F + 15) / 16; }
inline int fold_tiles16(const OnlineDev &d) { return ((d.F + 15) / 16) * ((d.K + 15) / 16); }

}  // namespace isnmf
