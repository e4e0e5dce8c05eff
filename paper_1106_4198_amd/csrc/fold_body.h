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

// A = rho A + sum_n r2 h W^2, B = rho B + sum_n r1 h (Algorithm 1), W = sqrt(A/B);
// w, a0, b0: the element's current W, A, B (a0, b0 with the pending column
// scale applied).  A and B are stored as computed here, with no pending scale.
__device__ inline void epilogue(const FoldArgs &a, int f, int k, double sa, double sb, double w,
                                double a0, double b0) {
    const size_t e = (size_t)f + (size_t)k * a.F;
    const double av = a.rho * a0 + sa * (w * w);
    const double bv = a.rho * b0 + sb;
    a.A[e] = av;
    a.B[e] = bv;
    if (a.update_w) {
        double wn = w;
        if (bv > 0.0 && av >= 0.0)
            wn = sqrt(av / bv);
        else
            atomicOr(a.flags, FLAG_GUARD_W);
        a.Wn[e] = wn;
    }
}

// Batched and served fold: one 16-row tile of f and every component k per
// 256-thread block (4 waves), KTM >= ceil(K / 16) tiles of 16 components, so
// each block reads its r1, r2 rows once for all components.  The frames are the
// contraction dimension of v_mfma_f32_16x16x4f32: wave w takes the groups of
// 4 frames with (n / 4) mod 4 == w, in increasing n, and reads each group's
// r1, r2 operand once for all component tiles; the four per-wave partials of
// an element are summed in wave order.  Wave w then applies the FP64
// epilogue to the component tiles kt = w (mod 4).
// The operands of CH frames at a time are first staged in LDS by the whole
// block with 16-byte loads, all issued before the first is waited for, so a
// block keeps its whole chunk in flight; frames past the minibatch and
// components past K are staged as zeros.  H rows sit HS floats apart in LDS,
// so that the four frames of one MFMA operand fall in disjoint bank ranges.
// One slice of at most SLICE frames (the batched forms' limit).
template <int KTM>
struct RowsFold {
    static constexpr int CH = KTM <= 2 ? 128 : 64;             // frames per staged chunk
    static constexpr int HS = KTM == 1 ? 16 : 16 * KTM + 16;   // LDS floats per H row
    static constexpr int HQ = 4 * KTM;                          // float4 of H data per row
    static constexpr int STAGE = CH * (32 + HS);                // floats: r2, r1, H
    static constexpr int RED = 4 * KTM * 2 * 64 * 4;            // floats: wave partials
    static constexpr int LDS = STAGE > RED ? STAGE : RED;
    static constexpr int RQ = CH * 4 / 256;                     // float4 of r2 (and r1) per thread
    static constexpr int HL = CH * HQ / 256;                    // float4 of H per thread
    static_assert(RQ * 256 == CH * 4 && HL * 256 == CH * HQ, "chunk must tile the block");
};

template <int KTM>
__device__ __forceinline__ void fold_rows_body(const FoldArgs &a, int ft) {
    using C = RowsFold<KTM>;
    constexpr int KE = (KTM + 3) / 4;           // epilogue tiles per wave
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

    // epilogue operands of this wave's component tiles, loaded before the frames
    double wq[KE][4], aq[KE][4], bq[KE][4];
#pragma unroll
    for (int u = 0; u < KE; ++u) {
        const int kc = 16 * (w + 4 * u) + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = f0 + 4 * sub + r;
            const bool ok = w + 4 * u < KT && f < a.F && kc < a.K;
            const size_t e = ok ? (size_t)f + (size_t)kc * a.F : 0;
            wq[u][r] = ok ? a.W64[e] : 0.0;
            aq[u][r] = ok ? a.A[e] / a.sc[kc] : 0.0;
            bq[u][r] = ok ? a.B[e] * a.sc[kc] : 0.0;
        }
    }

    // minibatch loss: wave 1 of tile 0, lane l sums frames l, l + 64, ... in
    // order, then a fixed xor butterfly over the lanes
    if (a.d_loss_sum && ft == 0 && w == 1) {
        double s = 0.0;
        for (int n = lane; n < a.b; n += 64) s += a.lossf[n];
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) s += __shfl_xor(s, m, 64);
        if (lane == 0) *a.d_loss_sum += s;
    }

    floatx4 ca[KTM], cb[KTM];
#pragma unroll
    for (int kt = 0; kt < KTM; ++kt) {
        ca[kt] = floatx4{0.f, 0.f, 0.f, 0.f};
        cb[kt] = floatx4{0.f, 0.f, 0.f, 0.f};
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
            *reinterpret_cast<float4 *>(sH + (e / C::HQ) * C::HS + 4 * (e % C::HQ)) = vh[i];
        }
        __syncthreads();
        const int nmax = min(C::CH, n_hi - c0);
#pragma unroll 4
        for (int g0 = 4 * w; g0 < nmax; g0 += 16) {
            const int nl = g0 + sub;
            const float r2 = sR2[nl * 16 + (lane & 15)];
            const float r1 = sR1[nl * 16 + (lane & 15)];
#pragma unroll
            for (int kt = 0; kt < KTM; ++kt) {
                if (kt < KT) {
                    const float hh = sH[nl * C::HS + 16 * kt + (lane & 15)];
                    ca[kt] = mfma16(r2, hh, ca[kt]);
                    cb[kt] = mfma16(r1, hh, cb[kt]);
                }
            }
        }
        __syncthreads();
    }
    floatx4 *red = reinterpret_cast<floatx4 *>(lds);   // [4][KTM][2][64], after the last chunk
#pragma unroll
    for (int kt = 0; kt < KTM; ++kt) {
        if (kt < KT) {
            red[((w * KTM + kt) * 2 + 0) * 64 + lane] = ca[kt];
            red[((w * KTM + kt) * 2 + 1) * 64 + lane] = cb[kt];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < KE; ++u) {
        const int kt = w + 4 * u;
        if (kt >= KT) continue;
        auto at = [&](int v, int c) { return red[((v * KTM + kt) * 2 + c) * 64 + lane]; };
        const floatx4 sa = ((at(0, 0) + at(1, 0)) + at(2, 0)) + at(3, 0);
        const floatx4 sb = ((at(0, 1) + at(1, 1)) + at(2, 1)) + at(3, 1);
        const int kc = 16 * kt + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = f0 + 4 * sub + r;
            if (f < a.F && kc < a.K)
                epilogue(a, f, kc, double(sa[r]), double(sb[r]), wq[u][r], aq[u][r], bq[u][r]);
        }
    }
}

// Single-stream fold: one 16 x 16 tile of (f, k) per 256-thread block (4
// waves), so a single minibatch spreads over ceil(F/16) ceil(K/16) blocks.
// Each element is computed exactly as fold_rows_body computes it (the same
// MFMA chain per wave over the frames with (n / 4) mod 4 == w, the same wave
// order, the same epilogue), so both give the same bits.
// nslices > 1: write the FP32 partial tile of slice `slice` instead of the
// epilogue.
__device__ __forceinline__ void fold_tile16_body(const FoldArgs &a, int tile, int slice,
                                                 int nslices) {
    __shared__ floatx4 red[4][2][64];
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

    // epilogue operands (wave 0 only), loaded before the frame rounds
    const int kc = k0 + (lane & 15);
    double wq[4], aq[4], bq[4];
    if (w == 0 && nslices == 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = f0 + 4 * sub + r;
            const bool ok = f < a.F && kc < a.K;
            const size_t e = ok ? (size_t)f + (size_t)kc * a.F : 0;
            wq[r] = ok ? a.W64[e] : 0.0;
            aq[r] = ok ? a.A[e] / a.sc[kc] : 0.0;
            bq[r] = ok ? a.B[e] * a.sc[kc] : 0.0;
        }
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
    red[w][0][lane] = ca;
    red[w][1][lane] = cb;
    __syncthreads();
    if (w != 0) return;
    ca = ((red[0][0][lane] + red[1][0][lane]) + red[2][0][lane]) + red[3][0][lane];
    cb = ((red[0][1][lane] + red[1][1][lane]) + red[2][1][lane]) + red[3][1][lane];
    if (nslices == 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = f0 + 4 * sub + r;
            if (f < a.F && kc < a.K)
                epilogue(a, f, kc, double(ca[r]), double(cb[r]), wq[r], aq[r], bq[r]);
        }
    } else {
        const size_t fk = (size_t)a.F * a.K;
        float *pa = a.part + (size_t)slice * 2 * fk;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = f0 + 4 * sub + r;
            if (f < a.F && kc < a.K) {
                pa[f + (size_t)kc * a.F] = ca[r];
                pa[fk + f + (size_t)kc * a.F] = cb[r];
            }
        }
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
