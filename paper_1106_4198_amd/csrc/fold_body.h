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
    double rho;
    int update_w;
    int tiles_f;           // ceil(F / 16)
    float *part;           // slices x 2 x F x K partials (multi-slice only)
    const double *lossf;   // frame losses of the minibatch (may be null)
    double *d_loss_sum;    // += sum of lossf (may be null)
    int *flags;
};

__device__ inline floatx4 mfma16(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// A = rho A + sum_n r2 h W^2, B = rho B + sum_n r1 h (Algorithm 1), W = sqrt(A/B);
// w, a0, b0: the element's current W, A, B.
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

// One 16 x 16 tile of (f, k) per 256-thread block (4 waves); frame groups of
// 4 dealt round-robin to the waves, partial tiles summed in wave order.
// nslices > 1: write the FP32 partial tile of slice `slice` instead of the
// epilogue.
__device__ __forceinline__ void fold_tile_body(const FoldArgs &a, int tile, int slice,
                                               int nslices) {
    __shared__ floatx4 red[4][2][64];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int f0 = (tile % a.tiles_f) * 16;
    const int k0 = (tile / a.tiles_f) * 16;
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
            aq[r] = ok ? a.A[e] : 0.0;
            bq[r] = ok ? a.B[e] : 0.0;
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
    a.Wn = d.Wn;
    a.rho = rho;
    a.update_w = update_w;
    a.tiles_f = (d.F + 15) / 16;
    a.part = part;
    a.lossf = d.lossf;
    a.d_loss_sum = d_loss_sum;
    a.flags = d.flags;
    return a;
}

inline int fold_tiles(const OnlineDev &d) { return ((d.F + 15) / 16) * ((d.K + 15) / 16); }

}  // namespace isnmf
