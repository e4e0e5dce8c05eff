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

#include "common.h"
#include "devmath.h"

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

template <int MT>
__device__ inline void body(const FitDesc &a, int n_first) {
    constexpr int P = pitch(MT);
    extern __shared__ float wl[];   // [16 T][P]
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int n = lane & 15;
    const int F = a.F, K = a.K;
    const int T = (F + 15) >> 4;
    const int fr = n_first + WF * w + n;   // this lane's frame (B / C column)
    const bool fok = fr < a.b;
    const float eps = a.eps;
    const float *vrow = a.V + (size_t)(fok ? fr : 0) * a.ldv;

    // ---- W into LDS (zero past F and K); consecutive threads read consecutive
    // rows of a column of the column-major FP32 copy
    {
        const int rows = 16 * T, cols = 16 * MT;
        for (int e = threadIdx.x; e < rows * cols; e += NWT * 64) {
            const int c = e / rows, r = e - c * rows;
            wl[r * P + c] = (r < F && c < K) ? a.W[r + (size_t)c * F] : 0.f;
        }
    }

    // eps + v at the lane's rows 16t + 4g + j of its frame (0 past F and for
    // frames past the minibatch)
    auto load_v = [&](int t) {
        f4 v;
        const int r0 = 16 * t + 4 * g;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (fok && r0 + j < F) ? eps + vrow[r0 + j] : 0.f;
        return v;
    };
    // X accumulator start: eps, or 1 on rows past F (W = 0 there; x only needs to be > 0)
    auto cinit = [&](int t) {
        f4 c = {eps, eps, eps, eps};
        const int r0 = 16 * t + 4 * g;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (r0 + j >= F) c[j] = 1.f;
        return c;
    };

    // ---- h (FP32): lane (g, n) holds components 16 mt + 4 g + j of frame n
    float hq[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 16 * mt + 4 * g + j;
            hq[mt][j] = k < K ? ((a.warm && fok) ? a.Hb[(size_t)fr * a.ldh + k] : 1.f) : 0.f;
        }
    // slots j of the last m-tile that hold any component < K
    const int jlast = min(4, K - 16 * (MT - 1));
    __syncthreads();   // W in LDS

    // X operands of row tile t: components 16 mt + 4g .. + 3 of row 16t + n
    auto load_wx = [&](int t, f4 (&o)[MT]) {
        const float *p = wl + (16 * t + n) * P + 4 * g;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) o[mt] = *reinterpret_cast<const f4 *>(p + 16 * mt);
    };
    auto model_ops = [&](int t, const f4 (&o)[MT]) {
        f4 x = cinit(t);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (mt < MT - 1 || j < jlast) x = mfma(o[mt][j], hq[mt][j], x);
        return x;
    };
    auto model = [&](int t) {
        f4 o[MT];
        load_wx(t, o);
        return model_ops(t, o);
    };

    int guard = 0;
    for (int it = 0; it < a.iters; ++it) {
        f4 na[MT], da[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            na[mt] = f4{0.f, 0.f, 0.f, 0.f};
            da[mt] = f4{0.f, 0.f, 0.f, 0.f};
        }
        // Software pipeline over the row tiles: tile t + 1's model products go
        // to the matrix pipe before tile t's ratios are formed, and v of tile
        // t + 2 is in flight meanwhile.  Same products and sums as tile by
        // tile, so the same bits.
        f4 x = model(0);
        f4 v0 = load_v(0);
        f4 v1 = T > 1 ? load_v(1) : v0;
        for (int t = 0; t < T; ++t) {
            f4 xn = x;
            if (t + 1 < T) xn = model(t + 1);
            f4 v2 = v1;
            if (t + 2 < T) v2 = load_v(t + 2);
            // W^T operands of the tile: component 16 mt + n of rows 16t + 4g + j
            float wt[4][MT];
            const float *p = wl + (16 * t + 4 * g) * P + n;
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) wt[j][mt] = p[j * P + 16 * mt];
            float r1[4], r2[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                r1[j] = __builtin_amdgcn_rcpf(x[j]);
                r2[j] = v0[j] * r1[j] * r1[j];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    na[mt] = mfma(wt[j][mt], r2[j], na[mt]);
                    da[mt] = mfma(wt[j][mt], r1[j], da[mt]);
                }
            x = xn;
            v0 = v1;
            v1 = v2;
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
    }
    if (guard) atomicOr(a.flags, FLAG_GUARD_H);

    // ---- final model: R1, R2 for the fold, the frame loss (FP64 terms, as the
    // objective), and the check of v
    double ls = 0.0;
    int bad = 0;
    f4 x = model(0);
    for (int t = 0; t < T; ++t) {
        f4 xn = x;
        if (t + 1 < T) xn = model(t + 1);
        const int r0 = 16 * t + 4 * g;
        f4 r1, r2;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool ok = fok && r0 + j < F;
            const float v = ok ? vrow[r0 + j] : 0.f;
            bad |= !isfinite(v);
            const float ve = eps + v;
            const float r = __builtin_amdgcn_rcpf(x[j]);
            r1[j] = ok ? r : 0.f;
            r2[j] = ok ? ve * r * r : 0.f;
            if (ok) ls += dis_term(a.epsd + double(v), double(x[j]));
        }
        // FR is a multiple of 64, so rows r0 .. r0 + 3 lie in the frame's buffer row
        if (fok) {
            *reinterpret_cast<f4 *>(a.R1 + (size_t)fr * a.FR + r0) = r1;
            *reinterpret_cast<f4 *>(a.R2 + (size_t)fr * a.FR + r0) = r2;
        }
        x = xn;
    }
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

template <int MT>
__global__ __launch_bounds__(NWT * 64) void fit_t32_kernel(FitDesc a) {
    body<MT>(a, blockIdx.x * FPW);
}

// Batched form: item = (stream, tile of 128 frames); tiles past the stream's
// minibatch of this step exit.
template <int MT>
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
    body<MT>(a, it.y * FPW);
}

// Served form: grid (chunk i, 128-frame tile j) over a step's work list.
template <int MT>
__global__ __launch_bounds__(NWT * 64) void fit_t32_work_kernel(const FitDesc *__restrict__ tab,
                                                                const ServeWork *__restrict__ work) {
    const ServeWork wk = work[blockIdx.x];
    if ((int)blockIdx.y * FPW >= wk.b) return;   // uniform per workgroup
    FitDesc a = tab[wk.sess];
    a.b = wk.b;
    a.V = wk.V;
    a.ldv = wk.ldv;
    body<MT>(a, blockIdx.y * FPW);
}

}  // namespace t32
}  // namespace isnmf
