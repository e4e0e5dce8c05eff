// Latency variant of the fused fit (FP32 products on the VALU): one frame per
// workgroup.
//
// It computes what fit_body.h computes for a frame (the inner problem of
// Algorithm 1, i.e. the argmin over h of eq. (4), by I multiplicative updates
// of Section 2.1, then the final model, the ratios 1/x and (eps+v)/x^2 the
// fold consumes, the frame loss and the fitted h), in the same output layouts.
// A minibatch of b frames occupies b CUs instead of b/4, which shortens the
// dependent chain of 2I+1 matrix-vector products when one stream runs alone.
//
// Mapping: 512 threads = 64 row groups p x 8 component groups q (q = t & 7,
// p = t >> 3).  Thread (p, q) keeps W[p + 64r][q + 8c] (r < RF, c < CK) in
// registers; RF = ceil(F / 64), CK = ceil(K / 8), so only the last row set
// can be partial and no thread holds a row set that is entirely past F.
//   x_f          : partial over the thread's components, summed over the 8
//                  q-lanes of the row with DPP (the same value in all 8);
//   num_k, den_k : partial over the thread's rows, summed over the wave with
//                  DPP row_ror 8 and the gfx950 permlane16/permlane32 swaps
//                  (four values per register afterwards), then over the 8
//                  waves by the lane owning k (8 + 8 values from LDS).
// Two workgroup barriers per update.  Every sum has a fixed order, so results
// are bitwise repeatable and independent of the other frames of a launch.
//
// 16-wave form (NW = 16, FP32): 1024 threads = 128 row groups x 8 component
// groups, rows p + 128 r, W read from the column-major FP32 copy, the
// partials of 16 waves summed per component.  It extends the variant past the
// 8-wave form's 17 row sets (F <= 1088) to F <= 1152 (9 row sets of 128 rows
// within the 128 registers of four waves per SIMD); where both forms fit, the
// 8-wave form is the faster (the per-wave reductions and the barrier grow with
// the wave count), so only RF = 9 is built.
//
// BF16 form (BF = true, the precision form's single-stream variant): the
// products W h, W^T r2 and W^T r1 take bf16 operands two at a time on
// v_dot2c_f32_bf16 (FP32 accumulation), with everything else (x, the ratios,
// the reductions, h) in FP32 as above.  The thread keeps W twice as packed
// bf16 pairs: pairs of components (c, c + 1) of one row for W h, and pairs of
// row sets (r, r + 1) of one component for the transposed products, so each
// product takes half the instructions.  bf16 has FP32's exponent range, so no
// operand is scaled.
#pragma once

#include <hip/hip_ext.h>

#include "common.h"
#include "devmath.h"

namespace isnmf {
namespace valu {

constexpr int VT = 512;   // threads per workgroup (8-wave form)

template <int CTRL>
__device__ inline float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// Sum over the 8 lanes with the same lane >> 3 (identical result in all 8).
__device__ inline float sum8(float v) {
    v += dpp<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);   // row_half_mirror: the other quad of the 8
    return v;
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));

// (a, b) rounded to bf16 (nearest even) in one word, a in the low half
__device__ inline uint32_t pack_bf2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){a, b}, bf16x2));
}

// c + a.lo * b.lo + a.hi * b.hi with bf16 operands
__device__ inline float dot2(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a),
                                           __builtin_bit_cast(bf16x2, b), c, false);
}

// a, b -> rows (a0+a1, b0+b1, a2+a3, b2+b3) of 16 lanes each
__device__ inline float swap16_add(float a, float b) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// a, b -> rows (a0+a2, a1+a3, b0+b2, b1+b3)
__device__ inline float swap32_add(float a, float b) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

template <int CK, int RF, bool BF, int NW = 8>
__device__ inline void body(const FitDesc &a, int fr) {
    static_assert(NW == 8 || (NW == 16 && !BF), "8 waves, or 16 waves in FP32");
    constexpr int PR = 8 * NW;              // row groups: rows p + PR r
    constexpr int KSW = 2 * NW + 4;         // LDS floats per component: N, D partials, pad
    constexpr int NV = 2 * CK;              // num/den values per thread
    constexpr int CH = (CK + 1) / 2;        // BF16: component pairs per row set
    constexpr int RH = (RF + 1) / 2;        // BF16: row-set pairs per component
    constexpr int NG = (CK + 1) / 2;        // registers after the in-wave reduction
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int w = t >> 6;
    const int q = t & 7;
    const int p = t >> 3;
    const int F = a.F, K = a.K;
    const float eps = a.eps;

    __shared__ float4 red4[8 * CK * KSW / 4];   // [k][N 0..NW-1 | D 0..NW-1 | pad] per wave w
    __shared__ float hsh[8 * CK];
    __shared__ double lred[NW];
    float *red = reinterpret_cast<float *>(red4);

    // the last row set holds rows p + PR (RF-1); it has rows below F in wave w
    // iff 8w + PR (RF-1) < F (uniform per wave)
    constexpr int RL = RF - 1;
    const bool last_live = 8 * w + PR * RL < F;
    const bool last_ok = p + PR * RL < F;

    // W: 8 waves read its register-order copy, one float4 per thread per 4
    // elements, contiguous over the workgroup (zero past F and K); 16 waves
    // read the column-major FP32 copy
    constexpr int NE = RF * CK;
    float wr[RF][CK];
    if constexpr (NW == 8) {
        const float4 *wv = reinterpret_cast<const float4 *>(a.Wv);
#pragma unroll
        for (int g = 0; g < (NE + 3) / 4; ++g) {
            const float4 v = wv[g * VT + t];
            const float e4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (4 * g + j < NE) wr[(4 * g + j) / CK][(4 * g + j) % CK] = e4[j];
        }
    } else {
#pragma unroll
        for (int r = 0; r < RF; ++r)
#pragma unroll
            for (int c = 0; c < CK; ++c) {
                const int f = p + PR * r, k = q + 8 * c;
                wr[r][c] = (f < F && k < K) ? a.W[(size_t)k * F + f] : 0.f;
            }
    }
    // BF16: W as pairs of components (model) and pairs of row sets (W^T)
    uint32_t wkp[BF ? RF : 1][BF ? CH : 1], wfp[BF ? RH : 1][BF ? CK : 1];
    if constexpr (BF) {
#pragma unroll
        for (int r = 0; r < RF; ++r)
#pragma unroll
            for (int i = 0; i < CH; ++i)
                wkp[r][i] = pack_bf2(wr[r][2 * i], 2 * i + 1 < CK ? wr[r][2 * i + 1] : 0.f);
#pragma unroll
        for (int j = 0; j < RH; ++j)
#pragma unroll
            for (int c = 0; c < CK; ++c)
                wfp[j][c] = pack_bf2(wr[2 * j][c], 2 * j + 1 < RF ? wr[2 * j + 1][c] : 0.f);
    }
    float ve[RF];   // eps + v (0 past F)
    int bad = 0;
#pragma unroll
    for (int r = 0; r < RF; ++r) {
        const int f = p + PR * r;
        const bool ok = r < RL || last_ok;
        const float v = ok ? a.V[(size_t)fr * a.ldv + f] : 0.f;
        bad |= !isfinite(v);
        ve[r] = ok ? eps + v : 0.f;
    }
    if (bad) atomicOr(a.flags, FLAG_NONFINITE_V);

    if (t < 8 * CK)   // thread t owns component k = t
        hsh[t] = t < K ? (a.warm ? a.Hb[(size_t)fr * a.ldh + t] : 1.f) : 0.f;
    __syncthreads();
    float hk[CK];
    uint32_t hkp[CH];   // BF16: h as pairs of components
    auto load_h = [&]() {
#pragma unroll
        for (int c = 0; c < CK; ++c) hk[c] = hsh[q + 8 * c];
        if constexpr (BF) {
#pragma unroll
            for (int i = 0; i < CH; ++i) hkp[i] = pack_bf2(hk[2 * i], 2 * i + 1 < CK ? hk[2 * i + 1] : 0.f);
        }
    };
    load_h();

    // eps enters the sum once, in the q = 0 lane of each row
    const float s0 = q == 0 ? eps : 0.f;
    float x[RF];
    auto row_model = [&](int r) {
        float s = s0;
        if constexpr (BF) {
#pragma unroll
            for (int i = 0; i < CH; ++i) s = dot2(wkp[r][i], hkp[i], s);
        } else {
#pragma unroll
            for (int c = 0; c < CK; ++c) s = fmaf(wr[r][c], hk[c], s);
        }
        return sum8(s);
    };
    auto model = [&]() {
#pragma unroll
        for (int r = 0; r < RL; ++r) x[r] = row_model(r);
        x[RL] = 1.f;
        if (last_live) {
            const float s = row_model(RL);
            x[RL] = last_ok ? s : 1.f;   // rows past F: W = 0 and v' = 0, any x > 0
        }
    };

    int guard = 0;
    for (int it = 0; it < a.iters; ++it) {
        model();
        float nd[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) nd[i] = 0.f;
        if constexpr (BF) {
            // ratios of the row sets in pairs; the last pair's second row set
            // (RF odd) and the dead last row set of a wave give r1 = r2 = 0
            // against W = 0 there
            float r1v[2 * RH], r2v[2 * RH];
#pragma unroll
            for (int r = 0; r < 2 * RH; ++r) {
                const bool live = r < RL || (r == RL && last_live);
                const float r1 = live ? __builtin_amdgcn_rcpf(x[r < RF ? r : 0]) : 0.f;
                r1v[r] = r1;
                r2v[r] = live ? ve[r < RF ? r : 0] * r1 * r1 : 0.f;
            }
#pragma unroll
            for (int j = 0; j < RH; ++j) {
                const uint32_t p1 = pack_bf2(r1v[2 * j], r1v[2 * j + 1]);
                const uint32_t p2 = pack_bf2(r2v[2 * j], r2v[2 * j + 1]);
#pragma unroll
                for (int c = 0; c < CK; ++c) {
                    nd[2 * c] = dot2(wfp[j][c], p2, nd[2 * c]);
                    nd[2 * c + 1] = dot2(wfp[j][c], p1, nd[2 * c + 1]);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const float r1 = __builtin_amdgcn_rcpf(x[r]);
                const float r2 = ve[r] * r1 * r1;
#pragma unroll
                for (int c = 0; c < CK; ++c) {
                    nd[2 * c] = fmaf(wr[r][c], r2, nd[2 * c]);
                    nd[2 * c + 1] = fmaf(wr[r][c], r1, nd[2 * c + 1]);
                }
            }
            if (last_live) {
                const float r1 = __builtin_amdgcn_rcpf(x[RL]);
                const float r2 = ve[RL] * r1 * r1;
#pragma unroll
                for (int c = 0; c < CK; ++c) {
                    nd[2 * c] = fmaf(wr[RL][c], r2, nd[2 * c]);
                    nd[2 * c + 1] = fmaf(wr[RL][c], r1, nd[2 * c + 1]);
                }
            }
        }
        // over the wave: lanes 8 apart, then rows 0+1 / 2+3, then halves
#pragma unroll
        for (int i = 0; i < NV; ++i) nd[i] += dpp<0x128>(nd[i]);   // row_ror 8
        float u[CK];
#pragma unroll
        for (int c = 0; c < CK; ++c) u[c] = swap16_add(nd[2 * c], nd[2 * c + 1]);
        float g4[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) g4[g] = swap32_add(u[2 * g], 2 * g + 1 < CK ? u[2 * g + 1] : 0.f);
        // register g, row j = lane >> 4 now holds value 4g + j: component
        // c = 2g + (j >> 1) (k = q + 8c), N for even j and D for odd j
        if ((lane & 8) == 0) {
            const int j = lane >> 4;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int c = 2 * g + (j >> 1);
                if (c < CK) red[(q + 8 * c) * KSW + (j & 1) * NW + w] = g4[g];
            }
        }
        __syncthreads();
        // penalty on H (section 2.2, Extensions): psi'(s) = lambda / (a + s) of
        // the column sum before the update joins every den_k.  K <= 64, so the
        // lanes t < K are wave 0's, which reads hsh before it writes it.
        float dpsi = 0.f;
        if (!BF && a.psi_lambda > 0.f && w == 0)
            dpsi = a.psi_lambda / (a.psi_a + wave_sum_f32(lane < K ? hsh[lane] : 0.f));
        if (t < K) {
            const float4 *pk = red4 + t * (KSW / 4);
            auto sum4 = [](float4 v) { return (v.x + v.y) + (v.z + v.w); };
            float N, D;
            if constexpr (NW == 8) {
                N = sum4(pk[0]) + sum4(pk[1]);
                D = (sum4(pk[2]) + sum4(pk[3])) + dpsi;
            } else {
                N = (sum4(pk[0]) + sum4(pk[1])) + (sum4(pk[2]) + sum4(pk[3]));
                D = ((sum4(pk[4]) + sum4(pk[5])) + (sum4(pk[6]) + sum4(pk[7]))) + dpsi;
            }
            float h = hsh[t];
            if (D > 0.f && N >= 0.f)
                h *= __builtin_amdgcn_sqrtf(N * __builtin_amdgcn_rcpf(D));
            else
                guard = 1;
            hsh[t] = h;
        }
        __syncthreads();
        load_h();
    }
    if (guard) atomicOr(a.flags, FLAG_GUARD_H);

    // final model; ratios for the fold and the frame loss.  Lane q takes row
    // set q (and q + 8), so each lane evaluates the loss term of at most two
    // rows and the 8 lanes of a row group cover its row sets without overlap.
    model();
    double lsum = 0.0;
    auto finish_row = [&](int base) {
        float xs = 1.f, es = 0.f;
#pragma unroll
        for (int r = base; r < RF && r < base + 8; ++r)
            if ((r & 7) == q) {
                xs = x[r];
                es = ve[r];
            }
        const int r = base + q;
        const int f = p + PR * r;
        if (r < RL || (r == RL && last_ok)) {
            const float ir = __builtin_amdgcn_rcpf(xs);
            a.R1[(size_t)fr * a.FR + f] = ir;
            a.R2[(size_t)fr * a.FR + f] = es * ir * ir;
            lsum += dis_term(double(es), double(xs));   // FP64 term, as the objective
        }
    };
    finish_row(0);
    if (RF > 8 && (RF > 9 || last_live)) finish_row(8);
    if (RF > 16 && last_live) finish_row(16);
    lsum = wave_sum_f64(lsum);
    if (lane == 0) lred[w] = lsum;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < NW; ++v) s += lred[v];
        a.lossf[fr] = s;
    }
    if (t < K) {
        a.Hi[(size_t)fr * a.KP + t] = hsh[t];
        if (a.Hb) a.Hb[(size_t)fr * a.ldh + t] = hsh[t];
    }
}

template <int CK, int RF, bool BF, int NW>
__global__ __launch_bounds__(64 * NW) void fit_valu_kernel(FitDesc a) {
    body<CK, RF, BF, NW>(a, blockIdx.x);
}

// Batched form: item = (stream, tile of NF frames); workgroup NF*i + j fits
// frame j of item i; frames past the stream's minibatch of this step exit.
template <int CK, int RF, bool BF, int NW>
__global__ __launch_bounds__(64 * NW) void fit_valu_multi_kernel(const FitDesc *__restrict__ descs,
                                                                 const int2 *__restrict__ items,
                                                                 const long long *__restrict__ cursor,
                                                                 const int *__restrict__ beff) {
    const int2 it = items[blockIdx.x / NF];
    const int fr = it.y * NF + (int)(blockIdx.x % NF);
    const int b = beff[it.x];
    if (fr >= b) return;   // uniform per workgroup
    FitDesc a = descs[it.x];
    const long long c = cursor[it.x];
    a.b = b;
    a.V += c * a.ldv;
    if (a.Hb) a.Hb += c * a.ldh;
    body<CK, RF, BF, NW>(a, fr);
}

// Served form: grid (frame j, chunk i) over a step's work list (the frame
// index in x, whose range is the larger); frames past the chunk exit.
template <int CK, int RF, bool BF, int NW>
__global__ __launch_bounds__(64 * NW) void fit_valu_work_kernel(const FitDesc *__restrict__ tab,
                                                                const ServeWork *__restrict__ work) {
    const ServeWork wk = work[blockIdx.y];
    if ((int)blockIdx.x >= wk.b) return;   // uniform per workgroup
    FitDesc a = tab[wk.sess];
    a.b = wk.b;
    a.V = wk.V;
    a.ldv = wk.ldv;
    body<CK, RF, BF, NW>(a, blockIdx.x);
}

// Single-stream launch of b frames of nt threads; with the handle's timing
// events pending, the events are attached to the dispatch (they then time the
// kernel alone).
inline void launch_single(void (*k)(FitDesc), FitDesc a, int b, int nt, hipStream_t s) {
    if (g_launch_timing.pending) {
        void *args[] = {&a};
        if (hipExtLaunchKernel(reinterpret_cast<const void *>(k), dim3(b), dim3(nt), args, 0, s,
                               g_launch_timing.start, g_launch_timing.stop, 0) == hipSuccess)
            g_launch_timing.pending = false;
        return;
    }
    k<<<b, nt, 0, s>>>(a);
}

// Launch of the (CK, rf, BF, NW) instance (rf = 1..17 with 8 waves, 9 with
// 16): b frames of *a (d and tab null), the frames of n batched items of d,
// or the frames of n served chunks of tab (at most max_b frames each).
// Explicitly instantiated per CK in fit_valu_ck*.hip, so the instances build
// in parallel.
template <int CK, bool BF, int NW>
hipError_t launch_any(const FitDesc *a, int rf, int b, const FitDesc *d, const int2 *items, int n,
                      const long long *cur, const int *beff, const FitDesc *tab,
                      const ServeWork *work, int max_b, hipStream_t s) {
    constexpr int nt = 64 * NW;
    constexpr int rf_min = NW == 8 ? 1 : 9, rf_max = NW == 8 ? 17 : 9;
    if (rf < rf_min || rf > rf_max) return hipErrorNotSupported;
    switch (rf) {
#define ISNMF_VALU_RF(RF)                                                                        \
    case RF:                                                                                     \
        if constexpr (RF >= rf_min && RF <= rf_max) {                                            \
            if (tab)                                                                             \
                fit_valu_work_kernel<CK, RF, BF, NW><<<dim3(max_b, n), nt, 0, s>>>(tab, work);    \
            else if (d)                                                                          \
                fit_valu_multi_kernel<CK, RF, BF, NW><<<n * NF, nt, 0, s>>>(d, items, cur, beff); \
            else                                                                                 \
                launch_single(&fit_valu_kernel<CK, RF, BF, NW>, *a, b, nt, s);                    \
        }                                                                                        \
        break;
        ISNMF_VALU_RF(1) ISNMF_VALU_RF(2) ISNMF_VALU_RF(3) ISNMF_VALU_RF(4)
        ISNMF_VALU_RF(5) ISNMF_VALU_RF(6) ISNMF_VALU_RF(7) ISNMF_VALU_RF(8)
        ISNMF_VALU_RF(9) ISNMF_VALU_RF(10) ISNMF_VALU_RF(11) ISNMF_VALU_RF(12)
        ISNMF_VALU_RF(13) ISNMF_VALU_RF(14) ISNMF_VALU_RF(15) ISNMF_VALU_RF(16)
        ISNMF_VALU_RF(17)
#undef ISNMF_VALU_RF
        default:
            return hipErrorNotSupported;
    }
    return hipGetLastError();
}

#define ISNMF_VALU_SIG(CKV, BFV, NWV)                                                           \
    hipError_t launch_any<CKV, BFV, NWV>(const FitDesc *, int, int, const FitDesc *, const int2 *, \
                                         int, const long long *, const int *, const FitDesc *,     \
                                         const ServeWork *, int, hipStream_t);
#define ISNMF_VALU_EXTERN(CKV)                                                      \
    extern template ISNMF_VALU_SIG(CKV, false, 8) extern template ISNMF_VALU_SIG(CKV, true, 8) \
    extern template ISNMF_VALU_SIG(CKV, false, 16)
#define ISNMF_VALU_INSTANTIATE(CKV)                                            \
    template ISNMF_VALU_SIG(CKV, false, 8) template ISNMF_VALU_SIG(CKV, true, 8) \
    template ISNMF_VALU_SIG(CKV, false, 16)

}  // namespace valu
}  // namespace isnmf
