// Fused inner fit of a tile of NF = 4 frames on gfx950 MFMA (device body,
// shared by the single-stream and the multi-stream kernels).
//
// What it computes (Algorithm 1, inner argmin truncated to I multiplicative
// updates, eps shift of section 2.3; the h update of section 2.1):
//   for each frame n, from h = 1 (or the caller's warm start), I times:
//     x = eps + W h ; r1 = 1/x ; r2 = (eps + v) r1^2
//     num = W^T r2 ; den = W^T r1 ; h <- h sqrt(num / den)
//   then once more x, r1, r2 with the final h, which are written out for the
//   fold of eq. (4), together with h and the frame loss sum_f d_IS(eps+v, x).
//
// Mapping.  Rows are cut into chunks of 64; wave w owns chunks w, w + NW, ...
// Both contractions use 4x4 MFMA blocks (16 independent blocks per wave):
//   X (reduce over k): block q = rows 4q..4q+3 of the chunk, columns = frames;
//      A operand lane l = W[f0 + l][k..], B operand lane 4q+n = h[k..][n].
//      Result lane 4q+n, register i = x[f0 + 4q + i][n].
//   num/den (reduce over f): block q = components 4q..4q+3 (of a half of 64
//      components), columns = frames; A operand lane l = W[f..][64h + l],
//      B operand lane 4q+n = r[f..][n] broadcast through LDS.
//      Result lane 4q+n, register m = num[64h + 4q + m][n].
// FP32 (PREC 0) runs v_mfma_f32_4x4x1_16b (one contraction step per
// instruction); the 16-bit forms (PREC 1 = BF16, 2 = FP16) run
// v_mfma_f32_4x4x4_16b (four steps) on W * 2^s and h * 2^-s (s = round(log2
// F), exact power-of-two scales so W h is unchanged); accumulation is FP32
// throughout.  FP16 also scales each frame's h operand by a power of two that
// brings its largest entry to [2^14, 2^15) at every update, undone on the FP32
// model values, so the operand keeps its range whatever the frame's amplitude
// (h grows with the amplitude of v, section 2.1's scale invariance).  W stays in registers in both operand
// layouts (WG = false) or, for shapes too large for the register file, is
// read from its 16-bit row- and column-major copies in HBM/L2 (WG = true).
// The per-wave num/den partials meet in LDS once per iteration; every wave then
// applies the same h update, so h needs no second exchange.  Rows past the last
// full chunk (F = 64 m + t, t <= TAIL_MAX: the Nyquist row of an STFT) run on
// the VALU in wave 0.  The IS ratios, the h update and the loss are FP32 /
// FP64 in every form.
#pragma once

#include "common.h"
#include "devmath.h"

namespace isnmf {

__device__ inline floatx4 mfma4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

typedef short v4h __attribute__((ext_vector_type(4)));      // four 16-bit values
typedef _Float16 halfx4 __attribute__((ext_vector_type(4)));

// Round to nearest even (finite inputs).
__device__ inline unsigned short to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

template <int PREC>
__device__ inline unsigned short to16(float f) {
    if constexpr (PREC == 1) return to_bf16(f);
    return __builtin_bit_cast(unsigned short, (_Float16)f);
}

template <int PREC>
__device__ inline v4h pack4(float a, float b, float c, float d) {
    return v4h{(short)to16<PREC>(a), (short)to16<PREC>(b), (short)to16<PREC>(c),
               (short)to16<PREC>(d)};
}

template <int PREC>
__device__ inline floatx4 mfma16b(v4h a, v4h b, floatx4 c) {
    if constexpr (PREC == 1) return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, b, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_4x4x4f16(__builtin_bit_cast(halfx4, a),
                                             __builtin_bit_cast(halfx4, b), c, 0, 0, 0);
}

// Maximum over the 16 lanes that share (lane & 3) (xor butterfly; every lane
// of the group ends with the same value).
__device__ inline float max_over_quads(float v) {
#pragma unroll
    for (int m = 4; m < 64; m <<= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
    return v;
}

// 2^(14 - e) for m in [2^e, 2^(e+1)): maps m into [2^14, 2^15).  1 for m = 0;
// the exponent is held to [-100, 100] so the scale and its inverse stay
// normal FP32 numbers.
__device__ inline float pow2_scale(float m) {
    if (!(m > 0.f) || !isfinite(m)) return 1.f;
    const int e = (int)((__float_as_uint(m) >> 23) & 0xff) - 127;
    return ldexpf(1.f, max(-100, min(100, 14 - e)));
}

// Scheduling fence: operand loads issued before it stay ahead of the MFMAs
// after it (the scheduler would otherwise sink them and expose the LDS
// latency), and no later load is hoisted above it (bounds live registers).
__device__ inline void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// Order LDS traffic between lanes of one wave (no workgroup barrier needed).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NW, int CPW, int KMAX, int PREC, bool WG>
__device__ __forceinline__ void fit_body(const FitDesc &a, int tile) {
    constexpr bool H16 = PREC != 0;
    constexpr int KH = (KMAX + 63) / 64;        // halves of 64 components
    constexpr int KG = KMAX / 4;                // groups of 4 components
    constexpr int NBUF = (NW * KH <= 8) ? 2 : 1;
    static_assert(KMAX % 4 == 0 && KMAX <= 128, "K class");
    static_assert(H16 || KMAX <= 64, "FP32 form covers K <= 64");
    static_assert(H16 || !WG, "W from memory needs the 16-bit copies");

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int q = lane >> 2;
    const int n = lane & 3;
    const int fr = tile * NF + n;  // frame of this lane's B/C column
    const bool fvalid = fr < a.b;
    const int F = a.F, K = a.K;
    const float eps = a.eps;

    // Rows of rl* and hs* are padded so that the four frames a vector read
    // touches fall in different LDS banks.
    __shared__ floatx4 red[NBUF][NW][2 * KH][64];              // per-wave num/den partials
    __shared__ float rl[NW][2][NF][H16 ? 4 : CHUNK + 4];        // r2/r1 of the current chunk
    __shared__ float hs[NW][NF][H16 ? 4 : KMAX + 4];            // per-wave copy of h
    __shared__ unsigned short rl16[NW][2][NF][H16 ? CHUNK + 8 : 4];
    __shared__ unsigned short hs16[NW][NF][H16 ? KMAX + 8 : 4];
    __shared__ double lred[NW][NF];

    // ---- registers: the wave's rows of W in both operand layouts, and v
    constexpr bool REG32 = !H16;
    constexpr bool REG16 = H16 && !WG;
    float wx[CPW][REG32 ? KMAX : 1];             // W[f0 + lane][k]
    float wn[CPW][REG32 ? CHUNK : 1];            // W[f0 + r][lane]
    v4h wx16[CPW][REG16 ? KG : 1];               // W[f0 + lane][4g..4g+3] * 2^s
    v4h wn16[CPW][REG16 ? KH * 16 : 1];          // W[f0 + 4g..4g+3][64h + lane] * 2^s
    float vr[CPW][4];                            // v[f0 + 4q + i][fr]
    bool cval[CPW];
    int bad = 0;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const int c = w + NW * j;
        cval[j] = c < a.main_chunks;
        const int f0 = c * CHUNK;
        if constexpr (REG32) {
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const int f = f0 + lane;
                wx[j][k] = (cval[j] && k < K && f < F) ? a.W[f + (size_t)k * F] : 0.f;
            }
#pragma unroll
            for (int r = 0; r < CHUNK; ++r) {
                const int f = f0 + r;
                wn[j][r] = (cval[j] && lane < K && f < F) ? a.W[f + (size_t)lane * F] : 0.f;
            }
        }
        if constexpr (REG16) {
            const int f = f0 + lane;
#pragma unroll
            for (int g = 0; g < KG; ++g)
                wx16[j][g] = (cval[j] && f < F && 4 * g < a.KP)
                                 ? *reinterpret_cast<const v4h *>(a.W16r + (size_t)f * a.KP + 4 * g)
                                 : v4h{0, 0, 0, 0};
#pragma unroll
            for (int h = 0; h < KH; ++h)
#pragma unroll
                for (int g = 0; g < 16; ++g)
                    wn16[j][h * 16 + g] =
                        (cval[j] && 64 * h + lane < K)
                            ? *reinterpret_cast<const v4h *>(a.W16c + (size_t)(64 * h + lane) * a.FR + f0 + 4 * g)
                            : v4h{0, 0, 0, 0};
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = f0 + 4 * q + i;
            float v = 1.f;
            if (cval[j] && fvalid && f < F) {
                v = a.V[(size_t)fr * a.ldv + f];
                bad |= !isfinite(v);
            }
            vr[j][i] = v;
        }
    }
    // tail rows (VALU, wave 0): lane 4q+n keeps W[f][64h + 4q + m] and v[f][n]
    float wt[TAIL_MAX][KH][4];
    float vt[TAIL_MAX];
#pragma unroll
    for (int t = 0; t < TAIL_MAX; ++t) {
        const int f = a.main_chunks * CHUNK + t;
        const bool tv = (w == 0) && t < a.tail;
#pragma unroll
        for (int h = 0; h < KH; ++h)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int k = 64 * h + 4 * q + m;
                wt[t][h][m] = (tv && k < K) ? a.W[f + (size_t)k * F] : 0.f;
            }
        float v = 1.f;
        if (tv && fvalid) {
            v = a.V[(size_t)fr * a.ldv + f];
            bad |= !isfinite(v);
        }
        vt[t] = v;
    }
    if (bad) atomicOr(a.flags, FLAG_NONFINITE_V);

    // ---- h in the "update" layout: lane 4q+n holds h[64h + 4q + m][fr]
    float hu[KH][4];
#pragma unroll
    for (int h = 0; h < KH; ++h)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int k = 64 * h + 4 * q + m;
            float v = 0.f;
            if (k < K) v = (a.warm && fvalid) ? a.Hb[(size_t)fr * a.ldh + k] : 1.f;
            hu[h][m] = v;
        }
    // the X operand copy of h (FP32, or 16-bit scaled by hscale; FP16 also by
    // the frame's power of two hsc, whose inverse hinv the model applies)
    float hinv = 1.f;
    auto store_h = [&]() {
        float hsc = a.hscale;
        if constexpr (PREC == 2) {
            float m = 0.f;
#pragma unroll
            for (int h = 0; h < KH; ++h)
#pragma unroll
                for (int i = 0; i < 4; ++i) m = fmaxf(m, hu[h][i]);
            const float p = pow2_scale(max_over_quads(m) * a.hscale);
            hsc = a.hscale * p;
            hinv = 1.f / p;   // exact: a power of two
        }
#pragma unroll
        for (int h = 0; h < KH; ++h) {
            const int k0 = 64 * h + 4 * q;
            if (k0 < KMAX) {
                if constexpr (!H16)
                    *reinterpret_cast<floatx4 *>(&hs[w][n][k0]) =
                        floatx4{hu[h][0], hu[h][1], hu[h][2], hu[h][3]};
                else
                    *reinterpret_cast<v4h *>(&hs16[w][n][k0]) =
                        pack4<PREC>(hu[h][0] * hsc, hu[h][1] * hsc, hu[h][2] * hsc, hu[h][3] * hsc);
            }
        }
    };
    store_h();
    wave_lds_sync();

    // X = eps + W h for chunk j: lane 4q+n gets rows f0+4q+i of frame fr.
    // Components k >= K hold h = 0 and W = 0, so all KMAX/4 groups run.
    auto model = [&](int j, float (&xv)[4]) {
        floatx4 x0 = {0.f, 0.f, 0.f, 0.f}, x1 = {0.f, 0.f, 0.f, 0.f};
        if constexpr (!H16) {
            floatx4 hn = *reinterpret_cast<const floatx4 *>(&hs[w][n][0]);
#pragma unroll
            for (int k4 = 0; k4 < KMAX; k4 += 4) {
                const floatx4 h4 = hn;
                if (k4 + 4 < KMAX) hn = *reinterpret_cast<const floatx4 *>(&hs[w][n][k4 + 4]);
                sched_fence();
                x0 = mfma4(wx[j][k4 + 0], h4[0], x0);
                x1 = mfma4(wx[j][k4 + 1], h4[1], x1);
                x0 = mfma4(wx[j][k4 + 2], h4[2], x0);
                x1 = mfma4(wx[j][k4 + 3], h4[3], x1);
            }
        } else {
            const int f = (w + NW * j) * CHUNK + lane;
            const bool frow = f < F;
            // operands two groups ahead (LDS for h; HBM/L2 for W when WG)
            constexpr int D = WG ? 3 : 2;
            v4h hp[D + 1], wp[WG ? D + 1 : 1];
#pragma unroll
            for (int g = 0; g < D && g < KG; ++g) {
                hp[g] = *reinterpret_cast<const v4h *>(&hs16[w][n][4 * g]);
                if constexpr (WG)
                    wp[g] = (frow && 4 * g < a.KP)
                                ? *reinterpret_cast<const v4h *>(a.W16r + (size_t)f * a.KP + 4 * g)
                                : v4h{0, 0, 0, 0};
            }
#pragma unroll
            for (int g = 0; g < KG; ++g) {
                if (g + D < KG) {
                    hp[(g + D) % (D + 1)] = *reinterpret_cast<const v4h *>(&hs16[w][n][4 * (g + D)]);
                    if constexpr (WG)
                        wp[(g + D) % (D + 1)] =
                            (frow && 4 * (g + D) < a.KP)
                                ? *reinterpret_cast<const v4h *>(a.W16r + (size_t)f * a.KP + 4 * (g + D))
                                : v4h{0, 0, 0, 0};
                }
                sched_fence();
                v4h wa;
                if constexpr (WG)
                    wa = wp[g % (D + 1)];
                else
                    wa = wx16[j][g];
                if (g & 1)
                    x1 = mfma16b<PREC>(wa, hp[g % (D + 1)], x1);
                else
                    x0 = mfma16b<PREC>(wa, hp[g % (D + 1)], x0);
            }
        }
        if constexpr (PREC == 2) {
#pragma unroll
            for (int i = 0; i < 4; ++i) xv[i] = eps + (x0[i] + x1[i]) * hinv;
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) xv[i] = eps + (x0[i] + x1[i]);
        }
    };
    // tail row t on the VALU: x for frame fr, identical in the 16 lanes of fr
    auto tail_model = [&](int t) {
        float p = 0.f;
#pragma unroll
        for (int h = 0; h < KH; ++h)
#pragma unroll
            for (int m = 0; m < 4; ++m) p += wt[t][h][m] * hu[h][m];
        return eps + sum_over_quads(p);
    };

    int buf = 0;
    int guard = 0;
    for (int it = 0; it < a.iters; ++it) {
        floatx4 num[KH], den[KH];
#pragma unroll
        for (int h = 0; h < KH; ++h) {
            num[h] = floatx4{0.f, 0.f, 0.f, 0.f};
            den[h] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            if (!cval[j]) continue;
            const int f0 = (w + NW * j) * CHUNK;
            float xv[4], r1[4], r2[4];
            model(j, xv);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool ok = f0 + 4 * q + i < F;
                const float ir = __builtin_amdgcn_rcpf(xv[i]);
                r1[i] = ok ? ir : 0.f;
                r2[i] = ok ? (eps + vr[j][i]) * ir * ir : 0.f;
            }
            // broadcast r to the k-major operand layout through LDS
            if constexpr (!H16) {
                *reinterpret_cast<floatx4 *>(&rl[w][0][n][4 * q]) = floatx4{r2[0], r2[1], r2[2], r2[3]};
                *reinterpret_cast<floatx4 *>(&rl[w][1][n][4 * q]) = floatx4{r1[0], r1[1], r1[2], r1[3]};
                wave_lds_sync();
                // r operands through LDS, two row-quads ahead of the MFMAs
                floatx4 a2p[3], a1p[3];
                a2p[0] = *reinterpret_cast<const floatx4 *>(&rl[w][0][n][0]);
                a1p[0] = *reinterpret_cast<const floatx4 *>(&rl[w][1][n][0]);
                a2p[1] = *reinterpret_cast<const floatx4 *>(&rl[w][0][n][4]);
                a1p[1] = *reinterpret_cast<const floatx4 *>(&rl[w][1][n][4]);
#pragma unroll
                for (int qq = 0; qq < CHUNK / 4; ++qq) {
                    if (qq + 2 < CHUNK / 4) {
                        a2p[(qq + 2) % 3] = *reinterpret_cast<const floatx4 *>(&rl[w][0][n][4 * qq + 8]);
                        a1p[(qq + 2) % 3] = *reinterpret_cast<const floatx4 *>(&rl[w][1][n][4 * qq + 8]);
                    }
                    sched_fence();
                    const floatx4 a2 = a2p[qq % 3], a1 = a1p[qq % 3];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        num[0] = mfma4(wn[j][4 * qq + i], a2[i], num[0]);
                        den[0] = mfma4(wn[j][4 * qq + i], a1[i], den[0]);
                    }
                }
            } else {
                // FP16: per (chunk, frame) power-of-two scales bring the largest r2
                // and r1 of the chunk to [2^14, 2^15); undone on the FP32 sums.
                float s2 = 1.f, s1 = 1.f;
                if constexpr (PREC == 2) {
                    float m2 = fmaxf(fmaxf(r2[0], r2[1]), fmaxf(r2[2], r2[3]));
                    float m1 = fmaxf(fmaxf(r1[0], r1[1]), fmaxf(r1[2], r1[3]));
                    m2 = max_over_quads(m2);
                    m1 = max_over_quads(m1);
                    s2 = pow2_scale(m2);
                    s1 = pow2_scale(m1);
                }
                *reinterpret_cast<v4h *>(&rl16[w][0][n][4 * q]) =
                    pack4<PREC>(r2[0] * s2, r2[1] * s2, r2[2] * s2, r2[3] * s2);
                *reinterpret_cast<v4h *>(&rl16[w][1][n][4 * q]) =
                    pack4<PREC>(r1[0] * s1, r1[1] * s1, r1[2] * s1, r1[3] * s1);
                wave_lds_sync();
                floatx4 numc[KH], denc[KH];
#pragma unroll
                for (int h = 0; h < KH; ++h) {
                    numc[h] = floatx4{0.f, 0.f, 0.f, 0.f};
                    denc[h] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
                constexpr int D = WG ? 3 : 2;
                v4h a2p[D + 1], a1p[D + 1], wq[WG ? (D + 1) * KH : 1];
                auto wload = [&](int g, int h) {
                    const int k = 64 * h + lane;
                    return k < K ? *reinterpret_cast<const v4h *>(a.W16c + (size_t)k * a.FR + f0 + 4 * g)
                                 : v4h{0, 0, 0, 0};
                };
#pragma unroll
                for (int g = 0; g < D; ++g) {
                    a2p[g] = *reinterpret_cast<const v4h *>(&rl16[w][0][n][4 * g]);
                    a1p[g] = *reinterpret_cast<const v4h *>(&rl16[w][1][n][4 * g]);
                    if constexpr (WG)
#pragma unroll
                        for (int h = 0; h < KH; ++h) wq[g * KH + h] = wload(g, h);
                }
#pragma unroll
                for (int qq = 0; qq < CHUNK / 4; ++qq) {
                    if (qq + D < CHUNK / 4) {
                        const int s = (qq + D) % (D + 1);
                        a2p[s] = *reinterpret_cast<const v4h *>(&rl16[w][0][n][4 * (qq + D)]);
                        a1p[s] = *reinterpret_cast<const v4h *>(&rl16[w][1][n][4 * (qq + D)]);
                        if constexpr (WG)
#pragma unroll
                            for (int h = 0; h < KH; ++h) wq[s * KH + h] = wload(qq + D, h);
                    }
                    sched_fence();
#pragma unroll
                    for (int h = 0; h < KH; ++h) {
                        v4h wa;
                        if constexpr (WG)
                            wa = wq[(qq % (D + 1)) * KH + h];
                        else
                            wa = wn16[j][h * 16 + qq];
                        numc[h] = mfma16b<PREC>(wa, a2p[qq % (D + 1)], numc[h]);
                        denc[h] = mfma16b<PREC>(wa, a1p[qq % (D + 1)], denc[h]);
                    }
                }
                const float u2 = 1.f / s2, u1 = 1.f / s1;   // exact: powers of two
#pragma unroll
                for (int h = 0; h < KH; ++h) {
                    num[h] += numc[h] * u2;
                    den[h] += denc[h] * u1;
                }
            }
            wave_lds_sync();
        }
        // tail rows on the VALU (wave 0)
        if (w == 0) {
#pragma unroll
            for (int t = 0; t < TAIL_MAX; ++t) {
                if (t < a.tail) {
                    const float x = tail_model(t);
                    const float ir = __builtin_amdgcn_rcpf(x);
                    const float rr2 = (eps + vt[t]) * ir * ir;
#pragma unroll
                    for (int h = 0; h < KH; ++h)
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            num[h][m] += wt[t][h][m] * rr2;
                            den[h][m] += wt[t][h][m] * ir;
                        }
                }
            }
        }
        // ---- combine the waves' partials (one barrier), then update h
#pragma unroll
        for (int h = 0; h < KH; ++h) {
            red[buf][w][2 * h][lane] = num[h];
            red[buf][w][2 * h + 1][lane] = den[h];
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < KH; ++h) {
            floatx4 N = red[buf][0][2 * h][lane], D = red[buf][0][2 * h + 1][lane];
#pragma unroll
            for (int v = 1; v < NW; ++v) {
                N += red[buf][v][2 * h][lane];
                D += red[buf][v][2 * h + 1][lane];
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (64 * h + 4 * q + m < K) {
                    if (D[m] > 0.f && N[m] >= 0.f)
                        hu[h][m] *= __builtin_amdgcn_sqrtf(N[m] * __builtin_amdgcn_rcpf(D[m]));
                    else
                        guard = 1;
                }
            }
        }
        if constexpr (NBUF == 2)
            buf ^= 1;
        else
            __syncthreads();   // single buffer: every wave has read it
        store_h();
        wave_lds_sync();
    }

    // ---- final model with the fitted h: ratios for the fold of eq. (4)
    float xf[CPW][4];
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        if (!cval[j]) continue;
        const int f0 = (w + NW * j) * CHUNK;
        model(j, xf[j]);
        float r1[4], r2[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool ok = f0 + 4 * q + i < F;
            const float ir = __builtin_amdgcn_rcpf(xf[j][i]);
            r1[i] = ok ? ir : 0.f;
            r2[i] = ok ? (eps + vr[j][i]) * ir * ir : 0.f;
        }
        if (fvalid) {
            const size_t o = (size_t)fr * a.FR + f0 + 4 * q;
            *reinterpret_cast<floatx4 *>(a.R1 + o) = floatx4{r1[0], r1[1], r1[2], r1[3]};
            *reinterpret_cast<floatx4 *>(a.R2 + o) = floatx4{r2[0], r2[1], r2[2], r2[3]};
        }
    }
    float xt[TAIL_MAX];
#pragma unroll
    for (int t = 0; t < TAIL_MAX; ++t) {
        xt[t] = 1.f;
        if (w == 0 && t < a.tail) {
            xt[t] = tail_model(t);
            if (q == 0 && fvalid) {
                const int f = a.main_chunks * CHUNK + t;
                const float ir = __builtin_amdgcn_rcpf(xt[t]);
                a.R1[(size_t)fr * a.FR + f] = ir;
                a.R2[(size_t)fr * a.FR + f] = (eps + vt[t]) * ir * ir;
            }
        }
    }
    // frame loss sum_f d_IS(eps + v, x) in FP64 (eq. (5) numerator)
    double lsum = 0.0;
    if (fvalid) {
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            if (!cval[j]) continue;
            const int f0 = (w + NW * j) * CHUNK;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (f0 + 4 * q + i < F) lsum += dis_term(a.epsd + double(vr[j][i]), double(xf[j][i]));
        }
        if (w == 0 && q == 0)
#pragma unroll
            for (int t = 0; t < TAIL_MAX; ++t)
                if (t < a.tail) lsum += dis_term(a.epsd + double(vt[t]), double(xt[t]));
    }
    if (guard && w == 0) atomicOr(a.flags, FLAG_GUARD_H);

    // ---- outputs: frame loss (fixed order), h
    lsum = sum_over_quads(lsum);
    if (q == 0) lred[w][n] = lsum;
    __syncthreads();
    if (w == 0 && q == 0 && fvalid) {
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < NW; ++v) s += lred[v][n];
        a.lossf[fr] = s;
    }
    if (w == 0 && fvalid) {
#pragma unroll
        for (int h = 0; h < KH; ++h)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int k = 64 * h + 4 * q + m;
                if (k < K) {
                    a.Hi[(size_t)fr * a.KP + k] = hu[h][m];
                    if (a.Hb) a.Hb[(size_t)fr * a.ldh + k] = hu[h][m];
                }
            }
    }
}

}  // namespace isnmf
