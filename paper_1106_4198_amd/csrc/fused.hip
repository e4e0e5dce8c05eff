// Fused inner fit of a minibatch on gfx950 MFMA (FP32).
//
// What it computes (Algorithm 1, inner argmin truncated to I multiplicative
// updates, eps shift of section 2.3; the h update of section 2.1):
//   for each frame n, from h = 1 (or the caller's warm start), I times:
//     x = eps + W h ; r1 = 1/x ; r2 = (eps + v) r1^2
//     num = W^T r2 ; den = W^T r1 ; h <- h sqrt(num / den)
//   then once more x, r1, r2 with the final h, which are written out for the
//   fold of eq. (4), together with h and the frame loss sum_f d_IS(eps+v, x).
//
// Mapping.  A workgroup owns NF = 4 frames.  Rows are cut into chunks of 64;
// wave w owns chunks w, w + NW, ...  Both contractions run on
// v_mfma_f32_4x4x1_16b (16 independent 4x4 blocks, rank-1 per instruction):
//   X (reduce over k): block q = rows 4q..4q+3 of the chunk, columns = frames;
//      A operand lane l = W[f0 + l][k], B operand lane 4q+n = h[k][n].
//      Result lane 4q+n, register i = x[f0 + 4q + i][n].
//   num/den (reduce over f): block q = components 4q..4q+3, columns = frames;
//      A operand lane l = W[f][l] (k = lane), B operand lane 4q+n = r[f][n]
//      broadcast through LDS.  Result lane 4q+n, register m = num[4q+m][n].
// Both W operands stay in registers for the whole minibatch (two layouts of
// the wave's rows of W).  The per-wave num/den partials meet in LDS once per
// iteration (one barrier); every wave then applies the same h update, so h
// needs no second exchange.  Rows past the last full chunk (F = 64 m + t,
// t <= 2: the Nyquist row of an STFT) are handled on the VALU by wave 0.
//
// Precision forms (PREC 1 = BF16, 2 = FP16): the same mapping on
// v_mfma_f32_4x4x4_16b_{bf16,f16}, four contraction steps per instruction,
// FP32 accumulation.  W is rounded to 16 bits as W * 2^s and h as h * 2^-s
// (s = round(log2 F), exact power-of-two scales, so W h is unchanged) which
// keeps L1-normalised columns and large activations inside FP16's range.  The
// IS ratios, the h update, the tail rows and the loss stay FP32/FP64.
#include "common.h"
#include "devmath.h"

namespace isnmf {
namespace {

struct FusedArgs {
    int F, K, b, ldv, ldh, iters, warm;
    int main_chunks;  // chunks of 64 rows handled on MFMA (last may be partial)
    int tail;         // rows after them handled on the VALU (<= TAIL_MAX)
    int FR, KP;
    float eps;
    double epsd;
    float wscale, hscale;   // 16-bit forms: W * wscale and h * hscale (powers of two)
    const float *V;
    const float *W;   // F x K, ld F (FP32 working copy)
    float *Hb;        // caller's K x b (warm start in / fitted h out) or null
    float *Hi;        // b x KP internal copy of the fitted h
    float *R1, *R2;   // b x FR
    double *lossf;    // b
    int *flags;
};

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

// Scheduling fence: the operand loads issued before it stay ahead of the
// MFMAs after it (the scheduler would otherwise sink them and expose the LDS
// latency), and no later load is hoisted above it (bounds live registers).
__device__ inline void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// Order LDS traffic between lanes of one wave (no workgroup barrier needed).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NW, int CPW, int KMAX, int PREC>
__global__ __launch_bounds__(NW * 64) void fused_fit_kernel(FusedArgs a) {
    static_assert(KMAX % 4 == 0 && KMAX <= 64, "K class");
    constexpr bool H16 = PREC != 0;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int q = lane >> 2;
    const int n = lane & 3;
    const int fr = blockIdx.x * NF + n;  // frame of this lane's B/C column
    const bool fvalid = fr < a.b;
    const int F = a.F, K = a.K;
    const float eps = a.eps;

    // Rows of rl and hs are padded by 4 floats so that the four frames a
    // b128 read touches fall in different LDS banks.
    __shared__ floatx4 red[2][NW][2][64];       // per-wave num/den partials
    __shared__ float rl[NW][2][NF][H16 ? 4 : CHUNK + 4];   // r2/r1 of the current chunk
    __shared__ float hs[NW][NF][H16 ? 4 : KMAX + 4];       // per-wave copy of h (X operand)
    __shared__ unsigned short rl16[NW][2][NF][H16 ? CHUNK + 8 : 4];
    __shared__ unsigned short hs16[NW][NF][H16 ? KMAX + 8 : 4];
    __shared__ double lred[NW][NF];

    // ---- registers: the wave's rows of W in both operand layouts, and v
    float wx[CPW][H16 ? 1 : KMAX];          // W[f0 + lane][k]
    float wn[CPW][H16 ? 1 : CHUNK];         // W[f0 + r][lane]
    v4h wx16[CPW][H16 ? KMAX / 4 : 1];      // W[f0 + lane][4g .. 4g+3] * wscale
    v4h wn16[CPW][H16 ? CHUNK / 4 : 1];     // W[f0 + 4g .. 4g+3][lane] * wscale
    float vr[CPW][4];         // v[f0 + 4q + i][fr]
    bool cval[CPW];
    int bad = 0;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const int c = w + NW * j;
        cval[j] = c < a.main_chunks;
        const int f0 = c * CHUNK;
        auto wxv = [&](int k) {
            const int f = f0 + lane;
            return (cval[j] && k < K && f < F) ? a.W[f + (size_t)k * F] : 0.f;
        };
        auto wnv = [&](int r) {
            const int f = f0 + r;
            return (cval[j] && lane < K && f < F) ? a.W[f + (size_t)lane * F] : 0.f;
        };
        if constexpr (!H16) {
#pragma unroll
            for (int k = 0; k < KMAX; ++k) wx[j][k] = wxv(k);
#pragma unroll
            for (int r = 0; r < CHUNK; ++r) wn[j][r] = wnv(r);
        } else {
            const float sc = a.wscale;
#pragma unroll
            for (int g = 0; g < KMAX / 4; ++g)
                wx16[j][g] = pack4<PREC>(wxv(4 * g) * sc, wxv(4 * g + 1) * sc,
                                         wxv(4 * g + 2) * sc, wxv(4 * g + 3) * sc);
#pragma unroll
            for (int g = 0; g < CHUNK / 4; ++g)
                wn16[j][g] = pack4<PREC>(wnv(4 * g) * sc, wnv(4 * g + 1) * sc,
                                         wnv(4 * g + 2) * sc, wnv(4 * g + 3) * sc);
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
    // tail rows (VALU, wave 0): lane 4q+n keeps W[f][4q+m] and v[f][n]
    float wt[TAIL_MAX][4];
    float vt[TAIL_MAX];
#pragma unroll
    for (int t = 0; t < TAIL_MAX; ++t) {
        const int f = a.main_chunks * CHUNK + t;
        const bool tv = (w == 0) && t < a.tail;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int k = 4 * q + m;
            wt[t][m] = (tv && k < K) ? a.W[f + (size_t)k * F] : 0.f;
        }
        float v = 1.f;
        if (tv && fvalid) {
            v = a.V[(size_t)fr * a.ldv + f];
            bad |= !isfinite(v);
        }
        vt[t] = v;
    }
    if (bad) atomicOr(a.flags, FLAG_NONFINITE_V);

    // ---- h in the "update" layout: lane 4q+n holds h[4q+m][fr]
    float hu[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int k = 4 * q + m;
        float h = 0.f;
        if (k < K) h = (a.warm && fvalid) ? a.Hb[(size_t)fr * a.ldh + k] : 1.f;
        hu[m] = h;
    }
    // the X operand copy of h (FP32, or 16-bit scaled by hscale)
    auto store_h = [&]() {
        if (4 * q < KMAX) {
            if constexpr (!H16)
                *reinterpret_cast<floatx4 *>(&hs[w][n][4 * q]) = floatx4{hu[0], hu[1], hu[2], hu[3]};
            else
                *reinterpret_cast<v4h *>(&hs16[w][n][4 * q]) =
                    pack4<PREC>(hu[0] * a.hscale, hu[1] * a.hscale, hu[2] * a.hscale,
                                hu[3] * a.hscale);
        }
    };
    store_h();
    wave_lds_sync();

    // X = eps + W h for chunk j: lane 4q+n gets rows f0+4q+i of frame fr.
    auto model = [&](int j, float (&xv)[4]) {
        floatx4 x0 = {0.f, 0.f, 0.f, 0.f}, x1 = {0.f, 0.f, 0.f, 0.f};
        // h operand through LDS, one group of 4 components ahead of the MFMAs.
        // Components k >= K hold h = 0 and W = 0, so all KMAX/4 groups run.
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
            v4h hp[3];
            hp[0] = *reinterpret_cast<const v4h *>(&hs16[w][n][0]);
            if (KMAX > 4) hp[1] = *reinterpret_cast<const v4h *>(&hs16[w][n][4]);
#pragma unroll
            for (int g = 0; g < KMAX / 4; ++g) {
                if (g + 2 < KMAX / 4) hp[(g + 2) % 3] = *reinterpret_cast<const v4h *>(&hs16[w][n][4 * g + 8]);
                sched_fence();
                if (g & 1)
                    x1 = mfma16b<PREC>(wx16[j][g], hp[g % 3], x1);
                else
                    x0 = mfma16b<PREC>(wx16[j][g], hp[g % 3], x0);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) xv[i] = eps + (x0[i] + x1[i]);
    };
    // tail row t on the VALU: x for frame fr, identical in the 16 lanes of fr
    auto tail_model = [&](int t) {
        float p = 0.f;
#pragma unroll
        for (int m = 0; m < 4; ++m) p += wt[t][m] * hu[m];
        return eps + sum_over_quads(p);
    };

    int buf = 0;
    int guard = 0;
    for (int it = 0; it < a.iters; ++it) {
        floatx4 num = {0.f, 0.f, 0.f, 0.f}, den = {0.f, 0.f, 0.f, 0.f};
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
                        num = mfma4(wn[j][4 * qq + i], a2[i], num);
                        den = mfma4(wn[j][4 * qq + i], a1[i], den);
                    }
                }
            } else {
                *reinterpret_cast<v4h *>(&rl16[w][0][n][4 * q]) = pack4<PREC>(r2[0], r2[1], r2[2], r2[3]);
                *reinterpret_cast<v4h *>(&rl16[w][1][n][4 * q]) = pack4<PREC>(r1[0], r1[1], r1[2], r1[3]);
                wave_lds_sync();
                v4h a2p[3], a1p[3];
                a2p[0] = *reinterpret_cast<const v4h *>(&rl16[w][0][n][0]);
                a1p[0] = *reinterpret_cast<const v4h *>(&rl16[w][1][n][0]);
                a2p[1] = *reinterpret_cast<const v4h *>(&rl16[w][0][n][4]);
                a1p[1] = *reinterpret_cast<const v4h *>(&rl16[w][1][n][4]);
#pragma unroll
                for (int qq = 0; qq < CHUNK / 4; ++qq) {
                    if (qq + 2 < CHUNK / 4) {
                        a2p[(qq + 2) % 3] = *reinterpret_cast<const v4h *>(&rl16[w][0][n][4 * qq + 8]);
                        a1p[(qq + 2) % 3] = *reinterpret_cast<const v4h *>(&rl16[w][1][n][4 * qq + 8]);
                    }
                    sched_fence();
                    num = mfma16b<PREC>(wn16[j][qq], a2p[qq % 3], num);
                    den = mfma16b<PREC>(wn16[j][qq], a1p[qq % 3], den);
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
                    for (int m = 0; m < 4; ++m) {
                        num[m] += wt[t][m] * rr2;
                        den[m] += wt[t][m] * ir;
                    }
                }
            }
        }
        // ---- combine the waves' partials (one barrier), then update h
        red[buf][w][0][lane] = num;
        red[buf][w][1][lane] = den;
        __syncthreads();
        floatx4 N = red[buf][0][0][lane], D = red[buf][0][1][lane];
#pragma unroll
        for (int v = 1; v < NW; ++v) {
            N += red[buf][v][0][lane];
            D += red[buf][v][1][lane];
        }
        buf ^= 1;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (4 * q + m < K) {
                if (D[m] > 0.f && N[m] >= 0.f)
                    hu[m] *= __builtin_amdgcn_sqrtf(N[m] * __builtin_amdgcn_rcpf(D[m]));
                else
                    guard = 1;
            }
        }
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
        for (int m = 0; m < 4; ++m) {
            const int k = 4 * q + m;
            if (k < K) {
                a.Hi[(size_t)fr * a.KP + k] = hu[m];
                if (a.Hb) a.Hb[(size_t)fr * a.ldh + k] = hu[m];
            }
        }
    }
}

struct Plan {
    int main_chunks, tail, nw;
};

Plan plan_for(int F) {
    Plan p;
    p.main_chunks = F / CHUNK;
    p.tail = F % CHUNK;
    if (p.tail > TAIL_MAX) {
        p.main_chunks += 1;  // last chunk partially valid (masked)
        p.tail = 0;
    }
    int nw = p.main_chunks < 1 ? 1 : p.main_chunks;
    p.nw = nw <= 1 ? 1 : nw <= 2 ? 2 : nw <= 4 ? 4 : 8;
    return p;
}

template <int NW, int KMAX, int PREC>
hipError_t launch_t(const FusedArgs &a, int grid, hipStream_t s) {
    fused_fit_kernel<NW, 1, KMAX, PREC><<<grid, NW * 64, 0, s>>>(a);
    return hipGetLastError();
}

template <int NW, int PREC>
hipError_t launch_k(const FusedArgs &a, int grid, hipStream_t s) {
    if (a.K <= 8) return launch_t<NW, 8, PREC>(a, grid, s);
    if (a.K <= 16) return launch_t<NW, 16, PREC>(a, grid, s);
    if (a.K <= 24) return launch_t<NW, 24, PREC>(a, grid, s);
    if (a.K <= 32) return launch_t<NW, 32, PREC>(a, grid, s);
    if (a.K <= 40) return launch_t<NW, 40, PREC>(a, grid, s);
    if (a.K <= 52) return launch_t<NW, 52, PREC>(a, grid, s);
    return launch_t<NW, 64, PREC>(a, grid, s);
}

template <int PREC>
hipError_t launch_p(const FusedArgs &a, int nw, int grid, hipStream_t s) {
    switch (nw) {
        case 1: return launch_k<1, PREC>(a, grid, s);
        case 2: return launch_k<2, PREC>(a, grid, s);
        case 4: return launch_k<4, PREC>(a, grid, s);
        default: return launch_k<8, PREC>(a, grid, s);
    }
}

}  // namespace

bool fused_supported(int F, int K) {
    if (F < 1 || K < 1 || K > 64) return false;
    const Plan p = plan_for(F);
    return p.main_chunks <= 8;
}

hipError_t launch_fused_fit(const OnlineDev &d, const float *V, int ldv, int b, int iters,
                            double eps, int warm, float *Hb, int ldh, int prec, hipStream_t s) {
    if (!fused_supported(d.F, d.K)) return hipErrorNotSupported;
    const Plan p = plan_for(d.F);
    FusedArgs a;
    a.F = d.F;
    a.K = d.K;
    a.b = b;
    a.ldv = ldv;
    a.ldh = ldh;
    a.iters = iters;
    a.warm = warm;
    a.main_chunks = p.main_chunks;
    a.tail = p.tail;
    a.FR = d.FR;
    a.KP = d.KP;
    a.eps = float(eps);
    a.epsd = eps;
    a.V = V;
    a.W = d.W32;
    a.Hb = Hb;
    a.Hi = (float *)d.Hi;
    a.R1 = (float *)d.R1;
    a.R2 = (float *)d.R2;
    a.lossf = d.lossf;
    a.flags = d.flags;
    const int sexp = (int)lrint(log2((double)d.F));
    a.wscale = ldexpf(1.f, sexp);
    a.hscale = ldexpf(1.f, -sexp);
    const int grid = (b + NF - 1) / NF;
    if (prec == 1) return launch_p<1>(a, p.nw, grid, s);
    if (prec == 2) return launch_p<2>(a, p.nw, grid, s);
    return launch_p<0>(a, p.nw, grid, s);
}

}  // namespace isnmf
