// Device math shared by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace isnmf {

// Coefficients (-1)^j / j of the series of  d - log(1 + d),  j = 2..24.
struct DisSeries {
    double c[25];
    constexpr DisSeries() : c() {
        for (int j = 2; j <= 24; ++j) c[j] = ((j & 1) ? -1.0 : 1.0) / double(j);
    }
};

// One Itakura-Saito term  y/x - log(y/x) - 1  in FP64 (section 2.1).  With
// u = y/x and d = u - 1, |d| < 0.1 sums the Taylor series of d - log(1+d)
// (to d^24) instead of the cancelling difference.
__device__ inline double dis_term(double y, double x) {
    constexpr DisSeries S;
    const double u = y / x;
    const double d = u - 1.0;
    if (fabs(d) < 0.1) {
        double s = 0.0;
#pragma unroll
        for (int j = 24; j >= 2; --j) s = fma(s, d, S.c[j]);
        return s * d * d;
    }
    return d - log(u);
}

// The same term in FP32 from y and r = 1/x (the reciprocal the fit already
// has): u = y r, d = u - 1; |d| < 1/8 sums the series of d - log(1 + d) to
// d^9 (truncation below 2^-24 of the term), else d - log u.  The fused FP32
// and 16-bit fits evaluate the frame loss with it and sum it in FP64.
__device__ inline float dis_term32(float y, float r) {
    const float u = y * r;
    const float d = u - 1.f;
    if (fabsf(d) < 0.125f) {
        float s = -1.f / 9.f;
        s = fmaf(s, d, 1.f / 8.f);
        s = fmaf(s, d, -1.f / 7.f);
        s = fmaf(s, d, 1.f / 6.f);
        s = fmaf(s, d, -1.f / 5.f);
        s = fmaf(s, d, 1.f / 4.f);
        s = fmaf(s, d, -1.f / 3.f);
        s = fmaf(s, d, 1.f / 2.f);
        return s * d * d;
    }
    return d - __logf(u);
}

// Sum over the 64 lanes of a wave in a fixed order, the result in every
// lane: 8-lane groups with DPP (xor 1, xor 2, half-row mirror), lanes 8 apart
// (row_ror 8), then 16-lane rows and 32-lane halves with the gfx950
// permlane16/permlane32 swaps.  No LDS and no barrier.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const unsigned lo = __builtin_amdgcn_update_dpp(0u, (unsigned)u, CTRL, 0xf, 0xf, false);
    const unsigned hi = __builtin_amdgcn_update_dpp(0u, (unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, (uint64_t)hi << 32 | lo);
}

__device__ inline double join_f64(unsigned lo, unsigned hi) {
    return __builtin_bit_cast(double, (uint64_t)hi << 32 | lo);
}

__device__ inline double wave_sum_f64(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x128>(v);
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    auto l16 = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
    auto h16 = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    v = join_f64(l16[0], h16[0]) + join_f64(l16[1], h16[1]);
    u = __builtin_bit_cast(uint64_t, v);
    auto l32 = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
    auto h32 = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    return join_f64(l32[0], h32[0]) + join_f64(l32[1], h32[1]);
}

// Sum over the wave in a fixed order (same value in every lane): the xor
// butterfly over lane bits 0..5.
__device__ inline float wave_sum_f32(float v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Sum over the 16 lanes that share (lane & 3): xor butterfly over lane bits
// 2..5.  Every lane of the group ends with the same, order-independent value.
__device__ inline double sum_over_quads(double v) {
#pragma unroll
    for (int m = 4; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ inline float sum_over_quads(float v) {
#pragma unroll
    for (int m = 4; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

}  // namespace isnmf
