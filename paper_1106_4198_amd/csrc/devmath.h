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
