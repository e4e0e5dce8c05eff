// Plain (unfused) fit of a minibatch: one simple kernel per operation, launched
// 2*I + 2 times per minibatch.  This is the comparison point of the fused
// path and, instantiated in FP64, the logic check against the FP64 oracle.
//
// One multiplicative update of h for frame n (section 2.1 "similar updates";
// Algorithm 1, inner argmin with the eps shift of section 2.3):
//   x_f = eps + sum_k W_fk h_k,  r1_f = 1/x_f,  r2_f = (eps + v_f) r1_f^2
//   h_k <- h_k sqrt( sum_f W_fk r2_f / sum_f W_fk r1_f )
// With the penalty on H (section 2.2, Extensions; psi(s) = lambda log(a + s)
// of the column sum s = sum_k h_k), lambda / (a + s) joins the denominator,
// s taken before the update.
#include <type_traits>

#include "common.h"
#include "devmath.h"

namespace isnmf {
namespace {

template <typename T>
__global__ void plain_hinit(int K, int b, int KP, int warm, const float *__restrict__ Hin, int ldh,
                            T *__restrict__ H) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y;
    if (k >= KP || n >= b) return;
    T v = T(0);
    if (k < K) v = warm ? T(Hin[(size_t)n * ldh + k]) : T(1);
    H[(size_t)n * KP + k] = v;
}

// Model, ratios and (optionally) the per-element loss.  Thread per (f, n).
template <typename T>
__global__ void plain_model(int F, int K, int b, const float *__restrict__ V, int ldv,
                            const T *__restrict__ W, const T *__restrict__ H, int KP, T eps,
                            T *__restrict__ R1, T *__restrict__ R2, int FR,
                            double *__restrict__ lossel, int *__restrict__ flags) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y;
    if (f >= F || n >= b) return;
    const T *h = H + (size_t)n * KP;
    T x = eps;
    for (int k = 0; k < K; ++k) x += W[f + (size_t)k * F] * h[k];
    const float vin = V[(size_t)n * ldv + f];
    if (!isfinite(vin)) atomicOr(flags, FLAG_NONFINITE_V);
    const T y = eps + T(vin);
    const T r1 = T(1) / x;
    R1[(size_t)n * FR + f] = r1;
    R2[(size_t)n * FR + f] = y / (x * x);
    if (lossel) lossel[(size_t)n * FR + f] = dis_term(double(eps) + double(vin), double(x));
}

// Column sums of H in index order (penalty on H).  Thread per frame.
template <typename T>
__global__ void plain_hsum(int K, int b, int KP, const T *__restrict__ H, T *__restrict__ S) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= b) return;
    T s = T(0);
    for (int k = 0; k < K; ++k) s += H[(size_t)n * KP + k];
    S[n] = s;
}

// num/den and the multiplicative update of h.  Thread per (k, n).  S: null,
// or the column sums for the penalty term lambda / (a + S[n]).
template <typename T>
__global__ void plain_numden(int F, int K, int b, const T *__restrict__ W,
                             const T *__restrict__ R1, const T *__restrict__ R2, int FR,
                             T *__restrict__ H, int KP, const T *__restrict__ S, T lam, T pa,
                             int *__restrict__ flags) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y;
    if (k >= K || n >= b) return;
    const T *r1 = R1 + (size_t)n * FR;
    const T *r2 = R2 + (size_t)n * FR;
    const T *wk = W + (size_t)k * F;
    T num = T(0), den = T(0);
    for (int f = 0; f < F; ++f) {
        num += wk[f] * r2[f];
        den += wk[f] * r1[f];
    }
    if (S) den += lam / (pa + S[n]);
    T hk = H[(size_t)n * KP + k];
    if (den > T(0) && num >= T(0))
        hk *= sqrt(num / den);
    else
        atomicOr(flags, FLAG_GUARD_H);
    H[(size_t)n * KP + k] = hk;
}

// Per-frame sum of the loss terms in a fixed order.  Block per frame.
__global__ void plain_loss_frames(int F, int FR, const double *__restrict__ lossel,
                                  double *__restrict__ lossf) {
    __shared__ double red[256];
    const int n = blockIdx.x;
    double s = 0.0;
    for (int f = threadIdx.x; f < F; f += 256) s += lossel[(size_t)n * FR + f];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) lossf[n] = red[0];
}

template <typename T>
__global__ void plain_hout(int K, int b, int KP, const T *__restrict__ H, float *__restrict__ Hb,
                           int ldh) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y;
    if (k >= K || n >= b) return;
    Hb[(size_t)n * ldh + k] = float(H[(size_t)n * KP + k]);
}

}  // namespace

template <typename T>
hipError_t launch_plain_fit(const OnlineDev &d, const float *V, int ldv, int b, int iters,
                            double eps, int warm, float *Hb, int ldh, hipStream_t s) {
    const T *W = std::is_same<T, double>::value ? (const T *)d.W64 : (const T *)d.W32;
    T *H = (T *)d.Hi;
    T *R1 = (T *)d.R1;
    T *R2 = (T *)d.R2;
    const T e = T(eps);
    T *S = d.psi_lambda > 0.0 ? (T *)d.hsum : nullptr;
    if (d.psi_lambda > 0.0 && !S) return hipErrorInvalidValue;
    dim3 gk((d.KP + 63) / 64, b), gf((d.F + 255) / 256, b), gkk((d.K + 63) / 64, b);
    plain_hinit<T><<<gk, 64, 0, s>>>(d.K, b, d.KP, warm, Hb, ldh, H);
    for (int it = 0; it < iters; ++it) {
        plain_model<T><<<gf, 256, 0, s>>>(d.F, d.K, b, V, ldv, W, H, d.KP, e, R1, R2, d.FR,
                                          nullptr, d.flags);
        if (S) plain_hsum<T><<<(b + 63) / 64, 64, 0, s>>>(d.K, b, d.KP, H, S);
        plain_numden<T><<<gkk, 64, 0, s>>>(d.F, d.K, b, W, R1, R2, d.FR, H, d.KP, S,
                                           T(d.psi_lambda), T(d.psi_a), d.flags);
    }
    plain_model<T><<<gf, 256, 0, s>>>(d.F, d.K, b, V, ldv, W, H, d.KP, e, R1, R2, d.FR,
                                      d.lossel, d.flags);
    if (d.lossel) plain_loss_frames<<<b, 256, 0, s>>>(d.F, d.FR, d.lossel, d.lossf);
    if (Hb) plain_hout<T><<<gkk, 64, 0, s>>>(d.K, b, d.KP, H, Hb, ldh);
    return hipGetLastError();
}

template hipError_t launch_plain_fit<float>(const OnlineDev &, const float *, int, int, int,
                                            double, int, float *, int, hipStream_t);
template hipError_t launch_plain_fit<double>(const OnlineDev &, const float *, int, int, int,
                                             double, int, float *, int, hipStream_t);

}  // namespace isnmf
