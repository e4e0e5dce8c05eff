// Dictionary update of one online step (Algorithm 1, body of "if t = 0 mod
// beta"; eq. (4) summed over the minibatch; scaling of past data and rescaling
// of W, section 2.3):
//   fold:    A <- rho A + (sum_n r2_n h_n^T) o W^2,   B <- rho B + sum_n r1_n h_n^T
//            Wn = sqrt(A / B)
//   rescale: s_k = sum_f Wn_fk;  W = Wn / s,  A /= s,  B *= s,  warm H[k,:] *= s;
//            dW = ||W_new - W_old||_F;  loss_sum += sum_n loss_n
// A, B and the master W are FP64.  A /= s and B *= s are deferred: the
// rescale records s in sc, and whoever reads A and B next (the next fold,
// isnmf_online_get) divides and multiplies by it, so they are read and written
// once per step instead of twice.  Every sum runs in a fixed order, so the
// results are bitwise repeatable.
#include "common.h"
#include "state_body.h"

namespace isnmf {
namespace {

// Thread per (f, k); f fastest so the R reads coalesce and h is uniform.
template <typename TR>
__global__ void fold_kernel(int F, int K, int b, int FR, int KP, const TR *__restrict__ R1,
                            const TR *__restrict__ R2, const TR *__restrict__ H,
                            const double *__restrict__ W64, double *__restrict__ A,
                            double *__restrict__ B, const double *__restrict__ sc,
                            double *__restrict__ Wn, double rho, int update_w,
                            int *__restrict__ flags) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)F * K) return;
    const int f = (int)(e % F);
    const int k = (int)(e / F);
    double sa = 0.0, sb = 0.0;
    for (int n = 0; n < b; ++n) {
        const double h = double(H[(size_t)n * KP + k]);
        sa += double(R2[(size_t)n * FR + f]) * h;
        sb += double(R1[(size_t)n * FR + f]) * h;
    }
    const double w = W64[e];
    const double a = rho * (A[e] / sc[k]) + sa * (w * w);
    const double bb = rho * (B[e] * sc[k]) + sb;
    A[e] = a;
    B[e] = bb;
    if (update_w) {
        double wn = w;
        if (bb > 0.0 && a >= 0.0)
            wn = sqrt(a / bb);
        else
            atomicOr(flags, FLAG_GUARD_W);
        Wn[e] = wn;
    }
}

__global__ __launch_bounds__(64) void rescale_kernel(RescaleArgs a, int b) {
    rescale_body(a, blockIdx.x, b);
}

// Warm-start activations times their column's scale, H[n][k] *= s_k, one
// thread per entry (the multiplication rescale_body applies per column, here
// over rows of H in memory order).
__global__ void scale_h_kernel(float *__restrict__ Hb, int ldh, int b, int K,
                               const double *__restrict__ sc) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)b * K) return;
    const int n = (int)(i / K), k = (int)(i % K);
    Hb[(size_t)n * ldh + k] *= float(sc[k]);
}

__global__ void unit_scale_kernel(double *__restrict__ sc, int K) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K) sc[k] = 1.0;
}

// The statistics with the pending scale applied: A[:,k] / sc[k], B[:,k] * sc[k]
// into Ao, Bo (either may be null); in place when they are A and B themselves.
__global__ void apply_scale_kernel(int F, int K, const double *A, const double *B,
                                   const double *__restrict__ sc, double *Ao, double *Bo) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)F * K) return;
    const int k = (int)(e / F);
    if (Ao) Ao[e] = A[e] / sc[k];
    if (Bo) Bo[e] = B[e] * sc[k];
}

// ||W_new - W_old||_F from the per-column partials, in column order.
__global__ void dw_total_kernel(int K, const double *__restrict__ dwpart, int update_w,
                                double *__restrict__ out) {
    if (threadIdx.x == 0) {
        double s = 0.0;
        if (update_w)
            for (int k = 0; k < K; ++k) s += dwpart[k];
        *out = sqrt(s);
    }
}

__global__ void set_w_kernel(int F, int K, const float *__restrict__ W, int ldw,
                             const double *__restrict__ Wd, double *__restrict__ W64,
                             float *__restrict__ W32, W16Out w16, WvOut wv) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)F * K) return;
    const int f = (int)(e % F);
    const int k = (int)(e / F);
    const double v = Wd ? Wd[e] : double(W[f + (size_t)k * ldw]);
    W64[e] = v;
    W32[e] = float(v);
    store_w16(w16, f, k, v);
    store_wv(wv, f, k, v);
}

// Same order as the MFMA fold's loss sum: lane l adds frames l, l + 64, ...,
// then a fixed xor butterfly (one wave).
__global__ void loss_total_kernel(const double *__restrict__ lossf, int b,
                                  double *__restrict__ out) {
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int n = lane; n < b; n += 64) s += lossf[n];
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) s += __shfl_xor(s, m, 64);
    if (lane == 0) *out += s;
}

__global__ void row_swap_kernel(const RowSwap a) {
    const int t = threadIdx.x;
    if ((int)blockIdx.x < a.n_in) {
        const int i = blockIdx.x;
        const long long r = a.in_idx[i];
        const bool ok = r >= 0 && r < a.N;
        if (!ok && t == 0) atomicOr(a.flags, FLAG_BAD_INDEX);
        const float *v = a.V + (ok ? r : 0) * a.ldv;
        const float *h = a.H + (ok ? r : 0) * a.ldh;
        for (int j = t; j < a.F; j += 256) a.Vg[(size_t)i * a.F + j] = ok ? v[j] : 0.f;
        for (int j = t; j < a.K; j += 256) a.Hg_in[(size_t)i * a.K + j] = ok ? h[j] : 0.f;
    } else {
        const int i = blockIdx.x - a.n_in;
        const long long r = a.out_idx[i];
        if (r < 0 || r >= a.N) return;
        for (int j = t; j < a.K; j += 256) a.H[r * a.ldh + j] = a.Hg_out[(size_t)i * a.K + j];
    }
}

}  // namespace

hipError_t launch_row_swap(const RowSwap &a, hipStream_t s) {
    if (a.n_in + a.n_out < 1) return hipSuccess;
    row_swap_kernel<<<a.n_in + a.n_out, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_loss_total(const double *lossf, int b, double *d_loss_sum, hipStream_t s) {
    loss_total_kernel<<<1, 64, 0, s>>>(lossf, b, d_loss_sum);
    return hipGetLastError();
}

hipError_t launch_fold(const OnlineDev &d, int b, double rho, int update_w, int is_double,
                       hipStream_t s) {
    const long n = (long)d.F * d.K;
    const int blocks = (int)((n + 255) / 256);
    if (is_double)
        fold_kernel<double><<<blocks, 256, 0, s>>>(d.F, d.K, b, d.FR, d.KP, (const double *)d.R1,
                                                   (const double *)d.R2, (const double *)d.Hi,
                                                   d.W64, d.A, d.B, d.sc, d.Wn, rho, update_w,
                                                   d.flags);
    else
        fold_kernel<float><<<blocks, 256, 0, s>>>(d.F, d.K, b, d.FR, d.KP, (const float *)d.R1,
                                                  (const float *)d.R2, (const float *)d.Hi,
                                                  d.W64, d.A, d.B, d.sc, d.Wn, rho, update_w,
                                                  d.flags);
    return hipGetLastError();
}

// Warm frames per step above which H is scaled by its own launch.
constexpr int SCALE_H_APART = 2048;

hipError_t launch_rescale(const OnlineDev &d, int b, int update_w, int normalize, int warm,
                          float *Hb, int ldh, double *d_dw, hipStream_t s) {
    if (update_w) {
        RescaleArgs a = rescale_args(d, normalize, warm, Hb, ldh);
        if (!d_dw) a.dwpart = nullptr;
        // Many warm frames (batch MU's whole set): the per-column loop over H
        // strides by ldh, so a separate launch scales H row by row instead.
        const bool h_apart = warm && Hb && normalize && b > SCALE_H_APART;
        if (h_apart) a.Hb = nullptr;
        rescale_kernel<<<d.K, 64, 0, s>>>(a, b);
        if (h_apart) {
            const long n = (long)b * d.K;
            scale_h_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(Hb, ldh, b, d.K, d.sc);
        }
    } else {
        // the fold stored A and B with no pending scale
        unit_scale_kernel<<<(d.K + 63) / 64, 64, 0, s>>>(d.sc, d.K);
    }
    if (d_dw) dw_total_kernel<<<1, 64, 0, s>>>(d.K, d.dwpart, update_w, d_dw);
    return hipGetLastError();
}

hipError_t launch_unit_scale(const OnlineDev &d, hipStream_t s) {
    unit_scale_kernel<<<(d.K + 63) / 64, 64, 0, s>>>(d.sc, d.K);
    return hipGetLastError();
}

hipError_t launch_get_ab(const OnlineDev &d, double *A, double *B, hipStream_t s) {
    const long n = (long)d.F * d.K;
    if (!A && !B) return hipSuccess;
    apply_scale_kernel<<<(int)((n + 255) / 256), 256, 0, s>>>(d.F, d.K, d.A, d.B, d.sc, A, B);
    return hipGetLastError();
}

hipError_t launch_settle_ab(const OnlineDev &d, hipStream_t s) {
    hipError_t e = launch_get_ab(d, d.A, d.B, s);
    if (e == hipSuccess) e = launch_unit_scale(d, s);
    return e;
}

hipError_t launch_set_w(const OnlineDev &d, const float *W, int ldw, const double *W64,
                        hipStream_t s) {
    const long n = (long)d.F * d.K;
    set_w_kernel<<<(int)((n + 255) / 256), 256, 0, s>>>(d.F, d.K, W, ldw, W64, d.W64, d.W32,
                                                        w16_out(d), wv_out(d));
    return hipGetLastError();
}

hipError_t launch_get_w(const OnlineDev &d, float *W, hipStream_t s) {
    return hipMemcpyAsync(W, d.W32, sizeof(float) * (size_t)d.F * d.K, hipMemcpyDeviceToDevice, s);
}

}  // namespace isnmf
