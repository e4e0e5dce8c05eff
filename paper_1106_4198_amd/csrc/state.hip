// Dictionary update of one online step (Algorithm 1, body of "if t = 0 mod
// beta"; eq. (4) summed over the minibatch; scaling of past data and rescaling
// of W, section 2.3):
//   fold:    A <- rho A + (sum_n r2_n h_n^T) o W^2,   B <- rho B + sum_n r1_n h_n^T
//            Wn = sqrt(A / B)
//   rescale: s_k = sum_f Wn_fk;  W = Wn / s,  A /= s,  B *= s,  warm H[k,:] *= s;
//            dW = ||W_new - W_old||_F;  loss_sum += sum_n loss_n
// A, B and the master W are FP64.  Every sum runs in a fixed order, so the
// results are bitwise repeatable.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "common.h"

namespace isnmf {
namespace {

// Thread per (f, k); f fastest so the R reads coalesce and h is uniform.
template <typename TR>
__global__ void fold_kernel(int F, int K, int b, int FR, int KP, const TR *__restrict__ R1,
                            const TR *__restrict__ R2, const TR *__restrict__ H,
                            const double *__restrict__ W64, double *__restrict__ A,
                            double *__restrict__ B, double *__restrict__ Wn, double rho,
                            int update_w, int *__restrict__ flags) {
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
    const double a = rho * A[e] + sa * (w * w);
    const double bb = rho * B[e] + sb;
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

__device__ inline uint16_t to_half_bits(double v, int kind) {
    if (kind == 1) {
        __hip_bfloat16 h = __float2bfloat16(float(v));
        return *reinterpret_cast<uint16_t *>(&h);
    }
    __half h = __float2half(float(v));
    return *reinterpret_cast<uint16_t *>(&h);
}

// Block per column k.  The last block to finish (ticket counter) writes the
// scalar diagnostics, summing the per-column and per-frame partials in index
// order.
__global__ void rescale_kernel(int F, int K, int b, const double *__restrict__ Wn,
                               double *__restrict__ W64, float *__restrict__ W32,
                               uint16_t *__restrict__ W16, int w16_kind, double *__restrict__ A,
                               double *__restrict__ B, int update_w, int normalize, int warm,
                               float *__restrict__ Hb, int ldh, double *__restrict__ dwpart,
                               const double *__restrict__ lossf, double *__restrict__ d_loss_sum,
                               double *__restrict__ d_dw, unsigned *__restrict__ counter,
                               int *__restrict__ flags) {
    __shared__ double red[256];
    __shared__ bool last;
    const int k = blockIdx.x;
    const int tid = threadIdx.x;
    const size_t col = (size_t)k * F;
    if (update_w) {
        double s = 0.0;
        for (int f = tid; f < F; f += 256) s += Wn[col + f];
        red[tid] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        double scale = 1.0;
        if (normalize) {
            if (red[0] > 0.0)
                scale = red[0];
            else if (tid == 0)
                atomicOr(flags, FLAG_GUARD_W);
        }
        __syncthreads();
        double dw = 0.0;
        for (int f = tid; f < F; f += 256) {
            const double wn = Wn[col + f] / scale;
            const double dlt = wn - W64[col + f];
            dw += dlt * dlt;
            W64[col + f] = wn;
            W32[col + f] = float(wn);
            if (W16) W16[col + f] = to_half_bits(wn, w16_kind);
            if (normalize) {
                A[col + f] /= scale;
                B[col + f] *= scale;
            }
        }
        if (warm && Hb && normalize)
            for (int n = tid; n < b; n += 256) Hb[(size_t)n * ldh + k] *= float(scale);
        red[tid] = dw;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0) dwpart[k] = red[0];
    } else if (tid == 0) {
        dwpart[k] = 0.0;
    }
    // last-block diagnostics.  The agent-scope fences write back / invalidate
    // the per-XCD L2 so the partials of blocks on other XCDs are visible.
    __threadfence();
    __syncthreads();
    if (tid == 0) last = atomicAdd(counter, 1u) == (unsigned)(gridDim.x - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (tid == 0) {
        double dw2 = 0.0;
        for (int j = 0; j < K; ++j) dw2 += dwpart[j];
        double ls = 0.0;
        if (d_loss_sum && lossf)
            for (int n = 0; n < b; ++n) ls += lossf[n];
        if (d_dw) *d_dw = sqrt(dw2);
        if (d_loss_sum) *d_loss_sum += ls;
        *counter = 0u;
    }
}

__global__ void set_w_kernel(int F, int K, const float *__restrict__ W, int ldw,
                             const double *__restrict__ Wd, double *__restrict__ W64,
                             float *__restrict__ W32, uint16_t *__restrict__ W16, int w16_kind) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)F * K) return;
    const int f = (int)(e % F);
    const int k = (int)(e / F);
    const double v = Wd ? Wd[e] : double(W[f + (size_t)k * ldw]);
    W64[e] = v;
    W32[e] = float(v);
    if (W16) W16[e] = to_half_bits(v, w16_kind);
}

}  // namespace

hipError_t launch_fold(const OnlineDev &d, int b, double rho, int update_w, int is_double,
                       hipStream_t s) {
    const long n = (long)d.F * d.K;
    const int blocks = (int)((n + 255) / 256);
    if (is_double)
        fold_kernel<double><<<blocks, 256, 0, s>>>(d.F, d.K, b, d.FR, d.KP, (const double *)d.R1,
                                                   (const double *)d.R2, (const double *)d.Hi,
                                                   d.W64, d.A, d.B, d.Wn, rho, update_w, d.flags);
    else
        fold_kernel<float><<<blocks, 256, 0, s>>>(d.F, d.K, b, d.FR, d.KP, (const float *)d.R1,
                                                  (const float *)d.R2, (const float *)d.Hi,
                                                  d.W64, d.A, d.B, d.Wn, rho, update_w, d.flags);
    return hipGetLastError();
}

hipError_t launch_rescale(const OnlineDev &d, int b, int update_w, int normalize, int warm,
                          float *Hb, int ldh, double *d_loss_sum, double *d_dw, int w16_kind,
                          hipStream_t s) {
    rescale_kernel<<<d.K, 256, 0, s>>>(d.F, d.K, b, d.Wn, d.W64, d.W32, w16_kind ? d.W16 : nullptr,
                                       w16_kind, d.A, d.B, update_w, normalize, warm, Hb, ldh,
                                       d.dwpart, d.lossf, d_loss_sum, d_dw, d.counter, d.flags);
    return hipGetLastError();
}

hipError_t launch_set_w(const OnlineDev &d, const float *W, int ldw, const double *W64,
                        int w16_kind, hipStream_t s) {
    const long n = (long)d.F * d.K;
    set_w_kernel<<<(int)((n + 255) / 256), 256, 0, s>>>(d.F, d.K, W, ldw, W64, d.W64, d.W32,
                                                        w16_kind ? d.W16 : nullptr, w16_kind);
    return hipGetLastError();
}

hipError_t launch_get_w(const OnlineDev &d, float *W, hipStream_t s) {
    return hipMemcpyAsync(W, d.W32, sizeof(float) * (size_t)d.F * d.K, hipMemcpyDeviceToDevice, s);
}

}  // namespace isnmf
