// Objective of eq. (1) with the eps shift of section 2.3:
//   (1/N) sum_n sum_f d_IS(eps + V_fn, eps + (W H)_fn)
// The model value is formed in FP32, every divergence term and every sum in
// FP64, in a fixed order (per-frame block sums, then frames in index order).
#include "common.h"
#include "devmath.h"

namespace isnmf {
namespace {

// Block per frame n.
__global__ void objective_frames(const float *__restrict__ V, int ldv,
                                 const float *__restrict__ W, int ldw,
                                 const float *__restrict__ H, int ldh, int F, int K,
                                 double eps, double *__restrict__ frame_buf) {
    __shared__ double red[256];
    const int n = blockIdx.x;
    const float *h = H + (size_t)n * ldh;
    const float *v = V + (size_t)n * ldv;
    const float epsf = float(eps);
    double s = 0.0;
    for (int f = threadIdx.x; f < F; f += 256) {
        float x = epsf;
        for (int k = 0; k < K; ++k) x += W[f + (size_t)k * ldw] * h[k];
        s += dis_term(eps + double(v[f]), double(x));
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) frame_buf[n] = red[0];
}

// One block: fixed-order total of the frame sums, scaled by 1/N.
__global__ void objective_total(int N, const double *__restrict__ frame_buf,
                                double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    const int per = (N + 255) / 256;
    const int lo = threadIdx.x * per;
    const int hi = min(N, lo + per);
    for (int n = lo; n < hi; ++n) s += frame_buf[n];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = N > 0 ? red[0] / double(N) : 0.0;
}

}  // namespace

hipError_t launch_objective(const float *V, int ldv, const float *W, int ldw, const float *H,
                            int ldh, int F, int K, int N, double eps, double *frame_buf,
                            double *d_out, hipStream_t s) {
    if (N > 0)
        objective_frames<<<N, 256, 0, s>>>(V, ldv, W, ldw, H, ldh, F, K, eps, frame_buf);
    objective_total<<<1, 256, 0, s>>>(N, frame_buf, d_out);
    return hipGetLastError();
}

}  // namespace isnmf
