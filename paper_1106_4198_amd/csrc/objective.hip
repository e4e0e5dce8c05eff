// Objective of eq. (1) with the eps shift of section 2.3:
//   (1/N) sum_n sum_f d_IS(eps + V_fn, eps + (W H)_fn)
// The model value is formed in FP32, every divergence term and every sum in
// FP64, in a fixed order (per-frame block sums, then frames in index order).
#include <mutex>

#include "common.h"
#include "devmath.h"

namespace isnmf {
namespace {

// Per-frame partial sums of isnmf_objective_noalloc, for callers that cannot
// allocate: one copy per GPU, held until the process ends.  Host code never
// uses this name as an address; it takes the device address from
// hipGetSymbolAddress (scratch_ptr below) on each device.
__device__ __align__(256) double scratch[ISNMF_OBJECTIVE_NOALLOC_MAX_FRAMES];

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

// The same sums as objective_frames, with W read once per block instead of
// once per frame: thread t keeps its rows t, t + 256, ... of W (RF =
// ceil(F / 256) rows, K <= KM components) in registers and the block loops
// over frames n = blockIdx.x, blockIdx.x + gridDim.x, ...  Each model value
// is the same FMA chain over k in increasing order (the KM - K padded steps
// add 0 * 0, which leaves a chain that starts at eps >= 0 with non-negative
// W and H unchanged), the thread adds its terms in row order, and the 256
// thread sums meet in the same tree: the two levels across waves through LDS,
// the last six within wave 0 by shuffles that pair the same lanes.  So every
// frame sum has objective_frames' bits for W, H >= 0.
template <int RF, int KM>
__global__ __launch_bounds__(256) void objective_frames_reg(const float *__restrict__ V, int ldv,
                                                            const float *__restrict__ W, int ldw,
                                                            const float *__restrict__ H, int ldh,
                                                            int F, int K, int N, double eps,
                                                            double *__restrict__ frame_buf) {
    __shared__ double red[2][256];   // alternate frames, so one barrier less per frame
    const int t = threadIdx.x, lane = t & 63;
    const float epsf = float(eps);
    float w[RF][KM];
#pragma unroll
    for (int r = 0; r < RF; ++r) {
        const int f = t + 256 * r;
#pragma unroll
        for (int k = 0; k < KM; ++k) w[r][k] = (f < F && k < K) ? W[f + (size_t)k * ldw] : 0.f;
    }
    // a frame's h (lane k of every wave holds h_k, zero past K) and the
    // thread's v values, loaded one frame ahead
    auto load = [&](int n, float &hv, float (&vv)[RF]) {
        hv = (n < N && lane < K) ? H[(size_t)n * ldh + lane] : 0.f;
#pragma unroll
        for (int r = 0; r < RF; ++r) {
            const int f = t + 256 * r;
            vv[r] = (n < N && f < F) ? V[(size_t)n * ldv + f] : 0.f;
        }
    };
    float hv, vv[RF];
    load(blockIdx.x, hv, vv);
    int p = 0;
    for (int n = blockIdx.x; n < N; n += gridDim.x, p ^= 1) {
        float hn, vn[RF];
        load(n + gridDim.x, hn, vn);
        float x[RF];
#pragma unroll
        for (int r = 0; r < RF; ++r) x[r] = epsf;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const float hk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hv), k));
#pragma unroll
            for (int r = 0; r < RF; ++r) x[r] = __builtin_fmaf(w[r][k], hk, x[r]);
        }
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < RF; ++r)
            if (t + 256 * r < F) s += dis_term(eps + double(vv[r]), double(x[r]));
        double *rd = red[p];
        rd[t] = s;
        __syncthreads();
        if (t < 128) rd[t] += rd[t + 128];
        __syncthreads();
        if (t < 64) {
            double v = rd[t] + rd[t + 64];
#pragma unroll
            for (int m = 32; m > 0; m >>= 1) v += __shfl_down(v, m, 64);
            if (t == 0) frame_buf[n] = v;
        }
        hv = hn;
#pragma unroll
        for (int r = 0; r < RF; ++r) vv[r] = vn[r];
    }
}

// One block: fixed-order total of the frame sums, scaled by 1/N.
__global__ void objective_total(int N, const double *__restrict__ frame_buf,
                                double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    const int per = (N + 255) / 256;
    const int lo = threadIdx.x * per;
    const int hi = min(N, lo + per);
    // the thread's frames in index order; eight loads are issued before
    // their adds, so the adds do not wait on one load at a time
    for (int n = lo; n < hi; n += 8) {
        double b[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) b[j] = n + j < hi ? frame_buf[n + j] : 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (n + j < hi) s += b[j];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = N > 0 ? red[0] / double(N) : 0.0;
}

}  // namespace

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES] = {};

hipError_t scratch_ptr(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = (double *)g_scratch[dev];
    return hipSuccess;
}

namespace {

// Register-resident form for RF = ceil(F / 256) <= 4 rows per thread and K
// components rounded up to KM (a multiple of 4) with RF * KM <= 160 floats of
// W per thread (two blocks per CU); false where it has no instance.
constexpr int OBJ_BLOCKS = 512;   // two 4-wave blocks per CU

template <int RF>
bool launch_reg(int KM, const float *V, int ldv, const float *W, int ldw, const float *H, int ldh,
                int F, int K, int N, double eps, double *frame_buf, hipStream_t s) {
    const int grid = N < OBJ_BLOCKS ? N : OBJ_BLOCKS;
    switch (KM) {
#define ISNMF_OBJ_KM(M)                                                                          \
    case M:                                                                                      \
        if constexpr (RF * M <= 160) {                                                           \
            objective_frames_reg<RF, M><<<grid, 256, 0, s>>>(V, ldv, W, ldw, H, ldh, F, K, N, eps, \
                                                             frame_buf);                         \
            return true;                                                                         \
        }                                                                                        \
        return false;
        ISNMF_OBJ_KM(4) ISNMF_OBJ_KM(8) ISNMF_OBJ_KM(12) ISNMF_OBJ_KM(16)
        ISNMF_OBJ_KM(20) ISNMF_OBJ_KM(24) ISNMF_OBJ_KM(28) ISNMF_OBJ_KM(32)
        ISNMF_OBJ_KM(36) ISNMF_OBJ_KM(40) ISNMF_OBJ_KM(44) ISNMF_OBJ_KM(48)
        ISNMF_OBJ_KM(52) ISNMF_OBJ_KM(56) ISNMF_OBJ_KM(60) ISNMF_OBJ_KM(64)
#undef ISNMF_OBJ_KM
        default: return false;
    }
}

}  // namespace

hipError_t launch_objective(const float *V, int ldv, const float *W, int ldw, const float *H,
                            int ldh, int F, int K, int N, double eps, double *frame_buf,
                            double *d_out, hipStream_t s) {
    if (N > 0) {
        const int RF = (F + 255) / 256, KM = (K + 3) / 4 * 4;
        bool done = false;
        switch (RF) {
            case 1: done = launch_reg<1>(KM, V, ldv, W, ldw, H, ldh, F, K, N, eps, frame_buf, s); break;
            case 2: done = launch_reg<2>(KM, V, ldv, W, ldw, H, ldh, F, K, N, eps, frame_buf, s); break;
            case 3: done = launch_reg<3>(KM, V, ldv, W, ldw, H, ldh, F, K, N, eps, frame_buf, s); break;
            case 4: done = launch_reg<4>(KM, V, ldv, W, ldw, H, ldh, F, K, N, eps, frame_buf, s); break;
            default: break;
        }
        if (!done)
            objective_frames<<<N, 256, 0, s>>>(V, ldv, W, ldw, H, ldh, F, K, eps, frame_buf);
    }
    objective_total<<<1, 256, 0, s>>>(N, frame_buf, d_out);
    return hipGetLastError();
}

}  // namespace isnmf

extern "C" int isnmf_objective_noalloc(const float *V, int ldv, const float *W, int ldw,
                                       const float *H, int ldh, int F, int K, int N, double eps,
                                       double *d_out, void *stream) {
    using namespace isnmf;
    if (!V || !W || !H || !d_out || F < 1 || K < 1 || N < 0 || ldv < F || ldw < F || ldh < K ||
        !(eps >= 0.0))
        return ISNMF_EINVAL;
    if (N > ISNMF_OBJECTIVE_NOALLOC_MAX_FRAMES) return ISNMF_EINVAL;
    double *buf = nullptr;
    if (scratch_ptr(&buf) != hipSuccess) return ISNMF_EDEVICE;
    // every partial the total reads is written by the same call first
    return launch_objective(V, ldv, W, ldw, H, ldh, F, K, N, eps, buf, d_out,
                            (hipStream_t)stream) == hipSuccess
               ? ISNMF_OK
               : ISNMF_EDEVICE;
}
