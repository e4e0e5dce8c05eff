// Fold of a minibatch into the running statistics on gfx950 MFMA (FP32
// products, FP64 statistics).  Eq. (4) summed over the minibatch with the
// past scaled by rho (section 2.3):
//   dA' = R2 H^T,  dB = R1 H^T          (F x K, reduction over the b frames)
//   A <- rho A + dA' o W^2,  B <- rho B + dB,  Wn = sqrt(A / B)
// with R2 = (eps + v)/x^2 and R1 = 1/x of the final inner-fit model.
//
// Mapping: one block of 4 waves per 16 x 16 tile of (f, k),
// v_mfma_f32_16x16x4f32 with the frames as the contraction dimension (4 per
// instruction, groups of 4 frames dealt round-robin to the waves):
//   A operand lane l = R2[frame n0 + l/16][f0 + l%16]
//   B operand lane l = H[frame n0 + l/16][k0 + l%16]
//   result lane l, register r = dA'[f0 + 4(l/16) + r][k0 + l%16]
// Minibatches longer than SLICE frames are cut into slices whose FP32 partial
// tiles are summed in slice order (FP64) by a second kernel.
#include "common.h"
#include "fold_body.h"

namespace isnmf {
namespace {

// Blocks reach the 8 XCDs round-robin by launch index.  Work item g = (tile,
// slice) in slice-major order is given to blocks so that each XCD takes one
// contiguous range of items: the tiles of a slice, which read the same H and
// r1, r2 rows, meet in one L2.  Every item is the same computation whichever
// block runs it.
__global__ __launch_bounds__(256) void fold_mfma_kernel(FoldArgs a) {
    const unsigned T = gridDim.x * gridDim.y;
    const unsigned L = blockIdx.y * gridDim.x + blockIdx.x;
    const unsigned x = L % 8, pos = L / 8;
    const unsigned g = x * (T / 8) + (x < T % 8 ? x : T % 8) + pos;
    fold_tile16_body(a, (int)(g % gridDim.x), (int)(g / gridDim.x), gridDim.y);
}


// Multi-slice: sum the slice partials in slice order, then the epilogue.
__global__ void fold_reduce_kernel(FoldArgs a, int slices) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t fk = (size_t)a.F * a.K;
    if (e >= (long)fk) return;
    double sa = 0.0, sb = 0.0;
    int s = 0;
    // eight slices' loads issued before their adds, which stay in slice order
    for (; s + 8 <= slices; s += 8) {
        float pa[8], pb[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            pa[j] = a.part[(size_t)(s + j) * 2 * fk + e];
            pb[j] = a.part[(size_t)(s + j) * 2 * fk + fk + e];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            sa += double(pa[j]);
            sb += double(pb[j]);
        }
    }
    for (; s < slices; ++s) {
        sa += double(a.part[(size_t)s * 2 * fk + e]);
        sb += double(a.part[(size_t)s * 2 * fk + fk + e]);
    }
    const int k = (int)(e / a.F);
    epilogue(a, (int)(e % a.F), k, sa, sb, a.W64[e], a.A[e] / a.sc[k], a.B[e] * a.sc[k]);
}

}  // namespace

size_t fold_partial_bytes(int F, int K, int b) {
    const int slices = (b + SLICE - 1) / SLICE;
    return slices > 1 ? (size_t)slices * 2 * F * K * sizeof(float) : 0;
}

hipError_t launch_fold_mfma(const OnlineDev &d, int b, double rho, int update_w, float *part,
                            double *d_loss_sum, hipStream_t s) {
    FoldArgs a = fold_args(d, b, rho, update_w, part, d_loss_sum);
    const int slices = (b + SLICE - 1) / SLICE;
    if (slices > 1 && !part) return hipErrorInvalidValue;
    fold_mfma_kernel<<<dim3(fold_tiles16(d), slices), 256, 0, s>>>(a);
    if (slices > 1) {
        a.d_loss_sum = nullptr;
        const long fk = (long)d.F * d.K;
        fold_reduce_kernel<<<(int)((fk + 255) / 256), 256, 0, s>>>(a, slices);
    }
    return hipGetLastError();
}

}  // namespace isnmf
