// Host side of the fused fit: the kernel variant for a shape and the
// single-stream launch.  The kernel body is in fit_body.h; its instantiations
// are in fit_f32.hip, fit_bf16.hip and fit_f16.hip.
//
// Variants (register budget of one CU: 4 SIMDs x 512 x 64 x 4 B):
//   chunks <= 8 (F <= 516):   NW = 1, 2, 4 or 8 waves, one 64-row chunk each,
//                             K <= 64 (FP32) or K <= 128 (16-bit), W in registers
//   chunks 9..16, 16-bit:     K <= 64: 8 waves x 2 chunks, W in registers;
//                             K > 64:  16 waves x 1 chunk, W read from its
//                             16-bit copies in L2 (too large for registers)
//   FP32, F <= 1088, K <= 64: the VALU variant (one frame per workgroup) where
//                             no MFMA tile fits, and as a tuning candidate
//                             elsewhere
//   BF16, F <= 640, K <= 64:  the 16-frame tile variant, a tuning candidate
//                             (throughput over many frames)
//   BF16, F <= 1088, K <= 64: the VALU variant on bf16 dot products, the
//                             default where no MFMA tile fits and a tuning
//                             candidate elsewhere (latency of one minibatch)
//   FP32, K <= 64:            the FP32 16-frame tile variant (16x16x4 FP32
//                             MFMA, W in LDS), a tuning candidate (throughput)
#include <math.h>

#include "common.h"

namespace isnmf {

namespace {
int kclass(int K, int prec) {
    static const int ks[] = {8, 16, 24, 32, 40, 52, 64, 80, 96, 112, 128};
    for (int k : ks) {
        if (k > 64 && prec == 0) return 0;
        if (K <= k) return k;
    }
    return 0;
}
}  // namespace

FitClass fit_class(int F, int K, int prec) {
    FitClass c = {};
    if (F < 1 || K < 1) return c;
    c.main_chunks = F / CHUNK;
    c.tail = F % CHUNK;
    if (c.tail > TAIL_MAX) {
        c.main_chunks += 1;   // last chunk partially valid (masked)
        c.tail = 0;
    }
    c.kmax = kclass(K, prec);
    if (!c.kmax) return c;
    const int nch = c.main_chunks < 1 ? 1 : c.main_chunks;
    if (nch <= 8) {
        c.cpw = 1;
        c.nw = nch <= 1 ? 1 : nch <= 2 ? 2 : nch <= 4 ? 4 : 8;
        c.wg = 0;
        c.ok = 1;
    } else if (nch <= 16 && prec != 0) {
        if (c.kmax <= 64) {
            c.nw = 8;
            c.cpw = 2;
            c.wg = 0;
        } else {
            c.nw = 16;
            c.cpw = 1;
            c.wg = 1;
        }
        c.ok = 1;
    }
    // FP32 and BF16 beyond the register-resident MFMA tiles: one frame per
    // workgroup (FP32 past the 8-wave form's rows: its 16-wave form)
    if (!c.ok && prec == 0) return valu_class(F, K).ok ? valu_class(F, K) : valu16_class(F, K);
    if (!c.ok && prec == 1) return vbf_class(F, K);
    return c;
}

bool fused_supported(int F, int K, int prec) { return fit_class(F, K, prec).ok != 0; }

int fit_candidates(int F, int K, int prec, FitClass *out, int max_out) {
    const FitClass d = fit_class(F, K, prec);
    if (!d.ok) return 0;
    int n = 0;
    auto add = [&](FitClass c) {
        if (n < max_out) out[n++] = c;
    };
    add(d);
    if (prec == 0 && d.cpw != 0) {   // the VALU variant, when the default is an MFMA tile
        const FitClass v = valu_class(F, K);
        if (v.ok) add(v);
    }
    if (prec == 0) {                 // the FP32 16-frame tile variant (throughput)
        const FitClass t = t32_class(F, K);
        if (t.ok) add(t);
    }
    if (prec == 1 && d.cpw != -4) {   // the VALU variant on bf16 dot products (latency)
        const FitClass v = vbf_class(F, K);
        if (v.ok) add(v);
    }
    if (prec == 1) {                 // the 16-frame tile variants (BF16)
        const FitClass t = tile_class(F, K);
        if (t.ok) add(t);
        const FitClass st = stile_class(F, K);
        if (st.ok) add(st);
    }
    if (prec != 0 && d.kmax <= 64) {
        const int nch = d.main_chunks < 1 ? 1 : d.main_chunks;
        if (nch > 4 && nch <= 8) {   // 4 waves x 2 chunks instead of 8 x 1
            FitClass c = d;
            c.nw = 4;
            c.cpw = 2;
            add(c);
        }
        if (nch > 8 && nch <= 16) {  // 16 waves x 1 chunk, W from its 16-bit copies
            FitClass c = d;
            c.nw = 16;
            c.cpw = 1;
            c.wg = 1;
            add(c);
        }
    }
    return n;
}

FitDesc make_fit_desc(const OnlineDev &d, const float *V, int ldv, int b, int iters, double eps,
                      int warm, float *Hb, int ldh) {
    const FitClass c = fit_class(d.F, d.K, d.w16_kind);
    FitDesc a;
    a.F = d.F;
    a.K = d.K;
    a.b = b;
    a.ldv = ldv;
    a.ldh = ldh;
    a.iters = iters;
    a.warm = warm;
    a.main_chunks = c.main_chunks;
    a.tail = c.tail;
    a.FR = d.FR;
    a.KP = d.KP;
    a.eps = float(eps);
    a.psi_lambda = float(d.psi_lambda);
    a.psi_a = float(d.psi_a);
    a.epsd = eps;
    a.wscale = ldexpf(1.f, d.wexp);
    a.hscale = ldexpf(1.f, -d.wexp);
    a.V = V;
    a.W = d.W32;
    a.W16r = d.W16r;
    a.W16c = d.W16c;
    a.Wv = d.Wv;
    a.Hb = Hb;
    a.Hi = (float *)d.Hi;
    a.R1 = (float *)d.R1;
    a.R2 = (float *)d.R2;
    a.lossf = d.lossf;
    a.flags = d.flags;
    a.fold = nullptr;
    a.rs = nullptr;
    return a;
}

hipError_t launch_fused_fit(const OnlineDev &d, const FitClass &c, const float *V, int ldv, int b,
                            int iters, double eps, int warm, float *Hb, int ldh, int prec,
                            hipStream_t s) {
    if (!c.ok) return hipErrorNotSupported;
    const FitDesc a = make_fit_desc(d, V, ldv, b, iters, eps, warm, Hb, ldh);
    if (c.cpw == 0) return prec == 0 ? launch_fit_valu(a, c, b, s) : hipErrorNotSupported;
    if (c.cpw == -4) return prec == 1 ? launch_fit_valu(a, c, b, s) : hipErrorNotSupported;
    if (d.psi_lambda > 0.0) return hipErrorNotSupported;   // penalty: VALU variant only
    if (c.cpw == -1) return prec == 1 ? launch_fit_tile(a, c, b, s) : hipErrorNotSupported;
    if (c.cpw == -2) return prec == 1 ? launch_fit_stile(a, c, b, s) : hipErrorNotSupported;
    if (c.cpw == -3) return prec == 0 ? launch_fit_t32(a, c, b, s) : hipErrorNotSupported;
    const int grid = (b + NF - 1) / NF;
    if (prec == 1) return launch_fit_single_p<1>(a, c, grid, s);
    if (prec == 2) return launch_fit_single_p<2>(a, c, grid, s);
    return launch_fit_single_p<0>(a, c, grid, s);
}

}  // namespace isnmf
