// Internal declarations of the gfx950 online IS-NMF library (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "isnmf.h"

namespace isnmf {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Sticky device flag bits (isnmf_online_status).
enum : int {
    FLAG_NONFINITE_V = 1,
    FLAG_GUARD_H = 2,
    FLAG_GUARD_W = 4,
    FLAG_BAD_INDEX = 8,
};

// Rows per MFMA chunk of the fused fit: 16 blocks x 4 rows of v_mfma_f32_4x4x1_16b.
constexpr int CHUNK = 64;
// Frames per workgroup of the fused fit (the 4 columns of each 4x4 block).
constexpr int NF = 4;
// Rows past the last full chunk that the fused fit handles on the VALU
// (F = 64 m + 1 for the STFT sizes 129, 257, 513, 1025).
constexpr int TAIL_MAX = 2;

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Register order of W for the VALU fit (512 threads, thread t = 8p + q holds
// W[p + 64r][q + 8c], r < ceil(F/64), c < ck): element e = r ck + c of thread t
// sits at float index 4 (512 (e / 4) + t) + e mod 4, so each thread reads its
// elements as float4 and a wave's read is one contiguous 1 KiB block.
// Entries of rows >= F or columns >= K are zero.
__host__ __device__ inline size_t wv_index(int f, int k, int ck) {
    const int e = (f >> 6) * ck + (k >> 3);
    const int t = ((f & 63) << 3) | (k & 7);
    return ((size_t)((e >> 2) * 512 + t) << 2) | (size_t)(e & 3);
}
inline size_t wv_floats(int F, int K) {
    const int e = ((F + 63) / 64) * ((K + 7) / 8);
    return (size_t)512 * 4 * ((e + 3) / 4);
}

// Device-side state of one online stream (views into the caller's workspace).
struct OnlineDev {
    int F, K, b_max;
    int FR;              // padded row stride of the R buffers (multiple of 4)
    int KP;              // padded row stride of the internal H buffer
    double *W64;         // F x K, ld F: master W (FP64)
    float *W32;          // F x K, ld F: working copy (FP32)
    uint16_t *W16r;      // F x KP row-major: W * 2^wexp in BF16/FP16 (precision forms)
    uint16_t *W16c;      // K x FR (column k at k*FR): the same values, column-major
    int w16_kind;        // 0 none, 1 BF16, 2 FP16
    int w16_rows;        // 1: W16r is kept current (0 when the fit variant reads only W16c)
    int wexp;            // s = round(log2 F): 16-bit copies hold W * 2^s
    float *Wv;           // W in the register order of the VALU fit (see wv_index) or null
    int wv_ck;           // ceil(K / 8): components per thread of that order
    int wv_live;         // 1: Wv is kept current (0 when the handle's fit variant does
                         // not read it; it then holds W(0) for the autotuner's trials)
    double *A, *B;       // F x K, ld F, stored before the last column rescale:
                         // the statistics are A[:,k] / sc[k] and B[:,k] * sc[k]
    double *sc;          // K: column scale of A and B not yet applied (1 = none)
    double *Wn;          // F x K: sqrt(A/B) before rescaling
    double *dwpart;      // K: per-column sum of squared change of W
    double *lossf;       // b_max: per-frame loss of the current minibatch
    void *R1, *R2;       // b_max x FR (float, or double in FP64 mode): 1/x and (eps+v)/x^2
    void *Hi;            // b_max x KP (float or double): fitted h of the minibatch
    void *hsum;          // plain path with the penalty on H: b_max column sums of H
                         // (float, or double in FP64 mode), else null
    double psi_lambda;   // penalty on H: psi(s) = psi_lambda log(psi_a + s) of each
    double psi_a;        // column sum (psi_lambda = 0: none)
    double *lossel;      // plain path: b_max x FR per-element loss terms
    float *part;         // fold slice partials (b_max > 512) or null
    float *Vg, *Hg;      // warm multi-pass: gathered minibatch frames (b_max x F) and h
                         // (two buffers of b_max x K, alternating between minibatches)
    int *flags;          // sticky flags
    unsigned *counter;   // spare device word (zeroed at init)
};

// Start/stop events for the next single-stream fit launch, set by a handle's
// timing hook.  A launcher that attaches them to its dispatch (the VALU
// variants, through hipExtLaunchKernel) clears `pending`.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
    bool pending = false;
};
extern thread_local LaunchTiming g_launch_timing;

struct FoldArgs;      // fold_body.h
struct RescaleArgs;   // state_body.h

// One stream's fit problem for the fused kernels (by value for a single
// stream, an array in device memory for the batched form).
struct FitDesc {
    int F, K, b, ldv, ldh, iters, warm;
    int main_chunks;   // chunks of 64 rows on MFMA (the last may be partial)
    int tail;          // rows after them on the VALU (<= TAIL_MAX)
    int FR, KP;
    float eps, wscale, hscale;
    float psi_lambda, psi_a;   // penalty on H (VALU variant only; 0 elsewhere)
    double epsd;
    const float *V;            // frame 0 of the minibatch
    const float *W;            // F x K, ld F (FP32 working copy)
    const uint16_t *W16r;      // F x KP, 16-bit W * wscale
    const uint16_t *W16c;      // K x FR, 16-bit W * wscale
    const float *Wv;           // W in the VALU fit's register order (or null)
    float *Hb;                 // caller's K x b (warm start in / fitted h out) or null
    float *Hi;                 // b x KP internal copy of the fitted h
    float *R1, *R2;            // b x FR
    double *lossf;             // b
    int *flags;
    // The stream's fold (device memory) when the fit launch folds the minibatch
    // itself (the batched form's 16-frame tile streams of at most 128 frames),
    // else null: the fit then writes R1, R2 for a separate fold.
    const FoldArgs *fold;
    // With fold: the stream's column rescale (device memory) when the fit
    // launch also rescales W after its fold (the BF16 16-frame tile variant),
    // else null.
    const RescaleArgs *rs;
};

// One chunk of a served step: session (index in the server's device tables),
// frame count, frames (the session's frame stride ldv).
struct ServeWork {
    int sess;
    int b;
    const float *V;
    int ldv, pad;
};

// Kernel variant of the fused fit for a shape: an MFMA tile variant of
// fit_body.h (cpw >= 1: NW waves x CPW chunks of 64 rows, NF frames per
// workgroup), the VALU variant of fit_valu.h (cpw = 0: one frame per
// workgroup of nw = 8 or 16 waves, rf row sets of 8 nw rows and kmax / 8
// components per thread; cpw = -4 is its BF16 form, 8 waves), the 16-frame tile variant of fit_tile.h (cpw = -1: BF16
// products, nw = 8 waves of 16 frames each, rf = ceil(F / 32) contraction
// steps of 32 rows, kmax = 32 ceil(K / 32)), its streamed form of
// fit_stile.h (cpw = -2), or the FP32 16-frame tile variant of fit_t32.h
// (cpw = -3: nw = 8 waves of 16 frames, rf = ceil(F / 16) row tiles,
// kmax = K).
struct FitClass {
    int ok;
    int nw, cpw, kmax, wg;
    int main_chunks, tail;
    int rf;
};
FitClass fit_class(int F, int K, int prec);
// The VALU variant for (F, K) with FP32 products, or ok = 0.
FitClass valu_class(int F, int K);
// The VALU variant with bf16 products on v_dot2c_f32_bf16 (cpw = -4; the
// same shapes as valu_class), or ok = 0.
FitClass vbf_class(int F, int K);
// The 16-wave form of the FP32 VALU variant for the rows past the 8-wave
// form (cpw = 0, nw = 16, 1088 < F <= 1152, rf = 9, K <= 64; W read from the
// FP32 working copy), or ok = 0.
FitClass valu16_class(int F, int K);
// The 16-frame tile variant for (F, K) with BF16 products, or ok = 0.
FitClass tile_class(int F, int K);
FitClass stile_class(int F, int K);
// The FP32 16-frame tile variant for (F, K), or ok = 0.
FitClass t32_class(int F, int K);
FitDesc make_fit_desc(const OnlineDev &d, const float *V, int ldv, int b, int iters, double eps,
                      int warm, float *Hb, int ldh);

// Single-stream and batched launches of one fit class, per product precision.
template <int PREC>
hipError_t launch_fit_single_p(const FitDesc &a, const FitClass &c, int grid, hipStream_t s);
template <int PREC>
hipError_t launch_fit_multi_p(const FitClass &c, const FitDesc *descs, const int2 *items,
                              int nitems, const long long *cursor, const int *beff, hipStream_t s);

// ---------------------------------------------------------------- launchers

// Plain (unfused) fit of all frames of a minibatch; T = float or double.
// Hb: caller's K x b activations (warm start in, fitted h out) or nullptr.
template <typename T>
hipError_t launch_plain_fit(const OnlineDev &d, const float *V, int ldv, int b, int iters,
                            double eps, int warm, float *Hb, int ldh, hipStream_t s);

// Fused MFMA fit; prec 0 = FP32, 1 = BF16, 2 = FP16 products.  Returns
// hipErrorNotSupported for shapes it does not cover.
hipError_t launch_fused_fit(const OnlineDev &d, const FitClass &c, const float *V, int ldv, int b,
                            int iters, double eps, int warm, float *Hb, int ldh, int prec,
                            hipStream_t s);
bool fused_supported(int F, int K, int prec);
// VALU variant launches (class from valu_class): b frames, or the frames of
// n batched items of NF frames each.
hipError_t launch_fit_valu(const FitDesc &a, const FitClass &c, int b, hipStream_t s);
hipError_t launch_fit_valu_work(const FitClass &c, const FitDesc *tab, const ServeWork *work, int n,
                                int max_b, hipStream_t s);
hipError_t launch_fit_valu_multi(const FitClass &c, const FitDesc *d, const int2 *items, int n,
                                 const long long *cur, const int *beff, hipStream_t s);
// 16-frame tile variant launches: b frames, or n batched items (stream, tile of 16 frames).
hipError_t launch_fit_tile(const FitDesc &a, const FitClass &c, int b, hipStream_t s);
// fold: the launch folds each minibatch itself (every descriptor's fold is set;
// tile_fold_fits(c) holds).
hipError_t launch_fit_tile_multi(const FitClass &c, const FitDesc *d, const int2 *items, int n,
                                 const long long *cur, const int *beff, bool fold, hipStream_t s);
// The 16-frame tile variant of class c can fold in its launch (its LDS holds the
// fold's staging beside the X operands).
bool tile_fold_fits(const FitClass &c);
// ... and over a served step's work list: n chunks, `tiles` tiles of 128 frames each.
hipError_t launch_fit_tile_work(const FitClass &c, const FitDesc *tab, const ServeWork *work, int n,
                                int tiles, hipStream_t s);
// Frames per batched work item of a fit class.
hipError_t launch_fit_stile(const FitDesc &a, const FitClass &c, int b, hipStream_t s);
hipError_t launch_fit_stile_multi(const FitClass &c, const FitDesc *d, const int2 *items, int n,
                                  const long long *cur, const int *beff, hipStream_t s);
hipError_t launch_fit_stile_work(const FitClass &c, const FitDesc *tab, const ServeWork *work, int n,
                                 int tiles, hipStream_t s);
// FP32 16-frame tile variant launches: b frames, n batched items (fold: as
// for launch_fit_tile_multi), or a served work list.
hipError_t launch_fit_t32(const FitDesc &a, const FitClass &c, int b, hipStream_t s);
hipError_t launch_fit_t32_multi(const FitClass &c, const FitDesc *d, const int2 *items, int n,
                                const long long *cur, const int *beff, bool fold, hipStream_t s);
// The FP32 16-frame tile variant of class c can fold in its launch (its LDS holds
// the fold's staging beside W).
bool t32_fold_fits(const FitClass &c);
hipError_t launch_fit_t32_work(const FitClass &c, const FitDesc *tab, const ServeWork *work, int n,
                               int tiles, hipStream_t s);
// Frames per batched item: 128 for the 16-frame tile variants (8 waves of
// 16), NF (the workgroups of one item) for the MFMA tile and VALU variants.
inline int frames_per_item(const FitClass &c) {
    return c.cpw == -1 || c.cpw == -2 || c.cpw == -3 ? 128 : NF;
}
// Every fit variant valid for the shape (the default first); returns the count.
int fit_candidates(int F, int K, int prec, FitClass *out, int max_out);
// The variant the autotuner chose for (F, K, prec, b), or the default.
FitClass tuned_class(int F, int K, int prec, int b);

// Fold the minibatch into A, B and (optionally) form sqrt(A/B).
// Rin/Hin element type: float (is_double = 0) or double (1).
hipError_t launch_fold(const OnlineDev &d, int b, double rho, int update_w, int is_double,
                       hipStream_t s);

// MFMA fold (FP32 R and H).  part: slice partials when b > 512 (see
// fold_partial_bytes), else unused.  Adds the minibatch loss to d_loss_sum.
hipError_t launch_fold_mfma(const OnlineDev &d, int b, double rho, int update_w, float *part,
                            double *d_loss_sum, hipStream_t s);
size_t fold_partial_bytes(int F, int K, int b);

// Column rescale (when update_w), W copies, warm-H compensation; d_dw (if
// not null) receives ||W_new - W_old||_F.
// A, B with the pending column scale applied, into A and B (device F x K, or
// null); settle applies it in place and clears it; unit_scale clears it.
hipError_t launch_get_ab(const OnlineDev &d, double *A, double *B, hipStream_t s);
hipError_t launch_settle_ab(const OnlineDev &d, hipStream_t s);
hipError_t launch_unit_scale(const OnlineDev &d, hipStream_t s);
hipError_t launch_rescale(const OnlineDev &d, int b, int update_w, int normalize, int warm,
                          float *Hb, int ldh, double *d_dw, hipStream_t s);

// *d_loss_sum += sum of lossf[0..b) in index order (one block).
hipError_t launch_loss_total(const double *lossf, int b, double *d_loss_sum, hipStream_t s);

// One launch that moves minibatches between a resident set of N frames (V: F
// floats per frame, stride ldv; H: K floats, stride ldh) and the packed
// buffers of one step: frames in_idx[0..n_in) are gathered into Vg and Hg_in
// (rows of F and K floats), and rows 0..n_out of Hg_out are written back to H
// at out_idx.  An index outside [0, N) gathers zeros and sets FLAG_BAD_INDEX,
// and is skipped on write-back.  The two index sets must be disjoint: a frame
// both read and written in one launch sees either value.
struct RowSwap {
    const float *V;
    float *H;
    long long ldv, ldh, N;
    int F, K;
    const int *in_idx;
    int n_in;
    float *Vg, *Hg_in;
    const int *out_idx;
    int n_out;
    const float *Hg_out;
    int *flags;
};
hipError_t launch_row_swap(const RowSwap &a, hipStream_t s);

// Copy helpers.
hipError_t launch_set_w(const OnlineDev &d, const float *W, int ldw, const double *W64,
                        hipStream_t s);
hipError_t launch_get_w(const OnlineDev &d, float *W, hipStream_t s);

// Objective of eq. (1): per-frame sums into frame_out (double, N entries) then a
// fixed-order total into d_out (scaled by 1/N).
hipError_t launch_objective(const float *V, int ldv, const float *W, int ldw, const float *H,
                            int ldh, int F, int K, int N, double eps, double *frame_buf,
                            double *d_out, hipStream_t s);

}  // namespace isnmf
