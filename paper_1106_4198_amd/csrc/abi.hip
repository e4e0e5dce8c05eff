// C ABI of the library (declared in include/isnmf.h): argument checks,
// workspace carving and the kernel sequence of each call.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "common.h"

using namespace isnmf;

thread_local LaunchTiming isnmf::g_launch_timing;

struct isnmf_online {
    OnlineDev d;
    isnmf_params p;
    long long t;
    hipStream_t last;
    int kernel_used;
    FitClass cls;   // fused fit variant (tuned or default)
    // per-launch timing of the fit kernel (isnmf_online_set_timing)
    bool timing = false;
    std::vector<hipEvent_t> ev0, ev1;
    size_t timed = 0;
};

namespace {

int elem_size(const isnmf_params &p) { return p.precision == ISNMF_FP64 ? 8 : 4; }

// Product precision of the fused kernels: 0 FP32, 1 BF16, 2 FP16.
int prec_code(const isnmf_params &p) {
    return p.precision == ISNMF_BF16 ? 1 : p.precision == ISNMF_FP16 ? 2 : 0;
}

bool params_ok(const isnmf_params &p) {
    if (!(p.eps >= 0.0) || !isfinite(p.eps)) return false;
    if (p.inner_iters < 0) return false;
    if (!(p.rho >= 0.0 && p.rho <= 1.0)) return false;
    if (p.h_init != ISNMF_H_ONES && p.h_init != ISNMF_H_WARM) return false;
    if (p.precision < ISNMF_FP32 || p.precision > ISNMF_FP64) return false;
    if (p.kernel < ISNMF_KERNEL_AUTO || p.kernel > ISNMF_KERNEL_FUSED) return false;
    if (!(p.psi_lambda >= 0.0) || !isfinite(p.psi_lambda)) return false;
    if (!(p.psi_a > 0.0) || !isfinite(p.psi_a)) return false;
    return true;
}

isnmf_params resolve(const isnmf_params *p) {
    isnmf_params q;
    isnmf_params_default(&q);
    if (p) q = *p;
    return q;
}

// Carve the online workspace; with base == nullptr only sizes are computed.
// with_lossel: keep the per-element loss buffer of the plain path.
size_t carve_online(int F, int K, int b_max, const isnmf_params &p, bool with_lossel, char *base,
                    OnlineDev *d) {
    const size_t fk = (size_t)F * K;
    const int FR = round_up(F, CHUNK);
    const int KP = round_up(K, 4);
    const int es = elem_size(p);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *ptr = base ? base + off : nullptr;
        off += align256(bytes);
        return ptr;
    };
    OnlineDev t;
    t.F = F;
    t.K = K;
    t.b_max = b_max;
    t.FR = FR;
    t.KP = KP;
    t.flags = (int *)take(sizeof(int));
    t.counter = (unsigned *)take(sizeof(unsigned));
    t.W64 = (double *)take(fk * 8);
    t.W32 = (float *)take(fk * 4);
    t.W16r = (uint16_t *)take((size_t)F * KP * 2);
    t.W16c = (uint16_t *)take((size_t)K * FR * 2);
    t.w16_kind = prec_code(p);
    t.w16_rows = 1;
    t.wexp = (int)lrint(log2((double)F));
    // register-order copy for the VALU fit variant (FP32 and BF16 shapes it covers)
    const bool wv = (p.precision == ISNMF_FP32 || p.precision == ISNMF_BF16) && valu_class(F, K).ok;
    t.Wv = wv ? (float *)take(wv_floats(F, K) * 4) : nullptr;
    t.wv_ck = (K + 7) / 8;
    t.wv_live = 1;
    t.A = (double *)take(fk * 8);
    t.B = (double *)take(fk * 8);
    t.Wn = (double *)take(fk * 8);
    t.dwpart = (double *)take((size_t)K * 8);
    t.sc = (double *)take((size_t)K * 8);
    t.lossf = (double *)take((size_t)b_max * 8);
    t.R1 = take((size_t)b_max * FR * es);
    t.R2 = take((size_t)b_max * FR * es);
    t.Hi = take((size_t)b_max * KP * es);
    t.psi_lambda = p.psi_lambda;
    t.psi_a = p.psi_a;
    t.hsum = p.psi_lambda > 0.0 ? take((size_t)b_max * es) : nullptr;
    t.lossel = with_lossel ? (double *)take((size_t)b_max * FR * 8) : nullptr;
    const size_t pb = fold_partial_bytes(F, K, b_max);
    t.part = pb ? (float *)take(pb) : nullptr;
    const bool warm = p.h_init == ISNMF_H_WARM;   // gather buffers of isnmf_online_passes
    t.Vg = warm ? (float *)take((size_t)b_max * F * 4) : nullptr;
    t.Hg = warm ? (float *)take((size_t)b_max * K * 8) : nullptr;
    if (d) *d = t;
    return off;
}

bool penalized(const isnmf_params &p) { return p.psi_lambda > 0.0; }

// With the penalty on H the fused fit is the VALU variant (FP32 only).
int use_fused(const isnmf_params &p, int F, int K) {
    if (p.precision == ISNMF_FP64) return 0;
    if (p.kernel == ISNMF_KERNEL_PLAIN) return 0;
    if (penalized(p)) return p.precision == ISNMF_FP32 && valu_class(F, K).ok ? 1 : 0;
    return fused_supported(F, K, prec_code(p)) ? 1 : 0;
}

// Zero the 16-bit and register-order copies once (their padding is never written),
// then write W into every copy.
hipError_t init_w(const OnlineDev &d, const float *W, int ldw, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (d.w16_kind) {
        e = hipMemsetAsync(d.W16r, 0, (size_t)d.F * d.KP * 2, s);
        if (e == hipSuccess) e = hipMemsetAsync(d.W16c, 0, (size_t)d.K * d.FR * 2, s);
    }
    if (d.Wv && e == hipSuccess) e = hipMemsetAsync(d.Wv, 0, wv_floats(d.F, d.K) * 4, s);
    if (e == hipSuccess) e = launch_set_w(d, W, ldw, nullptr, s);
    return e;
}

// 16-bit product forms exist only as fused kernels.
bool is16(const isnmf_params &p) { return p.precision == ISNMF_BF16 || p.precision == ISNMF_FP16; }

int run_fit(isnmf_online *h, const float *V, int ldv, int b, int iters, int warm, float *Hb,
            int ldh, hipStream_t s) {
    const isnmf_params &p = h->p;
    const bool timed = h->timing && h->timed < h->ev0.size();
    // the VALU variants take the event pair on their dispatch (one launch)
    const bool fused = p.precision != ISNMF_FP64 && h->kernel_used == ISNMF_KERNEL_FUSED;
    const bool on_dispatch = timed && fused && (h->cls.cpw == 0 || h->cls.cpw == -4);
    if (on_dispatch) g_launch_timing = LaunchTiming{h->ev0[h->timed], h->ev1[h->timed], true};
    if (timed && !on_dispatch && hipEventRecord(h->ev0[h->timed], s) != hipSuccess)
        return ISNMF_EDEVICE;
    hipError_t e;
    if (p.precision == ISNMF_FP64)
        e = launch_plain_fit<double>(h->d, V, ldv, b, iters, p.eps, warm, Hb, ldh, s);
    else if (fused)
        e = launch_fused_fit(h->d, h->cls, V, ldv, b, iters, p.eps, warm, Hb, ldh, prec_code(p), s);
    else
        e = launch_plain_fit<float>(h->d, V, ldv, b, iters, p.eps, warm, Hb, ldh, s);
    const bool attached = on_dispatch && !g_launch_timing.pending;
    g_launch_timing = LaunchTiming{};
    if (e != hipSuccess || (on_dispatch && !attached)) return ISNMF_EDEVICE;
    if (timed) {
        if (!on_dispatch && hipEventRecord(h->ev1[h->timed], s) != hipSuccess) return ISNMF_EDEVICE;
        ++h->timed;
    }
    return ISNMF_OK;
}

// Fold, W = sqrt(A/B) and rescale (the "if t = 0 mod beta" body of Algorithm 1).
int run_update(isnmf_online *h, int b, double rho, int update_w, int normalize, int warm,
               float *Hb, int ldh, double *d_loss_sum, double *d_dw, hipStream_t s) {
    const isnmf_params &p = h->p;
    hipError_t e;
    if (h->kernel_used == ISNMF_KERNEL_FUSED && p.precision != ISNMF_FP64) {
        e = launch_fold_mfma(h->d, b, rho, update_w, h->d.part, d_loss_sum, s);
    } else {
        e = launch_fold(h->d, b, rho, update_w, p.precision == ISNMF_FP64, s);
        if (e == hipSuccess && d_loss_sum) e = launch_loss_total(h->d.lossf, b, d_loss_sum, s);
    }
    if (e == hipSuccess)
        e = launch_rescale(h->d, b, update_w, normalize, warm, Hb, ldh, d_dw, s);
    return e == hipSuccess ? ISNMF_OK : ISNMF_EDEVICE;
}

void free_events(isnmf_online *h) {
    for (auto e : h->ev0) hipEventDestroy(e);
    for (auto e : h->ev1) hipEventDestroy(e);
    h->ev0.clear();
    h->ev1.clear();
    h->timed = 0;
}

}  // namespace

// Accessors used by the batched form (multi.hip).
const OnlineDev *isnmf_handle_dev(const isnmf_online *h) { return &h->d; }
const FitClass *isnmf_handle_class(const isnmf_online *h) { return &h->cls; }
const isnmf_params *isnmf_handle_params(const isnmf_online *h) { return &h->p; }
int isnmf_handle_kernel(const isnmf_online *h) { return h->kernel_used; }
void isnmf_handle_advance(isnmf_online *h, long long frames, hipStream_t s) {
    h->t += frames;
    h->last = s;
}

extern "C" {

void isnmf_params_default(isnmf_params *p) {
    if (!p) return;
    p->eps = 1e-12;
    p->inner_iters = 20;
    p->rho = 1.0;
    p->normalize = 1;
    p->h_init = ISNMF_H_ONES;
    p->precision = ISNMF_FP32;
    p->kernel = ISNMF_KERNEL_AUTO;
    p->update_w = 1;
    p->psi_lambda = 0.0;
    p->psi_a = 1.0;
}

const char *isnmf_strerror(int status) {
    switch (status) {
        case ISNMF_OK: return "ok";
        case ISNMF_EINVAL: return "invalid argument";
        case ISNMF_ENOMEM: return "workspace too small or host allocation failed";
        case ISNMF_EDEVICE: return "HIP runtime error";
        case ISNMF_ENONFINITE: return "non-finite value met on the device";
        case ISNMF_ESTATE: return "handle in an unusable state";
        case ISNMF_EUNSUPPORTED: return "shape or precision not supported";
        default: return "unknown status";
    }
}

int isnmf_forgetting_rho(double r, long long beta, long long n_frames, double *host_rho) {
    if (!host_rho || !(r >= 0.0 && r <= 1.0) || beta < 1 || n_frames < 1) return ISNMF_EINVAL;
    // r^(beta/N): the past is discounted by r per pass over N frames whatever
    // the minibatch size; pow(0, x > 0) = 0 gives the batch reading at r = 0
    *host_rho = pow(r, (double)beta / (double)n_frames);
    return ISNMF_OK;
}

size_t isnmf_online_workspace_size(int F, int K, int b_max, const isnmf_params *pp) {
    if (F < 1 || K < 1 || b_max < 1) return 0;
    const isnmf_params p = resolve(pp);
    return carve_online(F, K, b_max, p, true, nullptr, nullptr);
}

int isnmf_online_init(isnmf_online **out, int F, int K, int b_max, const isnmf_params *pp,
                      const float *W0, int ldw, const double *A0, const double *B0,
                      void *workspace, size_t ws_bytes, void *stream) {
    if (!out) return ISNMF_EINVAL;
    *out = nullptr;
    const isnmf_params p = resolve(pp);
    if (F < 1 || K < 1 || b_max < 1 || !W0 || ldw < F || !workspace || !params_ok(p))
        return ISNMF_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return ISNMF_EINVAL;
    if ((p.kernel == ISNMF_KERNEL_FUSED || is16(p)) && !use_fused(p, F, K))
        return ISNMF_EUNSUPPORTED;
    if (is16(p) && p.kernel == ISNMF_KERNEL_PLAIN) return ISNMF_EUNSUPPORTED;
    if (is16(p) && penalized(p)) return ISNMF_EUNSUPPORTED;
    const size_t need = carve_online(F, K, b_max, p, true, nullptr, nullptr);
    if (ws_bytes < need) return ISNMF_ENOMEM;
    isnmf_online *h = new (std::nothrow) isnmf_online;
    if (!h) return ISNMF_ENOMEM;
    carve_online(F, K, b_max, p, true, (char *)workspace, &h->d);
    h->p = p;
    h->t = 0;
    h->last = (hipStream_t)stream;
    h->kernel_used = use_fused(p, F, K) ? ISNMF_KERNEL_FUSED : ISNMF_KERNEL_PLAIN;
    h->cls = penalized(p) ? valu_class(F, K) : tuned_class(F, K, prec_code(p), b_max);
    h->d.w16_rows = h->cls.cpw != -1;   // the 16-frame tile variant reads only W16c
    hipStream_t s = (hipStream_t)stream;
    const size_t fk8 = sizeof(double) * (size_t)F * K;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemsetAsync(h->d.flags, 0, sizeof(int), s);
    if (e == hipSuccess) e = hipMemsetAsync(h->d.counter, 0, sizeof(unsigned), s);
    if (e == hipSuccess) e = init_w(h->d, W0, ldw, s);
    if (e == hipSuccess)
        e = A0 ? hipMemcpyAsync(h->d.A, A0, fk8, hipMemcpyDeviceToDevice, s)
               : hipMemsetAsync(h->d.A, 0, fk8, s);
    if (e == hipSuccess)
        e = B0 ? hipMemcpyAsync(h->d.B, B0, fk8, hipMemcpyDeviceToDevice, s)
               : hipMemsetAsync(h->d.B, 0, fk8, s);
    if (e == hipSuccess) e = launch_unit_scale(h->d, s);
    if (e != hipSuccess) {
        delete h;
        return ISNMF_EDEVICE;
    }
    // the register-order copy is written above; only the VALU variants read it later
    h->d.wv_live = (h->cls.cpw == 0 && h->cls.nw == 8) || h->cls.cpw == -4;
    *out = h;
    return ISNMF_OK;
}

int isnmf_online_step(isnmf_online *h, const float *Vb, int ldv, int b, float *Hb, int ldh,
                      double *d_loss_sum, double *d_dw, void *stream) {
    if (!h) return ISNMF_EINVAL;
    const isnmf_params &p = h->p;
    const int warm = p.h_init == ISNMF_H_WARM;
    if (!Vb || b < 1 || b > h->d.b_max || ldv < h->d.F) return ISNMF_EINVAL;
    if (warm && !Hb) return ISNMF_EINVAL;
    if (Hb && ldh < h->d.K) return ISNMF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int st = run_fit(h, Vb, ldv, b, p.inner_iters, warm, Hb, ldh, s);
    if (st != ISNMF_OK) return st;
    st = run_update(h, b, p.rho, p.update_w, p.normalize, warm, Hb, ldh, d_loss_sum, d_dw, s);
    if (st != ISNMF_OK) return st;
    h->t += b;
    h->last = s;
    return ISNMF_OK;
}

int isnmf_online_pass(isnmf_online *h, const float *V, int ldv, long long n_frames, int b,
                      float *H, int ldh, double *d_loss_sum, void *stream) {
    if (!h || !V || n_frames < 1 || b < 1 || b > h->d.b_max || ldv < h->d.F) return ISNMF_EINVAL;
    if (h->p.h_init == ISNMF_H_WARM && !H) return ISNMF_EINVAL;
    if (H && ldh < h->d.K) return ISNMF_EINVAL;
    for (long long s0 = 0; s0 < n_frames; s0 += b) {
        const int bb = (int)(n_frames - s0 < b ? n_frames - s0 : b);
        const int st = isnmf_online_step(h, V + (size_t)s0 * ldv, ldv, bb,
                                         H ? H + (size_t)s0 * ldh : nullptr, ldh, d_loss_sum,
                                         nullptr, stream);
        if (st != ISNMF_OK) return st;
    }
    return ISNMF_OK;
}

int isnmf_online_passes(isnmf_online *h, const float *V, int ldv, long long N, const int *perm,
                        int passes, int b, float *H, int ldh, double *d_loss_sum, void *stream) {
    if (!h || !V || !perm || !H || N < 1 || passes < 1 || b < 1 || b > h->d.b_max) return ISNMF_EINVAL;
    if (ldv < h->d.F || ldh < h->d.K || h->p.h_init != ISNMF_H_WARM || !h->d.Vg || !h->d.Hg)
        return ISNMF_EINVAL;
    const OnlineDev &d = h->d;
    hipStream_t s = (hipStream_t)stream;
    // Minibatch m runs on Hg buffer m % 2; the launch that gathers minibatch m
    // also writes minibatch m-1 back when both lie in one pass (a permutation
    // keeps their frames disjoint).  Across a pass boundary they may share
    // frames, so the write-back goes first, on its own.
    RowSwap a = {};
    a.V = V;
    a.H = H;
    a.ldv = ldv;
    a.ldh = ldh;
    a.N = N;
    a.F = d.F;
    a.K = d.K;
    a.Vg = d.Vg;
    a.flags = d.flags;
    const size_t hsz = (size_t)d.b_max * d.K;
    int buf = 0;
    for (int p = 0; p < passes; ++p) {
        for (long long s0 = 0; s0 < N; s0 += b) {
            const int bb = (int)(N - s0 < b ? N - s0 : b);
            if (s0 == 0 && a.n_out > 0) {
                RowSwap w = a;
                w.n_in = 0;
                if (launch_row_swap(w, s) != hipSuccess) return ISNMF_EDEVICE;
                a.n_out = 0;
            }
            a.in_idx = perm + (size_t)p * N + s0;
            a.n_in = bb;
            a.Hg_in = d.Hg + buf * hsz;
            if (launch_row_swap(a, s) != hipSuccess) return ISNMF_EDEVICE;
            const int st = isnmf_online_step(h, d.Vg, d.F, bb, a.Hg_in, d.K, d_loss_sum, nullptr, stream);
            if (st != ISNMF_OK) return st;
            a.out_idx = a.in_idx;
            a.n_out = bb;
            a.Hg_out = a.Hg_in;
            buf ^= 1;
        }
    }
    a.n_in = 0;
    return launch_row_swap(a, s) == hipSuccess ? ISNMF_OK : ISNMF_EDEVICE;
}

int isnmf_online_fit(isnmf_online *h, const float *Vb, int ldv, int b, float *Hb, int ldh,
                     double *d_loss_sum, void *stream) {
    if (!h) return ISNMF_EINVAL;
    const int warm = h->p.h_init == ISNMF_H_WARM;
    if (!Vb || b < 1 || b > h->d.b_max || ldv < h->d.F) return ISNMF_EINVAL;
    if (warm && !Hb) return ISNMF_EINVAL;
    if (Hb && ldh < h->d.K) return ISNMF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int st = run_fit(h, Vb, ldv, b, h->p.inner_iters, warm, Hb, ldh, s);
    if (st != ISNMF_OK) return st;
    if (d_loss_sum && launch_loss_total(h->d.lossf, b, d_loss_sum, s) != hipSuccess)
        return ISNMF_EDEVICE;
    h->last = s;
    return ISNMF_OK;
}

int isnmf_online_set_timing(isnmf_online *h, int enable, int capacity) {
    if (!h || (enable && capacity < 1)) return ISNMF_EINVAL;
    if (!enable) {
        h->timing = false;
        return ISNMF_OK;
    }
    if (hipStreamSynchronize(h->last) != hipSuccess) return ISNMF_EDEVICE;
    free_events(h);
    try {
        h->ev0.resize(capacity);
        h->ev1.resize(capacity);
    } catch (...) {
        h->ev0.clear();
        h->ev1.clear();
        return ISNMF_ENOMEM;
    }
    for (int i = 0; i < capacity; ++i) {
        if (hipEventCreate(&h->ev0[i]) != hipSuccess || hipEventCreate(&h->ev1[i]) != hipSuccess) {
            h->ev0.resize(i);
            h->ev1.resize(i);
            free_events(h);
            return ISNMF_EDEVICE;
        }
    }
    h->timed = 0;
    h->timing = true;
    return ISNMF_OK;
}

int isnmf_online_timing(isnmf_online *h, long long *host_launches, double *host_total_ms) {
    if (!h) return ISNMF_EINVAL;
    if (hipStreamSynchronize(h->last) != hipSuccess) return ISNMF_EDEVICE;
    double tot = 0.0;
    for (size_t i = 0; i < h->timed; ++i) {
        if (hipEventSynchronize(h->ev1[i]) != hipSuccess) return ISNMF_EDEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev0[i], h->ev1[i]) != hipSuccess) return ISNMF_EDEVICE;
        tot += ms;
    }
    if (host_launches) *host_launches = (long long)h->timed;
    if (host_total_ms) *host_total_ms = tot;
    h->timed = 0;
    return ISNMF_OK;
}

int isnmf_online_get(const isnmf_online *h, float *W, double *A, double *B, long long *host_t,
                     void *stream) {
    if (!h) return ISNMF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (W && e == hipSuccess) e = launch_get_w(h->d, W, s);
    if (e == hipSuccess) e = launch_get_ab(h->d, A, B, s);
    if (host_t) *host_t = h->t;
    return e == hipSuccess ? ISNMF_OK : ISNMF_EDEVICE;
}

int isnmf_online_get_w64(const isnmf_online *h, double *W, void *stream) {
    if (!h || !W) return ISNMF_EINVAL;
    const size_t fk = (size_t)h->d.F * h->d.K;
    return hipMemcpyAsync(W, h->d.W64, fk * 8, hipMemcpyDeviceToDevice, (hipStream_t)stream) ==
                   hipSuccess
               ? ISNMF_OK
               : ISNMF_EDEVICE;
}

int isnmf_online_set(isnmf_online *h, const float *W, const double *A, const double *B,
                     long long t, void *stream) {
    if (!h || t < 0) return ISNMF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const size_t fk = (size_t)h->d.F * h->d.K;
    hipError_t e = hipSuccess;
    if (W) e = launch_set_w(h->d, W, h->d.F, nullptr, s);
    if ((A || B) && e == hipSuccess) e = launch_settle_ab(h->d, s);   // the one not given keeps its value
    if (A && e == hipSuccess) e = hipMemcpyAsync(h->d.A, A, fk * 8, hipMemcpyDeviceToDevice, s);
    if (B && e == hipSuccess) e = hipMemcpyAsync(h->d.B, B, fk * 8, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return ISNMF_EDEVICE;
    h->t = t;
    h->last = s;
    return ISNMF_OK;
}

int isnmf_online_set_w64(isnmf_online *h, const double *W, void *stream) {
    if (!h || !W) return ISNMF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (launch_set_w(h->d, nullptr, h->d.F, W, s) != hipSuccess) return ISNMF_EDEVICE;
    h->last = s;
    return ISNMF_OK;
}

int isnmf_online_status(isnmf_online *h, int *host_flags) {
    if (!h) return ISNMF_EINVAL;
    if (hipStreamSynchronize(h->last) != hipSuccess) return ISNMF_EDEVICE;
    int f = 0;
    if (hipMemcpy(&f, h->d.flags, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return ISNMF_EDEVICE;
    if (hipMemset(h->d.flags, 0, sizeof(int)) != hipSuccess) return ISNMF_EDEVICE;
    if (host_flags) *host_flags = f;
    return (f & FLAG_NONFINITE_V) ? ISNMF_ENONFINITE : ISNMF_OK;
}

int isnmf_online_info(const isnmf_online *h, int *F, int *K, int *b_max, int *kernel_used) {
    if (!h) return ISNMF_EINVAL;
    if (F) *F = h->d.F;
    if (K) *K = h->d.K;
    if (b_max) *b_max = h->d.b_max;
    if (kernel_used) *kernel_used = h->kernel_used;
    return ISNMF_OK;
}

int isnmf_online_destroy(isnmf_online *h) {
    if (!h) return ISNMF_EINVAL;
    hipError_t e = hipStreamSynchronize(h->last);
    free_events(h);
    delete h;
    return e == hipSuccess ? ISNMF_OK : ISNMF_EDEVICE;
}

// ------------------------------------------------------------------- batch

size_t isnmf_batch_workspace_size(int F, int K, int N, const isnmf_params *pp) {
    if (F < 1 || K < 1 || N < 1) return 0;
    isnmf_params p = resolve(pp);
    // the online layout with b_max = N, without the per-element loss buffer
    return carve_online(F, K, N, p, false, nullptr, nullptr);
}

int isnmf_batch_mu(const float *V, int ldv, int F, int N, float *W, int ldw, float *H, int ldh,
                   int K, int cycles, const isnmf_params *pp, double *d_obj_trace,
                   void *workspace, size_t ws_bytes, void *stream) {
    isnmf_params p = resolve(pp);
    if (!V || !W || !H || !workspace || F < 1 || K < 1 || N < 1 || cycles < 0 || ldv < F ||
        ldw < F || ldh < K || !params_ok(p))
        return ISNMF_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return ISNMF_EINVAL;
    if (is16(p) && (p.kernel == ISNMF_KERNEL_PLAIN || !use_fused(p, F, K)))
        return ISNMF_EUNSUPPORTED;
    if (penalized(p)) return ISNMF_EUNSUPPORTED;
    if (ws_bytes < isnmf_batch_workspace_size(F, K, N, &p)) return ISNMF_ENOMEM;
    // an online handle over the whole set: beta = N, rho = 0, warm restarts,
    // one h update per cycle (section 2.3, overview).
    isnmf_online h;
    carve_online(F, K, N, p, false, (char *)workspace, &h.d);
    h.p = p;
    h.p.rho = 0.0;
    h.p.h_init = ISNMF_H_WARM;
    h.p.update_w = 1;
    h.t = 0;
    h.kernel_used = use_fused(p, F, K) ? ISNMF_KERNEL_FUSED : ISNMF_KERNEL_PLAIN;
    h.cls = tuned_class(F, K, prec_code(p), N);   // as an online handle of N frames
    hipStream_t s = (hipStream_t)stream;
    if (hipMemsetAsync(h.d.flags, 0, sizeof(int), s) != hipSuccess) return ISNMF_EDEVICE;
    if (hipMemsetAsync(h.d.counter, 0, sizeof(unsigned), s) != hipSuccess) return ISNMF_EDEVICE;
    if (init_w(h.d, W, ldw, s) != hipSuccess) return ISNMF_EDEVICE;
    // A(0) = B(0) = 0: rho = 0 multiplies them, and 0 times a non-finite
    // leftover of the workspace would not be 0
    const size_t fk8 = sizeof(double) * (size_t)F * K;
    if (hipMemsetAsync(h.d.A, 0, fk8, s) != hipSuccess ||
        hipMemsetAsync(h.d.B, 0, fk8, s) != hipSuccess || launch_unit_scale(h.d, s) != hipSuccess)
        return ISNMF_EDEVICE;
    for (int c = 0; c < cycles; ++c) {
        int st = run_fit(&h, V, ldv, N, 1, 1, H, ldh, s);
        if (st != ISNMF_OK) return st;
        st = run_update(&h, N, 0.0, 1, p.normalize, 1, H, ldh, nullptr, nullptr, s);
        if (st != ISNMF_OK) return st;
        if (d_obj_trace &&
            launch_objective(V, ldv, h.d.W32, F, H, ldh, F, K, N, p.eps, h.d.lossf,
                             d_obj_trace + c, s) != hipSuccess)
            return ISNMF_EDEVICE;
    }
    if (hipMemcpy2DAsync(W, sizeof(float) * ldw, h.d.W32, sizeof(float) * F, sizeof(float) * F, K,
                         hipMemcpyDeviceToDevice, s) != hipSuccess)
        return ISNMF_EDEVICE;
    return ISNMF_OK;
}

size_t isnmf_objective_workspace_size(int F, int K, int N) {
    if (F < 1 || K < 1 || N < 0) return 0;
    return align256((size_t)(N > 0 ? N : 1) * 8);
}

int isnmf_objective(const float *V, int ldv, const float *W, int ldw, const float *H, int ldh,
                    int F, int K, int N, double eps, double *d_out, void *workspace,
                    size_t ws_bytes, void *stream) {
    if (!V || !W || !H || !d_out || !workspace || F < 1 || K < 1 || N < 0 || ldv < F ||
        ldw < F || ldh < K || !(eps >= 0.0))
        return ISNMF_EINVAL;
    if (ws_bytes < isnmf_objective_workspace_size(F, K, N)) return ISNMF_ENOMEM;
    return launch_objective(V, ldv, W, ldw, H, ldh, F, K, N, eps, (double *)workspace, d_out,
                            (hipStream_t)stream) == hipSuccess
               ? ISNMF_OK
               : ISNMF_EDEVICE;
}

}  // extern "C"
