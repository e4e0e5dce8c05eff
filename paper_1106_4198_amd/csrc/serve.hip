// Served form: a continuous-batching engine over many online sessions.
//
// Sessions (isnmf_online handles, W/A/B resident on the device) register
// with the server; their kernel descriptors are written once into device
// tables.  Clients submit chunks (frames already on the device).  Each engine
// step takes at most one pending chunk per session (per-session order is
// kept, and consecutive steps of one session are ordered on the stream, so
// each session still follows Algorithm 1 minibatch by minibatch),
// up to max_frames frames in total, and runs one minibatch step for all of
// them: one fit launch per kernel variant in use, then one fold and one
// rescale launch per variant (the variants' chains side by side on up to four
// streams), reading a small work list (session, frames,
// count) that reaches the device through a pinned ring buffer.  Up to
// `inflight` steps are enqueued at once; chunks that arrive meanwhile join
// the next step.  A chunk's latency is arrival to the end of its step.
//
// Each chunk's arithmetic is that of isnmf_online_step on its session with
// b = chunk length (same kernel bodies and variant, fixed-order sums), so a
// session's result does not depend on what else shares the step.
//
// Admission: a session is resident (its descriptors in a row of the device
// tables, its footprint charged to the HBM budget) or waiting in a FIFO.
// The head of the FIFO is admitted as soon as a table row is free and its
// footprint fits what the resident sessions leave of the budget; closing a
// session returns its row and footprint once its last chunk has completed,
// and the engine admits from the FIFO on its next pump.  Chunks of a waiting
// session queue up and are served after admission.
#include <math.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "common.h"
#include "fit_body.h"
#include "fold_body.h"
#include "state_body.h"

using namespace isnmf;

const OnlineDev *isnmf_handle_dev(const isnmf_online *h);
const FitClass *isnmf_handle_class(const isnmf_online *h);
const isnmf_params *isnmf_handle_params(const isnmf_online *h);
int isnmf_handle_kernel(const isnmf_online *h);
void isnmf_handle_advance(isnmf_online *h, long long frames, hipStream_t s);

namespace {

typedef ServeWork Work;

// ---- kernels (grids: x = work item of the class range, y = tile / column)

template <int NW, int CPW, int KMAX, int PREC, bool WG>
__global__ __launch_bounds__(NW * 64) void serve_fit_kernel(const FitDesc *__restrict__ tab,
                                                            const Work *__restrict__ work) {
    const Work wk = work[blockIdx.x];
    if ((int)blockIdx.y * NF >= wk.b) return;
    FitDesc a = tab[wk.sess];
    a.b = wk.b;
    a.V = wk.V;
    a.ldv = wk.ldv;
    fit_body<NW, CPW, KMAX, PREC, WG>(a, blockIdx.y);
}

template <int KTM>
__global__ __launch_bounds__(256, 4) void serve_fold_kernel(const FoldArgs *__restrict__ tab,
                                                         const Work *__restrict__ work) {
    const Work wk = work[blockIdx.x];
    FoldArgs a = tab[wk.sess];
    a.b = wk.b;
    fold_rows_body<KTM>(a, blockIdx.y);
}

__global__ __launch_bounds__(64) void serve_rescale_kernel(const RescaleArgs *__restrict__ tab,
                                                            const int *__restrict__ upd,
                                                            const Work *__restrict__ work) {
    const Work wk = work[blockIdx.x];
    if (!upd[wk.sess]) {   // the fold stored A and B with no pending scale
        if (threadIdx.x == 0) tab[wk.sess].sc[blockIdx.y] = 1.0;
        return;
    }
    rescale_body(tab[wk.sess], blockIdx.y, wk.b);
}

template <int NW, int CPW, int KMAX, int PREC, bool WG>
struct ServeL {
    static hipError_t run(const FitDesc *tab, const Work *work, int n, int tiles, hipStream_t s) {
        serve_fit_kernel<NW, CPW, KMAX, PREC, WG><<<dim3(n, tiles), NW * 64, 0, s>>>(tab, work);
        return hipGetLastError();
    }
};

// The variant dispatch of fit_launch.h, restated for the serving wrapper.
template <int PREC>
hipError_t serve_fit(const FitClass &c, const FitDesc *tab, const Work *work, int n, int tiles,
                     hipStream_t s) {
#define ISNMF_SK(NW, CPW, WG)                                                           \
    switch (c.kmax) {                                                                   \
        case 8: return ServeL<NW, CPW, 8, PREC, WG>::run(tab, work, n, tiles, s);       \
        case 16: return ServeL<NW, CPW, 16, PREC, WG>::run(tab, work, n, tiles, s);     \
        case 24: return ServeL<NW, CPW, 24, PREC, WG>::run(tab, work, n, tiles, s);     \
        case 32: return ServeL<NW, CPW, 32, PREC, WG>::run(tab, work, n, tiles, s);     \
        case 40: return ServeL<NW, CPW, 40, PREC, WG>::run(tab, work, n, tiles, s);     \
        case 52: return ServeL<NW, CPW, 52, PREC, WG>::run(tab, work, n, tiles, s);     \
        case 64: return ServeL<NW, CPW, 64, PREC, WG>::run(tab, work, n, tiles, s);     \
        default: break;                                                                 \
    }
    if (!c.wg && c.cpw == 1) {
        switch (c.nw) {
            case 4: { ISNMF_SK(4, 1, false) break; }
            case 8: { ISNMF_SK(8, 1, false) break; }
            default: break;
        }
    }
#undef ISNMF_SK
    return hipErrorNotSupported;
}

// tiles: of NF frames for the MFMA tile variants, recomputed for the
// 16-frame tile variant's 128-frame workgroups from max_b.
hipError_t serve_fit_any(int prec, const FitClass &c, const FitDesc *tab, const Work *work, int n,
                         int tiles, int max_b, hipStream_t s) {
    if (c.cpw == -1)
        return prec == 1 ? launch_fit_tile_work(c, tab, work, n, (max_b + 127) / 128, s)
                         : hipErrorNotSupported;
    if (c.cpw == -2)
        return prec == 1 ? launch_fit_stile_work(c, tab, work, n, (max_b + 127) / 128, s)
                         : hipErrorNotSupported;
    if (c.cpw == -3)
        return prec == 0 ? launch_fit_t32_work(c, tab, work, n, (max_b + 127) / 128, s)
                         : hipErrorNotSupported;
    if (c.cpw == 0 || c.cpw == -4)   // VALU variants: one workgroup per frame
        return prec == (c.cpw == 0 ? 0 : 1) ? launch_fit_valu_work(c, tab, work, n, max_b, s)
                                            : hipErrorNotSupported;
    if (prec == 1) return serve_fit<1>(c, tab, work, n, tiles, s);
    if (prec == 2) return serve_fit<2>(c, tab, work, n, tiles, s);
    return serve_fit<0>(c, tab, work, n, tiles, s);
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct isnmf_server {
    // configuration
    size_t budget = 0, used = 0;
    int max_frames = 0, max_sessions = 0, inflight = 2;
    hipStream_t stream = nullptr;
    // sessions (ids are indices of `sess`, never reused)
    struct Sess {
        isnmf_online *h;
        int prec;
        FitClass cls;
        int F, K;
        size_t footprint;
        int slot = -1;                 // row of the device tables while resident
        int state = ISNMF_SESSION_WAITING;
        bool closing = false;          // no more submits; release when idle
        int inflight = 0;              // chunks launched and not yet retired
        double *loss = nullptr;        // running-loss target (set_loss)
        std::deque<long long> queue;   // pending request ids, FIFO
    };
    std::vector<Sess> sess;
    std::vector<int> slot_owner;       // session holding each table row, or -1
    std::vector<int> free_slots;
    std::deque<int> admit_q;           // waiting sessions, FIFO
    int resident = 0;
    // host mirrors of the device tables (the source of the admission copies)
    std::vector<FitDesc> h_fit;
    std::vector<FoldArgs> h_fold;
    std::vector<RescaleArgs> h_rs;
    std::vector<int> h_upd;
    FitDesc *d_fit = nullptr;
    FoldArgs *d_fold = nullptr;
    RescaleArgs *d_rs = nullptr;
    int *d_upd = nullptr;
    // requests
    struct Req {
        int sess, n, ldv;
        const float *V;
        double arrival, start, done;
        int state;   // 0 queued, 1 launched, 2 done
    };
    std::vector<Req> reqs;
    std::vector<long long> done_list;
    size_t done_read = 0;
    // step ring (pinned host work lists, device work lists, events)
    struct Slot {
        Work *host = nullptr;
        Work *dev = nullptr;
        hipEvent_t ev = nullptr;
        bool busy = false;
        std::vector<long long> reqs;
    };
    std::vector<Slot> slots;
    int next_slot = 0;
    // The groups of a step (one per variant and shape) touch disjoint
    // sessions, so their fit -> fold -> rescale chains are forked over up to
    // LANES streams (one event after the work-list copy, one join per side
    // stream before the step's completion event).
    static constexpr int LANES = 4;
    hipStream_t side[LANES - 1] = {};
    hipEvent_t ev_fork = nullptr, ev_join[LANES - 1] = {};
    long long steps = 0, frames = 0;
    double busy_since = 0.0;
};

namespace {

int prec_of(const isnmf_params &p) {
    return p.precision == ISNMF_BF16 ? 1 : p.precision == ISNMF_FP16 ? 2 : 0;
}

// Write session `id`'s descriptors into its table row (host mirror, then an
// asynchronous copy on the engine stream, ahead of any step that reads it).
bool write_row(isnmf_server *s, int id) {
    const auto &ss = s->sess[id];
    const int r = ss.slot;
    const OnlineDev &d = *isnmf_handle_dev(ss.h);
    const isnmf_params &p = *isnmf_handle_params(ss.h);
    s->h_fit[r] = make_fit_desc(d, nullptr, d.F, 1, p.inner_iters, p.eps, 0, nullptr, d.K);
    s->h_fold[r] = fold_args(d, 1, p.rho, p.update_w, nullptr, ss.loss);
    RescaleArgs ra = rescale_args(d, p.normalize, 0, nullptr, d.K);
    ra.dwpart = nullptr;   // served steps report no dW
    s->h_rs[r] = ra;
    s->h_upd[r] = p.update_w;
    hipStream_t st = s->stream;
    return hipMemcpyAsync(s->d_fit + r, &s->h_fit[r], sizeof(FitDesc), hipMemcpyHostToDevice,
                          st) == hipSuccess &&
           hipMemcpyAsync(s->d_fold + r, &s->h_fold[r], sizeof(FoldArgs), hipMemcpyHostToDevice,
                          st) == hipSuccess &&
           hipMemcpyAsync(s->d_rs + r, &s->h_rs[r], sizeof(RescaleArgs), hipMemcpyHostToDevice,
                          st) == hipSuccess &&
           hipMemcpyAsync(s->d_upd + r, &s->h_upd[r], sizeof(int), hipMemcpyHostToDevice, st) ==
               hipSuccess;
}

// Admit waiting sessions in FIFO order while a row is free and the head's
// footprint fits the budget.
bool admit(isnmf_server *s) {
    while (!s->admit_q.empty() && !s->free_slots.empty()) {
        const int id = s->admit_q.front();
        auto &ss = s->sess[id];
        if (s->used + ss.footprint > s->budget) break;   // head-of-line: FIFO order is kept
        s->admit_q.pop_front();
        ss.slot = s->free_slots.back();
        s->free_slots.pop_back();
        s->slot_owner[ss.slot] = id;
        s->used += ss.footprint;
        ss.state = ss.closing ? ISNMF_SESSION_CLOSING : ISNMF_SESSION_RESIDENT;
        ++s->resident;
        if (!write_row(s, id)) return false;
    }
    return true;
}

// Return a closing session's row and footprint once nothing of it is left.
void release_if_idle(isnmf_server *s, int id) {
    auto &ss = s->sess[id];
    if (!ss.closing || ss.state == ISNMF_SESSION_CLOSED || !ss.queue.empty() || ss.inflight)
        return;
    if (ss.slot >= 0) {
        s->slot_owner[ss.slot] = -1;
        s->free_slots.push_back(ss.slot);
        s->used -= ss.footprint;
        --s->resident;
        ss.slot = -1;
    } else {
        for (auto it = s->admit_q.begin(); it != s->admit_q.end(); ++it)
            if (*it == id) {
                s->admit_q.erase(it);
                break;
            }
    }
    ss.state = ISNMF_SESSION_CLOSED;
}

// Retire finished steps: stamp completion times, release sessions closed
// meanwhile and admit waiting ones into the rows and budget they free.
bool retire(isnmf_server *s) {
    std::vector<int> touched;
    for (auto &sl : s->slots) {
        if (!sl.busy) continue;
        if (hipEventQuery(sl.ev) != hipSuccess) continue;
        const double t = now_s();
        for (long long r : sl.reqs) {
            auto &q = s->reqs[r];
            q.state = 2;
            q.done = t;
            s->done_list.push_back(r);
            auto &ss = s->sess[q.sess];
            --ss.inflight;
            if (ss.closing) touched.push_back(q.sess);
        }
        sl.reqs.clear();
        sl.busy = false;
    }
    for (const int id : touched) release_if_idle(s, id);
    return admit(s);
}

// Form and enqueue one step from the pending chunks; returns frames launched.
int launch_step(isnmf_server *s) {
    isnmf_server::Slot *slot = nullptr;
    for (int i = 0; i < (int)s->slots.size(); ++i) {
        auto &c = s->slots[(s->next_slot + i) % s->slots.size()];
        if (!c.busy) {
            slot = &c;
            s->next_slot = (s->next_slot + i + 1) % (int)s->slots.size();
            break;
        }
    }
    if (!slot) return 0;
    // at most one chunk per resident session, oldest request first across sessions
    std::vector<std::pair<double, int>> cand;
    for (const int i : s->slot_owner) {
        if (i < 0) continue;
        const auto &ss = s->sess[i];
        if (!ss.queue.empty()) cand.push_back({s->reqs[ss.queue.front()].arrival, i});
    }
    if (cand.empty()) return 0;
    std::sort(cand.begin(), cand.end());
    std::vector<int> pick;
    int frames = 0;
    for (auto &c : cand) {
        const auto &q = s->reqs[s->sess[c.second].queue.front()];
        if (frames + q.n > s->max_frames && !pick.empty()) continue;
        pick.push_back(c.second);
        frames += q.n;
        if ((int)pick.size() >= s->max_sessions) break;
    }
    // group by (kernel variant, precision, shape) so each launch has one shape
    std::sort(pick.begin(), pick.end(), [&](int a, int b) {
        const auto &A = s->sess[a], &B = s->sess[b];
        return std::make_tuple(A.prec, A.cls.nw, A.cls.kmax, A.F, A.K) <
               std::make_tuple(B.prec, B.cls.nw, B.cls.kmax, B.F, B.K);
    });
    const double t = now_s();
    for (int i = 0; i < (int)pick.size(); ++i) {
        auto &ss = s->sess[pick[i]];
        const long long r = ss.queue.front();
        ss.queue.pop_front();
        auto &q = s->reqs[r];
        q.state = 1;
        q.start = t;
        slot->host[i] = Work{ss.slot, q.n, q.V, q.ldv, 0};
        slot->reqs.push_back(r);
        ++ss.inflight;
    }
    const int n = (int)pick.size();
    hipStream_t st = s->stream;
    if (hipMemcpyAsync(slot->dev, slot->host, sizeof(Work) * n, hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return -1;
    // groups of equal (variant, shape): [lo, hi) ranges of the sorted pick
    struct Span {
        int lo, hi, maxb;
        double cost;
        int lane;
    };
    std::vector<Span> spans;
    for (int lo = 0; lo < n;) {
        const auto &A = s->sess[pick[lo]];
        int hi = lo + 1, maxb = s->reqs[slot->reqs[lo]].n;
        while (hi < n) {
            const auto &B = s->sess[pick[hi]];
            if (B.prec != A.prec || B.cls.nw != A.cls.nw || B.cls.cpw != A.cls.cpw ||
                B.cls.kmax != A.cls.kmax || B.F != A.F || B.K != A.K)
                break;
            maxb = std::max(maxb, s->reqs[slot->reqs[hi]].n);
            ++hi;
        }
        double cost = 0.0;
        for (int i = lo; i < hi; ++i) cost += (double)s->reqs[slot->reqs[i]].n * A.F * A.K;
        spans.push_back(Span{lo, hi, maxb, cost, 0});
        lo = hi;
    }
    // lanes: largest group first onto the least loaded lane
    const int nlanes = std::min((int)spans.size(), isnmf_server::LANES);
    {
        std::vector<int> order(spans.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return spans[x].cost > spans[y].cost; });
        double load[isnmf_server::LANES] = {};
        for (const int gi : order) {
            int best = 0;
            for (int l = 1; l < nlanes; ++l)
                if (load[l] < load[best]) best = l;
            spans[gi].lane = best;
            load[best] += spans[gi].cost;
        }
    }
    if (nlanes > 1) {
        if (hipEventRecord(s->ev_fork, st) != hipSuccess) return -1;
        for (int i = 0; i < nlanes - 1; ++i)
            if (hipStreamWaitEvent(s->side[i], s->ev_fork, 0) != hipSuccess) return -1;
    }
    for (const Span &sp : spans) {
        const auto &A = s->sess[pick[sp.lo]];
        const hipStream_t ls = sp.lane ? s->side[sp.lane - 1] : st;
        const int lo = sp.lo, cnt = sp.hi - sp.lo;
        const int tiles = (sp.maxb + NF - 1) / NF;
        if (serve_fit_any(A.prec, A.cls, s->d_fit, slot->dev + lo, cnt, tiles, sp.maxb, ls) !=
            hipSuccess)
            return -1;
        const dim3 fg(cnt, (A.F + 15) / 16);
        switch (fold_ktm(A.K)) {
            case 1: serve_fold_kernel<1><<<fg, 256, 0, ls>>>(s->d_fold, slot->dev + lo); break;
            case 2: serve_fold_kernel<2><<<fg, 256, 0, ls>>>(s->d_fold, slot->dev + lo); break;
            case 4: serve_fold_kernel<4><<<fg, 256, 0, ls>>>(s->d_fold, slot->dev + lo); break;
            default: serve_fold_kernel<8><<<fg, 256, 0, ls>>>(s->d_fold, slot->dev + lo); break;
        }
        serve_rescale_kernel<<<dim3(cnt, A.K), 64, 0, ls>>>(s->d_rs, s->d_upd, slot->dev + lo);
    }
    if (hipGetLastError() != hipSuccess) return -1;
    for (int i = 0; i < nlanes - 1; ++i)
        if (hipEventRecord(s->ev_join[i], s->side[i]) != hipSuccess ||
            hipStreamWaitEvent(st, s->ev_join[i], 0) != hipSuccess)
            return -1;
    for (int i = 0; i < n; ++i) {
        auto &ss = s->sess[pick[i]];
        isnmf_handle_advance(ss.h, s->reqs[slot->reqs[i]].n, st);
    }
    if (hipEventRecord(slot->ev, st) != hipSuccess) return -1;
    slot->busy = true;
    s->steps += 1;
    s->frames += frames;
    return frames;
}

// frees the server's host resources (pinned work lists, events, side streams)
void release(isnmf_server *s) {
    for (auto &sl : s->slots) {
        if (sl.host) hipHostFree(sl.host);
        if (sl.ev) hipEventDestroy(sl.ev);
    }
    for (int i = 0; i < isnmf_server::LANES - 1; ++i) {
        if (s->side[i]) hipStreamDestroy(s->side[i]);
        if (s->ev_join[i]) hipEventDestroy(s->ev_join[i]);
    }
    if (s->ev_fork) hipEventDestroy(s->ev_fork);
    delete s;
}

}  // namespace

extern "C" {

size_t isnmf_server_workspace_size(int max_sessions, int max_per_step, int inflight) {
    if (max_sessions < 1 || max_per_step < 1 || inflight < 1) return 0;
    return align256(sizeof(FitDesc) * max_sessions) + align256(sizeof(FoldArgs) * max_sessions) +
           align256(sizeof(RescaleArgs) * max_sessions) + align256(sizeof(int) * max_sessions) +
           (size_t)inflight * align256(sizeof(Work) * max_per_step);
}

int isnmf_server_create(isnmf_server **out, int max_sessions, int max_per_step, int max_frames,
                        int inflight, size_t hbm_budget, void *workspace, size_t ws_bytes,
                        void *stream) {
    if (!out) return ISNMF_EINVAL;
    *out = nullptr;
    if (max_sessions < 1 || max_per_step < 1 || max_frames < 1 || inflight < 1 || inflight > 8 ||
        !workspace || ((uintptr_t)workspace & 255))
        return ISNMF_EINVAL;
    if (ws_bytes < isnmf_server_workspace_size(max_sessions, max_per_step, inflight))
        return ISNMF_ENOMEM;
    isnmf_server *s = new (std::nothrow) isnmf_server;
    if (!s) return ISNMF_ENOMEM;
    s->budget = hbm_budget;
    s->max_frames = max_frames;
    s->max_sessions = max_per_step;
    s->inflight = inflight;
    s->stream = (hipStream_t)stream;
    char *p = (char *)workspace;
    s->d_fit = (FitDesc *)p;
    p += align256(sizeof(FitDesc) * max_sessions);
    s->d_fold = (FoldArgs *)p;
    p += align256(sizeof(FoldArgs) * max_sessions);
    s->d_rs = (RescaleArgs *)p;
    p += align256(sizeof(RescaleArgs) * max_sessions);
    s->d_upd = (int *)p;
    p += align256(sizeof(int) * max_sessions);
    s->slot_owner.assign(max_sessions, -1);
    for (int r = max_sessions - 1; r >= 0; --r) s->free_slots.push_back(r);   // row 0 first
    s->h_fit.resize(max_sessions);
    s->h_fold.resize(max_sessions);
    s->h_rs.resize(max_sessions);
    s->h_upd.resize(max_sessions);
    s->slots.resize(inflight);
    for (auto &sl : s->slots) {
        sl.dev = (Work *)p;
        p += align256(sizeof(Work) * max_per_step);
        if (hipHostMalloc((void **)&sl.host, sizeof(Work) * max_per_step, 0) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
            for (auto &c : s->slots) {
                if (c.host) hipHostFree(c.host);
                if (c.ev) hipEventDestroy(c.ev);
            }
            delete s;
            return ISNMF_ENOMEM;
        }
    }
    bool ok = hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < isnmf_server::LANES - 1; ++i)
        ok = hipStreamCreateWithFlags(&s->side[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&s->ev_join[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        release(s);
        return ISNMF_EDEVICE;
    }
    *out = s;
    return ISNMF_OK;
}

int isnmf_server_open(isnmf_server *s, isnmf_online *h, size_t footprint, int *session) {
    if (!s || !h || !session) return ISNMF_EINVAL;
    const isnmf_params &p = *isnmf_handle_params(h);
    if (p.h_init == ISNMF_H_WARM) return ISNMF_EINVAL;
    if (isnmf_handle_kernel(h) != ISNMF_KERNEL_FUSED) return ISNMF_EUNSUPPORTED;
    if (p.psi_lambda > 0.0) return ISNMF_EUNSUPPORTED;   // no penalty on H
    const OnlineDev &d = *isnmf_handle_dev(h);
    const FitClass &c = *isnmf_handle_class(h);
    // variants with a served kernel of their own: the 16-frame tiles and the VALU forms
    const bool own = ((c.cpw == -1 || c.cpw == -2 || c.cpw == -4) && prec_of(p) == 1) ||
                     ((c.cpw == -3 || c.cpw == 0) && prec_of(p) == 0);
    if (((c.cpw == 0 && c.nw == 8) || c.cpw == -4) && !d.Wv) return ISNMF_EUNSUPPORTED;
    if (!own && (c.wg || c.cpw != 1 || (c.nw != 4 && c.nw != 8) || c.kmax > 64))
        return ISNMF_EUNSUPPORTED;
    if (footprint > s->budget) return ISNMF_ENOMEM;   // could never be admitted
    for (const auto &o : s->sess)
        if (o.h == h && o.state != ISNMF_SESSION_CLOSED) return ISNMF_EINVAL;   // already open
    isnmf_server::Sess ss;
    ss.h = h;
    ss.prec = prec_of(p);
    ss.cls = c;
    ss.F = d.F;
    ss.K = d.K;
    ss.footprint = footprint;
    const int id = (int)s->sess.size();
    try {
        s->sess.push_back(ss);
        s->admit_q.push_back(id);
    } catch (...) {
        if ((int)s->sess.size() > id) s->sess.pop_back();
        return ISNMF_ENOMEM;
    }
    if (!admit(s)) return ISNMF_EDEVICE;
    *session = id;
    return ISNMF_OK;
}

int isnmf_server_close(isnmf_server *s, int session) {
    if (!s || session < 0 || session >= (int)s->sess.size()) return ISNMF_EINVAL;
    auto &ss = s->sess[session];
    if (ss.closing) return ISNMF_OK;
    ss.closing = true;
    if (ss.state == ISNMF_SESSION_RESIDENT) ss.state = ISNMF_SESSION_CLOSING;
    release_if_idle(s, session);
    return admit(s) ? ISNMF_OK : ISNMF_EDEVICE;
}

int isnmf_server_session_state(const isnmf_server *s, int session, int *state) {
    if (!s || !state || session < 0 || session >= (int)s->sess.size()) return ISNMF_EINVAL;
    const auto &ss = s->sess[session];
    *state = (ss.closing && ss.state == ISNMF_SESSION_WAITING) ? ISNMF_SESSION_CLOSING : ss.state;
    return ISNMF_OK;
}

int isnmf_server_admission(const isnmf_server *s, size_t *host_used, int *host_resident,
                           int *host_waiting) {
    if (!s) return ISNMF_EINVAL;
    if (host_used) *host_used = s->used;
    if (host_resident) *host_resident = s->resident;
    if (host_waiting) *host_waiting = (int)s->admit_q.size();
    return ISNMF_OK;
}

int isnmf_server_set_loss(isnmf_server *s, int session, double *d_loss_sum) {
    if (!s || session < 0 || session >= (int)s->sess.size()) return ISNMF_EINVAL;
    auto &ss = s->sess[session];
    if (ss.state == ISNMF_SESSION_CLOSED) return ISNMF_ESTATE;
    ss.loss = d_loss_sum;
    if (ss.slot < 0) return ISNMF_OK;   // waiting: written at admission
    const isnmf_params &p = *isnmf_handle_params(ss.h);
    const int r = ss.slot;
    s->h_fold[r] = fold_args(*isnmf_handle_dev(ss.h), 1, p.rho, p.update_w, nullptr, d_loss_sum);
    // on the engine stream: steps enqueued before keep the previous target
    if (hipMemcpyAsync(s->d_fold + r, &s->h_fold[r], sizeof(FoldArgs), hipMemcpyHostToDevice,
                       s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return ISNMF_EDEVICE;
    return ISNMF_OK;
}

int isnmf_server_submit(isnmf_server *s, int session, const float *V, int ldv, int n_frames,
                        double arrival, long long *request) {
    if (!s || session < 0 || session >= (int)s->sess.size() || !V || n_frames < 1) return ISNMF_EINVAL;
    auto &ss = s->sess[session];
    if (ss.closing) return ISNMF_ESTATE;
    const OnlineDev &d = *isnmf_handle_dev(ss.h);
    if (ldv < d.F || n_frames > d.b_max || n_frames > 512 || n_frames > s->max_frames)
        return ISNMF_EINVAL;
    isnmf_server::Req q;
    q.sess = session;
    q.n = n_frames;
    q.ldv = ldv;
    q.V = V;
    q.arrival = arrival < 0 ? now_s() : arrival;
    q.start = q.done = 0.0;
    q.state = 0;
    try {
        s->reqs.push_back(q);
        ss.queue.push_back((long long)s->reqs.size() - 1);
    } catch (...) {
        return ISNMF_ENOMEM;
    }
    if (request) *request = (long long)s->reqs.size() - 1;
    return ISNMF_OK;
}

int isnmf_server_pump(isnmf_server *s, int *launched_frames) {
    if (!s) return ISNMF_EINVAL;
    if (!retire(s)) return ISNMF_EDEVICE;
    int total = 0;
    for (;;) {
        const int f = launch_step(s);
        if (f < 0) return ISNMF_EDEVICE;
        if (f == 0) break;
        total += f;
    }
    if (launched_frames) *launched_frames = total;
    return ISNMF_OK;
}

int isnmf_server_pending(const isnmf_server *s, long long *queued, long long *inflight) {
    if (!s) return ISNMF_EINVAL;
    long long qn = 0, fl = 0;
    for (const auto &ss : s->sess) qn += (long long)ss.queue.size();
    for (const auto &sl : s->slots) fl += (long long)sl.reqs.size();
    if (queued) *queued = qn;
    if (inflight) *inflight = fl;
    return ISNMF_OK;
}

int isnmf_server_drain(isnmf_server *s) {
    if (!s) return ISNMF_EINVAL;
    for (;;) {
        if (isnmf_server_pump(s, nullptr) != ISNMF_OK) return ISNMF_EDEVICE;
        long long q = 0, f = 0;
        isnmf_server_pending(s, &q, &f);
        if (q == 0 && f == 0) return ISNMF_OK;
        // nothing in flight after a pump: what is queued belongs to waiting
        // sessions that no release can admit until the caller closes some
        if (f == 0) return ISNMF_ESTATE;
        if (hipStreamSynchronize(s->stream) != hipSuccess) return ISNMF_EDEVICE;
    }
}

int isnmf_server_results(isnmf_server *s, int max_out, long long *req, int *session,
                         int *n_frames, double *arrival, double *start, double *done, int *count) {
    if (!s || !count || max_out < 0) return ISNMF_EINVAL;
    int c = 0;
    while (s->done_read < s->done_list.size() && c < max_out) {
        const long long r = s->done_list[s->done_read++];
        const auto &q = s->reqs[r];
        if (req) req[c] = r;
        if (session) session[c] = q.sess;
        if (n_frames) n_frames[c] = q.n;
        if (arrival) arrival[c] = q.arrival;
        if (start) start[c] = q.start;
        if (done) done[c] = q.done;
        ++c;
    }
    *count = c;
    return ISNMF_OK;
}

int isnmf_server_stats(const isnmf_server *s, long long *steps, long long *frames) {
    if (!s) return ISNMF_EINVAL;
    if (steps) *steps = s->steps;
    if (frames) *frames = s->frames;
    return ISNMF_OK;
}

double isnmf_server_clock(void) { return now_s(); }

int isnmf_server_destroy(isnmf_server *s) {
    if (!s) return ISNMF_EINVAL;
    hipError_t e = hipStreamSynchronize(s->stream);
    for (int i = 0; i < isnmf_server::LANES - 1; ++i)
        if (s->side[i] && hipStreamSynchronize(s->side[i]) != hipSuccess) e = hipErrorUnknown;
    release(s);
    return e == hipSuccess ? ISNMF_OK : ISNMF_EDEVICE;
}

}  // extern "C"
