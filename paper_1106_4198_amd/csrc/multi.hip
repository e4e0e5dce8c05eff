// Batched form: many independent online streams (each its own W, A, B, F, K,
// minibatch size) advanced by one minibatch per step with one fit launch per
// kernel variant in use, side by side on up to four streams (lanes), each lane
// followed by one fold launch and one rescale launch for its streams.  A step reads its per-stream frame cursors on the device, so it can
// be captured once into a hipGraph and replayed.  Also the autotuner that picks
// the fit variant for a shape.
//
// Each stream's arithmetic is exactly that of isnmf_online_step with the same
// handle (same kernel bodies, same variant, fixed-order sums), so a stream's
// result does not depend on which other streams share the launch.
#include <math.h>

#include <map>
#include <algorithm>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "common.h"
#include "fold_body.h"
#include "state_body.h"

using namespace isnmf;

// ----------------------------------------------------------------- tuning cache

namespace isnmf {
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, FitClass> g_tune;
}  // namespace

FitClass tuned_class(int F, int K, int prec, int /*b*/) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find({F, K, prec});
    if (it != g_tune.end()) return it->second;
    return fit_class(F, K, prec);
}
}  // namespace isnmf

// ----------------------------------------------------------------- kernels

namespace {

__global__ void prepare_kernel(int S, const int *__restrict__ b, const long long *__restrict__ nf,
                               const long long *__restrict__ cursor, int *__restrict__ beff) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const long long left = nf[s] - cursor[s];
    beff[s] = left <= 0 ? 0 : (int)(left < b[s] ? left : b[s]);
}

__global__ void advance_kernel(int S, const int *__restrict__ beff, long long *__restrict__ cursor) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S) cursor[s] += beff[s];
}

template <int KTM>
__global__ __launch_bounds__(256, 4) void fold_multi_kernel(const FoldArgs *__restrict__ fa,
                                                         const int2 *__restrict__ items,
                                                         const int *__restrict__ beff) {
    const int2 it = items[blockIdx.x];
    const int b = beff[it.x];
    if (b == 0) return;
    FoldArgs a = fa[it.x];
    a.b = b;
    fold_rows_body<KTM>(a, it.y);
}

__global__ __launch_bounds__(64) void rescale_multi_kernel(const RescaleArgs *__restrict__ ra,
                                                            const int *__restrict__ upd,
                                                            const int2 *__restrict__ items,
                                                            const int *__restrict__ beff) {
    const int2 it = items[blockIdx.x];
    const int b = beff[it.x];
    if (b == 0) return;   // no step: A, B and their pending scale are untouched
    if (!upd[it.x]) {     // the fold stored A and B with no pending scale
        if (threadIdx.x == 0) ra[it.x].sc[it.y] = 1.0;
        return;
    }
    rescale_body(ra[it.x], it.y, b);
}

// Positive pseudo-random fill (splitmix hash of the index) for tuning inputs.
__global__ void fill_kernel(float *x, long n, float lo, float span, unsigned seed) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned long long z = (unsigned long long)i * 0x9E3779B97F4A7C15ull + seed;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = lo + span * (float)(z >> 40) * (1.0f / 16777216.0f);
}

}  // namespace

struct isnmf_multi {
    int S = 0;
    std::vector<isnmf_online *> hs;
    std::vector<long long> nframes, cursor;
    std::vector<int> b;
    FitDesc *d_fit = nullptr;
    FoldArgs *d_fold = nullptr;
    RescaleArgs *d_rs = nullptr;
    int *d_upd = nullptr, *d_b = nullptr, *d_beff = nullptr;
    long long *d_cursor = nullptr, *d_nf = nullptr;
    int2 *d_items = nullptr;
    struct Group {
        FitClass c;
        int prec, off, n;
        bool fold;     // the fit launch folds its streams' minibatches itself
        double cost;   // frames x F x K over its items (for the lane balance)
        int lane;      // 0: the step's stream; i > 0: side[i - 1]
    };
    std::vector<Group> groups;
    // The fit groups are independent (each stream is in exactly one), so a
    // step forks them over up to LANES streams: one event after prepare, one
    // join per side stream before the fold.  Each launch is bounded by its
    // slowest workgroup; side by side those tails overlap instead of adding.
    static constexpr int LANES = 4;
    int nlanes = 1;
    hipStream_t side[LANES - 1] = {};
    hipEvent_t ev_fork = nullptr, ev_join[LANES - 1] = {};
    // Per lane: the fold and rescale items of the streams whose fit groups run
    // on it, launched on the lane right after its fits (a lane's streams do
    // not wait for the other lanes' fits), and the fold instance that covers
    // the lane's widest stream.
    int fold_off[LANES] = {}, fold_n[LANES] = {}, rs_off[LANES] = {}, rs_n[LANES] = {};
    int fold_ktm[LANES] = {1, 1, 1, 1};
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last = nullptr;
};

// Host accessors of the online handle (defined in abi.hip).
extern "C++" {
const OnlineDev *isnmf_handle_dev(const isnmf_online *h);
const FitClass *isnmf_handle_class(const isnmf_online *h);
const isnmf_params *isnmf_handle_params(const isnmf_online *h);
int isnmf_handle_kernel(const isnmf_online *h);
void isnmf_handle_advance(isnmf_online *h, long long frames, hipStream_t s);
}

namespace {

int prec_of(const isnmf_params &p) {
    return p.precision == ISNMF_BF16 ? 1 : p.precision == ISNMF_FP16 ? 2 : 0;
}

struct Layout {
    size_t fit, fold, rs, upd, b, beff, cur, nf, items, total;
};

Layout layout(int S, size_t nitems) {
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.fit = take(sizeof(FitDesc) * S);
    L.fold = take(sizeof(FoldArgs) * S);
    L.rs = take(sizeof(RescaleArgs) * S);
    L.upd = take(sizeof(int) * S);
    L.b = take(sizeof(int) * S);
    L.beff = take(sizeof(int) * S);
    L.cur = take(sizeof(long long) * S);
    L.nf = take(sizeof(long long) * S);
    L.items = take(sizeof(int2) * (nitems ? nitems : 1));
    L.total = off;
    return L;
}

// Workgroup i of a launch is dispatched to XCD i mod 8.  Ordering a launch's
// items so that all items of a stream share an XCD lets that XCD's L2 merge
// the partial cache lines that neighbouring tiles of the stream write (the
// fold's 16-row column segments, the rescale's row-major 16-bit W) and serve
// the lines they both read, instead of each XCD fetching and writing back its
// own partial copy.  xcd[s] is the XCD of stream s; the queues are
// interleaved, and once the shorter ones run out the rest keeps its order.
constexpr int XCDS = 8;

std::vector<int> xcd_assign(const std::vector<size_t> &load_per_stream) {
    const int S = (int)load_per_stream.size();
    std::vector<int> order(S), xcd(S, 0);
    for (int s = 0; s < S; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return load_per_stream[a] > load_per_stream[b]; });
    size_t load[XCDS] = {};
    for (int s : order) {
        int x = 0;
        for (int y = 1; y < XCDS; ++y)
            if (load[y] < load[x]) x = y;
        xcd[s] = x;
        load[x] += load_per_stream[s];
    }
    return xcd;
}

void push_xcd_ordered(std::vector<int2> &out, const std::vector<int2> &items,
                      const std::vector<int> &xcd) {
    std::vector<int2> q[XCDS];
    for (const int2 &it : items) q[xcd[it.x]].push_back(it);
    size_t longest = 0;
    for (int x = 0; x < XCDS; ++x) longest = std::max(longest, q[x].size());
    for (size_t j = 0; j < longest; ++j)
        for (int x = 0; x < XCDS; ++x)
            if (j < q[x].size()) out.push_back(q[x][j]);
}

size_t count_items(isnmf_online *const *h, const int *b, int S) {
    size_t n = 0;
    for (int s = 0; s < S; ++s) {
        const OnlineDev &d = *isnmf_handle_dev(h[s]);
        n += (size_t)((b[s] + NF - 1) / NF) + fold_tiles(d) + d.K;
    }
    return n;
}

hipError_t enqueue_step(isnmf_multi *m, hipStream_t s) {
    const int blocks = (m->S + 255) / 256;
    prepare_kernel<<<blocks, 256, 0, s>>>(m->S, m->d_b, m->d_nf, m->d_cursor, m->d_beff);
    if (m->nlanes > 1) {
        hipError_t e = hipEventRecord(m->ev_fork, s);
        for (int i = 0; e == hipSuccess && i < m->nlanes - 1; ++i)
            e = hipStreamWaitEvent(m->side[i], m->ev_fork, 0);
        if (e != hipSuccess) return e;
    }
    for (const auto &g : m->groups) {
        hipError_t e;
        const hipStream_t gs = g.lane ? m->side[g.lane - 1] : s;
        if (g.c.cpw == 0 || g.c.cpw == -4)
            e = launch_fit_valu_multi(g.c, m->d_fit, m->d_items + g.off, g.n, m->d_cursor, m->d_beff, gs);
        else if (g.c.cpw == -1)
            e = launch_fit_tile_multi(g.c, m->d_fit, m->d_items + g.off, g.n, m->d_cursor, m->d_beff,
                                      g.fold, gs);
        else if (g.c.cpw == -2)
            e = launch_fit_stile_multi(g.c, m->d_fit, m->d_items + g.off, g.n, m->d_cursor, m->d_beff, gs);
        else if (g.c.cpw == -3)
            e = launch_fit_t32_multi(g.c, m->d_fit, m->d_items + g.off, g.n, m->d_cursor, m->d_beff,
                                     g.fold, gs);
        else if (g.prec == 1)
            e = launch_fit_multi_p<1>(g.c, m->d_fit, m->d_items + g.off, g.n, m->d_cursor, m->d_beff, gs);
        else if (g.prec == 2)
            e = launch_fit_multi_p<2>(g.c, m->d_fit, m->d_items + g.off, g.n, m->d_cursor, m->d_beff, gs);
        else
            e = launch_fit_multi_p<0>(g.c, m->d_fit, m->d_items + g.off, g.n, m->d_cursor, m->d_beff, gs);
        if (e != hipSuccess) return e;
    }
    for (int l = 0; l < m->nlanes; ++l) {
        const hipStream_t ls = l ? m->side[l - 1] : s;
        const int nf = m->fold_n[l];
        if (nf) {
            const int2 *fi = m->d_items + m->fold_off[l];
            switch (m->fold_ktm[l]) {
                case 1: fold_multi_kernel<1><<<nf, 256, 0, ls>>>(m->d_fold, fi, m->d_beff); break;
                case 2: fold_multi_kernel<2><<<nf, 256, 0, ls>>>(m->d_fold, fi, m->d_beff); break;
                case 4: fold_multi_kernel<4><<<nf, 256, 0, ls>>>(m->d_fold, fi, m->d_beff); break;
                case 8: fold_multi_kernel<8><<<nf, 256, 0, ls>>>(m->d_fold, fi, m->d_beff); break;
                default: return hipErrorNotSupported;
            }
        }
        if (m->rs_n[l])
            rescale_multi_kernel<<<m->rs_n[l], 64, 0, ls>>>(m->d_rs, m->d_upd,
                                                            m->d_items + m->rs_off[l], m->d_beff);
    }
    if (m->nlanes > 1) {
        hipError_t e = hipSuccess;
        for (int i = 0; e == hipSuccess && i < m->nlanes - 1; ++i) {
            e = hipEventRecord(m->ev_join[i], m->side[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, m->ev_join[i], 0);
        }
        if (e != hipSuccess) return e;
    }
    advance_kernel<<<blocks, 256, 0, s>>>(m->S, m->d_beff, m->d_cursor);
    return hipGetLastError();
}

void release_lanes(isnmf_multi *m) {
    for (int i = 0; i < isnmf_multi::LANES - 1; ++i) {
        if (m->side[i]) hipStreamDestroy(m->side[i]);
        if (m->ev_join[i]) hipEventDestroy(m->ev_join[i]);
        m->side[i] = nullptr;
        m->ev_join[i] = nullptr;
    }
    if (m->ev_fork) hipEventDestroy(m->ev_fork);
    m->ev_fork = nullptr;
}

void host_advance(isnmf_multi *m, hipStream_t s) {
    for (int i = 0; i < m->S; ++i) {
        const long long left = m->nframes[i] - m->cursor[i];
        const long long step = left <= 0 ? 0 : (left < m->b[i] ? left : m->b[i]);
        m->cursor[i] += step;
        if (step) isnmf_handle_advance(m->hs[i], step, s);
    }
}

}  // namespace

extern "C" {

size_t isnmf_multi_workspace_size(isnmf_online *const *handles, int S, const int *b) {
    if (!handles || !b || S < 1) return 0;
    for (int s = 0; s < S; ++s)
        if (!handles[s] || b[s] < 1) return 0;
    return layout(S, count_items(handles, b, S)).total;
}

int isnmf_multi_create(isnmf_multi **out, isnmf_online *const *handles, int S,
                       const float *const *V, const int *ldv, const long long *n_frames,
                       const int *b, double *d_loss, void *workspace, size_t ws_bytes,
                       void *stream) {
    if (!out) return ISNMF_EINVAL;
    *out = nullptr;
    if (!handles || !V || !ldv || !n_frames || !b || S < 1 || !workspace) return ISNMF_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return ISNMF_EINVAL;
    for (int s = 0; s < S; ++s) {
        if (!handles[s] || !V[s] || n_frames[s] < 0 || b[s] < 1) return ISNMF_EINVAL;
        const OnlineDev &d = *isnmf_handle_dev(handles[s]);
        const isnmf_params &p = *isnmf_handle_params(handles[s]);
        if (ldv[s] < d.F || b[s] > d.b_max) return ISNMF_EINVAL;
        if (p.h_init == ISNMF_H_WARM) return ISNMF_EINVAL;            // fresh restarts only
        if (isnmf_handle_kernel(handles[s]) != ISNMF_KERNEL_FUSED) return ISNMF_EUNSUPPORTED;
        if (p.psi_lambda > 0.0) return ISNMF_EUNSUPPORTED;            // no penalty on H
        if (b[s] > 512) return ISNMF_EUNSUPPORTED;                   // single fold slice
        const FitClass &c = *isnmf_handle_class(handles[s]);
        if (((c.cpw == 0 && c.nw == 8) || c.cpw == -4) && !d.Wv) return ISNMF_EUNSUPPORTED;
        for (int r = 0; r < s; ++r)
            if (handles[r] == handles[s]) return ISNMF_EINVAL;        // one entry per stream
    }
    const size_t nitems = count_items(handles, b, S);
    const Layout L = layout(S, nitems);
    if (ws_bytes < L.total) return ISNMF_ENOMEM;

    isnmf_multi *m = new (std::nothrow) isnmf_multi;
    if (!m) return ISNMF_ENOMEM;
    char *base = (char *)workspace;
    m->S = S;
    m->hs.assign(handles, handles + S);
    m->nframes.assign(n_frames, n_frames + S);
    m->cursor.assign(S, 0);
    m->b.assign(b, b + S);
    m->d_fit = (FitDesc *)(base + L.fit);
    m->d_fold = (FoldArgs *)(base + L.fold);
    m->d_rs = (RescaleArgs *)(base + L.rs);
    m->d_upd = (int *)(base + L.upd);
    m->d_b = (int *)(base + L.b);
    m->d_beff = (int *)(base + L.beff);
    m->d_cursor = (long long *)(base + L.cur);
    m->d_nf = (long long *)(base + L.nf);
    m->d_items = (int2 *)(base + L.items);
    m->last = (hipStream_t)stream;

    std::vector<FitDesc> fit(S);
    std::vector<FoldArgs> fold(S);
    std::vector<RescaleArgs> rs(S);
    std::vector<int> upd(S);
    std::vector<long long> zero(S, 0);
    std::vector<int2> items;
    items.reserve(nitems);
    // fit items grouped by (variant, precision, fold in the fit).  When every
    // stream is on a 16-frame tile variant (BF16 or FP32) with a minibatch that
    // fits one workgroup, each fit launch folds its streams itself (the same
    // bits as the separate fold) and the step has no fold launch.  With any
    // other stream the fold launch stays, and moving work from it into the fit
    // lanes (the step's critical path) only lengthens them, so then no stream
    // is folded in its fit.
    std::vector<std::pair<std::tuple<int, int, int, int, int, int, int>, std::vector<int2>>> groups;
    bool fold_in_fit = true;
    for (int s = 0; s < S && fold_in_fit; ++s) {
        const FitClass &c = *isnmf_handle_class(handles[s]);
        fold_in_fit = b[s] <= frames_per_item(c) &&
                      ((c.cpw == -1 && tile_fold_fits(c)) || (c.cpw == -3 && t32_fold_fits(c)));
    }
    std::vector<char> folded(S, fold_in_fit ? 1 : 0);
    // Folding BF16 tile fits also rescale their streams in the same workgroup.
    // The FP32 tile fit keeps the rescale launch: at its register budget the
    // rescale body spills inside its fold rounds and costs more than the launch.
    std::vector<char> rescaled(S, 0);
    for (int s = 0; s < S; ++s) {
        const OnlineDev &d = *isnmf_handle_dev(handles[s]);
        const isnmf_params &p = *isnmf_handle_params(handles[s]);
        const FitClass &c = *isnmf_handle_class(handles[s]);
        fit[s] = make_fit_desc(d, V[s], ldv[s], b[s], p.inner_iters, p.eps, 0, nullptr, d.K);
        fold[s] = fold_args(d, b[s], p.rho, p.update_w, nullptr, d_loss ? d_loss + s : nullptr);
        if (folded[s]) {
            fit[s].fold = m->d_fold + s;
            if (c.cpw == -1) {
                fit[s].rs = m->d_rs + s;
                rescaled[s] = 1;
            }
        }
        rs[s] = rescale_args(d, p.normalize, 0, nullptr, d.K);
        rs[s].dwpart = nullptr;   // the batched step reports no dW
        upd[s] = p.update_w;
        const auto key = std::make_tuple(c.nw, c.cpw, c.kmax, c.wg, c.rf, prec_of(p), (int)folded[s]);
        size_t gi = 0;
        while (gi < groups.size() && groups[gi].first != key) ++gi;
        if (gi == groups.size()) groups.push_back({key, {}});
        const int per = frames_per_item(c);
        for (int t = 0; t < (b[s] + per - 1) / per; ++t) groups[gi].second.push_back(int2{s, t});
    }
    for (auto &g : groups) {
        isnmf_multi::Group G;
        G.c = *isnmf_handle_class(handles[g.second.front().x]);
        G.prec = std::get<5>(g.first);
        G.fold = std::get<6>(g.first) != 0;
        G.off = (int)items.size();
        G.n = (int)g.second.size();
        G.cost = 0.0;
        for (const int2 &it : g.second) {
            const OnlineDev &d = *isnmf_handle_dev(handles[it.x]);
            G.cost += (double)frames_per_item(G.c) * d.F * d.K;
        }
        G.lane = 0;
        items.insert(items.end(), g.second.begin(), g.second.end());
        m->groups.push_back(G);
    }
    // lanes: largest group first onto the least loaded lane
    m->nlanes = std::min((int)m->groups.size(), isnmf_multi::LANES);
    {
        std::vector<int> order(m->groups.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return m->groups[x].cost > m->groups[y].cost; });
        double load[isnmf_multi::LANES] = {};
        for (const int gi : order) {
            int best = 0;
            for (int l = 1; l < m->nlanes; ++l)
                if (load[l] < load[best]) best = l;
            m->groups[gi].lane = best;
            load[best] += m->groups[gi].cost;
        }
    }
    // fold and rescale items per lane (each stream's fit group sits on one
    // lane), and within a lane streams to XCDs by their fold tiles x
    // components (the state they move)
    std::vector<int> lane_of(S, 0);
    for (const auto &G : m->groups)
        for (int i = 0; i < G.n; ++i) lane_of[items[G.off + i].x] = G.lane;
    for (int l = 0; l < m->nlanes; ++l) {
        std::vector<size_t> state(S, 0);
        for (int s = 0; s < S; ++s) {
            const OnlineDev &d = *isnmf_handle_dev(handles[s]);
            if (lane_of[s] == l) state[s] = (size_t)d.F * d.K;
        }
        const std::vector<int> xcd = xcd_assign(state);
        std::vector<int2> list;
        m->fold_off[l] = (int)items.size();
        for (int s = 0; s < S; ++s) {
            if (lane_of[s] != l || folded[s]) continue;
            const int nt = fold_tiles(*isnmf_handle_dev(handles[s]));
            m->fold_ktm[l] = std::max(m->fold_ktm[l], fold_ktm(isnmf_handle_dev(handles[s])->K));
            for (int t = 0; t < nt; ++t) list.push_back(int2{s, t});
        }
        push_xcd_ordered(items, list, xcd);
        m->fold_n[l] = (int)items.size() - m->fold_off[l];
        m->rs_off[l] = (int)items.size();
        list.clear();
        for (int s = 0; s < S; ++s) {
            if (lane_of[s] != l || rescaled[s]) continue;
            const int K = isnmf_handle_dev(handles[s])->K;
            for (int k = 0; k < K; ++k) list.push_back(int2{s, k});
        }
        push_xcd_ordered(items, list, xcd);
        m->rs_n[l] = (int)items.size() - m->rs_off[l];
    }

    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    auto cp = [&](void *dst, const void *src, size_t n) {
        if (e == hipSuccess) e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, st);
    };
    cp(m->d_fit, fit.data(), sizeof(FitDesc) * S);
    cp(m->d_fold, fold.data(), sizeof(FoldArgs) * S);
    cp(m->d_rs, rs.data(), sizeof(RescaleArgs) * S);
    cp(m->d_upd, upd.data(), sizeof(int) * S);
    cp(m->d_b, b, sizeof(int) * S);
    cp(m->d_cursor, zero.data(), sizeof(long long) * S);
    cp(m->d_nf, n_frames, sizeof(long long) * S);
    cp(m->d_items, items.data(), sizeof(int2) * items.size());
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // host vectors go out of scope
    if (m->nlanes > 1 && e == hipSuccess) {
        e = hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming);
        for (int i = 0; e == hipSuccess && i < m->nlanes - 1; ++i) {
            e = hipStreamCreateWithFlags(&m->side[i], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_join[i], hipEventDisableTiming);
        }
    }
    if (e != hipSuccess) {
        release_lanes(m);
        delete m;
        return ISNMF_EDEVICE;
    }
    *out = m;
    return ISNMF_OK;
}

int isnmf_multi_step(isnmf_multi *m, void *stream) {
    if (!m) return ISNMF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (enqueue_step(m, s) != hipSuccess) return ISNMF_EDEVICE;
    host_advance(m, s);
    m->last = s;
    return ISNMF_OK;
}

int isnmf_multi_run(isnmf_multi *m, int steps, int use_graph, void *stream) {
    if (!m || steps < 0) return ISNMF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph) {
        for (int i = 0; i < steps; ++i) {
            const int st = isnmf_multi_step(m, stream);
            if (st != ISNMF_OK) return st;
        }
        return ISNMF_OK;
    }
    if (!m->exec) {
        if (!m->cap && hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking) != hipSuccess)
            return ISNMF_EDEVICE;
        if (hipStreamBeginCapture(m->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return ISNMF_EDEVICE;
        const hipError_t e1 = enqueue_step(m, m->cap);
        const hipError_t e2 = hipStreamEndCapture(m->cap, &m->graph);
        if (e1 != hipSuccess || e2 != hipSuccess) return ISNMF_EDEVICE;
        if (hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0) != hipSuccess) {
            m->exec = nullptr;
            return ISNMF_EDEVICE;
        }
    }
    for (int i = 0; i < steps; ++i) {
        if (hipGraphLaunch(m->exec, s) != hipSuccess) return ISNMF_EDEVICE;
        host_advance(m, s);
    }
    m->last = s;
    return ISNMF_OK;
}

int isnmf_multi_frames_left(const isnmf_multi *m, long long *host_max_left) {
    if (!m || !host_max_left) return ISNMF_EINVAL;
    long long mx = 0;
    for (int i = 0; i < m->S; ++i) {
        const long long left = m->nframes[i] - m->cursor[i];
        if (left > mx) mx = left;
    }
    *host_max_left = mx;
    return ISNMF_OK;
}

int isnmf_multi_launches(const isnmf_multi *m, int *fit_launches, int *fold_launches,
                         int *rescale_launches) {
    if (!m || !fit_launches || !fold_launches || !rescale_launches) return ISNMF_EINVAL;
    *fit_launches = (int)m->groups.size();
    *fold_launches = 0;
    *rescale_launches = 0;
    for (int l = 0; l < m->nlanes; ++l) {
        *fold_launches += m->fold_n[l] > 0 ? 1 : 0;
        *rescale_launches += m->rs_n[l] > 0 ? 1 : 0;
    }
    return ISNMF_OK;
}

int isnmf_multi_destroy(isnmf_multi *m) {
    if (!m) return ISNMF_EINVAL;
    hipError_t e = hipStreamSynchronize(m->last);
    if (m->exec) hipGraphExecDestroy(m->exec);
    if (m->graph) hipGraphDestroy(m->graph);
    if (m->cap) hipStreamDestroy(m->cap);
    for (int i = 0; i < m->nlanes - 1; ++i)
        if (m->side[i] && hipStreamSynchronize(m->side[i]) != hipSuccess) e = hipErrorUnknown;
    release_lanes(m);
    delete m;
    return e == hipSuccess ? ISNMF_OK : ISNMF_EDEVICE;
}

// ----------------------------------------------------------------- autotuner

size_t isnmf_autotune_workspace_size(int F, int K, int b, const isnmf_params *pp) {
    isnmf_params p;
    isnmf_params_default(&p);
    if (pp) p = *pp;
    if (F < 1 || K < 1 || b < 1) return 0;
    const size_t ows = isnmf_online_workspace_size(F, K, b, &p);
    if (ows == 0) return 0;
    return ows + align256(sizeof(float) * (size_t)F * b) + align256(sizeof(float) * (size_t)F * K);
}

int isnmf_autotune(int F, int K, int b, const isnmf_params *pp, int trials, int *out_variant,
                   double *out_us, void *workspace, size_t ws_bytes, void *stream) {
    isnmf_params p;
    isnmf_params_default(&p);
    if (pp) p = *pp;
    if (F < 1 || K < 1 || b < 1 || trials < 1 || !workspace || ((uintptr_t)workspace & 255))
        return ISNMF_EINVAL;
    if (p.precision == ISNMF_FP64) return ISNMF_EUNSUPPORTED;
    const int prec = prec_of(p);
    FitClass cand[8];
    const int nc = fit_candidates(F, K, prec, cand, 8);
    if (nc == 0) return ISNMF_EUNSUPPORTED;
    if (ws_bytes < isnmf_autotune_workspace_size(F, K, b, &p)) return ISNMF_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    // a scratch stream state, synthetic frames and W(0), all in the caller's workspace
    const size_t wsz = isnmf_online_workspace_size(F, K, b, &p);
    void *ws = workspace;
    float *V = (float *)((char *)workspace + wsz);
    float *W0 = (float *)((char *)V + align256(sizeof(float) * (size_t)F * b));
    const long nv = (long)F * b, nw = (long)F * K;
    fill_kernel<<<(int)((nv + 255) / 256), 256, 0, s>>>(V, nv, 0.01f, 10.f, 7u);
    fill_kernel<<<(int)((nw + 255) / 256), 256, 0, s>>>(W0, nw, 0.5f, 1.f, 11u);
    isnmf_online *h = nullptr;
    int st = isnmf_online_init(&h, F, K, b, &p, W0, F, nullptr, nullptr, ws, wsz, stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best = -1;
    double best_us = 1e30;
    if (st == ISNMF_OK && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        const OnlineDev &d = *isnmf_handle_dev(h);
        for (int c = 0; c < nc && st == ISNMF_OK; ++c) {
            float ms = 0.f;
            hipError_t e = launch_fused_fit(d, cand[c], V, F, b, p.inner_iters, p.eps, 0, nullptr,
                                            K, prec, s);   // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int t = 0; t < trials && e == hipSuccess; ++t)
                e = launch_fused_fit(d, cand[c], V, F, b, p.inner_iters, p.eps, 0, nullptr, K, prec, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                st = ISNMF_EDEVICE;
                break;
            }
            const double us = 1e3 * ms / trials;
            if (us < best_us) {
                best_us = us;
                best = c;
            }
        }
    } else if (st == ISNMF_OK) {
        st = ISNMF_EDEVICE;
    }
    if (h) isnmf_online_destroy(h);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (hipStreamSynchronize(s) != hipSuccess && st == ISNMF_OK) st = ISNMF_EDEVICE;
    if (st != ISNMF_OK) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[{F, K, prec}] = cand[best];
    }
    if (out_variant) *out_variant = best;
    if (out_us) *out_us = best_us;
    return ISNMF_OK;
}

int isnmf_tune_get(int F, int K, int precision, int *nw, int *cpw, int *wg) {
    isnmf_params p;
    isnmf_params_default(&p);
    p.precision = precision;
    const FitClass c = tuned_class(F, K, prec_of(p), 0);
    if (!c.ok) return ISNMF_EUNSUPPORTED;
    if (nw) *nw = c.nw;
    if (cpw) *cpw = c.cpw;
    if (wg) *wg = c.wg;
    return ISNMF_OK;
}

int isnmf_tune_set(int F, int K, int precision, int nw, int cpw, int wg) {
    isnmf_params p;
    isnmf_params_default(&p);
    p.precision = precision;
    const int prec = prec_of(p);
    FitClass cand[8];
    const int nc = fit_candidates(F, K, prec, cand, 8);
    for (int c = 0; c < nc; ++c)
        if (cand[c].nw == nw && cand[c].cpw == cpw && cand[c].wg == wg) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[{F, K, prec}] = cand[c];
            return ISNMF_OK;
        }
    return ISNMF_EINVAL;
}

void isnmf_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

}  // extern "C"
