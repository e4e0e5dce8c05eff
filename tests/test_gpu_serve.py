"""Served form: continuous batching over many sessions.

Each session's chunks are applied in submission order whatever else shares
the engine's steps, so every session ends bitwise equal to the same session
stepped alone chunk by chunk.  Admission by HBM footprint and the latency
records are checked too.
"""
import sys

import numpy as np
import pytest

from paper_1106_4198_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1106_4198_amd import binding as bd  # noqa: E402

DEV = "cuda"


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def sessions(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        F = int(rng.choice([257, 513]))
        K = int(rng.choice([32, 64]))
        prec = ["bf16", "fp32", "fp16"][i % 3]
        nch = int(rng.integers(1, 5))
        lens = rng.integers(1, 65, size=nch)
        V, W0 = synth.problem(F, K, int(lens.sum()), seed=seed * 100 + i)
        Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
        chunks, o = [], 0
        for L in lens:
            chunks.append(Vt[o:o + int(L)])
            o += int(L)
        out.append((torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), prec, chunks))
    return out


def test_served_sessions_equal_alone_bitwise():
    S = 24
    data = sessions(S, seed=7)
    say(f"served vs alone, {S} sessions")
    alone = []
    for W0, prec, chunks in data:
        g = bd.OnlineISNMF(W0, 64, precision=prec)
        for c in chunks:
            g.step(c)
        alone.append(g)
    srv = bd.Server(max_sessions=S, max_per_step=S, max_frames=600, inflight=2)
    served = []
    for W0, prec, chunks in data:
        g = bd.OnlineISNMF(W0, 64, precision=prec)
        served.append((g, srv.open(g)))
    # interleave submissions across sessions, per-session order kept
    rng = np.random.default_rng(3)
    order = [i for i, (_, _, ch) in enumerate(data) for _ in ch]
    rng.shuffle(order)
    nxt = [0] * S
    for k, i in enumerate(order):
        srv.submit(served[i][1], data[i][2][nxt[i]])
        nxt[i] += 1
        if k % 5 == 0:
            srv.pump()
    srv.drain()
    res = srv.results()
    assert len(res["req"]) == len(order)
    assert np.all(res["done"] >= res["start"]) and np.all(res["start"] >= res["arrival"])
    steps, frames = srv.stats()
    assert frames == sum(int(c.shape[0]) for _, _, ch in data for c in ch)
    torch.cuda.synchronize()
    for i, (ga, (gs, _)) in enumerate(zip(alone, served)):
        Wa, Aa, Ba, ta = ga.get()
        Ws, As, Bs, ts = gs.get()
        assert ta == ts
        assert torch.equal(ga.get_w64(), gs.get_w64()), i
        assert torch.equal(Aa, As) and torch.equal(Ba, Bs), i
    srv.close()


def test_served_loss_equals_alone_bitwise():
    """Each session's running loss (isnmf_server_set_loss) is the same FP64
    bits as the session stepped alone with loss_sum, chunk by chunk; a
    session without a target leaves the others' sums alone."""
    S = 12
    data = sessions(S, seed=21)
    say(f"served loss vs alone, {S} sessions")
    loss_alone = []
    for W0, prec, chunks in data:
        g = bd.OnlineISNMF(W0, 64, precision=prec)
        ls = torch.zeros((), dtype=torch.float64, device=DEV)
        for c in chunks:
            g.step(c, None, ls)
        loss_alone.append(ls)
    srv = bd.Server(max_sessions=S, max_per_step=S, max_frames=600, inflight=2)
    losses = torch.zeros(S, dtype=torch.float64, device=DEV)
    ids = []
    for i, (W0, prec, chunks) in enumerate(data):
        g = bd.OnlineISNMF(W0, 64, precision=prec)
        ids.append((g, srv.open(g)))
        if i != 3:                      # session 3 keeps no running loss
            srv.set_loss(ids[-1][1], losses[i:i + 1])
    rng = np.random.default_rng(5)
    order = [i for i, (_, _, ch) in enumerate(data) for _ in ch]
    rng.shuffle(order)
    nxt = [0] * S
    for k, i in enumerate(order):
        srv.submit(ids[i][1], data[i][2][nxt[i]])
        nxt[i] += 1
        if k % 4 == 0:
            srv.pump()
    srv.drain()
    torch.cuda.synchronize()
    for i in range(S):
        if i == 3:
            assert losses[i].item() == 0.0
        else:
            assert loss_alone[i].item() > 0.0
            assert torch.equal(losses[i], loss_alone[i]), (i, losses[i].item(), loss_alone[i].item())
    with pytest.raises(bd.IsnmfError):
        srv.set_loss(S + 5, losses[0:1])
    srv.close()


def test_admission_by_hbm_footprint():
    """A session whose footprint alone exceeds the budget is refused; one that
    does not fit beside the resident ones waits, and is admitted when a
    resident session closes."""
    say("admission")
    W0 = torch.rand((32, 257), device=DEV) + 0.5
    g1 = bd.OnlineISNMF(W0, 64, precision="bf16")
    g2 = bd.OnlineISNMF(W0, 64, precision="bf16")
    fp = g1.workspace.numel()
    srv = bd.Server(max_sessions=4, max_per_step=4, max_frames=256, hbm_budget=fp + fp // 2)
    s1 = srv.open(g1)
    s2 = srv.open(g2)
    assert srv.state(s1) == srv.RESIDENT and srv.state(s2) == srv.WAITING
    assert srv.admission() == (fp, 1, 1)
    with pytest.raises(bd.IsnmfError) as ei:
        srv.open(bd.OnlineISNMF(W0, 64, precision="bf16"), footprint=2 * fp)
    assert ei.value.code == bd.ENOMEM
    with pytest.raises(bd.IsnmfError) as ei:
        srv.open(g1)                       # already open
    assert ei.value.code == bd.EINVAL
    with pytest.raises(bd.IsnmfError):
        srv.submit(s1, torch.rand((300, 257), device=DEV))   # above max_frames
    srv.close_session(s1)                  # idle: released at once, s2 admitted
    assert srv.state(s1) == srv.CLOSED and srv.state(s2) == srv.RESIDENT
    assert srv.admission() == (fp, 1, 0)
    with pytest.raises(bd.IsnmfError) as ei:
        srv.submit(s1, torch.rand((8, 257), device=DEV))
    assert ei.value.code == bd.ESTATE
    srv.close()


def _admission_mix(budget_sessions, S, seed, max_sessions):
    data = sessions(S, seed=seed)
    alone = []
    for W0, prec, chunks in data:
        g = bd.OnlineISNMF(W0, 64, precision=prec)
        ls = torch.zeros((), dtype=torch.float64, device=DEV)
        for c in chunks:
            g.step(c, None, ls)
        alone.append((g, ls))
    fp = max(bd.OnlineISNMF(W0, 64, precision=prec).workspace.numel() for W0, prec, _ in data)
    budget = budget_sessions * fp
    srv = bd.Server(max_sessions=max_sessions, max_per_step=S, max_frames=600, inflight=2,
                    hbm_budget=budget)
    served, losses = [], torch.zeros(S, dtype=torch.float64, device=DEV)
    for i, (W0, prec, chunks) in enumerate(data):
        g = bd.OnlineISNMF(W0, 64, precision=prec)
        sid = srv.open(g, footprint=fp)
        srv.set_loss(sid, losses[i:i + 1])
        served.append((g, sid))
    assert srv.admission()[1] == min(budget_sessions, max_sessions)
    assert srv.admission()[2] == S - min(budget_sessions, max_sessions)
    # every chunk submitted up front; each session closed after its last chunk
    rng = np.random.default_rng(seed + 1)
    order = [i for i, (_, _, ch) in enumerate(data) for _ in ch]
    rng.shuffle(order)
    nxt = [0] * S
    peak = 0
    for k, i in enumerate(order):
        srv.submit(served[i][1], data[i][2][nxt[i]])
        nxt[i] += 1
        if nxt[i] == len(data[i][2]):
            srv.close_session(served[i][1])
        if k % 3 == 0:
            srv.pump()
        used, res, _ = srv.admission()
        assert used <= budget and res <= max_sessions
        peak = max(peak, res)
    srv.drain()
    assert all(srv.state(sid) == srv.CLOSED for _, sid in served)
    assert srv.admission() == (0, 0, 0)
    res = srv.results()
    assert len(res["req"]) == len(order)
    torch.cuda.synchronize()
    for i, ((ga, la), (gs, _)) in enumerate(zip(alone, served)):
        _, Aa, Ba, ta = ga.get()
        _, As, Bs, ts = gs.get()
        assert ta == ts
        assert torch.equal(ga.get_w64(), gs.get_w64()), i
        assert torch.equal(Aa, As) and torch.equal(Ba, Bs), i
        assert torch.equal(losses[i], la), i
    srv.close()
    return peak


@pytest.mark.parametrize("budget_sessions,max_sessions", [(2, 16), (5, 3)])
def test_admission_queue_serves_every_session_bitwise(budget_sessions, max_sessions):
    """A budget (or a table) smaller than the sessions forces queueing: sessions
    wait in order, are admitted as others close, and each ends bitwise equal to
    the same session stepped alone, running loss included."""
    say(f"admission queue: budget {budget_sessions} sessions, {max_sessions} rows")
    peak = _admission_mix(budget_sessions, 14, seed=41 + budget_sessions, max_sessions=max_sessions)
    assert peak <= min(budget_sessions, max_sessions)


def test_drain_reports_sessions_that_cannot_be_admitted():
    """With the budget held by an open, idle session, a waiting session's
    chunks cannot run: drain says so instead of spinning, and serves them once
    the holder closes."""
    say("drain with a blocked queue")
    W0 = torch.rand((32, 257), device=DEV) + 0.5
    g1 = bd.OnlineISNMF(W0, 64, precision="bf16")
    g2 = bd.OnlineISNMF(W0, 64, precision="bf16")
    fp = g1.workspace.numel()
    srv = bd.Server(max_sessions=4, max_per_step=4, max_frames=256, hbm_budget=fp)
    s1, s2 = srv.open(g1), srv.open(g2)
    V = torch.rand((16, 257), device=DEV) + 0.1
    srv.submit(s2, V)
    with pytest.raises(bd.IsnmfError) as ei:
        srv.drain()
    assert ei.value.code == bd.ESTATE
    srv.close_session(s1)
    srv.drain()
    assert srv.state(s2) == srv.RESIDENT
    assert len(srv.results()["req"]) == 1
    srv.close()


def test_server_keeps_chunks_and_loss_targets_alive():
    """The binding keeps submitted frames and running-loss targets alive on
    its own (by request id and by session id, separately): with the caller's
    references dropped and set_loss interleaved with submits, every session
    still ends bitwise equal to the session stepped alone."""
    say("server keep-alive")
    S = 6
    data = sessions(S, seed=77)
    alone = []
    for W0, prec, chunks in data:
        g = bd.OnlineISNMF(W0, 64, precision=prec)
        ls = torch.zeros((), dtype=torch.float64, device=DEV)
        for c in chunks:
            g.step(c, None, ls)
        alone.append((g, ls.item()))
    srv = bd.Server(max_sessions=S, max_per_step=S, max_frames=600, inflight=2)
    served = []
    for W0, prec, _ in data:
        g = bd.OnlineISNMF(W0, 64, precision=prec)
        served.append((g, srv.open(g)))
    order = [i for i, (_, _, ch) in enumerate(data) for _ in ch]
    nxt = [0] * S
    for k, i in enumerate(order):
        srv.submit(served[i][1], data[i][2][nxt[i]].clone())   # caller keeps no reference
        nxt[i] += 1
        if nxt[i] == 1:
            srv.set_loss(served[i][1], torch.zeros((1,), dtype=torch.float64, device=DEV))
    data = None
    import gc
    gc.collect()
    for _ in range(4):                       # churn the caching allocator
        torch.rand((1 << 20,), device=DEV).mul_(2.0)
    srv.drain()
    torch.cuda.synchronize()
    for i, ((ga, la), (gs, sid)) in enumerate(zip(alone, served)):
        assert torch.equal(ga.get_w64(), gs.get_w64()), i
        assert srv._loss[sid].item() == la, i
    srv.close()


def test_served_form_runs_the_valu_variant_at_wide_f():
    """At F = 1025 no FP32 MFMA tile holds W, so FP32 handles fit on the VALU
    variant by default (BF16 handles here by a tuning entry); the served form
    runs them on its kernel of its own (one workgroup per frame) and gives
    the bits of the sessions alone."""
    say("serve VALU at F = 1025")
    bd.tune_clear()
    bd.tune_set(1025, 40, "bf16", 8, -4, 0)
    W0 = torch.rand((40, 1025), device=DEV) + 0.5
    V = torch.rand((200, 1025), device=DEV) + 1e-3
    for prec in ("fp32", "bf16"):
        ga = bd.OnlineISNMF(W0, 128, precision=prec)
        assert bd.tune_get(1025, 40, prec)[1] == (0 if prec == "fp32" else -4)
        ga.step(V[:120])
        ga.step(V[120:])
        gs = bd.OnlineISNMF(W0, 128, precision=prec)
        srv = bd.Server(max_sessions=2, max_per_step=2, max_frames=256)
        sid = srv.open(gs)
        srv.submit(sid, V[:120])
        srv.submit(sid, V[120:])
        srv.drain()
        torch.cuda.synchronize()
        assert torch.equal(ga.get_w64(), gs.get_w64()), prec
        srv.close()
    bd.tune_clear()


@pytest.mark.parametrize("cpw", [-1, -2])
def test_served_tile_sessions_equal_alone_bitwise(cpw):
    """BF16 sessions on a 16-frame tile variant (W resident in LDS or streamed
    through it; chunks of 1..300 frames, several 128-frame tiles) are served
    bitwise as they run alone."""
    say(f"served tile sessions vs alone, cpw {cpw}")
    bd.tune_clear()
    for F, K in ((257, 32), (513, 64), (513, 32)):
        bd.tune_set(F, K, "bf16", 8, cpw, 0)
    try:
        rng = np.random.default_rng(11)
        data = []
        for i in range(9):
            F, K = [(257, 32), (513, 64), (513, 32)][i % 3]
            lens = rng.integers(1, 301, size=3)
            V, W0 = synth.problem(F, K, int(lens.sum()), seed=1100 + i)
            Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
            chunks, o = [], 0
            for L in lens:
                chunks.append(Vt[o:o + int(L)])
                o += int(L)
            data.append((torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), chunks))
        alone = []
        for W0, chunks in data:
            g = bd.OnlineISNMF(W0, 300, precision="bf16")
            for c in chunks:
                g.step(c)
            alone.append(g)
        srv = bd.Server(max_sessions=9, max_per_step=9, max_frames=2700, inflight=2)
        served = []
        for W0, chunks in data:
            g = bd.OnlineISNMF(W0, 300, precision="bf16")
            served.append((g, srv.open(g)))
        for k in range(3):
            for i in range(len(data)):
                srv.submit(served[i][1], data[i][1][k])
            srv.pump()
        srv.drain()
        torch.cuda.synchronize()
        for i, (ga, (gs, _)) in enumerate(zip(alone, served)):
            Wa, Aa, Ba, ta = ga.get()
            Ws, As, Bs, ts = gs.get()
            assert ta == ts
            assert torch.equal(ga.get_w64(), gs.get_w64()), i
            assert torch.equal(Aa, As) and torch.equal(Ba, Bs), i
        srv.close()
    finally:
        bd.tune_clear()


@pytest.mark.parametrize("precision,cpw", [("fp32", -3), ("fp32", 0), ("bf16", -4), ("fp32", None)])
def test_served_own_kernel_sessions_equal_alone_bitwise(precision, cpw):
    """Sessions on the variants with served kernels of their own (the FP32
    16-frame tile, and the VALU variant in FP32 and BF16: one workgroup per
    frame; cpw None: the VALU variant's 16-wave form, the FP32 default past
    F = 1088) give the bits of the same sessions run alone."""
    say(f"served {precision} cpw={cpw}")
    bd.tune_clear()
    shapes = [(513, 64), (257, 32)] if cpw is not None else [(1100, 64), (1130, 32)]
    for F, K in shapes:
        if cpw is not None:
            bd.tune_set(F, K, precision, 8, cpw, 0)
        else:
            assert bd.tune_get(F, K, precision) == (16, 0, 0)
    try:
        rng = np.random.default_rng(9)
        data = []
        for i in range(6):
            F, K = shapes[i % 2]
            lens = rng.integers(1, 300, size=3)
            V, W0 = synth.problem(F, K, int(lens.sum()), seed=700 + i)
            Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
            o, chunks = 0, []
            for L in lens:
                chunks.append(Vt[o:o + int(L)])
                o += int(L)
            data.append((torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), chunks))
        alone = []
        for W0, chunks in data:
            g = bd.OnlineISNMF(W0, 512, precision=precision)
            for c in chunks:
                g.step(c)
            alone.append(g)
        srv = bd.Server(max_sessions=6, max_per_step=6, max_frames=4096, inflight=2)
        served = []
        for W0, _ in data:
            g = bd.OnlineISNMF(W0, 512, precision=precision)
            served.append((g, srv.open(g)))
        for k in range(3):
            for i, (_, chunks) in enumerate(data):
                srv.submit(served[i][1], chunks[k])
            srv.pump()
        srv.drain()
        torch.cuda.synchronize()
        for i, (ga, (gs, _)) in enumerate(zip(alone, served)):
            assert torch.equal(ga.get_w64(), gs.get_w64()), i
            _, Aa, Ba, _ = ga.get()
            _, As, Bs, _ = gs.get()
            assert torch.equal(Aa, As) and torch.equal(Ba, Bs), i
        srv.close()
    finally:
        bd.tune_clear()
