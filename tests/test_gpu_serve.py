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
    say("admission")
    W0 = torch.rand((32, 257), device=DEV) + 0.5
    g1 = bd.OnlineISNMF(W0, 64, precision="bf16")
    g2 = bd.OnlineISNMF(W0, 64, precision="bf16")
    fp = g1.workspace.numel()
    srv = bd.Server(max_sessions=4, max_per_step=4, max_frames=256, hbm_budget=fp + fp // 2)
    srv.open(g1)
    with pytest.raises(bd.IsnmfError) as ei:
        srv.open(g2)
    assert ei.value.code == bd.ENOMEM
    with pytest.raises(bd.IsnmfError):
        srv.submit(0, torch.rand((300, 257), device=DEV))   # above max_frames
    srv.close()


def test_served_form_rejects_the_valu_variant():
    """The served form runs MFMA tile variants only; a handle whose fit is the
    one-frame-per-workgroup VALU variant is refused, not silently rerouted."""
    say("serve rejects VALU")
    W0 = torch.rand((40, 1025), device=DEV) + 0.5
    g = bd.OnlineISNMF(W0, 16)   # FP32, F = 1025: the VALU variant
    srv = bd.Server(max_sessions=2, max_per_step=2, max_frames=64)
    with pytest.raises(bd.IsnmfError) as ei:
        srv.open(g)
    assert ei.value.code == bd.EUNSUPPORTED
    srv.close()


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
