"""Batched form: many streams of uneven F, K, b in shared launches.

A stream's result must not depend on which other streams share its launches:
each stream of a mixed batch is compared bitwise with the same stream run
alone through isnmf_online_step (same kernel variant, fixed-order sums).
The hipGraph replay is checked against eager execution after every replay.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1106_4198_amd import synth
from tests.helpers import from_gpu_kf, rel_fro

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1106_4198_amd import binding as bd  # noqa: E402

DEV = "cuda"

# (F, K, b, precision, frames)
MIX = [(257, 16, 32, "bf16", 160), (513, 50, 64, "bf16", 256), (1025, 40, 32, "bf16", 96),
       (1025, 100, 16, "bf16", 64), (513, 128, 32, "fp16", 80), (257, 64, 128, "fp32", 384),
       (129, 8, 4, "fp32", 14), (513, 50, 128, "fp32", 200)]


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def inputs(seed0=300):
    out = []
    for i, (F, K, b, prec, N) in enumerate(MIX):
        V, W0 = synth.problem(F, K, N, seed=seed0 + i)
        out.append((torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV),
                    torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV), b, prec))
    return out


def handles(data):
    return [bd.OnlineISNMF(W0, b, precision=prec) for (W0, V, b, prec) in data]


def state(g):
    W, A, B, t = g.get()
    return g.get_w64(), A, B, t


def test_batched_equals_alone_bitwise():
    data = inputs()
    steps = 4
    say("batched vs alone, %d streams, %d steps" % (len(data), steps))
    alone = handles(data)
    loss_alone = []
    for g, (W0, V, b, prec) in zip(alone, data):
        ls = torch.zeros((), dtype=torch.float64, device=DEV)
        for s in range(steps):
            lo, hi = s * b, min((s + 1) * b, V.shape[0])
            if lo < hi:
                g.step(V[lo:hi], None, ls)
        loss_alone.append(ls)
    mixed = handles(data)
    m = bd.MultiISNMF(mixed, [d[1] for d in data], [d[2] for d in data])
    m.run(steps, graph=False)
    torch.cuda.synchronize()
    for i, (ga, gm) in enumerate(zip(alone, mixed)):
        sa, sm = state(ga), state(gm)
        assert sa[3] == sm[3], (i, sa[3], sm[3])
        for x, y in zip(sa[:3], sm[:3]):
            assert torch.equal(x, y), f"stream {i} {MIX[i]} differs alone vs batched"
        assert torch.equal(loss_alone[i], m.loss[i]), i
    assert m.frames_left() == max(0, max(N - steps * b for (_, _, b, _, N) in MIX))
    m.close()


def test_streams_that_run_out_keep_their_state():
    """Steps past a stream's last frame leave its W, A, B (and the column
    scale still pending on A and B) untouched while the others go on."""
    data = inputs(seed0=350)
    steps = 12
    say("streams running out, %d steps" % steps)
    alone = handles(data)
    for g, (W0, V, b, prec) in zip(alone, data):
        for s in range(steps):
            lo, hi = s * b, min((s + 1) * b, V.shape[0])
            if lo < hi:
                g.step(V[lo:hi])
    mixed = handles(data)
    m = bd.MultiISNMF(mixed, [d[1] for d in data], [d[2] for d in data], loss=False)
    m.run(steps, graph=True)
    torch.cuda.synchronize()
    assert m.frames_left() == 0
    for i, (ga, gm) in enumerate(zip(alone, mixed)):
        sa, sm = state(ga), state(gm)
        assert sa[3] == sm[3] == MIX[i][4], (i, sa[3], sm[3])
        for x, y in zip(sa[:3], sm[:3]):
            assert torch.equal(x, y), f"stream {i} {MIX[i]} differs after running out"
    m.close()


def test_graph_replays_match_eager_every_step():
    data = inputs(seed0=400)
    say("graph replay vs eager")
    ge, gg = handles(data), handles(data)
    me = bd.MultiISNMF(ge, [d[1] for d in data], [d[2] for d in data])
    mg = bd.MultiISNMF(gg, [d[1] for d in data], [d[2] for d in data])
    for step in range(6):
        mg.run(1, graph=True)
        torch.cuda.synchronize()
        me.run(1, graph=False)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(ge, gg)):
            sa, sb = state(a), state(b)
            assert sa[3] == sb[3]
            for x, y in zip(sa[:3], sb[:3]):
                assert torch.equal(x, y), f"replay {step} stream {i}"
        assert torch.equal(me.loss, mg.loss)
    me.close()
    mg.close()


def test_batched_streams_match_oracle():
    """Two streams of the mix against the FP64 oracle: FP32 at 1e-5, BF16 at
    the precision-form bound (2e-2 on W, A, B; 1e-3 on the loss)."""
    data = inputs(seed0=500)
    steps = 3
    say("batched vs oracle")
    hs = handles(data)
    m = bd.MultiISNMF(hs, [d[1] for d in data], [d[2] for d in data])
    m.run(steps, graph=True)
    torch.cuda.synchronize()
    for i, tol in ((5, 1e-5), (1, 2e-2), (3, 2e-2)):
        F, K, b, prec, N = MIX[i]
        W0 = data[i][0].cpu().double().numpy().T
        V = data[i][1].cpu().double().numpy().T
        st = oracle.OnlineState(W0)
        for s in range(steps):
            st.step(V[:, s * b:min((s + 1) * b, N)], iters=20)
        W64, A, B, t = state(hs[i])
        assert t == min(N, steps * b)
        for x, y, nm in ((from_gpu_kf(W64), st.W, "W"), (from_gpu_kf(A), st.A, "A"),
                         (from_gpu_kf(B), st.B, "B")):
            e = rel_fro(x, y)
            print(f"[batched] stream {i} {MIX[i]} {nm} rel {e:.2e}")
            assert e <= tol
        assert abs(m.loss[i].item() - st.loss_sum) <= 1e-3 * st.loss_sum
    m.close()


def test_autotune_picks_a_valid_variant_and_keeps_parity():
    say("autotune")
    bd.tune_clear()
    for F, K, prec in ((513, 50, "bf16"), (1025, 40, "bf16")):
        v, us = bd.autotune(F, K, 64, precision=prec, trials=3)
        nw, cpw, wg = bd.tune_get(F, K, prec)
        print(f"[autotune] F={F} K={K} {prec}: variant {v} nw={nw} cpw={cpw} wg={wg} {us:.1f} us")
        # an MFMA tile variant's waves x chunks cover the rows; the VALU (0, -4)
        # and 16-frame tile (-1, -2, -3) variants cover any F they are offered for
        assert us > 0 and (cpw <= 0 or nw * cpw * 64 >= (F // 64) * 64)
        V, W0 = synth.problem(F, K, 64, seed=7)
        g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), 64, precision=prec)
        g.step(torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV))
        st = oracle.OnlineState(W0.astype(np.float64))
        st.step(V.astype(np.float64), iters=20)
        assert rel_fro(from_gpu_kf(g.get_w64()), st.W) < 2e-2
    bd.tune_clear()


def test_batched_valu_streams_equal_alone_bitwise():
    """FP32 streams on the VALU fit variant (tuned, and by default for F = 1025)
    share launches with MFMA-tile streams and match their runs alone."""
    mix = [(513, 50, 128, "fp32", 300), (257, 64, 16, "fp32", 70), (1025, 40, 32, "fp32", 90),
           (513, 50, 64, "bf16", 200), (129, 8, 4, "fp32", 14)]
    say("batched VALU vs alone")
    bd.tune_clear()
    bd.tune_set(513, 50, "fp32", 8, 0, 0)
    bd.tune_set(257, 64, "fp32", 8, 0, 0)
    try:
        data = []
        for i, (F, K, b, prec, N) in enumerate(mix):
            V, W0 = synth.problem(F, K, N, seed=700 + i)
            data.append((torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV),
                         torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV), b, prec))
        steps = 3
        alone = handles(data)
        for g, (W0, V, b, prec) in zip(alone, data):
            for s in range(steps):
                lo, hi = s * b, min((s + 1) * b, V.shape[0])
                if lo < hi:
                    g.step(V[lo:hi])
        mixed = handles(data)
        m = bd.MultiISNMF(mixed, [d[1] for d in data], [d[2] for d in data])
        m.run(steps, graph=True)
        torch.cuda.synchronize()
        for i, (ga, gm) in enumerate(zip(alone, mixed)):
            sa, sm = state(ga), state(gm)
            assert sa[3] == sm[3], i
            for x, y in zip(sa[:3], sm[:3]):
                assert torch.equal(x, y), f"stream {i} {mix[i]} differs alone vs batched"
        # and one of them against the oracle
        W0 = data[0][0].cpu().double().numpy().T
        V = data[0][1].cpu().double().numpy().T
        st = oracle.OnlineState(W0)
        for s in range(steps):
            st.step(V[:, s * 128:(s + 1) * 128], iters=20)
        assert rel_fro(from_gpu_kf(state(mixed[0])[0]), st.W) <= 1e-5
        m.close()
    finally:
        bd.tune_clear()


def test_autotune_offers_the_valu_variant_for_fp32():
    say("autotune fp32")
    bd.tune_clear()
    v, us = bd.autotune(513, 50, 128, precision="fp32", trials=3)
    got = bd.tune_get(513, 50, "fp32")
    print(f"[autotune] F=513 K=50 fp32: variant {v} {got} {us:.1f} us")
    assert v in (0, 1) and (got == (8, 0, 0)) == (v == 1)
    bd.tune_clear()


TILE_FOLD_MIX = [(513, 50, 128, "bf16", 300), (257, 64, 40, "bf16", 100), (129, 8, 16, "bf16", 40),
                 (200, 33, 37, "bf16", 100), (608, 64, 128, "bf16", 260), (64, 1, 5, "bf16", 12),
                 (33, 20, 100, "bf16", 250)]
# FP32 16-frame tile streams: K splits into 1..4 matrix-pipe m-tiles and 0..4
# VALU remainder components (K = 50: 3 + 2, 33: 2 + 1, 20: 1 + 4), F up to the
# LDS bound of the folding pass at K = 64 (400 rows), ragged minibatches
T32_FOLD_MIX = [(513, 50, 128, "fp32", 300), (257, 48, 40, "fp32", 100), (129, 8, 16, "fp32", 40),
                (200, 33, 37, "fp32", 100), (400, 64, 128, "fp32", 260), (64, 1, 5, "fp32", 12),
                (33, 20, 100, "fp32", 250)]


@pytest.mark.parametrize("mixname", ["shared_fold", "bf16_fold_in_fit", "fp32_fold_in_fit"])
def test_batched_tile_streams_equal_alone_bitwise(mixname):
    """Streams on the 16-frame tile variants (ragged minibatches included)
    match their runs alone.  Mixed with other variants, they share the step's
    fold launch; alone in the step with at most 128 frames each, every fit
    launch folds its streams itself (no fold launch), while alone they run the
    separate fold: W, A, B and the running loss must agree bit for bit either
    way.  The fold-in-fit sets have an idle fold wave (K = 33), K = 1, row
    tiles past F (F = 200, 33), the largest F the LDS allows and b = 5."""
    fold_in_fit = mixname != "shared_fold"
    if mixname == "bf16_fold_in_fit":
        mix = TILE_FOLD_MIX
    elif mixname == "fp32_fold_in_fit":
        mix = T32_FOLD_MIX
    else:
        mix = [(513, 50, 128, "bf16", 300), (257, 64, 40, "bf16", 100), (129, 8, 16, "bf16", 40),
               (513, 50, 64, "fp32", 200), (1025, 40, 32, "bf16", 90), (200, 33, 37, "bf16", 100),
               (513, 50, 256, "bf16", 600)]
    say(f"batched tile vs alone, {mixname}")
    bd.tune_clear()
    for F, K, _, prec, _ in mix:
        if prec == "bf16" and F <= 640 and K <= 64:
            bd.tune_set(F, K, "bf16", 8, -1, 0)
        if prec == "fp32" and fold_in_fit:
            bd.tune_set(F, K, "fp32", 8, -3, 0)
    try:
        data = []
        for i, (F, K, b, prec, N) in enumerate(mix):
            V, W0 = synth.problem(F, K, N, seed=800 + i)
            data.append((torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV),
                         torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV), b, prec))
        steps = 3
        alone = handles(data)
        loss_alone = []
        for g, (W0, V, b, prec) in zip(alone, data):
            ls = torch.zeros((), dtype=torch.float64, device=DEV)
            for s in range(steps):
                lo, hi = s * b, min((s + 1) * b, V.shape[0])
                if lo < hi:
                    g.step(V[lo:hi], None, ls)
            loss_alone.append(ls)
        mixed = handles(data)
        m = bd.MultiISNMF(mixed, [d[1] for d in data], [d[2] for d in data])
        fits, folds, rescales = m.launches()
        assert folds == 0 if fold_in_fit else 1 <= folds <= min(fits, 4)
        # one rescale per lane (at most four), none where the BF16 tile fits rescale
        assert rescales == {"shared_fold": folds, "bf16_fold_in_fit": 0,
                            "fp32_fold_in_fit": min(fits, 4)}[mixname]
        m.run(1, graph=False)
        m.run(steps - 1, graph=True)
        torch.cuda.synchronize()
        for i, (ga, gm) in enumerate(zip(alone, mixed)):
            sa, sm = state(ga), state(gm)
            assert sa[3] == sm[3], i
            for x, y in zip(sa[:3], sm[:3]):
                assert torch.equal(x, y), f"stream {i} {mix[i]} differs alone vs batched"
            assert torch.equal(loss_alone[i], m.loss[i]), f"stream {i} loss differs"
        W0 = data[0][0].cpu().double().numpy().T
        V = data[0][1].cpu().double().numpy().T
        st = oracle.OnlineState(W0)
        for s in range(steps):
            st.step(V[:, s * 128:(s + 1) * 128], iters=20)
        assert rel_fro(from_gpu_kf(state(mixed[0])[0]), st.W) <= (1e-5 if mix[0][3] == "fp32" else 2e-2)
        m.close()
    finally:
        bd.tune_clear()


def test_batched_streamed_tile_streams_equal_alone_bitwise():
    """BF16 streams of different F and K on the streamed 16-frame tile variant
    share one launch per component class (the variant does not depend on F),
    beside streams on other variants, and match their runs alone."""
    mix = [(513, 50, 128, "bf16", 300), (1025, 100, 64, "bf16", 150), (1025, 40, 32, "bf16", 90),
           (257, 64, 40, "bf16", 100), (700, 128, 16, "bf16", 40), (513, 50, 64, "fp32", 200),
           (129, 8, 16, "bf16", 40)]
    say("batched streamed tile vs alone")
    bd.tune_clear()
    for (F, K, b, prec, N) in mix[:5]:
        bd.tune_set(F, K, "bf16", 8, -2, 0)
    try:
        data = []
        for i, (F, K, b, prec, N) in enumerate(mix):
            V, W0 = synth.problem(F, K, N, seed=850 + i)
            data.append((torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV),
                         torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV), b, prec))
        steps = 3
        alone = handles(data)
        for g, (W0, V, b, prec) in zip(alone, data):
            for s in range(steps):
                lo, hi = s * b, min((s + 1) * b, V.shape[0])
                if lo < hi:
                    g.step(V[lo:hi])
        mixed = handles(data)
        m = bd.MultiISNMF(mixed, [d[1] for d in data], [d[2] for d in data])
        m.run(steps, graph=True)
        torch.cuda.synchronize()
        for i, (ga, gm) in enumerate(zip(alone, mixed)):
            sa, sm = state(ga), state(gm)
            assert sa[3] == sm[3], i
            for x, y in zip(sa[:3], sm[:3]):
                assert torch.equal(x, y), f"stream {i} {mix[i]} differs alone vs batched"
        W0 = data[1][0].cpu().double().numpy().T
        V = data[1][1].cpu().double().numpy().T
        st = oracle.OnlineState(W0)
        for s in range(steps):
            st.step(V[:, s * 64:(s + 1) * 64], iters=20)
        assert rel_fro(from_gpu_kf(state(mixed[1])[0]), st.W) <= 2e-2
        m.close()
    finally:
        bd.tune_clear()


@pytest.mark.parametrize("precision,cpw", [("fp32", -3), ("fp32", 0), ("bf16", -4)])
def test_fp32_tile_and_valu_batched_equal_alone_bitwise(precision, cpw):
    """The FP32 16-frame tile variant (cpw -3) and the VALU variant in FP32 (0)
    and BF16 (-4) in the batched form: streams of one shape and of mixed
    shapes (several groups of the variant, ragged last minibatches) give the
    bits of the same streams run alone."""
    shapes = [(513, 50, 128, 300), (513, 50, 128, 256), (257, 64, 64, 200), (129, 8, 200, 390),
              (592, 64, 33, 70), (1025, 32, 128, 130)]
    if cpw == 0:   # and the 16-wave form past F = 1088 (the default there)
        shapes += [(1100, 40, 64, 130), (1152, 64, 17, 40)]
    say(f"{precision} cpw={cpw} batched vs alone")
    bd.tune_clear()
    for F, K, _, _ in shapes:
        if F <= 1088:
            bd.tune_set(F, K, precision, 8, cpw, 0)
    try:
        data = []
        for i, (F, K, b, N) in enumerate(shapes):
            V, W0 = synth.problem(F, K, N, seed=500 + i)
            data.append((torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV),
                         torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV), b))
        steps = 3
        alone, loss_alone = [], []
        for W0, V, b in data:
            g = bd.OnlineISNMF(W0, b, precision=precision)
            ls = torch.zeros((), dtype=torch.float64, device=DEV)
            for s in range(steps):
                lo, hi = s * b, min((s + 1) * b, V.shape[0])
                if lo < hi:
                    g.step(V[lo:hi], None, ls)
            alone.append(g)
            loss_alone.append(ls)
        mixed = [bd.OnlineISNMF(W0, b, precision=precision) for W0, _, b in data]
        m = bd.MultiISNMF(mixed, [d[1] for d in data], [d[2] for d in data])
        m.run(1, graph=False)
        m.run(steps - 1, graph=True)
        torch.cuda.synchronize()
        for i, (ga, gm) in enumerate(zip(alone, mixed)):
            sa, sm = state(ga), state(gm)
            assert sa[3] == sm[3], i
            for x, y in zip(sa[:3], sm[:3]):
                assert torch.equal(x, y), f"stream {i} {shapes[i]} differs alone vs batched"
            assert torch.equal(loss_alone[i], m.loss[i]), i
        m.close()
    finally:
        bd.tune_clear()


@pytest.mark.parametrize("precision,cpw", [("bf16", -1), ("fp32", -3)])
def test_fold_in_fit_with_step_options_equal_alone_bitwise(precision, cpw):
    """A plan whose fit launches fold (every stream on a 16-frame tile variant,
    b <= 128) with the step's options varied per stream: forgetting rho < 1,
    W frozen (update_w off: A and B still fold, no W update), no column
    rescale, eps = 0.  Each stream matches the same stream stepped alone (the
    separate fold), W, A, B, t and the running loss bit for bit."""
    opts = [dict(rho=0.7), dict(update_w=False), dict(normalize=False), dict(eps=0.0),
            dict(rho=0.5, normalize=False)]
    shapes = [(257, 40, 128, 300), (129, 8, 64, 200), (200, 33, 100, 250), (513, 50, 37, 100),
              (65, 16, 128, 260)]
    say(f"fold in fit with options, {precision}")
    bd.tune_clear()
    for F, K, _, _ in shapes:
        bd.tune_set(F, K, precision, 8, cpw, 0)
    try:
        data = []
        for i, (F, K, b, N) in enumerate(shapes):
            V, W0 = synth.problem(F, K, N, seed=900 + i)
            data.append((torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV),
                         torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV), b))

        def make():
            return [bd.OnlineISNMF(W0, b, precision=precision, **o) for (W0, _, b), o in zip(data, opts)]

        steps = 3
        alone, loss_alone = make(), []
        for g, (W0, V, b) in zip(alone, data):
            ls = torch.zeros((), dtype=torch.float64, device=DEV)
            for s in range(steps):
                g.step(V[s * b:(s + 1) * b], None, ls)
            loss_alone.append(ls)
        mixed = make()
        m = bd.MultiISNMF(mixed, [d[1] for d in data], [d[2] for d in data])
        fits, folds, rescales = m.launches()
        assert (folds, rescales) == (0, 0 if cpw == -1 else min(fits, 4))
        m.run(steps, graph=True)
        torch.cuda.synchronize()
        for i, (ga, gm) in enumerate(zip(alone, mixed)):
            sa, sm = state(ga), state(gm)
            assert sa[3] == sm[3], i
            for x, y in zip(sa[:3], sm[:3]):
                assert torch.equal(x, y), f"stream {i} {shapes[i]} {opts[i]} differs"
            assert torch.equal(loss_alone[i], m.loss[i]), i
        m.close()
    finally:
        bd.tune_clear()
