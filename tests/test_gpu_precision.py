"""Precision forms (BF16 / FP16 products, FP32 ratios, FP64 statistics)
against the FP64 oracle.

Gate (the stated accuracy of the forms): the online loss over a pass and the
final objective within rel 1e-3 of the oracle.  Per-step errors of W, A, B
are reported (printed) and bounded loosely (2e-2), not gated at 1e-5.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1106_4198_amd import synth
from tests.helpers import from_gpu_kf, rel_fro, to_gpu_kf

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1106_4198_amd import binding as bd  # noqa: E402

DEV = "cuda"


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
@pytest.mark.parametrize("F,K,b", [(513, 50, 128), (129, 8, 16), (257, 64, 33), (70, 5, 6),
                                   (257, 96, 7), (513, 128, 12), (1025, 50, 16), (1025, 100, 9),
                                   (1025, 16, 5), (700, 33, 4)])
def test_one_step_error_is_small(precision, F, K, b):
    say(f"precision step {precision} F={F} K={K} b={b}")
    V, W0 = synth.problem(F, K, 3 * b, seed=5)
    st = oracle.OnlineState(W0.astype(np.float64))
    st.step(V[:, :b].astype(np.float64), iters=20)
    st.step(V[:, b:2 * b].astype(np.float64), iters=20)
    g = bd.OnlineISNMF(to_gpu_kf(st.W, np.float32, torch), b, precision=precision,
                       A0=to_gpu_kf(st.A, np.float64, torch), B0=to_gpu_kf(st.B, np.float64, torch))
    assert g.kernel_used == "fused"
    g.set_w64(to_gpu_kf(st.W, np.float64, torch))
    Vb = V[:, 2 * b:3 * b]
    loss = torch.zeros((), dtype=torch.float64, device=DEV)
    g.step(torch.from_numpy(np.ascontiguousarray(Vb.T)).to(DEV), None, loss)
    st.step(Vb.astype(np.float64), iters=20)
    eW = rel_fro(from_gpu_kf(g.get_w64()), st.W)
    _, A, B, _ = g.get()
    eA = rel_fro(from_gpu_kf(A), st.A)
    eB = rel_fro(from_gpu_kf(B), st.B)
    el = abs(loss.item() - st.last_loss) / st.last_loss
    print(f"[precision] {precision} F={F} K={K} b={b}: W {eW:.2e} A {eA:.2e} B {eB:.2e} loss {el:.2e}")
    assert eW < 2e-2 and eA < 2e-2 and eB < 2e-2
    assert el < 1e-3
    assert g.status() == 0


def tile_variant(F, K, cpw=-1):
    """Make handles of shape (F, K) in BF16 use a 16-frame tile variant: W
    resident in LDS (cpw -1) or streamed through it (cpw -2); or the VALU
    variant on bf16 dot products (cpw -4)."""
    bd.tune_clear()
    bd.tune_set(F, K, "bf16", 8, cpw, 0)
    assert bd.tune_get(F, K, "bf16") == (8, cpw, 0)


TILE_SHAPES = [(513, 50, 128), (129, 8, 16), (257, 64, 33), (70, 5, 6), (513, 33, 7), (640, 64, 20),
               (16, 1, 3), (200, 40, 17), (257, 16, 1), (600, 64, 48), (513, 50, 300), (33, 32, 129)]
# the streamed variant also covers F > 640 and K > 64
STILE_SHAPES = TILE_SHAPES + [(1025, 128, 128), (1025, 100, 37), (1025, 40, 130), (1026, 97, 16),
                              (700, 65, 9), (257, 128, 64), (1025, 72, 1)]


# the VALU variant: F <= 1088, K <= 64, one frame per workgroup
VBF_SHAPES = [(513, 50, 128), (129, 8, 16), (257, 64, 33), (70, 5, 6), (513, 33, 7), (640, 64, 20),
              (16, 1, 3), (200, 40, 17), (257, 16, 1), (1025, 40, 130), (1088, 64, 5), (700, 57, 10),
              (1025, 1, 3), (577, 24, 4), (3, 2, 5), (66, 64, 5), (128, 9, 2)]


@pytest.mark.parametrize("cpw,F,K,b", [(-1,) + s for s in TILE_SHAPES] + [(-2,) + s for s in STILE_SHAPES]
                         + [(-4,) + s for s in VBF_SHAPES])
def test_tile_variant_one_step(cpw, F, K, b):
    """BF16 16-frame tile variants (16x16x32 MFMA; W resident in LDS, or
    streamed through it one 32-row step at a time) against the FP64 oracle at
    the precision-form bound, from a mid-stream state."""
    say(f"tile step cpw={cpw} F={F} K={K} b={b}")
    tile_variant(F, K, cpw)
    try:
        V, W0 = synth.problem(F, K, 3 * b, seed=6)
        st = oracle.OnlineState(W0.astype(np.float64))
        st.step(V[:, :b].astype(np.float64), iters=20)
        st.step(V[:, b:2 * b].astype(np.float64), iters=20)
        g = bd.OnlineISNMF(to_gpu_kf(st.W, np.float32, torch), b, precision="bf16",
                           A0=to_gpu_kf(st.A, np.float64, torch), B0=to_gpu_kf(st.B, np.float64, torch))
        g.set_w64(to_gpu_kf(st.W, np.float64, torch))
        Vb = V[:, 2 * b:3 * b]
        loss = torch.zeros((), dtype=torch.float64, device=DEV)
        H = torch.zeros((b, K), dtype=torch.float32, device=DEV)
        g.step(torch.from_numpy(np.ascontiguousarray(Vb.T)).to(DEV), H, loss)
        Hr, _, _ = st.step(Vb.astype(np.float64), iters=20)
        eW = rel_fro(from_gpu_kf(g.get_w64()), st.W)
        _, A, B, _ = g.get()
        eA = rel_fro(from_gpu_kf(A), st.A)
        eB = rel_fro(from_gpu_kf(B), st.B)
        eH = rel_fro(H.cpu().double().numpy().T, Hr)
        el = abs(loss.item() - st.last_loss) / st.last_loss
        print(f"[tile] F={F} K={K} b={b}: W {eW:.2e} A {eA:.2e} B {eB:.2e} H {eH:.2e} loss {el:.2e}")
        assert eW < 2e-2 and eA < 2e-2 and eB < 2e-2 and eH < 5e-2
        # one step's loss: 1e-3 once the minibatch averages the BF16 rounding of
        # its products; tiny shapes (K = 1: no averaging over components) 5e-3
        assert el < (1e-3 if F * K * b >= 4096 else 5e-3)
        assert g.status() == 0
        g.close()
    finally:
        bd.tune_clear()


@pytest.mark.parametrize("precision", ["bf16", "fp16", "fp32", "bf16_valu"])
def test_pass_accuracy_matches_stated_tolerance(precision):
    """F=513, K=50, b=128, I=20 over 24 minibatches (a prefix of the benchmark
    stream), with checkpoints of the relative error of W, A, B and the online
    loss against the FP64 oracle.  bf16_valu: BF16 on the VALU variant."""
    F, K, b, I, steps = 513, 50, 128, 20, 24
    say(f"precision pass {precision}")
    bd.tune_clear()
    if precision == "bf16_valu":
        precision = "bf16"
        bd.tune_set(F, K, "bf16", 8, -4, 0)
    V, W0 = synth.problem(F, K, steps * b, seed=2011)
    st = oracle.OnlineState(W0.astype(np.float64))
    oracle.set_threads(8)
    g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b,
                       precision=precision, inner_iters=I)
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
    loss = torch.zeros((), dtype=torch.float64, device=DEV)
    report = []
    for s in range(steps):
        g.step(Vt[s * b:(s + 1) * b], None, loss)
        st.step(V[:, s * b:(s + 1) * b].astype(np.float64), iters=I)
        if s + 1 in (1, 4, 12, 24):
            _, A, B, _ = g.get()
            report.append((s + 1, rel_fro(from_gpu_kf(g.get_w64()), st.W),
                           rel_fro(from_gpu_kf(A), st.A), rel_fro(from_gpu_kf(B), st.B),
                           abs(loss.item() - st.loss_sum) / st.loss_sum))
    oracle.set_threads(1)
    for r in report:
        print(f"[precision] {precision} step {r[0]:3d}: W {r[1]:.2e} A {r[2]:.2e} B {r[3]:.2e} loss {r[4]:.2e}")
    assert report[-1][4] < 1e-3            # online loss (eq. 5) over the pass
    # final objective of the learned dictionary on the pass's frames, refit by the oracle
    W = from_gpu_kf(g.get_w64())
    idx = range(0, steps * b, 97)
    Hg = np.column_stack([oracle.fit_h(V[:, n].astype(np.float64), W, iters=I)[0] for n in idx])
    Hr = np.column_stack([oracle.fit_h(V[:, n].astype(np.float64), st.W, iters=I)[0] for n in idx])
    og = oracle.objective(V[:, ::97].astype(np.float64), W, Hg)
    orf = oracle.objective(V[:, ::97].astype(np.float64), st.W, Hr)
    print(f"[precision] {precision} final objective rel {abs(og - orf) / orf:.2e}")
    assert abs(og - orf) <= 1e-3 * orf
    bd.tune_clear()


@pytest.mark.parametrize("precision", ["fp16", "bf16", "bf16_valu"])
@pytest.mark.parametrize("scale_exp", [-20, 20])
def test_step_is_amplitude_invariant(precision, scale_exp):
    """IS-NMF's fitted h scales with the frames' amplitude (section 2.1: the
    divergence is scale invariant, so h follows v).  The 16-bit forms keep
    their products in range whatever the amplitude: frames 2^-20 and 2^20
    times the generator's still meet the precision form's bounds against the
    FP64 oracle, which takes the same scaled frames."""
    F, K, b = 513, 50, 64
    say(f"amplitude {precision} 2^{scale_exp}")
    V, W0 = synth.problem(F, K, 3 * b, seed=12)
    V = (V.astype(np.float64) * 2.0 ** scale_exp).astype(np.float32)   # exact: a power of two
    st = oracle.OnlineState(W0.astype(np.float64))
    st.step(V[:, :b].astype(np.float64), iters=20)
    st.step(V[:, b:2 * b].astype(np.float64), iters=20)
    bd.tune_clear()
    if precision == "bf16_valu":
        precision = "bf16"
        bd.tune_set(F, K, "bf16", 8, -4, 0)
    g = bd.OnlineISNMF(to_gpu_kf(st.W, np.float32, torch), b, precision=precision,
                       A0=to_gpu_kf(st.A, np.float64, torch), B0=to_gpu_kf(st.B, np.float64, torch))
    bd.tune_clear()
    assert g.kernel_used == "fused"
    g.set_w64(to_gpu_kf(st.W, np.float64, torch))
    Vb = V[:, 2 * b:3 * b]
    loss = torch.zeros((), dtype=torch.float64, device=DEV)
    H = torch.zeros((b, K), dtype=torch.float32, device=DEV)
    g.step(torch.from_numpy(np.ascontiguousarray(Vb.T)).to(DEV), H, loss)
    Hr, _, _ = st.step(Vb.astype(np.float64), iters=20)
    eW = rel_fro(from_gpu_kf(g.get_w64()), st.W)
    _, A, B, _ = g.get()
    eA = rel_fro(from_gpu_kf(A), st.A)
    eB = rel_fro(from_gpu_kf(B), st.B)
    eH = rel_fro(H.cpu().double().numpy().T, Hr)
    el = abs(loss.item() - st.last_loss) / st.last_loss
    print(f"[amplitude] {precision} 2^{scale_exp}: W {eW:.2e} A {eA:.2e} B {eB:.2e} H {eH:.2e} "
          f"loss {el:.2e}")
    assert np.isfinite(H.cpu().numpy()).all()
    assert eW < 2e-2 and eA < 2e-2 and eB < 2e-2 and eH < 5e-2
    assert el < 1e-3
    assert g.status() == 0
