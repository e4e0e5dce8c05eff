"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances (norm-wise and elementwise, see helpers.assert_close):
  FP64 device mode, one step from identical state:   1e-12 (W, A, B)
  FP32 path, one step from identical state:           1e-5  (W, A, B, H)
  full pass, running loss and final objective:        1e-3
"""
import contextlib
import functools
import sys

import numpy as np
import pytest

import oracle
from paper_1106_4198_amd import synth
from tests.helpers import assert_close, from_gpu_kf, rel_fro, to_gpu_kf

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1106_4198_amd import binding as bd  # noqa: E402

DEV = "cuda"


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def make_state(F, K, seed, steps_before=0, b=8, iters=5):
    """An oracle state with nonzero A, B (a few warm-up steps from W0)."""
    V, W0 = synth.problem(F, K, steps_before * b + 1, seed)
    st = oracle.OnlineState(W0.astype(np.float64))
    for s in range(steps_before):
        st.step(V[:, s * b:(s + 1) * b].astype(np.float64), iters=iters)
    return st


def gpu_from_state(st, b_max, **kw):
    W32 = to_gpu_kf(st.W, np.float32, torch)
    A = to_gpu_kf(st.A, np.float64, torch)
    B = to_gpu_kf(st.B, np.float64, torch)
    g = bd.OnlineISNMF(W32, b_max, A0=A, B0=B, **kw)
    g.set_w64(to_gpu_kf(st.W, np.float64, torch))   # exact FP64 state
    return g


def run_step(g, Vb_fn, H0=None):
    Vb = torch.from_numpy(np.ascontiguousarray(Vb_fn.T)).to(DEV)
    if H0 is not None:
        H = torch.from_numpy(np.ascontiguousarray(H0.T).astype(np.float32)).to(DEV)
    else:
        H = torch.zeros((Vb.shape[0], g.K), dtype=torch.float32, device=DEV)
    loss = torch.zeros((), dtype=torch.float64, device=DEV)
    dw = torch.zeros((), dtype=torch.float64, device=DEV)
    g.step(Vb, H, loss, dw)
    torch.cuda.synchronize()
    return H.cpu().double().numpy().T, float(loss.item()), float(dw.item())


def compare_step(F, K, b, iters, precision, kernel, seed, tol, warm=False, rho=1.0,
                 normalize=True, update_w=True, steps_before=2, b_max=None, psi=None):
    say(f"step F={F} K={K} b={b} I={iters} {precision}/{kernel} warm={warm} rho={rho} "
        f"norm={normalize} upd={update_w} seed={seed} psi={psi}")
    st = make_state(F, K, seed, steps_before)
    Vb = synth.frames(F, K, b, seed + 1000)
    H0 = None
    if warm:
        H0 = np.asfortranarray(np.random.default_rng(seed).uniform(0.2, 2.0, size=(K, b)))
        H0 = H0.astype(np.float32).astype(np.float64)
    g = gpu_from_state(st, b_max or b, eps=1e-12, inner_iters=iters, rho=rho,
                       normalize=normalize, warm=warm, precision=precision, kernel=kernel,
                       update_w=update_w, psi=psi)
    if kernel == "fused":
        assert g.kernel_used == "fused"
    Hg, lg, dwg = run_step(g, Vb, H0)
    ref = st.copy()
    Hr, dwr, fl = ref.step(Vb.astype(np.float64), iters=iters, rho=rho, normalize=normalize,
                           H=H0, update_w=update_w, psi=psi)
    assert fl == 0
    W64 = from_gpu_kf(g.get_w64())
    Wg, Ag, Bg, t = g.get()
    assert t == b
    assert_close(W64, ref.W, tol, "W")
    assert_close(from_gpu_kf(Ag), ref.A, tol, "A")
    assert_close(from_gpu_kf(Bg), ref.B, tol, "B")
    assert_close(from_gpu_kf(Wg), ref.W, max(tol, 1e-7), "W32")
    assert_close(Hg, Hr, max(tol, 2e-7), "H")
    assert abs(lg - ref.last_loss) <= max(tol, 1e-9) * abs(ref.last_loss) + 1e-12, (lg, ref.last_loss)
    if update_w:
        assert abs(dwg - dwr) <= max(100 * tol, 1e-6) * max(dwr, 1e-30) + 1e-14, (dwg, dwr)
    assert g.status() == 0
    g.close()


# ---------------------------------------------------------------- one step, FP64 logic check

@pytest.mark.parametrize("F,K,b", [(129, 8, 1), (17, 5, 3), (513, 50, 16), (66, 64, 5), (3, 2, 4)])
def test_step_fp64_plain(F, K, b):
    compare_step(F, K, b, 10, "fp64", "plain", seed=11, tol=1e-12)


def test_step_fp64_variants():
    compare_step(40, 6, 7, 4, "fp64", "plain", seed=12, tol=1e-12, warm=True)
    compare_step(40, 6, 7, 4, "fp64", "plain", seed=13, tol=1e-12, rho=0.5)
    compare_step(40, 6, 7, 4, "fp64", "plain", seed=14, tol=1e-12, normalize=False)
    compare_step(40, 6, 7, 4, "fp64", "plain", seed=15, tol=1e-12, update_w=False)
    compare_step(40, 6, 7, 0, "fp64", "plain", seed=16, tol=1e-12)


# ---------------------------------------------------------------- one step, FP32

@pytest.mark.parametrize("kernel", ["plain", "fused"])
@pytest.mark.parametrize("F,K,b", [(129, 8, 1), (513, 50, 128), (257, 64, 7), (65, 16, 9),
                                   (64, 3, 4), (68, 33, 6), (3, 2, 5), (200, 52, 13)])
def test_step_fp32(F, K, b, kernel):
    compare_step(F, K, b, 20, "fp32", kernel, seed=21, tol=1e-5)


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_step_fp32_variants(kernel):
    compare_step(130, 10, 11, 6, "fp32", kernel, seed=22, tol=1e-5, warm=True)
    compare_step(130, 10, 11, 6, "fp32", kernel, seed=23, tol=1e-5, rho=0.7)
    compare_step(130, 10, 11, 6, "fp32", kernel, seed=24, tol=1e-5, normalize=False)
    compare_step(130, 10, 11, 6, "fp32", kernel, seed=25, tol=1e-5, update_w=False)
    compare_step(130, 10, 5, 6, "fp32", kernel, seed=26, tol=1e-5, b_max=16)   # ragged batch


# ---------------------------------------------------------------- one step, FP32 VALU variant

@contextlib.contextmanager
def valu_variant(F, K):
    """Handles of shape (F, K) created inside use the VALU fit variant (the
    default for FP32 where no MFMA tile fits, a tuning entry elsewhere)."""
    bd.tune_clear()
    if bd.tune_get(F, K, "fp32")[1] != 0:
        bd.tune_set(F, K, "fp32", 8, 0, 0)
    assert bd.tune_get(F, K, "fp32") == (8, 0, 0)
    try:
        yield
    finally:
        bd.tune_clear()


@pytest.mark.parametrize("F,K,b", [(129, 8, 1), (513, 50, 128), (257, 64, 7), (65, 16, 9),
                                   (64, 3, 4), (68, 33, 6), (3, 2, 5), (200, 52, 13),
                                   (1025, 40, 33), (1088, 64, 5), (700, 57, 10), (1025, 1, 3),
                                   (577, 24, 4)])
def test_step_fp32_valu(F, K, b):
    with valu_variant(F, K):
        compare_step(F, K, b, 20, "fp32", "fused", seed=27, tol=1e-5)


# the 16-wave form of the VALU variant: the FP32 default past the 8-wave form's
# rows (1088 < F <= 1152), 9 row sets of 128 rows with a ragged last set, K
# across the component groups of 8 (1..8, ragged)
@pytest.mark.parametrize("F,K,b", [(1089, 40, 3), (1152, 64, 5), (1100, 57, 33), (1120, 1, 4),
                                   (1150, 24, 9), (1130, 8, 1), (1097, 33, 130)])
def test_step_fp32_valu16(F, K, b):
    bd.tune_clear()
    assert bd.tune_get(F, K, "fp32") == (16, 0, 0)
    compare_step(F, K, b, 20, "fp32", "fused", seed=27, tol=1e-5)


def test_step_fp32_valu16_variants():
    bd.tune_clear()
    compare_step(1100, 10, 11, 6, "fp32", "fused", seed=22, tol=1e-5, warm=True)
    compare_step(1100, 10, 11, 6, "fp32", "fused", seed=23, tol=1e-5, rho=0.7)
    compare_step(1100, 10, 11, 6, "fp32", "fused", seed=24, tol=1e-5, normalize=False)
    compare_step(1100, 10, 11, 6, "fp32", "fused", seed=25, tol=1e-5, update_w=False)
    compare_step(1100, 10, 5, 6, "fp32", "fused", seed=26, tol=1e-5, b_max=16)
    compare_step(1100, 10, 5, 0, "fp32", "fused", seed=28, tol=1e-5)


def test_step_fp32_valu_variants():
    with valu_variant(130, 10):
        compare_step(130, 10, 11, 6, "fp32", "fused", seed=22, tol=1e-5, warm=True)
        compare_step(130, 10, 11, 6, "fp32", "fused", seed=23, tol=1e-5, rho=0.7)
        compare_step(130, 10, 11, 6, "fp32", "fused", seed=24, tol=1e-5, normalize=False)
        compare_step(130, 10, 11, 6, "fp32", "fused", seed=25, tol=1e-5, update_w=False)
        compare_step(130, 10, 5, 6, "fp32", "fused", seed=26, tol=1e-5, b_max=16)
        compare_step(130, 10, 5, 0, "fp32", "fused", seed=28, tol=1e-5)


def test_valu_large_config_and_repeatability():
    """The benchmark shape with the VALU variant (full and ragged minibatch),
    and two identical runs giving identical bits."""
    with valu_variant(513, 50):
        compare_step(513, 50, 128, 20, "fp32", "fused", seed=51, tol=1e-5, steps_before=3)
        compare_step(513, 50, 64, 20, "fp32", "fused", seed=52, tol=1e-5, steps_before=3, b_max=128)
        V, W0 = synth.problem(513, 50, 256, seed=53)
        Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
        outs = []
        for _ in range(2):
            g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), 128)
            H = torch.zeros((128, 50), dtype=torch.float32, device=DEV)
            for s in range(2):
                g.step(Vt[128 * s:128 * (s + 1)], H)
            outs.append((g.get_w64(), H.clone()))
            g.close()
        assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


# ---------------------------------------------------------------- one step, FP32 16-frame tile

@contextlib.contextmanager
def t32_variant(F, K):
    """Handles of shape (F, K) created inside use the FP32 16-frame tile
    variant (16x16x4 FP32 MFMA, W in LDS; a throughput tuning entry)."""
    bd.tune_clear()
    bd.tune_set(F, K, "fp32", 8, -3, 0)
    assert bd.tune_get(F, K, "fp32") == (8, -3, 0)
    try:
        yield
    finally:
        bd.tune_clear()


# shapes across every split of K into matrix-pipe m-tiles (1..4) and VALU
# remainder components (0..4: K = 8, 16, 33, 35, 49, 50, 52, 64, ...), row tiles
# from 1 to the LDS limit of each split (F <= 592 at 4 m-tiles, 784 at 3, 1136 at
# 2), ragged minibatches, one and several 128-frame workgroups
T32_SHAPES = [(129, 8, 1), (513, 50, 128), (257, 64, 7), (65, 16, 9), (64, 3, 4), (68, 33, 6),
              (3, 2, 5), (200, 52, 13), (592, 64, 20), (513, 50, 300), (784, 48, 40),
              (1025, 32, 33), (1088, 16, 129), (33, 32, 129), (16, 1, 3), (513, 17, 64),
              (577, 49, 17), (784, 52, 20), (300, 35, 40), (1088, 36, 8), (257, 20, 130)]


@pytest.mark.parametrize("F,K,b", T32_SHAPES)
def test_step_fp32_t32(F, K, b):
    with t32_variant(F, K):
        compare_step(F, K, b, 20, "fp32", "fused", seed=29, tol=1e-5)


def test_step_fp32_t32_variants():
    with t32_variant(130, 10):
        compare_step(130, 10, 11, 6, "fp32", "fused", seed=22, tol=1e-5, warm=True)
        compare_step(130, 10, 11, 6, "fp32", "fused", seed=23, tol=1e-5, rho=0.7)
        compare_step(130, 10, 11, 6, "fp32", "fused", seed=24, tol=1e-5, normalize=False)
        compare_step(130, 10, 11, 6, "fp32", "fused", seed=25, tol=1e-5, update_w=False)
        compare_step(130, 10, 5, 6, "fp32", "fused", seed=26, tol=1e-5, b_max=16)
        compare_step(130, 10, 5, 0, "fp32", "fused", seed=28, tol=1e-5)
    with t32_variant(513, 50):
        compare_step(513, 50, 128, 20, "fp32", "fused", seed=51, tol=1e-5, steps_before=3)
        compare_step(513, 50, 200, 20, "fp32", "fused", seed=53, tol=1e-5, warm=True)


def test_fp32_wide_F_uses_the_valu_variant():
    W0 = torch.rand((40, 1025), dtype=torch.float32, device=DEV) + 0.5
    g = bd.OnlineISNMF(W0, 4, kernel="auto")
    assert g.kernel_used == "fused"
    assert bd.tune_get(1025, 40, "fp32") == (8, 0, 0)
    W0 = torch.rand((40, 1089), dtype=torch.float32, device=DEV) + 0.5
    assert bd.OnlineISNMF(W0, 4, kernel="auto").kernel_used == "fused"
    assert bd.tune_get(1089, 40, "fp32") == (16, 0, 0)   # past the 8-wave form's rows
    W0 = torch.rand((40, 1153), dtype=torch.float32, device=DEV) + 0.5
    assert bd.OnlineISNMF(W0, 4, kernel="auto").kernel_used == "plain"


def test_auto_falls_back_to_plain_for_wide_K():
    W0 = torch.rand((80, 70), dtype=torch.float32, device=DEV) + 0.5
    g = bd.OnlineISNMF(W0, 4, kernel="auto")
    assert g.kernel_used == "plain"
    with pytest.raises(bd.IsnmfError):
        bd.OnlineISNMF(W0, 4, kernel="fused")


# ---------------------------------------------------------------- sequences and passes

@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_per_step_parity_over_a_sequence(kernel):
    """Ten consecutive steps, each compared from the oracle's state at that step."""
    F, K, b, I = 257, 20, 32, 20
    say(f"sequence F={F} K={K} b={b} {kernel}")
    V, W0 = synth.problem(F, K, 10 * b, seed=31)
    st = oracle.OnlineState(W0.astype(np.float64))
    g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b, kernel=kernel,
                       inner_iters=I)
    for s in range(10):
        g.set_w64(to_gpu_kf(st.W, np.float64, torch))
        g.set(A=to_gpu_kf(st.A, np.float64, torch), B=to_gpu_kf(st.B, np.float64, torch), t=st.t)
        Vb = V[:, s * b:(s + 1) * b]
        run_step(g, Vb)
        st.step(Vb.astype(np.float64), iters=I)
        assert_close(from_gpu_kf(g.get_w64()), st.W, 1e-5, f"W step {s}")
        _, A, B, _ = g.get()
        assert_close(from_gpu_kf(A), st.A, 1e-5, f"A step {s}")
        assert_close(from_gpu_kf(B), st.B, 1e-5, f"B step {s}")


@pytest.mark.parametrize("precision,kernel,tol", [("fp64", "plain", 1e-9), ("fp32", "plain", 1e-3),
                                                  ("fp32", "fused", 1e-3)])
def test_full_pass_small_config(precision, kernel, tol):
    """F=129, K=8, N=2000, b=1, I=10, one pass (the FP64 correctness workload)."""
    F, K, N, b, I = 129, 8, 2000, 1, 10
    say(f"full pass F={F} K={K} N={N} b={b} {precision}/{kernel}")
    V, W0 = synth.problem(F, K, N, seed=41)
    ref = oracle.online_pass(V.astype(np.float64), W0.astype(np.float64), b, iters=I)
    g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b, inner_iters=I,
                       precision=precision, kernel=kernel)
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
    loss = torch.zeros((), dtype=torch.float64, device=DEV)
    for s in range(0, N, b):
        g.step(Vt[s:s + b], None, loss)
    torch.cuda.synchronize()
    assert abs(loss.item() - ref.loss_sum) <= tol * ref.loss_sum
    W64 = from_gpu_kf(g.get_w64())
    assert rel_fro(W64, ref.W) <= tol
    _, A, B, t = g.get()
    assert t == N
    assert rel_fro(from_gpu_kf(A), ref.A) <= tol and rel_fro(from_gpu_kf(B), ref.B) <= tol
    # final objective of the learned dictionary, activations refit by the oracle
    Hfit = np.column_stack([oracle.fit_h(V[:, n].astype(np.float64), W64, iters=I)[0] for n in range(0, N, 20)])
    Href = np.column_stack([oracle.fit_h(V[:, n].astype(np.float64), ref.W, iters=I)[0] for n in range(0, N, 20)])
    og = oracle.objective(V[:, ::20].astype(np.float64), W64, Hfit)
    orf = oracle.objective(V[:, ::20].astype(np.float64), ref.W, Href)
    assert abs(og - orf) <= tol * orf


def test_large_config_one_step_fused():
    """The benchmark shape F=513, K=50, b=128, I=20 from a mid-stream state, with
    a ragged final minibatch of 64 (1e6 mod 128)."""
    compare_step(513, 50, 128, 20, "fp32", "fused", seed=51, tol=1e-5, steps_before=3)
    compare_step(513, 50, 64, 20, "fp32", "fused", seed=52, tol=1e-5, steps_before=3, b_max=128)


def test_full_size_pass_sampled_steps_match_oracle():
    """The benchmark's workload at full size, in the launch configuration it
    times: F=513, K=50, b=128, I=20 over N=10^6 resident frames (7812 full
    minibatches and a last one of 64), fused FP32 on the VALU fit variant.  At
    sampled minibatches the GPU's state before the step goes to the oracle,
    which takes the same step on the same frames; the GPU's state and h after
    it must match to 1e-5.  Over the whole pass: the online loss adds up step by
    step, W's columns sum to 1 after every rescale, and A, B stay positive."""
    F, K, b, I, N = 513, 50, 128, 20, 1_000_000
    nsteps = (N + b - 1) // b
    sampled = (0, 1, 3907, nsteps - 2, nsteps - 1)   # first, mid-stream, last full, tail of 64
    say(f"full-size pass F={F} K={K} b={b} N={N}, sampled steps {sampled}")
    V = synth.frames(F, K, N, 2011, threads=8)
    W0 = synth.initial_dictionary(F, K, 2011)
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
    with valu_variant(F, K):
        g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b, inner_iters=I)
    loss = torch.zeros((), dtype=torch.float64, device=DEV)
    step_losses = 0.0
    done = 0
    for s in sampled:
        if s > done:   # the steps between samples, one isnmf_online_step each
            g.run_pass(Vt[done * b:s * b], b, loss_sum=loss)
        lo, hi = s * b, min((s + 1) * b, N)
        W_before = from_gpu_kf(g.get_w64())
        _, A, B, t = g.get()
        assert t == lo
        st = oracle.OnlineState(W_before, from_gpu_kf(A), from_gpu_kf(B), t)
        l_before = loss.item()
        H = torch.zeros((hi - lo, K), dtype=torch.float32, device=DEV)
        g.step(Vt[lo:hi], H, loss)
        Hr, _, fl = st.step(V[:, lo:hi].astype(np.float64), iters=I)
        assert fl == 0
        _, A, B, t = g.get()
        assert t == hi
        assert_close(from_gpu_kf(g.get_w64()), st.W, 1e-5, f"W after step {s}")
        assert_close(from_gpu_kf(A), st.A, 1e-5, f"A after step {s}")
        assert_close(from_gpu_kf(B), st.B, 1e-5, f"B after step {s}")
        assert_close(H.cpu().double().numpy().T, Hr, 1e-5, f"H of step {s}")
        step_loss = loss.item() - l_before
        assert abs(step_loss - st.last_loss) <= 1e-6 * st.last_loss, (s, step_loss, st.last_loss)
        step_losses += step_loss
        done = s + 1
    assert done == nsteps
    W = from_gpu_kf(g.get_w64())
    _, A, B, _ = g.get()
    assert np.all(np.abs(W.sum(axis=0) - 1.0) <= 1e-12)
    assert np.all(from_gpu_kf(A) > 0) and np.all(from_gpu_kf(B) > 0)
    per_entry = loss.item() / N / F
    print(f"[full-size] online loss per entry {per_entry:.6f}")
    assert 0.5772 < per_entry < 0.7   # above the generator's floor (Euler's gamma), finite
    assert g.status() == 0
    g.close()


# ---------------------------------------------------------------- batch MU and objective

# W and H cross the batch ABI in FP32 between cycles, so even the FP64 device
# mode carries FP32 rounding from one cycle to the next.
@pytest.mark.parametrize("precision,kernel,tol", [("fp64", "plain", 1e-6), ("fp32", "plain", 1e-5),
                                                  ("fp32", "fused", 1e-5)])
def test_batch_mu_matches_oracle(precision, kernel, tol):
    F, K, N, C = 129, 8, 300, 6
    say(f"batch MU F={F} K={K} N={N} cycles={C} {precision}/{kernel}")
    V, W0 = synth.problem(F, K, N, seed=61)
    Wr, Hr = W0.astype(np.float64), np.ones((K, N))
    objs = []
    for _ in range(C):
        Wr, Hr, o, fl = oracle.batch_cycle(V.astype(np.float64), Wr, Hr)
        assert fl == 0
        objs.append(o)
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
    W = torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV)
    H = torch.ones((N, K), dtype=torch.float32, device=DEV)
    tr = bd.batch_mu(Vt, W, H, C, precision=precision, kernel=kernel)
    torch.cuda.synchronize()
    tr = tr.cpu().numpy()
    otol = max(tol, 1e-6) if precision == "fp32" else tol
    for c in range(C):
        assert abs(tr[c] - objs[c]) <= otol * objs[c], (c, tr[c], objs[c])
        if c:
            assert tr[c] <= tr[c - 1] * (1 + 1e-6)
    assert_close(from_gpu_kf(W), Wr, max(tol, 1e-5) * (10 if precision == "fp32" else 1), "W")
    assert rel_fro(H.cpu().double().numpy().T, Hr) <= max(tol, 1e-5) * 10


@functools.lru_cache(maxsize=1)
def _batch_mu_benchmark_shape_oracle(F, K, N, C, seed):
    """The oracle's C batch cycles from synth.problem(F, K, N, seed)."""
    V, W0 = synth.problem(F, K, N, seed=seed)
    oracle.set_threads(16)
    try:
        Wr, Hr, V64 = W0.astype(np.float64), np.ones((K, N)), V.astype(np.float64)
        objs = []
        for _ in range(C):
            Wr, Hr, o, fl = oracle.batch_cycle(V64, Wr, Hr)
            assert fl == 0
            objs.append(o)
    finally:
        oracle.set_threads(1)
    return V, W0, Wr, Hr, objs


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kernel", ["fused", "plain", "fused_t32"])
def test_batch_mu_at_benchmark_shape_matches_oracle(kernel):
    """Batch MU (section 2.1) at F = 513, K = 50 over N = 20480 frames: the
    fold sums 40 slices of 512 frames, and the warm H of all N frames is
    rescaled by its own launch; four cycles against the oracle's cycles,
    objective of every cycle and the final W and H.  fused_t32 runs the fit on
    the FP32 16-frame tile variant (the autotuner's pick for one update of
    many frames)."""
    F, K, N, C = 513, 50, 20480, 4
    say(f"batch MU F={F} K={K} N={N} cycles={C} fp32/{kernel}")
    V, W0, Wr, Hr, objs = _batch_mu_benchmark_shape_oracle(F, K, N, C, 62)
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
    W = torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV)
    H = torch.ones((N, K), dtype=torch.float32, device=DEV)
    bd.tune_clear()
    if kernel == "fused_t32":
        bd.tune_set(F, K, "fp32", 8, -3, 0)
    try:
        tr = bd.batch_mu(Vt, W, H, C, kernel="plain" if kernel == "plain" else "fused")
        torch.cuda.synchronize()
    finally:
        bd.tune_clear()
    tr = tr.cpu().numpy()
    for c in range(C):
        assert abs(tr[c] - objs[c]) <= 1e-6 * objs[c], (c, tr[c], objs[c])
        if c:
            assert tr[c] <= tr[c - 1] * (1 + 1e-6)
    assert_close(from_gpu_kf(W), Wr, 1e-4, "W")
    assert rel_fro(H.cpu().double().numpy().T, Hr) <= 1e-4


def test_objective_matches_oracle():
    F, K, N = 200, 12, 77
    say("objective")
    V, W0 = synth.problem(F, K, N, seed=71)
    H = np.random.default_rng(1).gamma(0.5, 1.0, size=(K, N)).astype(np.float32)
    ref = oracle.objective(V.astype(np.float64), W0.astype(np.float64), H.astype(np.float64))
    got = bd.objective(torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV),
                       torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV),
                       torch.from_numpy(np.ascontiguousarray(H.T)).to(DEV)).item()
    assert abs(got - ref) <= 1e-6 * ref


# ---------------------------------------------------------------- robustness

@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_nonfinite_input_sets_flag(kernel):
    F, K, b = 70, 4, 4
    say(f"nonfinite {kernel}")
    V, W0 = synth.problem(F, K, b, seed=81)
    V[5, 2] = np.nan
    g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b, kernel=kernel)
    g.step(torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV))
    assert g.status() & 1
    assert g.status() == 0   # cleared by the read


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_checkpoint_resume_is_bitwise(kernel):
    F, K, b = 130, 9, 8
    say(f"checkpoint {kernel}")
    V, W0 = synth.problem(F, K, 5 * b, seed=91)
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
    Wt = torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV)
    a = bd.OnlineISNMF(Wt, b, kernel=kernel)
    for s in range(5):
        a.step(Vt[s * b:(s + 1) * b])
    Wa, Aa, Ba, ta = a.get()
    Wa64 = a.get_w64()
    c = bd.OnlineISNMF(Wt, b, kernel=kernel)
    for s in range(3):
        c.step(Vt[s * b:(s + 1) * b])
    Wc, Ac, Bc, tc = c.get()
    Wc64 = c.get_w64()
    d = bd.OnlineISNMF(Wc, b, kernel=kernel, A0=Ac, B0=Bc)
    d.set_w64(Wc64)
    d.set(t=tc)
    for s in range(3, 5):
        d.step(Vt[s * b:(s + 1) * b])
    Wd, Ad, Bd, td = d.get()
    torch.cuda.synchronize()
    assert td == ta == 5 * b
    assert torch.equal(Wd, Wa) and torch.equal(Ad, Aa) and torch.equal(Bd, Ba)
    assert torch.equal(d.get_w64(), Wa64)


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_set_one_statistic_keeps_the_other(kernel):
    """After rescaling steps, setting A alone leaves B's value unchanged (and
    setting B alone leaves A's), bit for bit, and the next step continues from
    the mix exactly as a handle initialised with it does."""
    F, K, b = 97, 6, 16
    say(f"set one statistic {kernel}")
    V, W0 = synth.problem(F, K, 4 * b, seed=93)
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
    Wt = torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV)
    g = bd.OnlineISNMF(Wt, b, kernel=kernel)
    for s in range(3):
        g.step(Vt[s * b:(s + 1) * b])
    W1, A1, B1, t1 = g.get()
    A2 = A1 * 1.5
    g.set(A=A2, t=t1)
    _, Ag, Bg, _ = g.get()
    assert torch.equal(Ag, A2) and torch.equal(Bg, B1)
    B2 = B1 * 0.75
    g.set(B=B2, t=t1)
    _, Ag, Bg, _ = g.get()
    assert torch.equal(Ag, A2) and torch.equal(Bg, B2)
    W64 = g.get_w64()
    h = bd.OnlineISNMF(W1, b, kernel=kernel, A0=A2, B0=B2)
    h.set_w64(W64)
    h.set(t=t1)
    g.step(Vt[3 * b:])
    h.step(Vt[3 * b:])
    Wg, Ag, Bg, _ = g.get()
    Wh, Ah, Bh, _ = h.get()
    torch.cuda.synchronize()
    assert torch.equal(Wg, Wh) and torch.equal(Ag, Ah) and torch.equal(Bg, Bh)


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_repeatable_bitwise(kernel):
    F, K, b = 513, 50, 128
    say(f"repeatable {kernel}")
    V, W0 = synth.problem(F, K, b, seed=101)
    outs = []
    for _ in range(2):
        g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b, kernel=kernel)
        H = torch.zeros((b, K), dtype=torch.float32, device=DEV)
        g.step(torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV), H)
        W, A, B, _ = g.get()
        outs.append((W, A, B, H))
    torch.cuda.synchronize()
    for x, y in zip(*outs):
        assert torch.equal(x, y)


# ---------------------------------------------------------------- edge cases

@pytest.mark.parametrize("precision,variant", [("fp32", "valu"), ("fp32", "mfma"), ("bf16", "tile"),
                                               ("bf16", "mfma"), ("fp16", "mfma")])
def test_nonfinite_input_flag_every_fused_variant(precision, variant):
    F, K, b = 257, 20, 40
    say(f"nonfinite {precision}/{variant}")
    bd.tune_clear()
    if variant == "valu":
        bd.tune_set(F, K, "fp32", 8, 0, 0)
    if variant == "tile":
        bd.tune_set(F, K, "bf16", 8, -1, 0)
    try:
        for bad in (np.nan, np.inf):
            V, W0 = synth.problem(F, K, b, seed=83)
            V[100, 17] = bad
            g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b,
                               precision=precision)
            assert g.kernel_used == "fused"
            g.step(torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV))
            assert g.status() & 1, (precision, variant, bad)
            g.close()
    finally:
        bd.tune_clear()


@pytest.mark.parametrize("variant", ["mfma", "valu"])
def test_minibatch_above_one_fold_slice(variant):
    """b = 1300 frames: the fold sums three slices of 512 frames."""
    F, K = 257, 20
    with (valu_variant(F, K) if variant == "valu" else contextlib.nullcontext()):
        compare_step(F, K, 1300, 10, "fp32", "fused", seed=61, tol=1e-5, steps_before=1)


def test_tile_variant_above_one_fold_slice():
    F, K, b = 257, 40, 1100
    say("tile multi-slice")
    bd.tune_clear()
    bd.tune_set(F, K, "bf16", 8, -1, 0)
    try:
        V, W0 = synth.problem(F, K, b, seed=62)
        st = oracle.OnlineState(W0.astype(np.float64))
        g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b, precision="bf16")
        loss = torch.zeros((), dtype=torch.float64, device=DEV)
        g.step(torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV), None, loss)
        st.step(V.astype(np.float64), iters=20)
        assert rel_fro(from_gpu_kf(g.get_w64()), st.W) < 2e-2
        assert abs(loss.item() - st.loss_sum) <= 1e-3 * st.loss_sum
        assert g.status() == 0
    finally:
        bd.tune_clear()


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_silent_frames(kernel):
    """Frames that are entirely zero (v' = eps): every fit handles them."""
    F, K, b = 129, 8, 12
    say(f"silent frames {kernel}")
    st = make_state(F, K, 71, 2)
    Vb = synth.frames(F, K, b, 71 + 1000)
    Vb[:, [0, 5, 11]] = 0.0
    g = gpu_from_state(st, b, eps=1e-12, inner_iters=20, kernel=kernel)
    Hg, lg, _ = run_step(g, Vb)
    Hr, _, fl = st.step(Vb.astype(np.float64), iters=20)
    assert fl == 0
    assert_close(from_gpu_kf(g.get_w64()), st.W, 1e-5, "W")
    assert_close(Hg, Hr, 2e-6 if kernel == "plain" else 2e-5, "H")
    assert abs(lg - st.last_loss) <= 1e-5 * abs(st.last_loss)


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_eps_zero(kernel):
    """eps = 0 (the plain IS divergence of eq. 1) on strictly positive data."""
    F, K, b = 200, 12, 16
    say(f"eps 0 {kernel}")
    V, W0 = synth.problem(F, K, 2 * b, seed=73)
    V = np.maximum(V, 1e-6).astype(np.float32)
    st = oracle.OnlineState(W0.astype(np.float64))
    st.step(V[:, :b].astype(np.float64), iters=10, eps=0.0)
    g = bd.OnlineISNMF(to_gpu_kf(st.W, np.float32, torch), b, eps=0.0, inner_iters=10, kernel=kernel,
                       A0=to_gpu_kf(st.A, np.float64, torch), B0=to_gpu_kf(st.B, np.float64, torch))
    g.set_w64(to_gpu_kf(st.W, np.float64, torch))
    loss = torch.zeros((), dtype=torch.float64, device=DEV)
    g.step(torch.from_numpy(np.ascontiguousarray(V[:, b:].T)).to(DEV), None, loss)
    st.step(V[:, b:].astype(np.float64), iters=10, eps=0.0)
    assert_close(from_gpu_kf(g.get_w64()), st.W, 1e-5, "W")
    assert abs(loss.item() - st.last_loss) <= 1e-5 * st.last_loss
    assert g.status() == 0


# ---------------------------------------------------------------- multi-pass over a finite set

# FP64 mode: the resident H crosses the ABI in FP32, so every h is rounded to
# FP32 between visits (6e-8 relative) and the FP64 state follows it to ~1e-8.
@pytest.mark.parametrize("precision,kernel,variant,tol", [("fp64", "plain", "", 1e-7),
                                                          ("fp32", "plain", "", 1e-4),
                                                          ("fp32", "fused", "mfma", 1e-4),
                                                          ("fp32", "fused", "valu", 1e-4)])
def test_multipass_warm_restarts_match_oracle(precision, kernel, variant, tol):
    """Three passes over N = 100 frames, each in its own random order, minibatches
    of 16 (a short last one), warm restarts from the resident H (section 2.3)."""
    F, K, N, b, I, P = 129, 8, 100, 16, 10, 3
    say(f"multipass {precision}/{kernel}/{variant}")
    V, W0 = synth.problem(F, K, N, seed=121)
    rng = np.random.default_rng(122)
    perms = [rng.permutation(N) for _ in range(P)]
    st, Href = oracle.online_passes(V.astype(np.float64), W0.astype(np.float64), b, perms, iters=I)
    bd.tune_clear()
    if variant == "valu":
        bd.tune_set(F, K, "fp32", 8, 0, 0)
    try:
        g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b, warm=True,
                           inner_iters=I, precision=precision, kernel=kernel)
        H = torch.ones((N, K), dtype=torch.float32, device=DEV)
        perm = torch.from_numpy(np.stack(perms).astype(np.int32)).to(DEV)
        loss = torch.zeros((), dtype=torch.float64, device=DEV)
        g.run_passes(torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV), perm, b, H, loss)
        torch.cuda.synchronize()
        _, A, B, t = g.get()
        assert t == P * N
        assert rel_fro(from_gpu_kf(g.get_w64()), st.W) <= tol
        assert rel_fro(from_gpu_kf(A), st.A) <= tol and rel_fro(from_gpu_kf(B), st.B) <= tol
        assert rel_fro(H.cpu().double().numpy().T, Href) <= 10 * tol
        assert abs(loss.item() - st.loss_sum) <= tol * st.loss_sum
        assert g.status() == 0
        g.close()
    finally:
        bd.tune_clear()


@pytest.mark.parametrize("precision,kernel,variant,tol", [
    ("fp64", "plain", "", 1e-9), ("fp32", "plain", "", 1e-5), ("fp32", "fused", "mfma", 1e-5),
    ("fp32", "fused", "valu", 1e-5)])
def test_heldout_fit_and_objective_match_oracle(precision, kernel, variant, tol):
    """The held-out criterion of section 3: after a few training steps, fit the
    activations of unseen frames at the frozen W (the inner argmin only), then
    evaluate eq. (1) on them.  The fit leaves W, A, B and t untouched."""
    F, K, b, I, Nt = 129, 8, 16, 10, 77
    say(f"held-out fit {precision}/{kernel}/{variant}")
    V, W0 = synth.problem(F, K, 4 * b + Nt, seed=128)
    Vtr, Vte = V[:, :4 * b], V[:, 4 * b:]
    bd.tune_clear()
    if variant == "valu":
        bd.tune_set(F, K, "fp32", 8, 0, 0)
    try:
        g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b,
                           inner_iters=I, precision=precision, kernel=kernel)
        Vtr_t = torch.from_numpy(np.ascontiguousarray(Vtr.T)).to(DEV)
        for s0 in range(0, 4 * b, b):
            g.step(Vtr_t[s0:s0 + b])
        W, A, B, t = g.get()
        W64 = g.get_w64()
        torch.cuda.synchronize()
        Wf = from_gpu_kf(W)                 # the W the fit runs on, as the oracle's input
        if precision == "fp64":
            Wf = from_gpu_kf(W64)
        Vte_t = torch.from_numpy(np.ascontiguousarray(Vte.T)).to(DEV)
        H = torch.zeros((Nt, K), dtype=torch.float32, device=DEV)
        loss = torch.zeros((), dtype=torch.float64, device=DEV)
        for s0 in range(0, Nt, b):          # minibatches of at most b_max, a short last one
            g.fit(Vte_t[s0:s0 + b], H[s0:s0 + b], loss)
        W2, A2, B2, t2 = g.get()
        torch.cuda.synchronize()
        assert t2 == t and torch.equal(W2, W) and torch.equal(A2, A) and torch.equal(B2, B)
        Vd = Vte.astype(np.float64)
        Href = np.stack([oracle.fit_h(Vd[:, n], Wf, iters=I)[0] for n in range(Nt)], axis=1)
        lref = sum(oracle.dis(Vd[:, n], Wf @ Href[:, n], 1e-12) for n in range(Nt))
        Hg = H.cpu().double().numpy().T
        assert rel_fro(Hg, Href) <= max(10 * tol, 1e-7)   # H leaves the device in FP32
        assert abs(loss.item() - lref) <= 10 * tol * lref
        obj = bd.objective(Vte_t, W, H).item()
        assert abs(obj - oracle.objective(Vd, from_gpu_kf(W), Hg)) <= 1e-9 * obj
        assert abs(obj - lref / Nt) <= 10 * tol * obj
        assert g.status() == 0
        g.close()
    finally:
        bd.tune_clear()


@pytest.mark.parametrize("precision,kernel,tol", [("fp64", "plain", 1e-6), ("fp32", "fused", 1e-4)])
def test_multipass_with_beta_N_is_batch_mu_on_device(precision, kernel, tol):
    """With beta = N (one minibatch of all N frames), r = 0 and one h update per
    visit, each warm-restart pass is one batch MU cycle (section 2.3): the device
    multi-pass entry point against the device batch MU and the oracle's cycles."""
    F, K, N, C = 129, 8, 300, 4
    say(f"multipass beta=N {precision}/{kernel}")
    V, W0 = synth.problem(F, K, N, seed=126)
    Wr, Hr = W0.astype(np.float64), np.ones((K, N))
    for _ in range(C):
        Wr, Hr, _, _ = oracle.batch_cycle(V.astype(np.float64), Wr, Hr)
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
    W0t = torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV)
    g = bd.OnlineISNMF(W0t, N, warm=True, inner_iters=1, rho=0.0, precision=precision,
                       kernel=kernel)
    H = torch.ones((N, K), dtype=torch.float32, device=DEV)
    rng = np.random.default_rng(127)
    perm = torch.from_numpy(np.stack([rng.permutation(N) for _ in range(C)]).astype(np.int32))
    g.run_passes(Vt, perm.to(DEV), N, H)
    Wb = W0t.clone()
    Hb = torch.ones((N, K), dtype=torch.float32, device=DEV)
    bd.batch_mu(Vt, Wb, Hb, C, precision=precision, kernel=kernel, trace=False)
    torch.cuda.synchronize()
    Wo = from_gpu_kf(g.get_w64())
    assert g.status() == 0
    g.close()
    assert rel_fro(Wo, Wr) <= tol and rel_fro(Wo, from_gpu_kf(Wb)) <= tol
    Ho = H.cpu().double().numpy().T
    assert rel_fro(Ho, Hr) <= 10 * tol and rel_fro(Ho, Hb.cpu().double().numpy().T) <= 10 * tol


@pytest.mark.parametrize("b", [16, 40])
def test_multipass_frames_shared_across_a_pass_boundary(b):
    """Pass 2 runs pass 1 backwards, so the first minibatch of a pass revisits
    the frames the previous pass ended with (all of them when b = N): their h
    must come back from the previous visit before the next one starts."""
    F, K, N, I = 65, 8, 40, 10
    say(f"multipass boundary b={b}")
    V, W0 = synth.problem(F, K, N, seed=124)
    p0 = np.random.default_rng(125).permutation(N)
    perms = [p0, p0[::-1].copy(), p0]
    st, Href = oracle.online_passes(V.astype(np.float64), W0.astype(np.float64), b, perms, iters=I)
    g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b, warm=True,
                       inner_iters=I)
    H = torch.ones((N, K), dtype=torch.float32, device=DEV)
    perm = torch.from_numpy(np.stack(perms).astype(np.int32)).to(DEV)
    g.run_passes(torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV), perm, b, H)
    torch.cuda.synchronize()
    assert rel_fro(from_gpu_kf(g.get_w64()), st.W) <= 1e-4
    assert rel_fro(H.cpu().double().numpy().T, Href) <= 1e-3
    assert g.status() == 0
    g.close()


def test_multipass_out_of_range_index_is_flagged_not_read():
    F, K, N, b = 65, 4, 40, 8
    say("multipass bad index")
    V, W0 = synth.problem(F, K, N, seed=123)
    g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b, warm=True)
    H = torch.ones((N, K), dtype=torch.float32, device=DEV)
    p = np.arange(N, dtype=np.int32)
    p[5] = N + 1000           # outside [0, N): a zero frame, no write
    p[6] = -3
    perm = torch.from_numpy(p[None, :]).to(DEV)
    g.run_passes(torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV), perm, b, H)
    torch.cuda.synchronize()
    assert g.status() & 8
    g.close()
    cold = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b, warm=False)
    with pytest.raises(bd.IsnmfError):   # the passes entry point needs warm restarts
        cold.run_passes(torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV), perm, b, H)


@pytest.mark.parametrize("precision,cpw", [("fp32", 0), ("bf16", -4), ("fp32", 1)])
def test_fit_timing_hook_counts_launches_and_keeps_the_bits(precision, cpw):
    """The per-launch timing hook (the VALU variants time their dispatch
    itself, the others bracket the launch) counts every fit launch, reports a
    positive duration, and changes no result bit."""
    F, K, b = 257, 24, 64
    say(f"timing hook {precision} cpw={cpw}")
    bd.tune_clear()
    bd.tune_set(F, K, precision, 8 if cpw <= 0 else 4, cpw, 0)
    try:
        V, W0 = synth.problem(F, K, 5 * b, seed=77)
        Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
        W0t = torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV)
        plain = bd.OnlineISNMF(W0t, b, precision=precision)
        timed = bd.OnlineISNMF(W0t, b, precision=precision)
        timed.set_timing(True, 3)
        for s in range(5):
            plain.step(Vt[s * b:(s + 1) * b])
            timed.step(Vt[s * b:(s + 1) * b])
        n, ms = timed.timing()
        assert n == 3 and ms > 0.0
        assert torch.equal(plain.get_w64(), timed.get_w64())
        timed.set_timing(True, 8)
        timed.step(Vt[:b])
        assert timed.timing()[0] == 1
        assert plain.status() == 0 and timed.status() == 0
        plain.close()
        timed.close()
    finally:
        bd.tune_clear()
