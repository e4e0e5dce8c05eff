"""GPU parity of the penalty on H (section 2.2, Extensions) against the FP64
oracle: psi(s) = lambda log(a + s) of each column sum s = sum_k h_k, entering
the inner update through its tangent (lambda / (a + s) joins every den_k).

Tolerances as for the plain method: 1e-12 for the FP64 plain path, 1e-5 for
the FP32 paths (plain, and the VALU fit variant that FP32 handles run with the
penalty).  lambda is chosen per shape so that the penalty moves H by 20-80 %
(lambda = F/2 and 5F at a = 1 and 0.1), so a dropped or misplaced term fails.
"""
import numpy as np
import pytest

import oracle
from paper_1106_4198_amd import synth
from tests.helpers import from_gpu_kf, rel_fro
from tests.test_gpu_parity import DEV, bd, compare_step, say, torch

pytestmark = pytest.mark.gpu

SHAPES = [(129, 8, 1), (17, 5, 3), (513, 50, 16), (66, 64, 5), (3, 2, 4), (257, 33, 7)]


def psi_for(F, strong):
    return (5.0 * F, 0.1) if strong else (0.5 * F, 1.0)


@pytest.mark.parametrize("strong", [False, True])
@pytest.mark.parametrize("F,K,b", SHAPES)
def test_penalty_step_fp64_plain(F, K, b, strong):
    compare_step(F, K, b, 10, "fp64", "plain", seed=41, tol=1e-12, psi=psi_for(F, strong))


@pytest.mark.parametrize("kernel", ["plain", "fused"])
@pytest.mark.parametrize("strong", [False, True])
@pytest.mark.parametrize("F,K,b", SHAPES + [(513, 50, 128), (1025, 40, 9), (1088, 64, 3)])
def test_penalty_step_fp32(F, K, b, strong, kernel):
    compare_step(F, K, b, 20, "fp32", kernel, seed=42, tol=1e-5, psi=psi_for(F, strong))


@pytest.mark.parametrize("precision,kernel,tol", [("fp64", "plain", 1e-12), ("fp32", "plain", 1e-5),
                                                  ("fp32", "fused", 1e-5)])
def test_penalty_step_variants(precision, kernel, tol):
    psi = psi_for(130, False)
    compare_step(130, 10, 11, 6, precision, kernel, seed=43, tol=tol, warm=True, psi=psi)
    compare_step(130, 10, 11, 6, precision, kernel, seed=44, tol=tol, rho=0.7, psi=psi)
    compare_step(130, 10, 11, 6, precision, kernel, seed=45, tol=tol, normalize=False, psi=psi)
    compare_step(130, 10, 11, 6, precision, kernel, seed=46, tol=tol, update_w=False, psi=psi)
    compare_step(130, 10, 5, 0, precision, kernel, seed=47, tol=tol, psi=psi)


def test_penalty_uses_the_valu_variant_or_plain():
    """FP32 with the penalty runs the VALU fit where the shape has one (even when a
    tuning entry names another variant) and the plain path elsewhere."""
    bd.tune_clear()
    try:
        bd.tune_set(513, 50, "fp32", 8, -3, 0)          # the 16-frame tile variant
        W0 = torch.rand((50, 513), dtype=torch.float32, device=DEV) + 0.5
        g = bd.OnlineISNMF(W0, 8, psi=(10.0, 1.0))
        assert g.kernel_used == "fused"
        g.close()
    finally:
        bd.tune_clear()
    W0 = torch.rand((70, 80), dtype=torch.float32, device=DEV) + 0.5
    g = bd.OnlineISNMF(W0, 4, psi=(10.0, 1.0))
    assert g.kernel_used == "plain"
    g.close()
    with pytest.raises(bd.IsnmfError):
        bd.OnlineISNMF(W0, 4, kernel="fused", psi=(10.0, 1.0))
    W0 = torch.rand((8, 64), dtype=torch.float32, device=DEV) + 0.5
    for prec in ("bf16", "fp16"):
        with pytest.raises(bd.IsnmfError):
            bd.OnlineISNMF(W0, 4, precision=prec, psi=(10.0, 1.0))


@pytest.mark.parametrize("kernel", ["plain", "fused"])
def test_penalty_lambda_zero_is_the_plain_method_bitwise(kernel):
    """psi_lambda = 0 (any a) runs exactly the unpenalized arithmetic."""
    F, K, b = 257, 24, 16
    V, W0 = synth.problem(F, K, 3 * b, seed=48)
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
    W0t = torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV)
    outs = []
    for psi in (None, (0.0, 7.0)):
        g = bd.OnlineISNMF(W0t, b, inner_iters=12, kernel=kernel, psi=psi)
        H = torch.zeros((3 * b, K), dtype=torch.float32, device=DEV)
        for s0 in range(0, 3 * b, b):
            g.step(Vt[s0:s0 + b], H[s0:s0 + b])
        W, A, B, _ = g.get()
        torch.cuda.synchronize()
        outs.append((W.clone(), A.clone(), B.clone(), H.clone()))
        g.close()
    for x, y in zip(*outs):
        assert torch.equal(x, y)


def test_penalty_refused_by_batched_and_served_forms():
    W0 = torch.rand((8, 64), dtype=torch.float32, device=DEV) + 0.5
    g = bd.OnlineISNMF(W0, 4, kernel="fused", psi=(10.0, 1.0))
    V = torch.rand((16, 64), dtype=torch.float32, device=DEV)
    with pytest.raises(bd.IsnmfError) as ei:
        bd.MultiISNMF([g], [V], [4])
    assert ei.value.code == bd.EUNSUPPORTED
    srv = bd.Server(max_sessions=4, max_per_step=16, max_frames=64)
    with pytest.raises(bd.IsnmfError) as ei:
        srv.open(g)
    assert ei.value.code == bd.EUNSUPPORTED
    srv.close()
    g.close()


@pytest.mark.parametrize("precision,kernel,tol", [("fp64", "plain", 1e-9), ("fp32", "plain", 1e-5),
                                                  ("fp32", "fused", 1e-5)])
def test_penalty_heldout_fit_matches_oracle(precision, kernel, tol):
    """The held-out fit at a frozen W solves the penalized inner problem."""
    F, K, b, I, Nt = 129, 8, 16, 10, 37
    psi = psi_for(F, False)
    say(f"penalized held-out fit {precision}/{kernel}")
    V, W0 = synth.problem(F, K, 2 * b + Nt, seed=49)
    Vtr, Vte = V[:, :2 * b], V[:, 2 * b:]
    g = bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(DEV), b,
                       inner_iters=I, precision=precision, kernel=kernel, psi=psi)
    Vtr_t = torch.from_numpy(np.ascontiguousarray(Vtr.T)).to(DEV)
    for s0 in range(0, 2 * b, b):
        g.step(Vtr_t[s0:s0 + b])
    W, _, _, _ = g.get()
    Wf = from_gpu_kf(g.get_w64() if precision == "fp64" else W)
    Vte_t = torch.from_numpy(np.ascontiguousarray(Vte.T)).to(DEV)
    H = torch.zeros((Nt, K), dtype=torch.float32, device=DEV)
    loss = torch.zeros((), dtype=torch.float64, device=DEV)
    for s0 in range(0, Nt, b):
        g.fit(Vte_t[s0:s0 + b], H[s0:s0 + b], loss)
    torch.cuda.synchronize()
    Vd = Vte.astype(np.float64)
    Href = np.stack([oracle.fit_h_pen(Vd[:, n], Wf, psi[0], psi[1], iters=I)[0]
                     for n in range(Nt)], axis=1)
    lref = sum(oracle.dis(Vd[:, n], Wf @ Href[:, n], 1e-12) for n in range(Nt))
    assert rel_fro(H.cpu().double().numpy().T, Href) <= max(10 * tol, 1e-7)
    assert abs(loss.item() - lref) <= 10 * tol * lref
    assert g.status() == 0
    g.close()
