"""Shared test helpers: layout conversion between the oracle's Fortran (F, K)
arrays and the binding's row-major (K, F) torch tensors, and tolerances."""
import numpy as np


def rel_fro(x, y) -> float:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def assert_close(x, y, tol, what=""):
    """Norm-wise rel <= tol and elementwise |x-y| <= tol*|y| + tol*max|y|."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    assert x.shape == y.shape, (what, x.shape, y.shape)
    r = rel_fro(x, y)
    assert r <= tol, f"{what}: norm-wise rel error {r:.3e} > {tol:.1e}"
    bound = tol * np.abs(y) + tol * np.max(np.abs(y))
    bad = np.abs(x - y) > bound
    assert not bad.any(), f"{what}: {int(bad.sum())} elements out of bound, worst {np.max(np.abs(x - y) - bound):.3e}"


def to_gpu_kf(a_fk, dtype, torch, device="cuda"):
    """Fortran/numpy (F, K) -> torch (K, F) contiguous on device."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a_fk).T).astype(dtype)).to(device)


def from_gpu_kf(t):
    """torch (K, F) -> numpy float64 (F, K)."""
    return t.detach().cpu().double().numpy().T
