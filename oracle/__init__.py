"""FP64 CPU oracle for online Itakura-Saito NMF (arXiv:1106.4198).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The product path never imports this
package.  The arithmetic lives in ``isnmf_oracle.c`` (plain double-precision
loops); this module compiles it with gcc and wraps it with ctypes on numpy
float64 arrays.

Matrices are Fortran-ordered numpy arrays with the paper's shapes
(V: F x N, W: F x K, H: K x N; section 2.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "isnmf_oracle.c")
_LIB = os.path.join(_HERE, "libisnmf_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def build() -> str:
    """Compile the oracle shared library with gcc (OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.isnmf_ref_dis_term.restype = ctypes.c_double
    lib.isnmf_ref_dis_term.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.isnmf_ref_dis.restype = ctypes.c_double
    lib.isnmf_ref_dis.argtypes = [_dp, _dp, ctypes.c_long, ctypes.c_double]
    lib.isnmf_ref_objective.restype = ctypes.c_double
    lib.isnmf_ref_objective.argtypes = [ctypes.c_int] * 3 + [_dp, ctypes.c_long] * 3 + [ctypes.c_double]
    lib.isnmf_ref_fit_h.restype = ctypes.c_int
    lib.isnmf_ref_fit_h.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_long,
                                    _dp, ctypes.c_int, ctypes.c_double, _dp]
    lib.isnmf_ref_online_step.restype = ctypes.c_int
    lib.isnmf_ref_online_step.argtypes = [
        ctypes.c_int, ctypes.c_int, ctypes.c_int,
        _dp, ctypes.c_long, _dp, ctypes.c_long, _dp, _dp, _dp, ctypes.c_long,
        ctypes.c_int, ctypes.c_double, ctypes.c_double,
        ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.isnmf_ref_batch_stats.restype = None
    lib.isnmf_ref_batch_stats.argtypes = [ctypes.c_int] * 3 + [_dp, ctypes.c_long] * 3 + [
        ctypes.c_double, _dp, _dp]
    lib.isnmf_ref_batch_cycle.restype = ctypes.c_int
    lib.isnmf_ref_batch_cycle.argtypes = [ctypes.c_int] * 3 + [_dp, ctypes.c_long] * 3 + [
        ctypes.c_double, ctypes.c_int, _dp]
    lib.isnmf_ref_pen_objective_h.restype = ctypes.c_double
    lib.isnmf_ref_pen_objective_h.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_long,
                                              _dp, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double]
    lib.isnmf_ref_fit_h_pen.restype = ctypes.c_int
    lib.isnmf_ref_fit_h_pen.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_long, _dp,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, _dp]
    lib.isnmf_ref_online_step_pen.restype = ctypes.c_int
    lib.isnmf_ref_online_step_pen.argtypes = [
        ctypes.c_int, ctypes.c_int, ctypes.c_int,
        _dp, ctypes.c_long, _dp, ctypes.c_long, _dp, _dp, _dp, ctypes.c_long,
        ctypes.c_int, ctypes.c_double, ctypes.c_double,
        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp]
    lib.isnmf_ref_set_threads.restype = None
    lib.isnmf_ref_set_threads.argtypes = [ctypes.c_int]
    lib.isnmf_ref_get_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None) -> np.ndarray:
    out = np.asfortranarray(np.asarray(a, dtype=np.float64))
    if shape is not None and out.shape != shape:
        raise ValueError(f"expected shape {shape}, got {out.shape}")
    return out


def set_threads(n: int) -> None:
    _load().isnmf_ref_set_threads(int(n))


def get_threads() -> int:
    return int(_load().isnmf_ref_get_threads())


def dis_term(y: float, x: float) -> float:
    """y/x - log(y/x) - 1 (section 2.1)."""
    return float(_load().isnmf_ref_dis_term(float(y), float(x)))


def dis(y, x, eps: float = 0.0) -> float:
    """sum_i d_IS(eps + y_i, eps + x_i) (section 2.1, eps shift of section 2.3)."""
    y = np.ascontiguousarray(np.ravel(y), dtype=np.float64)
    x = np.ascontiguousarray(np.ravel(x), dtype=np.float64)
    if y.shape != x.shape:
        raise ValueError("shape mismatch")
    return float(_load().isnmf_ref_dis(_p(y), _p(x), y.size, float(eps)))


def objective(V, W, H, eps: float = 1e-12) -> float:
    """(1/N) sum_n d_IS(eps + v_n, eps + W h_n)  (eq. 1 with the eps shift)."""
    V = _f64(V)
    F, N = V.shape
    W = _f64(W)
    K = W.shape[1]
    H = _f64(H, (K, N))
    if W.shape[0] != F:
        raise ValueError("W rows != F")
    return float(_load().isnmf_ref_objective(F, K, N, _p(V), F, _p(W), F, _p(H), K, float(eps)))


def fit_h(v, W, h0=None, iters: int = 20, eps: float = 1e-12):
    """Inner multiplicative-update fit of one frame (Algorithm 1, inner argmin).

    Returns (h, flags)."""
    v = np.ascontiguousarray(np.ravel(v), dtype=np.float64)
    W = _f64(W)
    F, K = W.shape
    h = np.ones(K) if h0 is None else np.array(h0, dtype=np.float64).ravel().copy()
    scratch = np.zeros(F + K)
    fl = _load().isnmf_ref_fit_h(F, K, _p(v), _p(W), F, _p(h), int(iters), float(eps), _p(scratch))
    return h, int(fl)


def pen_objective_h(v, W, h, lam: float, a: float, eps: float = 1e-12) -> float:
    """sum_f d_IS(eps + v_f, eps + (W h)_f) + lam * log(a + sum_k h_k): the inner
    objective with the log penalty on H (section 2.2, Extensions)."""
    v = np.ascontiguousarray(np.ravel(v), dtype=np.float64)
    W = _f64(W)
    F, K = W.shape
    h = np.ascontiguousarray(np.ravel(h), dtype=np.float64)
    return float(_load().isnmf_ref_pen_objective_h(F, K, _p(v), _p(W), F, _p(h), float(eps),
                                                   float(lam), float(a)))


def fit_h_pen(v, W, lam: float, a: float, h0=None, iters: int = 20, eps: float = 1e-12):
    """Inner fit with the log penalty on H (section 2.2, Extensions).
    Returns (h, flags)."""
    v = np.ascontiguousarray(np.ravel(v), dtype=np.float64)
    W = _f64(W)
    F, K = W.shape
    h = np.ones(K) if h0 is None else np.array(h0, dtype=np.float64).ravel().copy()
    scratch = np.zeros(F + K)
    fl = _load().isnmf_ref_fit_h_pen(F, K, _p(v), _p(W), F, _p(h), int(iters), float(eps),
                                     float(lam), float(a), _p(scratch))
    return h, int(fl)


class OnlineState:
    """(W, A, B, t) of Algorithm 1, FP64, with one-minibatch steps."""

    def __init__(self, W0, A0=None, B0=None, t: int = 0):
        self.W = _f64(W0).copy(order="F")
        F, K = self.W.shape
        self.A = np.zeros((F, K), order="F") if A0 is None else _f64(A0, (F, K)).copy(order="F")
        self.B = np.zeros((F, K), order="F") if B0 is None else _f64(B0, (F, K)).copy(order="F")
        self.t = int(t)
        self.loss_sum = 0.0

    @property
    def F(self) -> int:
        return self.W.shape[0]

    @property
    def K(self) -> int:
        return self.W.shape[1]

    def copy(self) -> "OnlineState":
        s = OnlineState(self.W, self.A, self.B, self.t)
        s.loss_sum = self.loss_sum
        return s

    def step(self, Vb, iters: int = 20, eps: float = 1e-12, rho: float = 1.0,
             normalize: bool = True, H=None, update_w: bool = True, psi=None):
        """One online step on the minibatch Vb (F x b).

        H: None for fresh restarts (h = 1), else a K x b warm start (updated
        copy returned).  psi: None, or (lambda, a) of the log penalty on H
        (section 2.2, Extensions).  Returns (H_b, dW_fro, flags)."""
        Vb = _f64(Vb)
        F, b = Vb.shape
        if F != self.F:
            raise ValueError("frame length != F")
        warm = H is not None
        Hb = np.ones((self.K, b), order="F") if H is None else _f64(H, (self.K, b)).copy(order="F")
        loss = ctypes.c_double(0.0)
        dw = ctypes.c_double(0.0)
        if psi is not None:
            fl = _load().isnmf_ref_online_step_pen(
                F, self.K, b, _p(Vb), F, _p(self.W), F, _p(self.A), _p(self.B), _p(Hb), self.K,
                int(iters), float(eps), float(rho), int(bool(normalize)), int(warm),
                int(bool(update_w)), float(psi[0]), float(psi[1]), ctypes.byref(loss),
                ctypes.byref(dw))
        else:
            fl = _load().isnmf_ref_online_step(
                F, self.K, b, _p(Vb), F, _p(self.W), F, _p(self.A), _p(self.B), _p(Hb), self.K,
                int(iters), float(eps), float(rho), int(bool(normalize)), int(warm),
                int(bool(update_w)), ctypes.byref(loss), ctypes.byref(dw))
        if fl < 0:
            raise MemoryError("oracle allocation failed")
        self.t += b
        self.loss_sum += loss.value
        self.last_loss = loss.value
        return Hb, dw.value, int(fl)


def batch_stats(V, W, H, eps: float = 1e-12):
    """A, B of eq. (3) at fixed (W, H), eps-shifted."""
    V = _f64(V)
    F, N = V.shape
    W = _f64(W)
    K = W.shape[1]
    H = _f64(H, (K, N))
    A = np.zeros((F, K), order="F")
    B = np.zeros((F, K), order="F")
    _load().isnmf_ref_batch_stats(F, K, N, _p(V), F, _p(W), F, _p(H), K, float(eps), _p(A), _p(B))
    return A, B


def batch_cycle(V, W, H, eps: float = 1e-12, normalize: bool = True):
    """One batch MU cycle (section 2.1).  Returns (W_new, H_new, objective, flags)."""
    V = _f64(V)
    F, N = V.shape
    W = _f64(W).copy(order="F")
    K = W.shape[1]
    H = _f64(H, (K, N)).copy(order="F")
    obj = ctypes.c_double(0.0)
    fl = _load().isnmf_ref_batch_cycle(F, K, N, _p(V), F, _p(W), F, _p(H), K, float(eps),
                                       int(bool(normalize)), ctypes.byref(obj))
    if fl < 0:
        raise MemoryError("oracle allocation failed")
    return W, H, obj.value, int(fl)


def online_pass(V, W0, b: int, iters: int = 20, eps: float = 1e-12, rho: float = 1.0,
                normalize: bool = True, A0=None, B0=None, keep_h: bool = False,
                update_w: bool = True):
    """Fresh-restart one-pass run over all columns of V in minibatches of b
    (Algorithm 1 with beta = b; the final partial minibatch is a short step).
    update_w = False freezes W (statistics still accumulate).  Returns the
    final OnlineState (and the collected H if keep_h)."""
    V = _f64(V)
    st = OnlineState(W0, A0, B0)
    F, N = V.shape
    Hs = []
    for s in range(0, N, b):
        Hb, _, _ = st.step(V[:, s:s + b], iters=iters, eps=eps, rho=rho, normalize=normalize,
                           update_w=update_w)
        if keep_h:
            Hs.append(Hb)
    if keep_h:
        return st, np.asfortranarray(np.concatenate(Hs, axis=1)) if Hs else np.zeros((st.K, 0))
    return st


def online_passes(V, W0, b: int, perms, iters: int = 20, eps: float = 1e-12, rho: float = 1.0,
                  normalize: bool = True, H0=None, A0=None, B0=None):
    """Several passes of online IS-NMF over a finite set with warm restarts
    (section 2.3): the K x N activations stay resident, pass p visits the
    frames in the order perms[p] in minibatches of b (a short final one), and
    each frame's inner fit starts from its value of the previous visit (1 on
    the first, or H0).  Returns (OnlineState, H)."""
    V = _f64(V)
    F, N = V.shape
    st = OnlineState(W0, A0, B0)
    H = np.ones((st.K, N), order="F") if H0 is None else _f64(H0, (st.K, N)).copy(order="F")
    for order in perms:
        order = np.asarray(order, dtype=np.int64)
        if sorted(order.tolist()) != list(range(N)):
            raise ValueError("each pass must visit every frame once")
        for s in range(0, N, b):
            idx = order[s:s + b]
            Hb, _, _ = st.step(V[:, idx], iters=iters, eps=eps, rho=rho, normalize=normalize,
                               H=H[:, idx])
            H[:, idx] = Hb
    return st, H
