"""ctypes binding of libisnmf.so (C ABI in include/isnmf.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  torch supplies device memory and streams.  The library is
required: importing this module raises if it has not been built.

Matrix convention on the Python side.  The ABI is column-major; a column-major
F x N matrix is the same memory as a row-major (N, F) torch tensor.  So:
  V: (N, F) float32   frame n is row n
  W: (K, F) float32   component k is row k      (F x K column-major)
  H: (N, K) float32   activations of frame n   (K x N column-major)
  A, B: (K, F) float64
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisnmf.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
PREC = {"fp32": 0, "bf16": 1, "fp16": 2, "fp64": 3}
KERNEL = {"auto": 0, "plain": 1, "fused": 2}
KERNEL_NAME = {v: k for k, v in KERNEL.items()}


class Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("inner_iters", ctypes.c_int), ("rho", ctypes.c_double),
                ("normalize", ctypes.c_int), ("h_init", ctypes.c_int), ("precision", ctypes.c_int),
                ("kernel", ctypes.c_int), ("update_w", ctypes.c_int),
                ("psi_lambda", ctypes.c_double), ("psi_a", ctypes.c_double)]


class IsnmfError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1106_4198_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER(Params)
    sig = {
        "isnmf_params_default": (None, [P]),
        "isnmf_strerror": (ctypes.c_char_p, [i]),
        "isnmf_forgetting_rho": (i, [d, ctypes.c_longlong, ctypes.c_longlong,
                                     ctypes.POINTER(d)]),
        "isnmf_online_workspace_size": (sz, [i, i, i, P]),
        "isnmf_online_init": (i, [ctypes.POINTER(vp), i, i, i, P, vp, i, vp, vp, vp, sz, vp]),
        "isnmf_online_step": (i, [vp, vp, i, i, vp, i, vp, vp, vp]),
        "isnmf_online_get": (i, [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_longlong), vp]),
        "isnmf_online_get_w64": (i, [vp, vp, vp]),
        "isnmf_online_set": (i, [vp, vp, vp, vp, ctypes.c_longlong, vp]),
        "isnmf_online_set_w64": (i, [vp, vp, vp]),
        "isnmf_online_status": (i, [vp, ctypes.POINTER(i)]),
        "isnmf_online_info": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i),
                                  ctypes.POINTER(i)]),
        "isnmf_online_destroy": (i, [vp]),
        "isnmf_online_pass": (i, [vp, vp, i, ctypes.c_longlong, i, vp, i, vp, vp]),
        "isnmf_online_passes": (i, [vp, vp, i, ctypes.c_longlong, vp, i, i, vp, i, vp, vp]),
        "isnmf_online_fit": (i, [vp, vp, i, i, vp, i, vp, vp]),
        "isnmf_online_set_timing": (i, [vp, i, i]),
        "isnmf_online_timing": (i, [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(d)]),
        "isnmf_multi_workspace_size": (sz, [ctypes.POINTER(vp), i, ctypes.POINTER(i)]),
        "isnmf_multi_create": (i, [ctypes.POINTER(vp), ctypes.POINTER(vp), i, ctypes.POINTER(vp),
                                   ctypes.POINTER(i), ctypes.POINTER(ctypes.c_longlong),
                                   ctypes.POINTER(i), vp, vp, sz, vp]),
        "isnmf_multi_step": (i, [vp, vp]),
        "isnmf_multi_run": (i, [vp, i, i, vp]),
        "isnmf_multi_frames_left": (i, [vp, ctypes.POINTER(ctypes.c_longlong)]),
        "isnmf_multi_launches": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]),
        "isnmf_multi_destroy": (i, [vp]),
        "isnmf_autotune_workspace_size": (sz, [i, i, i, P]),
        "isnmf_autotune": (i, [i, i, i, P, i, ctypes.POINTER(i), ctypes.POINTER(d), vp, sz, vp]),
        "isnmf_tune_get": (i, [i, i, i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]),
        "isnmf_tune_set": (i, [i, i, i, i, i, i]),
        "isnmf_tune_clear": (None, []),
        "isnmf_server_workspace_size": (sz, [i, i, i]),
        "isnmf_server_create": (i, [ctypes.POINTER(vp), i, i, i, i, sz, vp, sz, vp]),
        "isnmf_server_open": (i, [vp, vp, sz, ctypes.POINTER(i)]),
        "isnmf_server_close": (i, [vp, i]),
        "isnmf_server_session_state": (i, [vp, i, ctypes.POINTER(i)]),
        "isnmf_server_admission": (i, [vp, ctypes.POINTER(sz), ctypes.POINTER(i),
                                       ctypes.POINTER(i)]),
        "isnmf_server_set_loss": (i, [vp, i, vp]),
        "isnmf_server_submit": (i, [vp, i, vp, i, i, d, ctypes.POINTER(ctypes.c_longlong)]),
        "isnmf_server_pump": (i, [vp, ctypes.POINTER(i)]),
        "isnmf_server_pending": (i, [vp, ctypes.POINTER(ctypes.c_longlong),
                                     ctypes.POINTER(ctypes.c_longlong)]),
        "isnmf_server_drain": (i, [vp]),
        "isnmf_server_results": (i, [vp, i, vp, vp, vp, vp, vp, vp, ctypes.POINTER(i)]),
        "isnmf_server_stats": (i, [vp, ctypes.POINTER(ctypes.c_longlong),
                                   ctypes.POINTER(ctypes.c_longlong)]),
        "isnmf_server_clock": (d, []),
        "isnmf_server_destroy": (i, [vp]),
        "isnmf_batch_workspace_size": (sz, [i, i, i, P]),
        "isnmf_batch_mu": (i, [vp, i, i, i, vp, i, vp, i, i, i, P, vp, vp, sz, vp]),
        "isnmf_objective_workspace_size": (sz, [i, i, i]),
        "isnmf_objective": (i, [vp, i, vp, i, vp, i, i, i, i, d, vp, vp, sz, vp]),
        "isnmf_objective_noalloc": (i, [vp, i, vp, i, vp, i, i, i, i, d, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("isnmf_params_default", "isnmf_strerror", "isnmf_forgetting_rho",
            "isnmf_online_workspace_size",
            "isnmf_online_init", "isnmf_online_step", "isnmf_online_get", "isnmf_online_get_w64",
            "isnmf_online_set", "isnmf_online_set_w64", "isnmf_online_status", "isnmf_online_info",
            "isnmf_online_destroy", "isnmf_online_pass", "isnmf_online_passes", "isnmf_online_fit",
            "isnmf_online_set_timing", "isnmf_online_timing",
            "isnmf_multi_workspace_size", "isnmf_multi_create", "isnmf_multi_step",
            "isnmf_multi_run", "isnmf_multi_frames_left", "isnmf_multi_launches", "isnmf_multi_destroy",
            "isnmf_autotune_workspace_size", "isnmf_autotune", "isnmf_tune_get", "isnmf_tune_set",
            "isnmf_tune_clear",
            "isnmf_server_workspace_size", "isnmf_server_create", "isnmf_server_open",
            "isnmf_server_close", "isnmf_server_session_state", "isnmf_server_admission",
            "isnmf_server_set_loss",
            "isnmf_server_submit", "isnmf_server_pump", "isnmf_server_pending",
            "isnmf_server_drain", "isnmf_server_results", "isnmf_server_stats",
            "isnmf_server_clock", "isnmf_server_destroy",
            "isnmf_batch_workspace_size", "isnmf_batch_mu",
            "isnmf_objective_workspace_size", "isnmf_objective", "isnmf_objective_noalloc")
OBJECTIVE_NOALLOC_MAX_FRAMES = 1 << 20   # ISNMF_OBJECTIVE_NOALLOC_MAX_FRAMES


def lib():
    return _lib


def strerror(code: int) -> str:
    return _lib.isnmf_strerror(int(code)).decode()


def _check(code: int, what: str):
    if code != OK:
        raise IsnmfError(code, what)


def forgetting_rho(r: float, beta: int, n_frames: int) -> float:
    """The weight of past statistics for forgetting factor r (section 2.3),
    computed by the library (isnmf_forgetting_rho): rho = r^(beta / N) with
    beta frames per W update and N frames in the set."""
    out = ctypes.c_double()
    code = _lib.isnmf_forgetting_rho(float(r), int(beta), int(n_frames), ctypes.byref(out))
    if code == EINVAL:
        raise ValueError("need 0 <= r <= 1, beta >= 1, n_frames >= 1")
    _check(code, "isnmf_forgetting_rho")
    return out.value


def make_params(eps=1e-12, inner_iters=20, rho=1.0, normalize=True, warm=False,
                precision="fp32", kernel="auto", update_w=True, psi=None) -> Params:
    """psi: None, or (lambda, a) of the penalty lambda log(a + sum_k h_k) on H."""
    p = Params()
    _lib.isnmf_params_default(ctypes.byref(p))
    if psi is not None:
        p.psi_lambda = float(psi[0])
        p.psi_a = float(psi[1])
    p.eps = float(eps)
    p.inner_iters = int(inner_iters)
    p.rho = float(rho)
    p.normalize = int(bool(normalize))
    p.h_init = 1 if warm else 0
    p.precision = PREC[precision]
    p.kernel = KERNEL[kernel]
    p.update_w = int(bool(update_w))
    return p


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _req(t, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.dim() == 2 and t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} rows must be contiguous")
    return t


def _ld(t):
    """Row stride in elements; a single row's stride is arbitrary (numpy and
    torch leave it so), and its row length serves."""
    if t.dim() != 2:
        return t.shape[-1]
    return t.stride(0) if t.shape[0] > 1 else t.shape[1]


class OnlineISNMF:
    """One online IS-NMF stream (Algorithm 1 with mini-batches) on the GPU."""

    def __init__(self, W0: torch.Tensor, b_max: int, *, eps=1e-12, inner_iters=20, rho=1.0,
                 normalize=True, warm=False, precision="fp32", kernel="auto", update_w=True,
                 A0=None, B0=None, stream=None, psi=None):
        _req(W0, torch.float32, name="W0")
        K, F = W0.shape
        self.F, self.K, self.b_max = int(F), int(K), int(b_max)
        self.params = make_params(eps, inner_iters, rho, normalize, warm, precision, kernel,
                                  update_w, psi)
        self.warm = bool(warm)
        nbytes = _lib.isnmf_online_workspace_size(self.F, self.K, self.b_max,
                                                  ctypes.byref(self.params))
        if nbytes == 0:
            raise IsnmfError(EINVAL, "isnmf_online_workspace_size")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=W0.device)
        if A0 is not None:
            _req(A0, torch.float64, (K, F), "A0")
        if B0 is not None:
            _req(B0, torch.float64, (K, F), "B0")
        h = ctypes.c_void_p()
        _check(_lib.isnmf_online_init(ctypes.byref(h), self.F, self.K, self.b_max,
                                      ctypes.byref(self.params), _ptr(W0), _ld(W0),
                                      _ptr(A0), _ptr(B0), _ptr(self.workspace),
                                      nbytes, _stream(stream)), "isnmf_online_init")
        self._h = h
        self.device = W0.device

    @property
    def kernel_used(self) -> str:
        k = ctypes.c_int()
        _check(_lib.isnmf_online_info(self._h, None, None, None, ctypes.byref(k)), "info")
        return KERNEL_NAME[k.value]

    def step(self, Vb: torch.Tensor, H: torch.Tensor | None = None, loss_sum=None, dw=None,
             stream=None):
        """Vb: (b, F) float32 frames.  H: (b, K) float32 out (in/out when warm).
        loss_sum, dw: optional float64 device scalars (loss is added)."""
        _req(Vb, torch.float32, name="Vb")
        b = Vb.shape[0]
        if Vb.shape[1] != self.F:
            raise ValueError("frame length != F")
        if H is not None:
            _req(H, torch.float32, (b, self.K), "H")
        _check(_lib.isnmf_online_step(self._h, _ptr(Vb), _ld(Vb), b, _ptr(H),
                                      _ld(H) if H is not None else self.K,
                                      _ptr(loss_sum), _ptr(dw), _stream(stream)),
               "isnmf_online_step")

    def run_pass(self, V: torch.Tensor, b: int, H: torch.Tensor | None = None, loss_sum=None,
                 stream=None):
        """Consecutive minibatches of b frames over all rows of V (N, F)."""
        _req(V, torch.float32, name="V")
        N = V.shape[0]
        if H is not None:
            _req(H, torch.float32, (N, self.K), "H")
        _check(_lib.isnmf_online_pass(self._h, _ptr(V), _ld(V), int(N), int(b), _ptr(H),
                                      _ld(H) if H is not None else self.K, _ptr(loss_sum),
                                      _stream(stream)), "isnmf_online_pass")

    def run_passes(self, V: torch.Tensor, perm: torch.Tensor, b: int, H: torch.Tensor,
                   loss_sum=None, stream=None):
        """Warm-restart passes over the finite set V (N, F): pass p visits the
        frames in the order perm[p] (perm: (passes, N) int32 on the device),
        in minibatches of b; H (N, K) holds every frame's h across passes."""
        _req(V, torch.float32, name="V")
        N = V.shape[0]
        _req(H, torch.float32, (N, self.K), "H")
        if perm.dtype != torch.int32 or perm.dim() != 2 or perm.shape[1] != N or \
                not perm.is_contiguous() or perm.device != V.device:
            raise ValueError("perm must be a contiguous (passes, N) int32 tensor on V's device")
        _check(_lib.isnmf_online_passes(self._h, _ptr(V), _ld(V), int(N), _ptr(perm),
                                        int(perm.shape[0]), int(b), _ptr(H), _ld(H),
                                        _ptr(loss_sum), _stream(stream)), "isnmf_online_passes")

    def fit(self, Vb: torch.Tensor, H: torch.Tensor | None = None, loss_sum=None, stream=None):
        """Inner fit only at the current W (A, B, W unchanged)."""
        _req(Vb, torch.float32, name="Vb")
        b = Vb.shape[0]
        if H is not None:
            _req(H, torch.float32, (b, self.K), "H")
        _check(_lib.isnmf_online_fit(self._h, _ptr(Vb), _ld(Vb), b, _ptr(H),
                                     _ld(H) if H is not None else self.K, _ptr(loss_sum),
                                     _stream(stream)), "isnmf_online_fit")

    def set_timing(self, enable: bool, capacity: int = 1 << 14):
        _check(_lib.isnmf_online_set_timing(self._h, int(bool(enable)), int(capacity)), "set_timing")

    def timing(self):
        """(timed fit launches, total milliseconds) since the last call."""
        n = ctypes.c_longlong()
        ms = ctypes.c_double()
        _check(_lib.isnmf_online_timing(self._h, ctypes.byref(n), ctypes.byref(ms)), "timing")
        return n.value, ms.value

    def get(self, stream=None):
        W = torch.empty((self.K, self.F), dtype=torch.float32, device=self.device)
        A = torch.empty((self.K, self.F), dtype=torch.float64, device=self.device)
        B = torch.empty_like(A)
        t = ctypes.c_longlong()
        _check(_lib.isnmf_online_get(self._h, _ptr(W), _ptr(A), _ptr(B), ctypes.byref(t),
                                     _stream(stream)), "isnmf_online_get")
        return W, A, B, t.value

    def get_w64(self, stream=None):
        W = torch.empty((self.K, self.F), dtype=torch.float64, device=self.device)
        _check(_lib.isnmf_online_get_w64(self._h, _ptr(W), _stream(stream)), "get_w64")
        return W

    def set(self, W=None, A=None, B=None, t=0, stream=None):
        for x, dt, nm in ((W, torch.float32, "W"), (A, torch.float64, "A"), (B, torch.float64, "B")):
            if x is not None:
                _req(x, dt, (self.K, self.F), nm)
        _check(_lib.isnmf_online_set(self._h, _ptr(W), _ptr(A), _ptr(B), int(t), _stream(stream)),
               "isnmf_online_set")

    def set_w64(self, W, stream=None):
        _req(W, torch.float64, (self.K, self.F), "W")
        _check(_lib.isnmf_online_set_w64(self._h, _ptr(W), _stream(stream)), "set_w64")

    def status(self) -> int:
        f = ctypes.c_int()
        code = _lib.isnmf_online_status(self._h, ctypes.byref(f))
        if code not in (OK, ENONFINITE):
            _check(code, "isnmf_online_status")
        return f.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.isnmf_online_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MultiISNMF:
    """Batched form: several OnlineISNMF streams advanced one minibatch per step
    in shared launches (optionally one replayed hipGraph per step)."""

    def __init__(self, streams, V, b, loss=True, stream=None):
        S = len(streams)
        if S < 1 or len(V) != S or len(b) != S:
            raise ValueError("need one V and one b per stream")
        for g, v in zip(streams, V):
            _req(v, torch.float32, name="V")
            if v.shape[1] != g.F:
                raise ValueError("frame length != F")
        self.streams = list(streams)
        self.V = list(V)
        H = (ctypes.c_void_p * S)(*[g._h for g in streams])
        Vp = (ctypes.c_void_p * S)(*[v.data_ptr() for v in V])
        ld = (ctypes.c_int * S)(*[_ld(v) for v in V])
        nf = (ctypes.c_longlong * S)(*[v.shape[0] for v in V])
        bb = (ctypes.c_int * S)(*[int(x) for x in b])
        dev = V[0].device
        self.loss = torch.zeros(S, dtype=torch.float64, device=dev) if loss else None
        nbytes = _lib.isnmf_multi_workspace_size(H, S, bb)
        if nbytes == 0:
            raise IsnmfError(EINVAL, "isnmf_multi_workspace_size")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        m = ctypes.c_void_p()
        _check(_lib.isnmf_multi_create(ctypes.byref(m), H, S, Vp, ld, nf, bb, _ptr(self.loss),
                                       _ptr(self.workspace), nbytes, _stream(stream)),
               "isnmf_multi_create")
        self._m = m

    def step(self, stream=None):
        _check(_lib.isnmf_multi_step(self._m, _stream(stream)), "isnmf_multi_step")

    def run(self, steps: int, graph: bool = True, stream=None):
        _check(_lib.isnmf_multi_run(self._m, int(steps), int(bool(graph)), _stream(stream)),
               "isnmf_multi_run")

    def frames_left(self) -> int:
        n = ctypes.c_longlong()
        _check(_lib.isnmf_multi_frames_left(self._m, ctypes.byref(n)), "frames_left")
        return n.value

    def launches(self) -> tuple:
        """(fit, fold, rescale) launches of one step; no fold or rescale launch
        when every fit launch folds and rescales its streams itself."""
        f, g, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.isnmf_multi_launches(self._m, ctypes.byref(f), ctypes.byref(g), ctypes.byref(r)),
               "launches")
        return f.value, g.value, r.value

    def close(self):
        if getattr(self, "_m", None):
            _lib.isnmf_multi_destroy(self._m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching engine over many sessions (see include/isnmf.h)."""

    def __init__(self, max_sessions=1024, max_per_step=1024, max_frames=65536, inflight=2,
                 hbm_budget=1 << 40, device="cuda", stream=None):
        nbytes = _lib.isnmf_server_workspace_size(max_sessions, max_per_step, inflight)
        if nbytes == 0:
            raise IsnmfError(EINVAL, "isnmf_server_workspace_size")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        s = ctypes.c_void_p()
        _check(_lib.isnmf_server_create(ctypes.byref(s), max_sessions, max_per_step, max_frames,
                                        inflight, int(hbm_budget), _ptr(self.workspace), nbytes,
                                        _stream(stream)), "isnmf_server_create")
        self._s = s
        self.sessions = {}
        self._loss = {}     # session id -> its running-loss tensor (read by the device)
        self._chunks = {}   # request id -> its frames (read by the device until done)

    WAITING, RESIDENT, CLOSING, CLOSED = 0, 1, 2, 3

    def open(self, g: "OnlineISNMF", footprint=None) -> int:
        """Open a session on handle g; it is admitted at once or waits for
        room (state()).  footprint defaults to g's workspace bytes."""
        fp = g.workspace.numel() if footprint is None else int(footprint)
        idx = ctypes.c_int()
        _check(_lib.isnmf_server_open(self._s, g._h, fp, ctypes.byref(idx)), "isnmf_server_open")
        self.sessions[idx.value] = g
        return idx.value

    def close_session(self, session: int) -> None:
        """No more chunks for this session; its footprint returns to the engine
        once its submitted chunks have completed."""
        _check(_lib.isnmf_server_close(self._s, int(session)), "isnmf_server_close")

    def state(self, session: int) -> int:
        st = ctypes.c_int()
        _check(_lib.isnmf_server_session_state(self._s, int(session), ctypes.byref(st)),
               "isnmf_server_session_state")
        if st.value == self.CLOSED:
            self._loss.pop(int(session), None)
        return st.value

    def admission(self):
        """(footprint bytes held by resident sessions, resident, waiting)."""
        u, r, w = ctypes.c_size_t(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.isnmf_server_admission(self._s, ctypes.byref(u), ctypes.byref(r),
                                           ctypes.byref(w)), "isnmf_server_admission")
        return u.value, r.value, w.value

    def set_loss(self, session: int, loss) -> None:
        """Accumulate the session's running loss (sum of d_IS over its served
        chunks, FP64) into `loss`, a float64 device scalar (None: stop)."""
        p = None
        if loss is not None:
            _req(loss, torch.float64, name="loss")
            if loss.numel() != 1:
                raise ValueError("loss must be a single float64 element")
            p = loss.data_ptr()
        _check(_lib.isnmf_server_set_loss(self._s, int(session), p), "isnmf_server_set_loss")
        if loss is None:
            self._loss.pop(int(session), None)
        else:
            self._loss[int(session)] = loss

    def submit(self, session: int, V: torch.Tensor, arrival: float = -1.0) -> int:
        """V: (n, F) float32 frames on the device (kept alive until done)."""
        _req(V, torch.float32, name="V")
        r = ctypes.c_longlong()
        _check(_lib.isnmf_server_submit(self._s, int(session), _ptr(V), _ld(V), V.shape[0],
                                        float(arrival), ctypes.byref(r)), "isnmf_server_submit")
        self._chunks[r.value] = V
        return r.value

    def pump(self) -> int:
        f = ctypes.c_int()
        _check(_lib.isnmf_server_pump(self._s, ctypes.byref(f)), "isnmf_server_pump")
        return f.value

    def pending(self):
        q, f = ctypes.c_longlong(), ctypes.c_longlong()
        _check(_lib.isnmf_server_pending(self._s, ctypes.byref(q), ctypes.byref(f)), "pending")
        return q.value, f.value

    def drain(self):
        _check(_lib.isnmf_server_drain(self._s), "isnmf_server_drain")

    def results(self, max_out=1 << 16):
        import numpy as np
        req = np.zeros(max_out, np.int64)
        ses = np.zeros(max_out, np.int32)
        nfr = np.zeros(max_out, np.int32)
        arr = np.zeros(max_out)
        sta = np.zeros(max_out)
        don = np.zeros(max_out)
        c = ctypes.c_int()
        P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(_lib.isnmf_server_results(self._s, max_out, P(req), P(ses), P(nfr), P(arr), P(sta),
                                         P(don), ctypes.byref(c)), "isnmf_server_results")
        n = c.value
        for r in req[:n]:
            self._chunks.pop(int(r), None)
        return {"req": req[:n], "session": ses[:n], "frames": nfr[:n], "arrival": arr[:n],
                "start": sta[:n], "done": don[:n]}

    def stats(self):
        st, fr = ctypes.c_longlong(), ctypes.c_longlong()
        _check(_lib.isnmf_server_stats(self._s, ctypes.byref(st), ctypes.byref(fr)), "stats")
        return st.value, fr.value

    @staticmethod
    def clock() -> float:
        return _lib.isnmf_server_clock()

    def close(self):
        if getattr(self, "_s", None):
            _lib.isnmf_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(F: int, K: int, b: int, precision="bf16", inner_iters=20, trials=5, stream=None):
    """Time the fit kernel variants for this shape; the fastest is used by
    handles created afterwards.  Returns (variant index, microseconds)."""
    p = make_params(inner_iters=inner_iters, precision=precision)
    v = ctypes.c_int()
    us = ctypes.c_double()
    nbytes = _lib.isnmf_autotune_workspace_size(int(F), int(K), int(b), ctypes.byref(p))
    if nbytes == 0:
        raise IsnmfError(EINVAL, "isnmf_autotune_workspace_size")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=torch.cuda.current_device())
    _check(_lib.isnmf_autotune(int(F), int(K), int(b), ctypes.byref(p), int(trials),
                               ctypes.byref(v), ctypes.byref(us), _ptr(ws), nbytes,
                               _stream(stream)), "isnmf_autotune")
    return v.value, us.value


def tune_get(F: int, K: int, precision="bf16"):
    nw, cpw, wg = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_lib.isnmf_tune_get(int(F), int(K), PREC[precision], ctypes.byref(nw), ctypes.byref(cpw),
                               ctypes.byref(wg)), "isnmf_tune_get")
    return nw.value, cpw.value, wg.value


def tune_set(F: int, K: int, precision: str, nw: int, cpw: int, wg: int):
    _check(_lib.isnmf_tune_set(int(F), int(K), PREC[precision], int(nw), int(cpw), int(wg)),
           "isnmf_tune_set")


def tune_clear():
    _lib.isnmf_tune_clear()


def save_tuning(path: str, shapes):
    """Write the tuning table entries for `shapes` [(F, K, precision)] as JSON."""
    import json
    rows = []
    for F, K, pr in shapes:
        nw, cpw, wg = tune_get(F, K, pr)
        rows.append({"F": F, "K": K, "precision": pr, "nw": nw, "cpw": cpw, "wg": wg})
    with open(path, "w") as f:
        json.dump(rows, f, indent=1)


def load_tuning(path: str):
    import json
    with open(path) as f:
        for r in json.load(f):
            tune_set(r["F"], r["K"], r["precision"], r["nw"], r["cpw"], r["wg"])


def batch_mu(V: torch.Tensor, W: torch.Tensor, H: torch.Tensor, cycles: int, *, eps=1e-12,
             normalize=True, precision="fp32", kernel="auto", trace=True, stream=None):
    """In-place batch MU cycles (section 2.1).  V (N, F), W (K, F), H (N, K) float32.
    Returns the device float64 objective trace (cycles,) or None."""
    _req(V, torch.float32, name="V")
    _req(W, torch.float32, name="W")
    N, F = V.shape
    K = W.shape[0]
    _req(H, torch.float32, (N, K), "H")
    p = make_params(eps=eps, normalize=normalize, precision=precision, kernel=kernel)
    nbytes = _lib.isnmf_batch_workspace_size(F, K, N, ctypes.byref(p))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=V.device)
    tr = torch.zeros(max(cycles, 1), dtype=torch.float64, device=V.device) if trace else None
    _check(_lib.isnmf_batch_mu(_ptr(V), _ld(V), F, N, _ptr(W), _ld(W), _ptr(H), _ld(H), K,
                               int(cycles), ctypes.byref(p), _ptr(tr), _ptr(ws), nbytes,
                               _stream(stream)), "isnmf_batch_mu")
    return tr[:cycles] if trace else None


def objective(V: torch.Tensor, W: torch.Tensor, H: torch.Tensor, eps=1e-12, stream=None):
    """(1/N) sum_n d_IS(eps + v_n, eps + W h_n) as a device float64 scalar."""
    _req(V, torch.float32, name="V")
    _req(W, torch.float32, name="W")
    N, F = V.shape
    K = W.shape[0]
    _req(H, torch.float32, (N, K), "H")
    nbytes = _lib.isnmf_objective_workspace_size(F, K, N)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=V.device)
    out = torch.zeros((), dtype=torch.float64, device=V.device)
    _check(_lib.isnmf_objective(_ptr(V), _ld(V), _ptr(W), _ld(W), _ptr(H), _ld(H), F, K, N,
                                float(eps), _ptr(out), _ptr(ws), nbytes, _stream(stream)),
           "isnmf_objective")
    return out


def objective_noalloc(V: torch.Tensor, W: torch.Tensor, H: torch.Tensor, out: torch.Tensor,
                      eps=1e-12, stream=None):
    """As objective(), through isnmf_objective_noalloc: no workspace, the
    library's own fixed per-device buffer (N <= OBJECTIVE_NOALLOC_MAX_FRAMES).
    out: a float64 device scalar the caller owns; the result is written there."""
    _req(V, torch.float32, name="V")
    _req(W, torch.float32, name="W")
    N, F = V.shape
    K = W.shape[0]
    _req(H, torch.float32, (N, K), "H")
    _req(out, torch.float64, name="out")
    _check(_lib.isnmf_objective_noalloc(_ptr(V), _ld(V), _ptr(W), _ld(W), _ptr(H), _ld(H), F, K,
                                        N, float(eps), _ptr(out), _stream(stream)),
           "isnmf_objective_noalloc")
    return out
