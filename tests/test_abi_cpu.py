"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device.  No
compute runs here (no GPU in this environment)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "isnmf.h")
LIB = os.path.join(ROOT, "paper_1106_4198_amd", "libisnmf.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(isnmf_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libisnmf.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["isnmf_online_init", "isnmf_online_step", "isnmf_batch_mu", "isnmf_objective",
                 "isnmf_online_get", "isnmf_online_set", "isnmf_online_destroy",
                 "isnmf_online_workspace_size", "isnmf_strerror"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_1106_4198_amd import binding
    assert sorted(binding.EXPORTED) == _declared()


def test_defaults_and_strerror():
    from paper_1106_4198_amd import binding as bd
    p = bd.Params()
    bd.lib().isnmf_params_default(ctypes.byref(p))
    assert p.eps == 1e-12 and p.inner_iters == 20 and p.rho == 1.0 and p.normalize == 1
    assert p.h_init == 0 and p.precision == 0 and p.kernel == 0 and p.update_w == 1
    for code in range(0, -7, -1):
        assert bd.strerror(code) and bd.strerror(code) != "unknown status"
    assert bd.strerror(-99) == "unknown status"


def test_params_default_has_no_penalty():
    from paper_1106_4198_amd import binding as bd
    p = bd.make_params()
    assert p.psi_lambda == 0.0 and p.psi_a == 1.0
    q = bd.make_params(psi=(2.5, 0.25))
    assert q.psi_lambda == 2.5 and q.psi_a == 0.25


def test_workspace_sizes_are_host_only_and_grow():
    from paper_1106_4198_amd import binding as bd
    L = bd.lib()
    p = bd.make_params()
    s1 = L.isnmf_online_workspace_size(513, 50, 128, ctypes.byref(p))
    s2 = L.isnmf_online_workspace_size(513, 50, 256, ctypes.byref(p))
    assert s1 > 0 and s2 > s1 and s1 % 256 == 0
    # F*K state: W64, W32, W16, A, B, Wn at least
    assert s1 >= 513 * 50 * (8 + 4 + 2 + 8 + 8 + 8)
    assert L.isnmf_online_workspace_size(0, 50, 128, ctypes.byref(p)) == 0
    assert L.isnmf_online_workspace_size(513, 0, 128, ctypes.byref(p)) == 0
    assert L.isnmf_batch_workspace_size(513, 50, 1000, ctypes.byref(p)) > 0
    assert L.isnmf_objective_workspace_size(513, 50, 1000) >= 8000


def test_einval_before_any_device_work():
    """These argument errors return before any HIP call (no GPU here)."""
    from paper_1106_4198_amd import binding as bd
    L = bd.lib()
    p = bd.make_params()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(256)            # never dereferenced: rejected first
    assert L.isnmf_online_init(None, 10, 2, 4, ctypes.byref(p), fake, 10, None, None, fake, 1 << 20, None) == bd.EINVAL
    assert L.isnmf_online_init(ctypes.byref(h), 0, 2, 4, ctypes.byref(p), fake, 10, None, None, fake, 1 << 20, None) == bd.EINVAL
    assert L.isnmf_online_init(ctypes.byref(h), 10, 2, 4, ctypes.byref(p), fake, 9, None, None, fake, 1 << 20, None) == bd.EINVAL
    bad = bd.make_params(rho=1.5)
    assert L.isnmf_online_init(ctypes.byref(h), 10, 2, 4, ctypes.byref(bad), fake, 10, None, None, fake, 1 << 20, None) == bd.EINVAL
    bad = bd.make_params(eps=-1.0)
    assert L.isnmf_online_init(ctypes.byref(h), 10, 2, 4, ctypes.byref(bad), fake, 10, None, None, fake, 1 << 20, None) == bd.EINVAL
    bad = bd.make_params(inner_iters=-1)
    assert L.isnmf_online_init(ctypes.byref(h), 10, 2, 4, ctypes.byref(bad), fake, 10, None, None, fake, 1 << 20, None) == bd.EINVAL
    # penalty on H: lambda >= 0 and a > 0, finite
    for psi in ((-1.0, 1.0), (1.0, 0.0), (1.0, -2.0), (float("nan"), 1.0), (1.0, float("inf"))):
        bad = bd.make_params(psi=psi)
        assert L.isnmf_online_init(ctypes.byref(h), 10, 2, 4, ctypes.byref(bad), fake, 10, None, None, fake, 1 << 20, None) == bd.EINVAL, psi
    # the penalty is refused by the 16-bit forms and by the batch MU
    for prec in ("bf16", "fp16"):
        pen = bd.make_params(precision=prec, psi=(1.0, 1.0))
        assert L.isnmf_online_init(ctypes.byref(h), 64, 8, 4, ctypes.byref(pen), fake, 64, None, None, fake, 1 << 30, None) == bd.EUNSUPPORTED
    pen = bd.make_params(kernel="fused", psi=(1.0, 1.0))       # no VALU variant at K = 65
    assert L.isnmf_online_init(ctypes.byref(h), 10, 65, 4, ctypes.byref(pen), fake, 10, None, None, fake, 1 << 30, None) == bd.EUNSUPPORTED
    pen = bd.make_params(psi=(1.0, 1.0))
    assert L.isnmf_batch_mu(fake, 10, 10, 5, fake, 10, fake, 2, 2, 1, ctypes.byref(pen), None, fake, 1 << 30, None) == bd.EUNSUPPORTED
    # misaligned workspace
    assert L.isnmf_online_init(ctypes.byref(h), 10, 2, 4, ctypes.byref(p), fake, 10, None, None, ctypes.c_void_p(260), 1 << 20, None) == bd.EINVAL
    # too small workspace
    assert L.isnmf_online_init(ctypes.byref(h), 10, 2, 4, ctypes.byref(p), fake, 10, None, None, fake, 16, None) == bd.ENOMEM
    # fused kernel requested for an unsupported shape
    fz = bd.make_params(kernel="fused")
    assert L.isnmf_online_init(ctypes.byref(h), 10, 65, 4, ctypes.byref(fz), fake, 10, None, None, fake, 1 << 30, None) == bd.EUNSUPPORTED
    assert h.value is None
    # null handle
    assert L.isnmf_online_step(None, fake, 10, 1, None, 2, None, None, None) == bd.EINVAL
    assert L.isnmf_batch_mu(None, 10, 10, 5, fake, 10, fake, 2, 2, 1, None, None, fake, 1 << 20, None) == bd.EINVAL
    assert L.isnmf_objective(fake, 9, fake, 10, fake, 2, 10, 2, 5, 0.0, fake, fake, 1 << 20, None) == bd.EINVAL
    # a served session's running loss needs a server (checked before any device work)
    assert L.isnmf_server_set_loss(None, 0, fake) == bd.EINVAL
    # a batched plan's launch count needs a plan and all three outputs
    n1, n2, n3 = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert L.isnmf_multi_launches(None, ctypes.byref(n1), ctypes.byref(n2), ctypes.byref(n3)) == bd.EINVAL
    assert L.isnmf_multi_launches(fake, None, ctypes.byref(n2), ctypes.byref(n3)) == bd.EINVAL
    assert L.isnmf_multi_launches(fake, ctypes.byref(n1), None, ctypes.byref(n3)) == bd.EINVAL
    assert L.isnmf_multi_launches(fake, ctypes.byref(n1), ctypes.byref(n2), None) == bd.EINVAL


def test_product_path_does_not_touch_the_oracle():
    """The package never imports the oracle (the oracle is test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_1106_4198_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in src and "from oracle" not in src, fn
                assert "isnmf_ref_" not in src, fn


def test_forgetting_rho_follows_section_2_3():
    """rho = r^(beta/N): r itself when beta = N, 1 in the limit of a large set,
    0 for the batch reading (r = 0, beta = N), and equal r^(1/N) per frame
    whatever beta (rho^(N/beta) = r)."""
    from paper_1106_4198_amd import binding
    assert binding.forgetting_rho(0.7, 1000, 1000) == pytest.approx(0.7, rel=0, abs=1e-15)
    assert binding.forgetting_rho(0.0, 500, 500) == 0.0
    assert binding.forgetting_rho(0.7, 1000, 10**12) == pytest.approx(1.0, abs=1e-9)
    for beta in (1, 10, 128, 1000):
        rho = binding.forgetting_rho(0.7, beta, 10**5)
        assert rho ** (10**5 / beta) == pytest.approx(0.7, rel=1e-9)
    with pytest.raises(ValueError):
        binding.forgetting_rho(1.5, 10, 10)


# a citation of the paper, an interface entry marked as not part of the
# method, or (the one no-allocation entry point) the callers it is for
CITE = re.compile(r"section \d|eq\. ?\(?\d|Algorithm 1|Not part of the method|"
                  r"callers that cannot allocate", re.I)


def _entries_with_comments():
    """(function name, the comment block directly above its declaration).
    Declarations that follow one another with no blank line share the
    comment above the first of them."""
    lines = open(HEADER).read().split("\n")
    out, in_comment = [], False
    for i, ln in enumerate(lines):
        starts_comment = ln.lstrip().startswith("/*")
        if not in_comment and not starts_comment:
            m = re.match(r"^\S.*?\b(isnmf_[a-z0-9_]+)\s*\(", ln)
            if m:
                j, comment = i - 1, ""
                while j >= 0 and lines[j].strip():
                    if lines[j].rstrip().endswith("*/"):
                        k = j
                        while "/*" not in lines[k]:
                            k -= 1
                        comment = "\n".join(lines[k:j + 1])
                        break
                    j -= 1
                out.append((m.group(1), comment))
        if "/*" in ln and "*/" not in ln[ln.index("/*"):]:
            in_comment = True
        if in_comment and "*/" in ln:
            in_comment = False
    return out


def test_every_header_entry_cites_its_passage():
    """Each declared entry point has a comment that cites the passage of the
    paper defining its operation (section, equation or Algorithm 1), or says
    it is not part of the method (interface bookkeeping)."""
    entries = _entries_with_comments()
    assert len({n for n, _ in entries}) == len(_declared())
    flat = [(n, re.sub(r"\s*\n\s*\*?\s*", " ", c)) for n, c in entries]
    missing = [n for n, c in flat if not CITE.search(c)]
    assert not missing, missing


def test_binding_holds_no_arithmetic_of_the_method():
    """The Python binding only marshals arguments: no power, exponential,
    logarithm, square root or division on values (sizes aside), no math or
    numpy arithmetic module calls."""
    import ast
    src = open(os.path.join(ROOT, "paper_1106_4198_amd", "binding.py")).read()
    tree = ast.parse(src)
    bad = []
    for node in ast.walk(tree):
        if isinstance(node, ast.BinOp) and isinstance(node.op, (ast.Pow, ast.Div)):
            bad.append(ast.unparse(node))
        if isinstance(node, (ast.Import, ast.ImportFrom)):
            names = [a.name for a in node.names] + [getattr(node, "module", None) or ""]
            if any(n in ("math", "cmath") for n in names):
                bad.append("import math")
        if isinstance(node, ast.Attribute) and isinstance(node.value, ast.Name) and \
                node.value.id in ("np", "numpy", "math", "torch") and \
                node.attr in ("exp", "log", "sqrt", "power", "pow", "log2", "log1p", "expm1"):
            bad.append(ast.unparse(node))
    assert not bad, bad


def test_forgetting_rho_is_a_library_call():
    """rho = r^(beta/N) (section 2.3) is computed by the library (a host-only
    call); the binding forwards to it."""
    from paper_1106_4198_amd import binding as bd
    r = ctypes.c_double()
    L = bd.lib()
    assert L.isnmf_forgetting_rho(0.7, 1000, 1000, ctypes.byref(r)) == bd.OK
    assert r.value == 0.7
    assert L.isnmf_forgetting_rho(0.7, 10, 0, ctypes.byref(r)) == bd.EINVAL
    assert L.isnmf_forgetting_rho(-0.1, 10, 10, ctypes.byref(r)) == bd.EINVAL
    assert L.isnmf_forgetting_rho(0.5, 0, 10, ctypes.byref(r)) == bd.EINVAL
    assert L.isnmf_forgetting_rho(0.5, 1, 10, None) == bd.EINVAL
    assert bd.forgetting_rho(0.25, 2, 4) == 0.5


def test_single_row_tensors_get_their_row_length_as_stride():
    """A one-row matrix (K = 1 as K x F, or one frame) may carry any row stride
    (numpy's relaxed strides give 1 for np.ascontiguousarray of a transposed
    F x 1 array); the binding passes its row length as the leading dimension."""
    import numpy as np
    import torch
    from paper_1106_4198_amd import binding as bd
    t = torch.from_numpy(np.ascontiguousarray(np.zeros((64, 1), dtype=np.float32).T))
    assert t.shape == (1, 64)
    assert bd._ld(t) == 64
    u = torch.zeros((5, 64), dtype=torch.float32)
    assert bd._ld(u) == 64 and bd._ld(u[:, :10]) == 64 and bd._ld(u[2:3]) == 64
    assert bd._ld(torch.zeros((3, 1))[:, :]) == 1
