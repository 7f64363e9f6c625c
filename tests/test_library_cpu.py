"""The C-ABI library on the CPU: it loads, exports every declared symbol, its
host eigensolver matches LAPACK, and argument checks that need no device
return the documented status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gleanvec.h")
LIB = os.path.join(ROOT, "paper_2410_22347_amd", "libgleanvec.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libgleanvec.so not built")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gv_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    syms = declared_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_covers_header():
    import paper_2410_22347_amd as gv
    assert sorted(gv.EXPORTED) == declared_symbols()


def test_status_strings():
    import paper_2410_22347_amd as gv
    assert gv.status_string(0) == "ok"
    assert gv.status_string(-1) == "invalid argument"
    assert gv.status_string(-6) == "unsupported"


@pytest.mark.parametrize("n", [1, 2, 7, 64, 257])
def test_host_eigensolver_matches_lapack(n):
    import paper_2410_22347_amd as gv
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n))
    A = M @ M.T / n
    lam, Vt = gv.host_eigh(A)
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    assert np.allclose(lam, ref, atol=1e-12 * max(1.0, ref[0]))
    assert np.allclose(Vt @ Vt.T, np.eye(n), atol=1e-12)
    assert np.allclose(A @ Vt.T, Vt.T * lam, atol=1e-11 * max(1.0, ref[0]))


def test_host_eigensolver_repeated_and_indefinite():
    import paper_2410_22347_amd as gv
    rng = np.random.default_rng(5)
    U, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam0 = np.repeat([3.0, -1.0, 0.0, 2.0], 10)
    A = (U * lam0) @ U.T
    lam, Vt = gv.host_eigh(A)
    assert np.allclose(lam, np.sort(lam0)[::-1], atol=1e-12)
    assert np.allclose(A @ Vt.T, Vt.T * lam, atol=1e-12)
    # a diagonal matrix and a 2x2 with a zero off-diagonal
    lam, Vt = gv.host_eigh(np.diag([1.0, 5.0, 3.0]))
    assert lam.tolist() == [5.0, 3.0, 1.0]


def test_host_argument_errors():
    import paper_2410_22347_amd as gv
    lib = gv._lib
    h = ctypes.c_void_p()
    mu = np.zeros((2, 4)); A = np.zeros((2, 3, 4))
    # d > D, C out of range, NULL inputs: rejected before any device call
    assert lib.gv_model_import(gv._np_ptr(mu), gv._np_ptr(A), gv._np_ptr(A), 2, 5, 4, ctypes.byref(h)) == -1
    assert lib.gv_model_import(gv._np_ptr(mu), gv._np_ptr(A), gv._np_ptr(A), 0, 3, 4, ctypes.byref(h)) == -1
    assert lib.gv_model_import(None, None, None, 2, 3, 4, ctypes.byref(h)) == -1
    assert h.value is None
    bad = A.copy(); bad[0, 0, 0] = np.nan
    assert lib.gv_model_import(gv._np_ptr(mu), gv._np_ptr(bad), gv._np_ptr(A), 2, 3, 4, ctypes.byref(h)) == -5
    assert b"d <= D" in lib.gv_last_error() or lib.gv_last_error() == b""
    # invalid handles
    assert lib.gv_model_shape(None, None, None, None) == -4
    assert lib.gv_index_shape(None, None, None, None, None, None) == -4
    assert lib.gv_search(None, None, None, 1, 10, 20, None, None, None) == -4
    assert lib.gv_model_stats(None, None, None, None, None, None, None, None) == -4
    assert lib.gv_host_eigh(0, None, None, None) == -1
    assert lib.gv_search_tuning(0, 48, 0) == -1
    assert lib.gv_search_tuning(0, 0, 100) == -1
    assert lib.gv_search_tuning(5000, 0, 0) == -1
    assert lib.gv_search_tuning(0, 0, 0) == 0
    lib.gv_model_destroy(None)
    lib.gv_index_destroy(None)


def test_padded_dim():
    import paper_2410_22347_amd as gv
    assert [gv.padded_dim(d) for d in (0, 1, 16, 32, 33, 64, 100, 128, 129, 160, 161, 192, 200, 256)] == \
        [0, 32, 32, 32, 64, 64, 128, 128, 160, 160, 192, 192, 256, 256]


def test_loss_argument_errors():
    """Invalid sizes or pointers are rejected before any device call."""
    import paper_2410_22347_amd as gv
    lib = gv._lib
    p = ctypes.c_void_p(16)  # never dereferenced: the checks fail first
    assert lib.gv_loss_grad(0, 4, 8, p, p, p, p, 1.0, p, None, None, None) == -1
    assert lib.gv_loss_grad(2, 9, 8, p, p, p, p, 1.0, p, None, None, None) == -1
    assert lib.gv_loss_grad(2, 4, 8, None, p, p, p, 1.0, p, None, None, None) == -1
    assert lib.gv_loss_grad(2, 4, 8, p, p, p, p, 0.0, p, None, None, None) == -1
    assert lib.gv_loss_grad(2, 4, 8, p, p, p, p, float("nan"), p, None, None, None) == -1
    assert lib.gv_moments(p, 10, 8, None, 2, p, None) == -1
    assert lib.gv_moments(p, 10, 0, None, 1, p, None) == -1
    assert lib.gv_moments(p, 10, 8, None, 1, None, None) == -1
    assert lib.gv_tags(None, p, 10, p, None) == -4
