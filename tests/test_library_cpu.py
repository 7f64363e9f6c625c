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


def test_host_eigensolver_reports_nonconvergence():
    """A step budget too small to deflate every off-diagonal entry is reported as
    GV_ENOCONV (the fit then fails instead of returning unconverged projections);
    the default budget converges on the same matrix."""
    import paper_2410_22347_amd as gv
    rng = np.random.default_rng(9)
    M = rng.standard_normal((48, 48))
    A = M @ M.T
    gv.eig_step_limit(3)
    try:
        with pytest.raises(gv.GleanVecError) as e:
            gv.host_eigh(A)
        assert e.value.status == -7
    finally:
        gv.eig_step_limit(0)
    lam, Vt = gv.host_eigh(A)
    assert np.allclose(A @ Vt.T, Vt.T * lam, atol=1e-10 * lam[0])
    assert gv._lib.gv_eig_step_limit(-1) == -1


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
    assert lib.gv_search_tuning(0, 0, 50) == -1
    assert lib.gv_search_tuning(5000, 0, 0) == -1
    assert lib.gv_search_tuning(0, 0, 0) == 0
    assert lib.gv_search_optimism(-2) == -1
    assert lib.gv_search_optimism(3) == 0 and lib.gv_search_optimism(-1) == 0 and lib.gv_search_optimism(0) == 0
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


class _ScanLevel(ctypes.Structure):
    _fields_ = [("stride", ctypes.c_int64), ("rows_per_level", ctypes.c_int64), ("query_blocks", ctypes.c_int64),
                ("dense", ctypes.c_int32), ("ranges", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("queries_per_wave", ctypes.c_int32), ("shared", ctypes.c_int32), ("xcd_map", ctypes.c_int32),
                ("tile_ring", ctypes.c_int32), ("workgroups_per_cu", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("staging", ctypes.c_int32), ("list_cap", ctypes.c_int32),
                ("list_limit", ctypes.c_int32)]


def _plan(lib, n, n_pad, C, fmt, d, ds, m, kappa):
    lv = (_ScanLevel * 8)()
    nl, keys, ws = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
    st = lib.gv_scan_plan(n, n_pad, C, fmt, d, ds, m, kappa, ctypes.cast(lv, ctypes.c_void_p), 8,
                          ctypes.byref(nl), ctypes.byref(keys), ctypes.byref(ws))
    return st, [lv[i] for i in range(nl.value)], keys.value, ws.value


def test_scan_plan_invariants():
    """The launch plans of S2/S3 over a grid of batch sizes, database sizes, cluster
    counts, kappa, reduced lengths, formats and tuning overrides keep the invariants
    the kernels rely on (two GPU faults of the scan came from launches that broke
    them: candidate scratch sized without a cascade, and compaction staging smaller
    than a list):
      * the scratch holds m x R x cap list slots for every filtering level, fewer
        than 2^32 of them;
      * a list checked every U tiles, compacted above list_limit, never outgrows
        its slots or the wavefront's LDS staging: list_limit + 32 (U + 1) <= min(cap, staging);
      * a compaction to the kappa best leaves room: list_limit > kappa;
      * without overrides every kappa <= 1024 is served for batches up to 4096;
      * the grid covers every (query block, range) work item exactly;
      * the cascade's dense sample comes first, the full scan last, strides nested."""
    import paper_2410_22347_amd as gv
    lib = gv._lib
    checked = refused = 0
    tunings = [(0, 0, 0), (24, 0, 0), (1, 0, 0), (4, 0, 640), (0, 64, 0), (0, 128, 0), (0, 32, 1024), (0, 0, 320)]
    for splits, qpw, cap in tunings:
        assert lib.gv_search_tuning(splits, qpw, cap) == 0
        try:
            for n in (40, 5_000, 300_000, 10_000_000, 60_000_000):
                for C in (1, 8, 32, 255):
                    n_pad = (n + 31 * C) // 32 * 32   # every segment padded: the most tiles
                    for d in (16, 40, 160, 256):
                        for fmt in (0, 1, 2, 3):
                            for m in (1, 33, 64, 65, 600, 4096, 20_000):
                                for kappa in (1, 50, 200, 256, 800, 1024):
                                    if kappa > n:
                                        continue
                                    st, lv, keys, ws = _plan(lib, n, n_pad, C, fmt, d, 0, m, kappa)
                                    if st != 0:
                                        assert st in (-6, -1), st
                                        # the automatic shapes serve every kappa <= 1024 for
                                        # batches whose lists fit the 32-bit slot space
                                        assert (splits, qpw, cap) != (0, 0, 0) or m > 4096, (n, C, d, fmt, m, kappa)
                                        refused += 1
                                        continue
                                    checked += 1
                                    assert lv[-1].stride == 1 and not lv[-1].dense
                                    for a, b in zip(lv[:-1], lv[1:]):
                                        assert a.stride % b.stride == 0 and a.stride > b.stride
                                    assert all(not x.dense for x in lv[1:])
                                    assert keys < 2 ** 32
                                    for x in lv:
                                        nb = x.queries_per_wave // 32
                                        assert x.query_blocks == -(-m // x.queries_per_wave)
                                        if x.shared:
                                            assert x.ranges % 4 == 0 and x.grid == x.query_blocks * x.ranges // 4
                                        else:
                                            assert x.grid == -(-x.query_blocks // 4) * x.ranges
                                            assert not x.xcd_map or x.ranges % 8 == 0
                                        assert 1 <= x.ranges <= 4096
                                        if x.dense:
                                            continue
                                        assert keys >= m * x.ranges * x.list_cap
                                        assert x.list_limit + 32 * (x.check_every + 1) <= min(x.list_cap, x.staging)
                                        assert x.list_limit > kappa
                                        assert nb in (1, 2, 4)
                                    assert ws >= 8 * keys
        finally:
            lib.gv_search_tuning(0, 0, 0)
    assert checked > 10_000 and refused < checked


def test_tuning_table_file_round_trip(tmp_path):
    """The autotuner's table as a text file: lines written by hand load, their
    shape classes look up (batch and size classes as documented), a malformed line
    is refused, and the saved table reads back the same."""
    import paper_2410_22347_amd as gv
    gv.tuning_table_clear()
    p = tmp_path / "tune.txt"
    p.write_text("# fmt d_pad batch_class size_class splits qpw cap ms\n"
                 "1 160 5 23 64 64 0 14.5\n"
                 "2 64 0 20 0 32 768 0.5\n")
    gv.tuning_table_load(str(p))
    assert gv.tuning_lookup("fp16", 160, 4096, 10_000_000) == (64, 64, 0)   # 2^23 <= 1e7 < 2^24
    assert gv.tuning_lookup("fp16", 160, 4000, 9_000_000) == (64, 64, 0)    # same classes
    assert gv.tuning_lookup("fp16", 160, 5000, 10_000_000) is None          # batch class 6
    assert gv.tuning_lookup("bf16", 64, 1, 1_500_000) == (0, 32, 768)
    q = tmp_path / "again.txt"
    gv.tuning_table_save(str(q))
    gv.tuning_table_clear()
    assert gv.tuning_lookup("bf16", 64, 1, 1_500_000) is None
    gv.tuning_table_load(str(q))
    assert gv.tuning_lookup("fp16", 160, 4096, 10_000_000) == (64, 64, 0)
    bad = tmp_path / "bad.txt"
    bad.write_text("1 160 5 23 64 48 0 1.0\n")                              # qpw 48 is not a shape
    with pytest.raises(gv.GleanVecError):
        gv.tuning_table_load(str(bad))
    gv.tuning_table_clear()
