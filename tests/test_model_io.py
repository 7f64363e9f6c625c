"""Model files (gv_model_save / gv_model_load / gv_model_file_info).

CPU: files written here from the documented layout, independently of the
library's writer, pass its validation; corrupt, truncated, foreign and
other-version files are refused with the documented status.  GPU: a fitted
model saved and loaded again gives back every value bit for bit, saving the
loaded model reproduces the file byte for byte, and searches with both models
agree bit for bit."""
import ctypes
import os
import struct
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2410_22347_amd", "libgleanvec.so")


def _fnv1a(b: bytes) -> int:
    h = 0xcbf29ce484222325
    for x in b:
        h ^= x
        h = (h * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def _write_model_file(path, C, d, D, stats, version=1, rng=None):
    """A model file from the layout stated in gleanvec.h (little-endian)."""
    rng = rng or np.random.default_rng(0)
    body = b"GLEANVEC" + struct.pack("<II", version, 1 if stats else 0) + struct.pack("<iiii", C, d, D, 7)
    for shape in [(C, D), (C, d, D), (C, d, D)]:
        body += rng.standard_normal(shape).astype("<f8").tobytes()
    if stats:
        for shape in [(D, D), (C, D, D), (D,), (C, D), (D, D), (D, D), (C, d, D)]:
            body += rng.standard_normal(shape).astype("<f8").tobytes()
        body += np.arange(C, dtype="<i8").tobytes() + np.zeros(C, np.uint8).tobytes()
    body += struct.pack("<Q", _fnv1a(body))
    with open(path, "wb") as f:
        f.write(body)
    return body


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgleanvec.so not built")
@pytest.mark.parametrize("stats", [False, True])
def test_model_file_validation(tmp_path, stats):
    import paper_2410_22347_amd as gv
    p = str(tmp_path / "m.gv")
    body = _write_model_file(p, 3, 4, 6, stats)
    assert gv.model_file_info(p) == (3, 4, 6, stats)

    def status_of(data):
        q = str(tmp_path / "bad.gv")
        with open(q, "wb") as f:
            f.write(data)
        C = ctypes.c_int32()
        return gv._lib.gv_model_file_info(os.fsencode(q), ctypes.byref(C), None, None, None)

    flipped = bytearray(body)
    flipped[60] ^= 1                                   # one bit of mu
    assert status_of(bytes(flipped)) == -1             # checksum mismatch
    assert status_of(body[:-9]) == -1                  # truncated
    assert status_of(b"NOTAMODL" + body[8:]) == -1     # magic
    other = str(tmp_path / "v2.gv")
    _write_model_file(other, 3, 4, 6, stats, version=2)
    assert gv._lib.gv_model_file_info(os.fsencode(other), None, None, None, None) == -6
    bad_shape = str(tmp_path / "shape.gv")
    _write_model_file(bad_shape, 3, 7, 6, stats)       # d > D
    assert gv._lib.gv_model_file_info(os.fsencode(bad_shape), None, None, None, None) == -1
    assert gv._lib.gv_model_file_info(os.fsencode(str(tmp_path / "missing.gv")), None, None, None, None) == -1
    assert gv._lib.gv_model_file_info(None, None, None, None, None) == -1
    assert gv._lib.gv_model_save(None, os.fsencode(p)) == -4


@pytest.mark.gpu
def test_model_round_trip_on_gpu(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_22347_amd as gv
    from helpers import problem
    print("[model io] fit, save, load", flush=True)
    sys.stdout.flush()
    X, QL, Q = problem(131, 64, 4, 20_000, 2_000, 33)
    Xd, QLd, Qd = (torch.from_numpy(a).cuda() for a in (X, QL, Q))
    model = gv.fit(Xd, QLd, 24, 4, seed=5)
    p = str(tmp_path / "fit.gv")
    model.save(p)
    assert gv.model_file_info(p) == (4, 24, 64, True)
    back = gv.model_load(p)
    for a, b in zip(model.export(), back.export()):
        assert np.array_equal(a, b)
    s0, s1 = model.stats(), back.stats()
    for key in s0:
        assert np.array_equal(s0[key], s1[key]), key
    for a, b in zip(model.sphering(), back.sphering()):
        assert np.array_equal(a, b)
    W, Wp, P = model.sphering()
    _, A, B = model.export()
    assert np.allclose(W @ W, s0["KQ"], rtol=0, atol=1e-10 * np.abs(s0["KQ"]).max())
    assert np.allclose(np.einsum("cjD,DE->cjE", P, W), B, rtol=0, atol=1e-12 * np.abs(B).max())
    # the loaded model writes the same bytes
    p2 = str(tmp_path / "again.gv")
    back.save(p2)
    assert open(p, "rb").read() == open(p2, "rb").read()
    # searches agree bit for bit
    for fmt in ("fp16", "fp8"):
        i0 = gv.encode(model, Xd, fmt)
        i1 = gv.encode(back, Xd, fmt)
        a0 = gv.search(model, i0, Qd, 10, 50)
        a1 = gv.search(back, i1, Qd, 10, 50)
        torch.cuda.synchronize()
        assert torch.equal(a0[0], a1[0]) and torch.equal(a0[1], a1[1])
    # an imported model keeps no statistics: the file says so and stats stay unsupported
    imp = gv.model_import(*model.export())
    p3 = str(tmp_path / "imp.gv")
    imp.save(p3)
    assert gv.model_file_info(p3) == (4, 24, 64, False)
    back3 = gv.model_load(p3)
    for a, b in zip(imp.export(), back3.export()):
        assert np.array_equal(a, b)
    with pytest.raises(gv.GleanVecError):
        back3.stats()
