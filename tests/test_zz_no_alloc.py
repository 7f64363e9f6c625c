"""gv_search_noalloc (the search with its scratch in a fixed per-device array)
through the C ABI: equal bit for bit to gv_search on two calls in a row, the
second with a smaller batch (the array keeps the first call's contents), and a
search larger than the array refused with GV_EINVAL."""
import sys

import numpy as np
import pytest

from helpers import problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_noalloc_search_equals_search():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_22347_amd as gv
    from oracle import gleanvec as G
    _say("[noalloc] setup")
    X, QL, Q = problem(141, 96, 6, 60_000, 3_000, 90)
    om = G.fit(X, QL, 40, 6, seed=4)
    model = gv.model_import(om.mu, om.A, om.B)
    Xd = torch.from_numpy(X).cuda()
    cap = gv.search_noalloc_capacity()
    assert cap == 64 << 20
    for fmt, kappa in (("fp16", 100), ("fp8", 60)):
        idx = gv.encode(model, Xd, fmt)
        for m in (90, 7):   # the second call is smaller and reuses the array
            _say(f"[noalloc] {fmt} m={m} kappa={kappa}")
            Qd = torch.from_numpy(Q[:m]).cuda()
            ids = torch.full((m, 10), -5, dtype=torch.int32, device="cuda")
            sc = torch.full((m, 10), -5.0, dtype=torch.float32, device="cuda")
            gv.search_noalloc_into(model, idx, Qd, 10, kappa, ids, sc)
            ref_ids, ref_sc = gv.search(model, idx, Qd, 10, kappa)
            torch.cuda.synchronize()
            assert torch.equal(ids, ref_ids) and torch.equal(sc, ref_sc)
        # more scratch than the array holds: refused before any device work
        big = torch.zeros((20_000, X.shape[1]), dtype=torch.float32, device="cuda")
        out = torch.empty((20_000, 10), dtype=torch.int32, device="cuda")
        with pytest.raises(gv.GleanVecError) as e:
            gv.search_noalloc_into(model, idx, big, 10, kappa, out)
        assert e.value.status == -1
        del idx
