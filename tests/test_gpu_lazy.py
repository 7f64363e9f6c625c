"""The lazy inner product (Algorithm 3) on the GPU: gv_search_lazy projects each
visited cluster's view inside the scan instead of in an S1 pass.  Its results
must equal the eager search's bit for bit (same arithmetic, made elsewhere),
and the eager search passes the oracle parity of verify_search on the same
inputs.  Unsupported shapes are refused."""
import sys

import numpy as np
import pytest

from helpers import oracle_model, problem, verify_search
from oracle import gleanvec as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_22347_amd as lib
    return lib


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


# d = 160 (the padded length the lazy kernel is built for); n large enough for a cascade
CASE = (171, 192, 6, 160_000, 3_000, 160, 6)


@pytest.mark.parametrize("m", [1, 5, 16])
def test_lazy_equals_eager_and_oracle(gv, m):
    cfg, D, J, n, ml, d, C = CASE
    _say(f"[lazy] m={m}")
    X, QL, Q = problem(cfg, D, J, n, ml, 16)
    Q = Q[:m]
    om = oracle_model(cfg, D, J, n, ml, d, C, 7)
    model = gv.model_import(om.mu, om.A, om.B)
    idx = gv.encode(model, dev(X), "fp16")
    Qd = dev(Q)
    for kappa in (50, 200):
        a_ids, a_sc = gv.search(model, idx, Qd, 10, kappa)
        l_ids, l_sc = gv.search_lazy(model, idx, Qd, 10, kappa)
        torch.cuda.synchronize()
        assert torch.equal(a_ids, l_ids) and torch.equal(a_sc, l_sc), f"kappa={kappa}"
    oi = G.encode(om.mu, om.B, X, "fp16")
    if np.array_equal(idx.export()["tags"], oi.tags):
        out = G.search(oi, om.A, Q, 10, 200)
        verify_search(gv, model, idx, X, Q, oi, out, 200, 10, "fp16", f"lazy m={m}")


def test_lazy_refuses_unsupported_shapes(gv):
    cfg, D, J, n, ml, d, C = CASE
    X, QL, Q = problem(cfg, D, J, n, ml, 40)
    om = oracle_model(cfg, D, J, n, ml, d, C, 7)
    model = gv.model_import(om.mu, om.A, om.B)
    idx8 = gv.encode(model, dev(X), "fp8")
    with pytest.raises(gv.GleanVecError):
        gv.search_lazy(model, idx8, dev(Q[:1]), 10, 50)      # not FP16
    idx = gv.encode(model, dev(X), "fp16")
    with pytest.raises(gv.GleanVecError):
        gv.search_lazy(model, idx, dev(Q[:17]), 10, 50)     # m > 16
