"""Streaming updates (Section 3, streaming vector search) on the GPU through the
C ABI: second-moment sums updated by inserting and removing vectors, the
projections recomputed from the kept statistics, and a search on the updated
index, each against the oracle."""
import sys

import numpy as np
import pytest

from helpers import problem, verify_search
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


def _stream_case():
    X, QL, Q = problem(131, 64, 4, 16_000, 2_000, 30)
    X0, ins = X[:12_000], X[12_000:]
    rng = np.random.default_rng(131)
    rm = np.sort(rng.choice(12_000, 2_500, replace=False))
    keep = np.setdiff1d(np.arange(12_000), rm)
    Xf = np.concatenate([X0[keep], ins])
    return X0, ins, rm, Xf, QL, Q


def test_moments_update_matches_oracle(gv):
    _say("[streaming] moment updates")
    X0, ins, rm, Xf, QL, Q = _stream_case()
    om = G.fit(X0, QL, 24, 4, seed=5)
    model = gv.model_import(om.mu, om.A, om.B)
    t0 = gv.tags(model, dev(X0))
    tins = gv.tags(model, dev(ins))
    K = gv.moments(dev(X0), t0, C=4)
    gv.moments_update(K, dev(ins), tins, +1)
    gv.moments_update(K, dev(X0[rm]), t0[torch.from_numpy(rm).cuda()].contiguous(), -1)
    Kf = gv.moments(dev(Xf), gv.tags(model, dev(Xf)), C=4)
    torch.cuda.synchronize()
    K = K.cpu().numpy(); Kf = Kf.cpu().numpy()
    ta = G.assign(X0.astype(np.float64), om.mu); tb = G.assign(ins.astype(np.float64), om.mu)
    K0 = np.stack([G.second_moment(X0[ta == c], mean=False) for c in range(4)])
    want = G.update_moments(G.update_moments(K0, ins, tb, +1), X0[rm], ta[rm], -1)
    scale = np.abs(want).max()
    assert np.allclose(K, want, rtol=0, atol=1e-11 * scale)
    assert np.allclose(K, Kf, rtol=0, atol=1e-11 * scale)
    with pytest.raises(gv.GleanVecError):
        gv.moments_update(torch.from_numpy(K).cuda(), dev(ins), tins, 0)


def test_fit_from_stats_matches_oracle(gv):
    _say("[streaming] refit from statistics")
    X0, ins, rm, Xf, QL, Q = _stream_case()
    om = G.fit(X0, QL, 24, 4, seed=5)
    model = gv.model_import(om.mu, om.A, om.B)
    tf = gv.tags(model, dev(Xf))
    KX = gv.moments(dev(Xf), tf, C=4)
    KQ = gv.moments(dev(QL), None, C=1)[0].contiguous()
    counts = np.bincount(tf.cpu().numpy(), minlength=4)
    new = gv.fit_from_stats(om.mu, KQ, QL.shape[0], KX, counts, 24)
    mu, A, B = new.export()
    st = new.stats()
    ta = G.assign(Xf.astype(np.float64), om.mu)
    assert np.array_equal(counts, np.bincount(ta, minlength=4))
    KXo = np.stack([G.second_moment(Xf[ta == c], mean=False) for c in range(4)])
    ref = G.fit_from_stats(om.mu, G.second_moment(QL, mean=False), QL.shape[0], KXo, counts, 24)
    assert np.array_equal(mu, om.mu)
    assert np.allclose(st["KQ"], ref.KQ, rtol=0, atol=1e-12 * np.abs(ref.KQ).max())
    for c in range(4):
        lam = ref.lam_c[c]
        assert np.allclose(st["lam_c"][c], lam, rtol=0, atol=1e-10 * lam[0])
        assert np.abs(A[c] - ref.A[c]).max() <= 1e-6 * np.abs(ref.A[c]).max()
        assert np.abs(B[c] - ref.B[c]).max() <= 1e-6 * np.abs(ref.B[c]).max()


def test_streaming_refit_then_search(gv):
    """Insert and remove, refit from the updated statistics, re-encode the current set and
    search it: the oracle's refit, encode and search of the same set agree."""
    _say("[streaming] refit, encode, search")
    X0, ins, rm, Xf, QL, Q = _stream_case()
    om = G.fit(X0, QL, 24, 4, seed=5)
    model = gv.model_import(om.mu, om.A, om.B)
    t0 = gv.tags(model, dev(X0))
    K = gv.moments(dev(X0), t0, C=4)
    gv.moments_update(K, dev(ins), gv.tags(model, dev(ins)), +1)
    gv.moments_update(K, dev(X0[rm]), t0[torch.from_numpy(rm).cuda()].contiguous(), -1)
    counts = np.bincount(gv.tags(model, dev(Xf)).cpu().numpy(), minlength=4)
    KQ = gv.moments(dev(QL), None, C=1)[0].contiguous()
    new = gv.fit_from_stats(om.mu, KQ, QL.shape[0], K, counts, 24)
    Xfd = dev(Xf)
    idx = gv.encode(new, Xfd, "fp16")
    ta = G.assign(Xf.astype(np.float64), om.mu)
    KXo = np.stack([G.second_moment(Xf[ta == c], mean=False) for c in range(4)])
    ref = G.fit_from_stats(om.mu, G.second_moment(QL, mean=False), QL.shape[0], KXo, counts, 24)
    for c in range(4):  # the refit agrees with the oracle's (as in the test above)
        _, A, B = new.export()
        assert np.abs(A[c].T @ B[c] - ref.A[c].T @ ref.B[c]).max() <= 1e-6 * np.abs(ref.A[c].T @ ref.B[c]).max()
    # search the GPU's refit model; the oracle encodes and searches with the same
    # (exported) projections, and every difference must be a proven near tie
    mu, A, B = new.export()
    oi = G.encode(mu, B, Xf, "fp16")
    out = G.search(oi, A, Q, 10, 80)
    verify_search(gv, new, idx, Xf, Q, oi, out, 80, 10, "fp16", "refit")
