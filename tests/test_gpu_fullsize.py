"""Parity at the benchmark's full size and launch configuration: 10M x 768 rows,
C = 32, d = 160, kappa = 200, fp16 storage, one batch of 4096 queries (the same
data, batch and launch shapes bench.py times).  The oracle fits its own model on
a subsample of the learn rows; the GPU imports that model, encodes all 10M rows
and searches the whole batch; sampled queries are then checked one by one
against the oracle's encode and search of the same rows: stored bits on sampled
rows, top-kappa sets and scores (within the derived tolerance), and the final
top-10 as the rerank of the GPU's own candidates -- every difference from the
oracle proven a near tie."""
import sys

import numpy as np
import pytest

import synth
from helpers import check_final_topk, check_topk_sets, decode_stored, exact_scores, reduced_score_tolerance
from oracle import gleanvec as G

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(1500)
def test_full_size_sampled_queries():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_22347_amd as gv
    wl = synth.WORKLOADS["mix32-10m-d768"]
    fmt, m, k = "fp16", 4096, 10
    dev = torch.device("cuda:0")
    _say("[fullsize] drawing data")
    geom = synth.make_geometry(wl.cfg, wl.D, wl.J, wl.law)
    Xd = synth.draw_torch(geom, wl.n, synth.S_DB, dev)
    Qd = synth.draw_torch(geom, wl.m_test, synth.S_QTEST, dev, queries_=True)[:m].contiguous()
    QLd = synth.draw_torch(geom, wl.m_learn, synth.S_QLEARN, dev, queries_=True)
    X = Xd.cpu().numpy()
    Q = Qd.cpu().numpy()
    QL = QLd.cpu().numpy()
    del QLd
    rows = synth.learn_rows(wl.n, 200_000, wl.cfg)
    _say("[fullsize] oracle fit")
    om = G.fit(X[rows], QL[:2000], wl.d, wl.C, seed=synth.fit_seed(wl.cfg))
    _say("[fullsize] GPU encode + search (bench launch shapes)")
    model = gv.model_import(om.mu, om.A, om.B)
    idx = gv.encode(model, Xd, fmt)
    _, t, qhat = gv.project(model, fmt, Qd, want_qc=False)
    cid, csc = gv.score_topk(idx, qhat, t, wl.kappa)
    ids, sc = gv.search(model, idx, Qd, k, wl.kappa)
    rid, rsc = gv.rerank(idx, Qd, cid, k)
    torch.cuda.synchronize()
    # the search is the composition of its stages, bit for bit
    assert torch.equal(ids, rid) and torch.equal(sc, rsc)
    del rid, rsc
    cid = cid.cpu().numpy(); csc = csc.cpu().numpy(); ids = ids.cpu().numpy(); sc = sc.cpu().numpy()
    ex = idx.export()
    del idx, Xd
    torch.cuda.empty_cache()

    _say("[fullsize] oracle encode")
    oi = G.encode(om.mu, om.B, X, fmt)
    # stored bits and grouping on sampled rows
    assert np.array_equal(ex["offsets"], oi.offsets) or (ex["tags"] != oi.tags).sum() <= 4
    rng = np.random.default_rng(3)
    same_tags = ex["tags"] == oi.tags
    assert same_tags.mean() > 0.99999
    if np.array_equal(ex["offsets"], oi.offsets):
        pos = rng.choice(wl.n, 200_000, replace=False)
        got = decode_stored(fmt, ex["xlow"][pos])[:, :wl.d]
        assert (got == oi.xq[pos]).mean() > 0.9999
    del ex

    # 32 sampled queries: the first and last of the batch, the rest seeded
    sample = sorted({0, m - 1, *np.random.default_rng(11).choice(m, 30, replace=False).tolist()})
    _say(f"[fullsize] oracle S1-S3 of {len(sample)} sampled queries")
    qc, t, qh = G.project_queries(om.A, Q[sample], fmt)
    S = G.reduced_scores(oi, t, qh)
    tol = reduced_score_tolerance({"qh": qh, "t": t, "scores": S}, oi, 160)
    near = 0
    for j, qi in enumerate(sample):
        by_id = np.empty(wl.n); by_id[oi.ids] = S[j]
        tol_id = np.empty(wl.n); tol_id[oi.ids] = tol[j]
        near += check_topk_sets(cid[qi], csc[qi], by_id, tol_id, wl.kappa, f"q{qi}")
        ex, tl = exact_scores(X, Q[qi], cid[qi])
        near += check_final_topk(ids[qi], cid[qi], ex, tl, k, f"q{qi}")
        exi, _ = exact_scores(X, Q[qi], ids[qi])
        assert np.allclose(sc[qi], exi.astype(np.float32), rtol=2 ** -23, atol=0)
    _say(f"[fullsize] {len(sample)} sampled queries verified ({near} proven near-tie differences)")
