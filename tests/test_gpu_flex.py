"""Flexible reduced dimension (Section 3.3) on the GPU, through the C ABI: an
index stores d coordinates per vector; searches score a leading d_search of
them, chosen per call, and rerank either from the full-dimension vectors or
from the stored ones.  Every stage is checked against the oracle's
search_flex on the same seeded inputs."""
import sys

import numpy as np
import pytest

from helpers import (U32, check_final_topk, check_topk_sets, exact_scores, oracle_model, problem,
                     reduced_score_tolerance)
from oracle import formats
from oracle import gleanvec as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (cfg, D, J, n, m_learn, d stored, C, m, kappa)
CASE = (111, 64, 4, 20_000, 2_000, 48, 4, 37, 60)


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


def _setup(gv, fmt, case=CASE, copy_X=False):
    cfg, D, J, n, ml, d, C, m, kappa = case
    X, QL, Q = problem(cfg, D, J, n, ml, m)
    om = oracle_model(cfg, D, J, n, ml, d, C, 9)
    oi = G.encode(om.mu, om.B, X, fmt)
    model = gv.model_import(om.mu, om.A, om.B)
    Xd = dev(X)
    idx = gv.encode(model, Xd, fmt, copy_X=copy_X)
    return X, Q, om, oi, model, idx, Xd, kappa


def _rerank_tol(oi, qc, cand, qi):
    """bound of the FP64-accumulated stored rerank against the oracle: FP32 rounding of q_c
    (one ulp per coordinate, both sides round the same FP64 sum) is the only gap."""
    pos_of = np.empty(oi.ids.shape[0], np.int64); pos_of[oi.ids] = np.arange(oi.ids.shape[0])
    out = np.empty(cand.shape[0])
    for r, i in enumerate(cand):
        c = oi.tags[i]
        out[r] = 4 * U32 * float(np.abs(qc[qi, c]) @ np.abs(oi.xq[pos_of[i]] * oi.scale[c])) + 1e-30
    return out


@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16", "fp8"])
@pytest.mark.parametrize("d_search", [16, 32, 48])
def test_flex_stages_match_oracle(gv, fmt, d_search):
    _say(f"[flex stages] {fmt} d_search={d_search}")
    X, Q, om, oi, model, idx, Xd, kappa = _setup(gv, fmt)
    out = G.search_flex(oi, om.A, Q, 10, kappa, d_search, "stored")
    qc, t, qhat = gv.project_flex(model, fmt, dev(Q), d_search)
    cid, csc = gv.score_topk_flex(idx, qhat, t, d_search, kappa)
    torch.cuda.synchronize()
    qc_h = qc.cpu().numpy()
    d = om.d
    # S1: q_c over all stored rows (FP64 sums rounded once to FP32), scales from the leading part
    assert np.allclose(qc_h[:, :, :d], out["qc"], rtol=2 ** -23, atol=0)
    assert np.all(qc_h[:, :, d:] == 0)
    assert np.array_equal(t.cpu().numpy(), out["t"]) or np.mean(t.cpu().numpy() == out["t"]) > 0.999
    # S2 + S3 on the leading coordinates
    tol = reduced_score_tolerance(out, oi, gv.padded_dim(d_search))
    n = X.shape[0]
    cid = cid.cpu().numpy(); csc = csc.cpu().numpy()
    flips = 0
    for qi in range(Q.shape[0]):
        by_id = np.empty(n); by_id[oi.ids] = out["scores"][qi]
        tol_id = np.empty(n); tol_id[oi.ids] = tol[qi]
        flips += check_topk_sets(cid[qi], csc[qi], by_id, tol_id, kappa, f"q{qi}")
    assert flips <= max(1, Q.shape[0] // 20)
    # S4 from the stored vectors, on the oracle's candidates
    ocand = out["cand_ids"].astype(np.int32)
    rid, rsc = gv.rerank_stored(idx, qc, dev(ocand), 10)
    torch.cuda.synchronize()
    rid = rid.cpu().numpy(); rsc = rsc.cpu().numpy()
    for qi in range(Q.shape[0]):
        ora = G.rerank_stored(oi, out["qc"], qi, out["cand_ids"][qi])
        tl = _rerank_tol(oi, out["qc"], out["cand_ids"][qi], qi)
        by = dict(zip(out["cand_ids"][qi].tolist(), zip(ora.tolist(), tl.tolist())))
        for i, s in zip(rid[qi].tolist(), rsc[qi].tolist()):
            o, e = by[i]
            assert abs(s - o) <= e + abs(o) * U32, f"q{qi} id {i}: {s} vs {o}"
        kth = out["out_scores"][qi, -1]
        for i in set(rid[qi].tolist()) ^ set(out["ids"][qi].tolist()):
            o, e = by[i]
            assert abs(o - kth) <= 2 * e + abs(kth) * U32, f"q{qi}: id {i} differs away from a tie"


def _verify_flex_search(gv, model, idx, X, Q, oi, om, fmt, kappa, d_search, rerank, what):
    """gv_search_flex against the oracle with every difference proven a near tie: the
    search equals the composition of its stages bit for bit; the GPU's candidates
    pass check_topk_sets against the oracle's leading-coordinate scores; its final
    ids are the rerank top-k of its own candidates, by the oracle's rerank scores
    (full or stored) within their tolerance."""
    out = G.search_flex(oi, om.A, Q, 10, kappa, d_search, rerank)
    Qd = dev(Q)
    ids, sc = gv.search_flex(model, idx, Qd, 10, kappa, d_search, rerank)
    qc, t, qhat = gv.project_flex(model, fmt, Qd, d_search)
    cid, csc = gv.score_topk_flex(idx, qhat, t, d_search, kappa)
    if rerank == "stored":
        rid, rsc = gv.rerank_stored(idx, qc, cid, 10)
    else:
        rid, rsc = gv.rerank(idx, Qd, cid, 10)
    torch.cuda.synchronize()
    assert torch.equal(ids, rid) and torch.equal(sc, rsc), f"{what}: search differs from its stages"
    ids = ids.cpu().numpy(); sc = sc.cpu().numpy(); cid = cid.cpu().numpy(); csc = csc.cpu().numpy()
    tol = reduced_score_tolerance(out, oi, gv.padded_dim(d_search))
    n = X.shape[0]
    agree = 0
    for qi in range(Q.shape[0]):
        by_id = np.empty(n); by_id[oi.ids] = out["scores"][qi]
        tol_id = np.empty(n); tol_id[oi.ids] = tol[qi]
        check_topk_sets(cid[qi], csc[qi], by_id, tol_id, kappa, f"{what} q{qi}")
        if rerank == "stored":
            fs = G.rerank_stored(oi, out["qc"], qi, cid[qi].astype(np.int64))
            ft = _rerank_tol(oi, out["qc"], cid[qi].astype(np.int64), qi) + np.abs(fs) * U32
        else:
            fs, ft = exact_scores(X, Q[qi], cid[qi])
        check_final_topk(ids[qi], cid[qi], fs, ft, 10, f"{what} q{qi}")
        by = dict(zip(cid[qi].tolist(), zip(fs.tolist(), ft.tolist())))
        for i, v in zip(ids[qi].tolist(), sc[qi].tolist()):
            o, e = by[i]
            assert abs(v - o) <= e + abs(o) * U32, f"{what} q{qi} id {i}: {v} vs {o}"
        agree += ids[qi].tolist() == out["ids"][qi].tolist()
    return agree


@pytest.mark.parametrize("fmt", ["fp16", "fp8"])
@pytest.mark.parametrize("rerank", ["full", "stored"])
def test_flex_search_matches_oracle(gv, fmt, rerank):
    _say(f"[flex search] {fmt} {rerank}")
    X, Q, om, oi, model, idx, Xd, kappa = _setup(gv, fmt, copy_X="none" if rerank == "stored" else False)
    for d_search in (16, 48):
        agree = _verify_flex_search(gv, model, idx, X, Q, oi, om, fmt, kappa, d_search, rerank,
                                    f"d_search={d_search}")
        _say(f"[flex search] d_search={d_search}: {agree}/{Q.shape[0]} equal the oracle, the rest near ties")


def test_flex_full_dimension_stored_rerank_is_exact(gv):
    """d = D, FP32 storage, no copy of X: the stored rerank gives the exact inner
    products (Section 3.3), so the result is the exact top-k where the k-th gap is wide."""
    case = (112, 32, 3, 8_000, 1_000, 32, 2, 20, 40)
    _say("[flex exact] d = D fp32")
    X, Q, om, oi, model, idx, Xd, kappa = _setup(gv, "fp32", case, copy_X="none")
    ids, sc = gv.search_flex(model, idx, dev(Q), 10, kappa, 16, "stored")
    torch.cuda.synchronize()
    gt, gs = G.exact_topk(X, Q, 11)
    ids = ids.cpu().numpy(); sc = sc.cpu().numpy()
    checked = 0
    for qi in range(Q.shape[0]):
        if gs[qi, 9] - gs[qi, 10] > 1e-4 * abs(gs[qi, 0]):
            cand = set(G.search_flex(oi, om.A, Q[qi:qi + 1], 10, kappa, 16, "stored")["cand_ids"][0].tolist())
            if set(gt[qi, :10].tolist()) <= cand:
                assert set(ids[qi].tolist()) == set(gt[qi, :10].tolist())
                assert np.allclose(np.sort(sc[qi])[::-1], gs[qi, :10], rtol=1e-5, atol=1e-5 * abs(gs[qi, 0]))
                checked += 1
    assert checked >= 5


def test_flex_index_wider_than_the_scan(gv):
    """d = 288 stored coordinates, more than the scan reads: the plain search refuses,
    the flexible search reads a leading part of at most 256."""
    case = (113, 320, 3, 6_000, 1_500, 288, 2, 9, 40)
    _say("[flex wide] d = 288 fp16")
    X, Q, om, oi, model, idx, Xd, kappa = _setup(gv, "fp16", case)
    with pytest.raises(gv.GleanVecError):
        gv.search(model, idx, dev(Q), 10, kappa)
    for d_search in (160, 256):
        _verify_flex_search(gv, model, idx, X, Q, oi, om, "fp16", kappa, d_search, "stored", f"d_search={d_search}")
    with pytest.raises(gv.GleanVecError):
        gv.search_flex(model, idx, dev(Q), 10, kappa, 288, "stored")


def test_flex_argument_errors(gv):
    X, Q, om, oi, model, idx, Xd, kappa = _setup(gv, "fp16", copy_X="none")
    Qd = dev(Q)
    for bad in (0, om.d + 1):
        with pytest.raises(gv.GleanVecError):
            gv.search_flex(model, idx, Qd, 10, kappa, bad, "stored")
    with pytest.raises(gv.GleanVecError):  # the index keeps no X
        gv.search_flex(model, idx, Qd, 10, kappa, 16, "full")
    with pytest.raises(gv.GleanVecError):
        gv.search(model, idx, Qd, 10, kappa)
